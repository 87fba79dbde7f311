// rf_poisson_dev.h -- the Poisson leaf (an unbinned Poisson PDF of an
// integer-valued observable n on the integer range [lo, hi] of its
// observable, K = hi - lo + 1 <= 2048 values).  Requires rf_dev.h.
//
//   u(n) = lambda^n e^-lambda / n! = exp(n log(lambda) - lambda - log n!),
//   N = sum over k = lo..hi of u(k)  (the range's probability),
//   d log u / d lambda = n / lambda - 1.
// The observable takes at most K values, so u is a function of lambda alone
// on a table of K entries: the block-wide prologue evaluates u(k) for the
// whole range (FP64, from the host's log k! table in the aux block) into
// LDS and forms N and sum k u(k) with a block-parallel sum in a fixed order.
// An event's value is a table read.  The table stays FP64 in both kernel
// precisions: the FP32 kernel's FP64 re-evaluation of events with tiny p
// reads the same table.
// Constants:
//   C[0] = 1/N, C[1] = d log N / d lambda + 1 = sum k u(k) / (lambda N),
//   C[2] = log lambda, C[3] = lambda, C[4] = 1/lambda.
// The derivative output is the event part n (factor C[4]); the -1 of
// d log u / d lambda is carried by C[1].  Without RF_VALIDATE an event off
// the integer range (or not an integer) reads the entry of its clamped,
// truncated count, and its derivative part is that same count.
#pragma once

enum { POISSON_NC = 5, POISSON_KMAX = 2048 };

template <int BS>
__device__ void poisson_prologue(const double* in, int lo, int K, const double* lf, double* C, double* tab,
                                 double* scratch /* [BS / 64][2] */) {
  const double lam = in[0], ll = ::log(lam);
  double s = 0.0, m = 0.0;
  for (int j = threadIdx.x; j < K; j += BS) {
    const double k = (double)(lo + j);
    const double u = ::exp(k * ll - lam - lf[j]);
    tab[j] = u;
    s += u;
    m += k * u;
  }
  s = wave_sum(s);
  m = wave_sum(m);
  if ((threadIdx.x & 63) == 0) {
    scratch[2 * (threadIdx.x >> 6)] = s;
    scratch[2 * (threadIdx.x >> 6) + 1] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, M = 0.0;
    for (int w = 0; w < BS / 64; ++w) {
      S += scratch[2 * w];
      M += scratch[2 * w + 1];
    }
    C[0] = 1.0 / S;
    C[1] = M / (lam * S);
    C[2] = ll;
    C[3] = lam;
    C[4] = 1.0 / lam;
  }
}

template <typename T> struct PoissonK {
  int lo, kmax;
  const double* tab;  // u(k) for k = lo .. lo + kmax (LDS)
  RF_DEV PoissonK make(const double* C, const double* tab, int lo, int K) {
    (void)C;
    PoissonK k;
    k.lo = lo;
    k.kmax = K - 1;
    k.tab = tab;
    return k;
  }
};

template <typename T> RF_DEV T poisson_eval(T n, const PoissonK<T>& k, T* d) {
  int j = (int)n - k.lo;  // events off the integer range are the caller's error: clamped
  j = j < 0 ? 0 : (j > k.kmax ? k.kmax : j);
  d[0] = (T)(j + k.lo);  // the count whose table entry was read, so the gradient matches the value
  return (T)k.tab[j];
}
