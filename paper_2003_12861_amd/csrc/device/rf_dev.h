// rf_dev.h -- device-side op library for the fused likelihood kernels.
//
// Every compiled model graph becomes one generated HIP source that includes
// this header.  For each PDF leaf the header provides
//   * <op>_prologue(): FP64, run once per workgroup per parameter point.  It
//     evaluates the normalisation integral N over the observable's range and
//     d log N / d(input) -- the parameter-only ("constant") branch that the
//     paper caches once per parameter point (Section 4) -- and the derived
//     constants the per-event code needs.  Layout of the constant block:
//       C[0] = 1/N, C[1..k] = d log N / d(shape input j), C[k+1..] = op data.
//   * <Op>K<T>: the constants as the per-event precision T (float or double),
//     with location-type constants split into hi + lo parts for T = float so
//     that (x - mu) keeps FP64 accuracy when mu is large compared to the
//     spread (e.g. a 5.28 GeV mass with a 3 MeV width).
//   * <op>_eval<T>(): per-event unnormalised shape u(x) and its derivative
//     with respect to shape input j, without the factors that depend on the
//     parameters only (those multiply the event sums once, in FP64, after
//     the reduction).  Most leaves give d log u / d(input) ("log form"); a
//     leaf that is linear in its inputs gives du / d(input) ("linear form"),
//     which needs no division by u.
// The shapes are the textbook PDFs of the batched RooFit work (Gaussian,
// exponential and sums of PDFs, Sections 4.1-4.2) and of the benchmark
// models (Chebyshev polynomial, decay (x) Gaussian resolution, ARGUS,
// Breit-Wigner, Breit-Wigner (x) Crystal Ball convolution, MLP surrogate).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RF_DEV static __device__ __forceinline__

// ------------------------------------------------------------------ math --
template <typename T> struct RM;
template <> struct RM<float> {
  RF_DEV float exp(float x) { return expf(x); }
  RF_DEV float log(float x) { return logf(x); }
  RF_DEV float erfc(float x) { return erfcf(x); }
  RF_DEV float erfcx(float x) { return erfcxf(x); }
  RF_DEV float sqrt(float x) { return sqrtf(x); }
  RF_DEV float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  // hardware square root (one transcendental instruction, ~1 ulp)
  RF_DEV float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
  // log p as accumulated by the event loop: log2 p (hardware instruction);
  // the FP64 flush multiplies the partial sums by ln 2
  RF_DEV float log_acc(float x) { return __builtin_amdgcn_logf(x); }
  RF_DEV bool finite(float x) { return isfinite(x); }
  RF_DEV float tiny() { return 1e-30f; }  // FP32 results below this are redone in FP64
};
// a * b + c as the three-operand FP64 FMA with the addend c -- a polynomial
// coefficient, the same on every lane -- in scalar registers.  Written as
// plain fma() in the large event loops, such steps compile to the
// two-operand form (the addend is also the destination) plus a 64-bit copy
// of the coefficient per step, and the hoisted coefficients hold vector
// registers.
__device__ __forceinline__ double rf_fma3s(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
}

// Natural logarithm in FP64 for the event loop's log p (normal, finite,
// positive x; other values give an unspecified result, which the callers
// discard): x = m 2^e with m in [sqrt(1/2), sqrt(2)), and
//   log x = e ln 2 + 2 atanh(s),  s = (m - 1)/(m + 1),  |s| <= 0.1716,
//   2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^20/21)   (truncation < 3e-17),
// the classical reduction of Cody and Waite ("Software Manual for the
// Elementary Functions", 1980, the logarithm chapter).  m - 1 is exact; s
// comes from the hardware reciprocal with one Newton step and one residual
// correction; ln 2 is split so that e ln2_hi is exact.  Measured against the
// host's correctly rounded log in the tests; it replaces a device-library
// call that costs about three times as many issue cycles.
RF_DEV double rf_log64(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double f = m - 1.0, d = m + 1.0;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  double sv = f * r;
  sv = fma(r, fma(-sv, d, f), sv);
  const double s2 = sv * sv;
  double q = 1.0 / 21.0;
  q = rf_fma3s(q, s2, 1.0 / 19.0);
  q = rf_fma3s(q, s2, 1.0 / 17.0);
  q = rf_fma3s(q, s2, 1.0 / 15.0);
  q = rf_fma3s(q, s2, 1.0 / 13.0);
  q = rf_fma3s(q, s2, 1.0 / 11.0);
  q = rf_fma3s(q, s2, 1.0 / 9.0);
  q = rf_fma3s(q, s2, 1.0 / 7.0);
  q = rf_fma3s(q, s2, 1.0 / 5.0);
  q = rf_fma3s(q, s2, 1.0 / 3.0);
  const double t = 2.0 * sv;
  const double lm = fma(t * s2, q, t);
  const double fe = (double)e;
  return fma(fe, 6.93147180369123816490e-01, fma(fe, 1.90821492927058770002e-10, lm));
}

static constexpr double RF_LOG2E = 1.44269504088896340736;
static constexpr double RF_LN2 = 0.69314718055994530942;
// ln 2 = RF_LN2_HI + RF_LN2_LO with RF_LN2_HI exact to 32 bits (its product
// with an integer below 2^21 is exact: Cody and Waite's split)
static constexpr double RF_LN2_HI = 6.93147180369123816490e-01;
static constexpr double RF_LN2_LO = 1.90821492927058770002e-10;

// The Gaussian's FP64 exponential in the event loop.  e^r for |r| <= ln2/2
// from its Taylor series to r^13 (the first omitted term is below 5e-18 of
// the result), evaluated by Horner's rule with the three-operand FMA and the
// coefficients in scalar registers; the power of two comes from ldexp
// (subnormal results rounded by the hardware).  (For the other leaves'
// general e^x the device library's exp is as short in their loops.)
__device__ __forceinline__ double rf_exp_taylor(double r) {
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = rf_fma3s(p, r, 1.0 / 479001600.0);
  p = rf_fma3s(p, r, 1.0 / 39916800.0);
  p = rf_fma3s(p, r, 1.0 / 3628800.0);
  p = rf_fma3s(p, r, 1.0 / 362880.0);
  p = rf_fma3s(p, r, 1.0 / 40320.0);
  p = rf_fma3s(p, r, 1.0 / 5040.0);
  p = rf_fma3s(p, r, 1.0 / 720.0);
  p = rf_fma3s(p, r, 1.0 / 120.0);
  p = rf_fma3s(p, r, 1.0 / 24.0);
  p = rf_fma3s(p, r, 1.0 / 6.0);
  p = rf_fma3s(p, r, 0.5);
  p = rf_fma3s(p, r, 1.0);
  return rf_fma3s(p, r, 1.0);
}
// 2^t for t <= 0 (the Gaussian's 2^(-q)): t = n + f, n = rint(t), |f| <= 1/2
// exact, 2^f = e^(f ln2); below -1100 the result is 0, NaN stays NaN.
RF_DEV double rf_exp2_neg(double t) {
  const double n = __builtin_rint(t);
  const double f = t - n;
  const double r = fma(f, RF_LN2_HI, f * RF_LN2_LO);
  const double v = __builtin_amdgcn_ldexp(rf_exp_taylor(r), (int)fmax(n, -1100.0));
  return t < -1100.0 ? 0.0 : v;
}

template <> struct RM<double> {
  RF_DEV double exp(double x) { return ::exp(x); }
  RF_DEV double log(double x) { return ::log(x); }
  RF_DEV double erfc(double x) { return ::erfc(x); }
  RF_DEV double erfcx(double x) { return ::erfcx(x); }
  RF_DEV double sqrt(double x) { return ::sqrt(x); }
  RF_DEV double rcp(double x) {
    // hardware estimate (measured on gfx950: within 2^-25 relative) and one
    // Newton step: within 11 ulp (a second step would give 0.5 ulp)
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
  }
  RF_DEV double sqrt_fast(double x) { return ::sqrt(x); }
  RF_DEV double log_acc(double x) { return rf_log64(x); }
  RF_DEV bool finite(double x) { return isfinite(x); }
  RF_DEV double tiny() { return 0.0; }
};

// A location constant: for float its value as hi + lo so that
// sub(x) = (x - hi) - lo keeps the FP64 value of the location.
template <typename T> struct Loc {
  T hi, lo;
  RF_DEV Loc make(double v) {
    Loc l;
    l.hi = (T)v;
    l.lo = (T)(v - (double)l.hi);
    return l;
  }
  __device__ __forceinline__ T sub(T x) const { return (x - hi) - lo; }
};
template <> struct Loc<double> {
  double hi;
  RF_DEV Loc make(double v) {
    Loc l;
    l.hi = v;
    return l;
  }
  __device__ __forceinline__ double sub(double x) const { return x - hi; }
};
// A scale constant for products x*s that must stay accurate when |x*s| is
// large: for float s = hi + lo and x*s ~ fma(x, hi, x*lo).
template <typename T> struct Scl {
  T hi, lo;
  RF_DEV Scl make(double v) {
    Scl s;
    s.hi = (T)v;
    s.lo = (T)(v - (double)s.hi);
    return s;
  }
  __device__ __forceinline__ T mul(T x) const { return fma(x, hi, x * lo); }
};
template <> struct Scl<double> {
  double hi;
  RF_DEV Scl make(double v) {
    Scl s;
    s.hi = v;
    return s;
  }
  __device__ __forceinline__ double mul(double x) const { return x * hi; }
};


// exp(s x) for a parameter-dependent rate s.  In float the rate is held in
// base-2 units, s log2(e) = hi + lo, and the product t = hi x is split
// exactly into t + t_lo with an FMA; 2^t comes from the hardware exp2
// instruction and the small remainder enters to first order,
// exp(s x) = 2^t (1 + ln2 t_lo + extra).  Without the split, an argument
// of -40 (a Gaussian 9 widths out) would carry an absolute rounding of
// 2.4e-6, i.e. that relative error in the result.  extra is an additional
// small correction in natural units (the low part of a squared argument).
template <typename T> struct ExpScl;
template <> struct ExpScl<float> {
  float hi, lo;
  RF_DEV ExpScl make(double s) {
    ExpScl e;
    const double v = s * RF_LOG2E;
    e.hi = (float)v;
    e.lo = (float)(v - (double)e.hi);
    return e;
  }
  __device__ __forceinline__ float exp(float x, float extra = 0.0f) const {
    const float t = hi * x;
    const float t_lo = fma(lo, x, fma(hi, x, -t));
    const float E = __builtin_amdgcn_exp2f(t);
    return fma(E, fma(t_lo, (float)RF_LN2, extra), E);
  }
};
template <> struct ExpScl<double> {
  double hi;
  RF_DEV ExpScl make(double s) {
    ExpScl e;
    e.hi = s;
    return e;
  }
  __device__ __forceinline__ double exp(double x, double extra = 0.0) const { return ::exp(fma(hi, x, extra)); }
};

static constexpr double RF_PI = 3.14159265358979323846;
static constexpr double RF_SQRT2 = 1.41421356237309504880;
static constexpr double RF_SQRTPI = 1.77245385090551602730;
static constexpr double RF_SQRT2PI = 2.50662827463100050242;
static constexpr double RF_INV_SQRT2PI = 0.39894228040143267794;

// ============================================================== Gaussian ==
// u = exp(-(x-mu)^2 / (2 sigma^2)); inputs (mu, sigma).
// N = sigma sqrt(pi/2) [erf(zb) - erf(za)], z = (y - mu)/(sqrt2 sigma);
// dN/dmu = u(lo) - u(hi);  dN/dsigma = (N - (hi-mu) u(hi) + (lo-mu) u(lo)) / sigma.
enum { GAUSS_NC = 5 };
// The same on two lanes of one wavefront (lanes l and l + 32, `upper` true on
// the second): each lane evaluates the error function and the exponential at
// its own end of the range, the partner's values come by a lane exchange, and
// the first lane writes the block -- the two library calls of each kind run
// side by side instead of one after the other (the prologue is on every
// workgroup's path to its event loop).
RF_DEV void gauss_prologue2(const double* in, double lo, double hi, double* C, bool upper) {
  const double mu = in[0], s = in[1];
  const double z = ((upper ? hi : lo) - mu) / (RF_SQRT2 * s);
  // the same branch on both lanes: erfc where the range lies on one side of
  // mu (no cancellation), erf where it straddles mu
  const int kase = lo >= mu ? 0 : (hi <= mu ? 1 : 2);
  const double F = kase == 0 ? ::erfc(z) : (kase == 1 ? ::erfc(-z) : ::erf(z));
  const double e = ::exp(-z * z);
  const double Fo = __shfl_xor(F, 32), eo = __shfl_xor(e, 32);
  if (upper) return;
  const double diff = kase == 0 ? F - Fo : Fo - F;  // F at lo, Fo at hi
  const double N = s * (0.5 * RF_SQRT2PI) * diff;
  const double ea = e, eb = eo;
  C[0] = 1.0 / N;
  C[1] = (ea - eb) / N;
  C[2] = (N - (hi - mu) * eb + (lo - mu) * ea) / (s * N);
  C[3] = mu;
  C[4] = 1.0 / s;
}
RF_DEV void gauss_prologue(const double* in, double lo, double hi, double* C) {
  const double mu = in[0], s = in[1];
  const double za = (lo - mu) / (RF_SQRT2 * s), zb = (hi - mu) / (RF_SQRT2 * s);
  double diff;
  if (za >= 0) diff = ::erfc(za) - ::erfc(zb);
  else if (zb <= 0) diff = ::erfc(-zb) - ::erfc(-za);
  else diff = ::erf(zb) - ::erf(za);
  const double N = s * (0.5 * RF_SQRT2PI) * diff;
  const double ea = ::exp(-za * za), eb = ::exp(-zb * zb);
  C[0] = 1.0 / N;
  C[1] = (ea - eb) / N;
  C[2] = (N - (hi - mu) * eb + (lo - mu) * ea) / (s * N);
  C[3] = mu;
  C[4] = 1.0 / s;
}
// With w = s (x - mu)/sigma, s = 1/sqrt(2 ln 2), the kernel is u = 2^(-w^2).
// In FP32 programs w and q = w^2 are formed in FP64 (one FP64 operation costs
// one FP32 issue slot here) and q is split into an FP32 pair qh + ql: the
// exponent is then exact to far below an FP32 unit, for any mu and sigma
// (an FP32 w would carry a relative error of 2^-24, which 2 q ln2 amplifies
// to several 1e-6 in u at |z| ~ 10).  Log form: d log u/d mu = z/sigma and
// d log u/d sigma = z^2/sigma with z = w/s; the event part is (w, w^2), the
// factors 1/(s sigma) and 1/(s^2 sigma) are applied to the sums.
static constexpr double RF_GW = 0.849321800288019042721502834103;      // 1/sqrt(2 ln 2)
static constexpr double RF_GW_INV = 1.17741002251547469101156932646;   // sqrt(2 ln 2)
static constexpr double RF_GW_INV2 = 1.38629436111989061883446424292;  // 2 ln 2
template <typename T> struct GaussK {
  double mis, is;  // -mu s / sigma and s / sigma
  RF_DEV GaussK load(const double* C) {
    GaussK k;
    k.is = C[4] * RF_GW;
    k.mis = -C[3] * k.is;
    return k;
  }
};
// w = x s/sigma - mu s/sigma in one FP64 FMA (mu s/sigma rounded once, to
// 2^-53 of itself)
template <typename T> RF_DEV T gauss_eval(T x, const GaussK<T>& k, T* d) {
  const double w = fma((double)x, k.is, k.mis);
  const double q = w * w;
  if constexpr (sizeof(T) == 4) {
    const float qh = (float)q;
    const float ql = (float)fma(w, w, -(double)qh);  // w^2 - qh
    d[0] = (float)w;
    d[1] = qh;
    const float E = __builtin_amdgcn_exp2f(-qh);
    return fma(E * ql, -(float)RF_LN2, E);  // 2^(-qh - ql) to first order in ql
  } else {
    d[0] = w;
    d[1] = q;
    const double E = rf_exp2_neg(-q);
    return fma(E * fma(w, w, -q), -RF_LN2, E);
  }
}

// ============================================================= Chebyshev ==
// u = 1 + sum_{k=1..n} c_k T_k(x'), x' = (2x - lo - hi)/(hi - lo); inputs c_1..c_n.
// N = (hi - lo) [1 + sum_{k even} c_k / (1 - k^2)].
template <int NC> RF_DEV void cheb_prologue(const double* in, double lo, double hi, double* C) {
  double s = 1.0;
  for (int k = 1; k <= NC; ++k)
    if ((k & 1) == 0) s += in[k - 1] / (1.0 - (double)(k * k));
  const double N = (hi - lo) * s;
  C[0] = 1.0 / N;
  for (int k = 1; k <= NC; ++k) C[k] = (k & 1) ? 0.0 : 1.0 / ((1.0 - (double)(k * k)) * s);
  C[NC + 1] = 2.0 / (hi - lo);
  C[NC + 2] = -(hi + lo) / (hi - lo);
  for (int k = 1; k <= NC; ++k) C[NC + 2 + k] = in[k - 1];
}
// Evaluated with y = 2x' and the doubled basis T'_k = 2 T_k, which obey
// T'_{k+1} = y T'_k - T'_{k-1} (T'_0 = 2, T'_1 = y): no separate doubling per
// step; y is exactly twice the FP32 x' (scaling by 2 is exact), and
// u = 1 + sum (c_k / 2) T'_k.  Linear form: d[j] = T'_{j+1} = 2 du/dc_{j+1};
// the factor 1/2 is applied to the sums.
template <typename T, int NC> struct ChebK {
  T a, b;      // 2 x (the affine map to [-1, 1])
  T c[NC];     // c_k / 2
  RF_DEV ChebK load(const double* C) {
    ChebK k;
    k.a = (T)(2.0 * C[NC + 1]);
    k.b = (T)(2.0 * C[NC + 2]);
    for (int j = 0; j < NC; ++j) k.c[j] = (T)(0.5 * C[NC + 3 + j]);
    return k;
  }
};
template <typename T, int NC> RF_DEV T cheb_eval(T x, const ChebK<T, NC>& k, T* d) {
  const T y = fma(x, k.a, k.b);
  T tkm = (T)2, tk = y, u = (T)1;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    u = fma(k.c[j], tk, u);
    d[j] = tk;
    const T tn = fma(y, tk, -tkm);
    tkm = tk;
    tk = tn;
  }
  return u;
}

// =========================================================== exponential ==
// form 0: u = exp(-x/tau), input tau;  N = tau e^{-lo/tau} (1 - e^{-(hi-lo)/tau}).
// form 1: u = exp(lam (x - xc)), input lam, xc = range midpoint (keeps u O(1));
//         N' = e^{lam(lo - xc)} expm1(lam (hi - lo)) / lam.
enum { EXP_NC = 5 };
RF_DEV void exp_prologue(const double* in, double lo, double hi, int form, double* C) {
  if (form == 0) {
    const double tau = in[0];
    const double ea = ::exp(-lo / tau), eb = ::exp(-hi / tau);
    const double N = -tau * ea * ::expm1(-(hi - lo) / tau);
    C[0] = 1.0 / N;
    C[1] = ((1.0 + lo / tau) * ea - (1.0 + hi / tau) * eb) / N;
    C[2] = -1.0 / tau;  // rate
    C[3] = 0.0;         // centre
    C[4] = 1.0 / (tau * tau);
  } else {
    const double lam = in[0], xc = 0.5 * (lo + hi);
    const double a = lo - xc, b = hi - xc;
    double N, dN;
    if (::fabs(lam) * (hi - lo) < 1e-8) {
      N = b - a;
      dN = 0.5 * (b * b - a * a);
    } else {
      const double ea = ::exp(lam * a), eb = ::exp(lam * b);
      N = ea * ::expm1(lam * (b - a)) / lam;
      dN = (b * eb - a * ea) / lam - N / lam;
    }
    C[0] = 1.0 / N;
    C[1] = dN / N;
    C[2] = lam;
    C[3] = xc;
    C[4] = 0.0;
  }
}
// Log form.  Form 0: d log u/d tau = x/tau^2 (event part x, factor C[4]);
// form 1: d log u/d lam = x - xc (factor 1).
template <typename T> struct ExpK {
  ExpScl<T> rate;
  Loc<T> xc;
  RF_DEV ExpK load(const double* C) {
    ExpK k;
    k.rate = ExpScl<T>::make(C[2]);
    k.xc = Loc<T>::make(C[3]);
    return k;
  }
};
template <typename T, int FORM> RF_DEV T exp_eval(T x, const ExpK<T>& k, T* d) {
  if (FORM == 0) {
    d[0] = x;
    return k.rate.exp(x);
  }
  const T xs = k.xc.sub(x);
  d[0] = xs;
  return k.rate.exp(xs);
}

// ========================================= decay (x) Gaussian resolution ==
// Single-sided decay exp(-t'/tau), t' >= 0, smeared by a Gaussian of width s
// and mean b.  With u = t - b:
//   F(t) = 1/2 exp(s^2/(2 tau^2) - u/tau) erfc((s^2/tau - u)/(sqrt2 s)),
//   antiderivative A(t) = tau [Phi(u/s) - F(t)],  N = A(hi) - A(lo).
// Inputs (tau, s, b).
enum { DECAY_NC = 12 };
RF_DEV double decay_F(double u, double tau, double s, double* dF) {
  const double w = (s * s / tau - u) / (RF_SQRT2 * s);
  const double G = ::exp(-u * u / (2 * s * s));
  double F;
  if (w > 4.0) F = 0.5 * G * ::erfcx(w);
  else F = 0.5 * ::exp(s * s / (2 * tau * tau) - u / tau) * ::erfc(w);
  dF[0] = F * (u / (tau * tau) - s * s / (tau * tau * tau)) + s * G * RF_INV_SQRT2PI / (tau * tau);
  dF[1] = F * s / (tau * tau) - G * (1.0 / tau + u / (s * s)) * RF_INV_SQRT2PI;
  dF[2] = F / tau - G * RF_INV_SQRT2PI / s;
  return F;
}
RF_DEV double decay_A(double t, double tau, double s, double b, double* dA) {
  const double u = t - b;
  double dF[3];
  const double F = decay_F(u, tau, s, dF);
  const double Phi = 0.5 * ::erfc(-u / (RF_SQRT2 * s));
  const double G = ::exp(-u * u / (2 * s * s));
  dA[0] = Phi - F - tau * dF[0];
  dA[1] = tau * (-u * G * RF_INV_SQRT2PI / (s * s) - dF[1]);
  dA[2] = tau * (-G * RF_INV_SQRT2PI / s - dF[2]);
  return tau * (Phi - F);
}
RF_DEV void decay_prologue(const double* in, double lo, double hi, double* C) {
  const double tau = in[0], s = in[1], b = in[2];
  double dh[3], dl[3];
  const double N = decay_A(hi, tau, s, b, dh) - decay_A(lo, tau, s, b, dl);
  C[0] = 1.0 / N;
  for (int j = 0; j < 3; ++j) C[1 + j] = (dh[j] - dl[j]) / N;
  C[4] = b;                                    // location
  C[5] = -1.0 / tau;                           // exponent slope
  C[6] = s * s / (2 * tau * tau);              // exponent offset
  C[7] = s * s / tau;                          // erfc shift
  C[8] = 1.0 / (RF_SQRT2 * s);                 // erfc scale
  C[9] = -1.0 / (2 * s * s);                   // resolution exponent factor
  C[10] = 1.0 / (tau * tau);
  C[11] = s / (tau * tau);
}
template <typename T> struct DecayK {
  Loc<T> b;
  Scl<T> slope;
  T off, shift, wscale, gfac, itau2, s_tau2, c_tau_s, c_s, c_b, itau, is2;
  RF_DEV DecayK load(const double* C) {
    DecayK k;
    k.b = Loc<T>::make(C[4]);
    k.slope = Scl<T>::make(C[5]);
    k.off = (T)C[6];
    k.shift = (T)C[7];
    k.wscale = (T)C[8];
    k.gfac = (T)C[9];
    k.itau2 = (T)C[10];
    k.s_tau2 = (T)C[11];
    const double s = 1.0 / (RF_SQRT2 * C[8]);
    const double tau = -1.0 / C[5];
    k.itau = (T)(1.0 / tau);
    k.is2 = (T)(1.0 / (s * s));
    k.c_tau_s = (T)(s * RF_INV_SQRT2PI / (tau * tau));  // coefficient of G/F in d/dtau
    k.c_s = (T)RF_INV_SQRT2PI;
    k.c_b = (T)(RF_INV_SQRT2PI / s);
    return k;
  }
};
template <typename T> RF_DEV T decay_eval(T x, const DecayK<T>& k, T* d) {
  const T u = k.b.sub(x);
  const T w = (k.shift - u) * k.wscale;
  const T G = RM<T>::exp(k.gfac * u * u);
  T F;
  if (w > (T)4) F = (T)0.5 * G * RM<T>::erfcx(w);
  else F = (T)0.5 * RM<T>::exp(k.slope.mul(u) + k.off) * RM<T>::erfc(w);
  const T r = F > (T)0 ? G * RM<T>::rcp(F) : (T)0;  // G / F
  // d log F / d(tau, s, b)
  d[0] = (u - k.shift) * k.itau2 + k.c_tau_s * r;
  d[1] = k.s_tau2 - r * (k.itau + u * k.is2) * k.c_s;
  d[2] = k.itau - r * k.c_b;
  return F;
}

// ================================================================= ARGUS ==
// u = m sqrt(U) exp(c U), U = 1 - (m/m0)^2 = (m0 - m)(m0 + m)/m0^2, m < m0;
// inputs (m0 -- must be a constant, c <= 0).  With k = -c:
//   J(U) = int_0^U v^{1/2} e^{-kv} dv,  J3(U) = int_0^U v^{3/2} e^{-kv} dv,
//   N = m0^2/2 [J(U(lo)) - J(U(min(hi, m0)))],  dN/dc = m0^2/2 [J3(U(lo)) - J3(U(top))].
enum { ARGUS_NC = 6 };
RF_DEV void argus_J(double U, double k, double* J, double* J3) {
  if (U <= 0) { *J = 0; *J3 = 0; return; }
  if (k * U < 1.0) {
    // alternating series, fast for kU < 1 where the closed form cancels
    double sJ = 0, sJ3 = 0, term = 1.0, Upow = U * ::sqrt(U);
    for (int n = 0; n < 40; ++n) {
      sJ += term * Upow / (n + 1.5);
      sJ3 += term * Upow * U / (n + 2.5);
      term *= -k * U / (n + 1);
    }
    *J = sJ; *J3 = sJ3;
    return;
  }
  const double sq = ::sqrt(k * U);
  const double e = ::exp(-k * U);
  *J = RF_SQRTPI / (2 * k * ::sqrt(k)) * ::erf(sq) - ::sqrt(U) * e / k;
  *J3 = 1.5 / k * (*J) - U * ::sqrt(U) * e / k;
}
RF_DEV void argus_prologue(const double* in, double lo, double hi, double* C) {
  const double m0 = in[0], c = in[1], k = -c;
  const double top = hi < m0 ? hi : m0;
  const double Ul = (m0 - lo) * (m0 + lo) / (m0 * m0);
  const double Ut = (m0 - top) * (m0 + top) / (m0 * m0);
  double Jl, J3l, Jt, J3t;
  argus_J(Ul, k, &Jl, &J3l);
  argus_J(Ut, k, &Jt, &J3t);
  const double N = 0.5 * m0 * m0 * (Jl - Jt);
  C[0] = 1.0 / N;
  C[1] = 0.0;
  C[2] = 0.5 * m0 * m0 * (J3l - J3t) / N;
  C[3] = m0;
  C[4] = 1.0 / (m0 * m0);
  C[5] = c;
}
// Log form: d log u/d c = U (input 0, m0, is a constant).
template <typename T> struct ArgusK {
  Loc<T> m0;
  T m0f, im02;
  ExpScl<T> c;
  RF_DEV ArgusK load(const double* C) {
    ArgusK k;
    k.m0 = Loc<T>::make(C[3]);
    k.m0f = (T)C[3];
    k.im02 = (T)C[4];
    k.c = ExpScl<T>::make(C[5]);
    return k;
  }
};
template <typename T> RF_DEV T argus_eval(T x, const ArgusK<T>& k, T* d) {
  const T dm = -k.m0.sub(x);  // m0 - x
  // U < 0 above the endpoint, where the shape is 0: clamping gives u = 0
  const T U = fmax(dm * (k.m0f + x) * k.im02, (T)0);
  d[0] = (T)0;
  d[1] = U;
  return x * RM<T>::sqrt_fast(U) * k.c.exp(U);
}

// ========================================================= Breit-Wigner ==
// u = 1/((x-M)^2 + Gamma^2/4);  inputs (M, Gamma);
// N = (2/Gamma)[atan(2(hi-M)/Gamma) - atan(2(lo-M)/Gamma)].
enum { BW_NC = 6 };
RF_DEV void bw_norm(double lo, double hi, double M, double G, double* N, double* dM, double* dG) {
  const double qh = 2 * (hi - M) / G, ql = 2 * (lo - M) / G;
  const double n = 2.0 / G * (::atan(qh) - ::atan(ql));
  const double bl = 1.0 / ((lo - M) * (lo - M) + 0.25 * G * G);
  const double bh = 1.0 / ((hi - M) * (hi - M) + 0.25 * G * G);
  *N = n;
  *dM = bl - bh;
  *dG = -n / G - 2.0 / (G * G) * (qh / (1 + qh * qh) - ql / (1 + ql * ql));
}
RF_DEV void bw_prologue(const double* in, double lo, double hi, double* C) {
  double N, dM, dG;
  bw_norm(lo, hi, in[0], in[1], &N, &dM, &dG);
  C[0] = 1.0 / N;
  C[1] = dM / N;
  C[2] = dG / N;
  C[3] = in[0];
  C[4] = 0.25 * in[1] * in[1];
  C[5] = -0.5 * in[1];
}
// Log form: d log u/d M = 2 q u, d log u/d Gamma = -(Gamma/2) u with
// q = x - M: event parts (q u, u), factors (2, C[5]).
template <typename T> struct BwK {
  Loc<T> M;
  T g2;
  RF_DEV BwK load(const double* C) {
    BwK k;
    k.M = Loc<T>::make(C[3]);
    k.g2 = (T)C[4];
    return k;
  }
};
template <typename T> RF_DEV T bw_eval(T x, const BwK<T>& k, T* d) {
  const T q = k.M.sub(x);
  const T b = RM<T>::rcp(fma(q, q, k.g2));
  d[0] = q * b;
  d[1] = b;
  return b;
}

// ====================================================== reductions, misc ==
// Cross-workgroup hand-off of the per-workgroup partial sums.  Partials are
// written with agent-scope atomic stores (written through to the level that
// is coherent across the whole device) and read back with agent-scope atomic
// loads, and nothing else is exchanged, so ordering them before the
// workgroup's ticket only needs the stores to be acknowledged: a wait on the
// vector-memory counter, with a compiler barrier.  A generic release fence
// would also write back the XCD's whole L2, once per workgroup.
RF_DEV void rf_wait_stores() { __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
RF_DEV unsigned rf_take_ticket(unsigned* t) {
  return __hip_atomic_fetch_add(t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
RF_DEV void rf_reset_ticket(unsigned* t) { __hip_atomic_store(t, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// one result word into mapped host memory, whole and straight through to it
RF_DEV void rf_store_host(double* h, double v) {
  __hip_atomic_store((uint64_t*)h, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// TwoSum (Knuth): s + e == a + b exactly.
RF_DEV void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// double-double accumulate (hi, lo) += (bh, bl)
RF_DEV void dd_add(double& hi, double& lo, double bh, double bl) {
  double s, e;
  two_sum(hi, bh, s, e);
  e += lo + bl;
  hi = s + e;
  lo = e - (hi - s);
}

// Wavefront sums with DPP lane moves (VALU, no LDS round trip).  Within each
// row of 16 lanes: partner xor 1, xor 2 (quad permutes), then the mirrored
// lane of the half row and of the row; IEEE addition is commutative, so both
// partners of every step hold bitwise equal values and each lane ends with
// its row's sum.  The four row sums (lanes 0, 16, 32, 48) are read into
// scalar registers and added in a fixed order.  Needs all 64 lanes active.
template <int CTRL> RF_DEV int dpp_i(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false); }
template <int CTRL> RF_DEV double dpp_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)u);
  const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
RF_DEV double lane_d(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
RF_DEV double row_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}
RF_DEV double wave_sum(double v) {
  v = row_sum(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}
RF_DEV unsigned wave_sum_u(unsigned x) {
  int v = (int)x;
  v += dpp_i<0xB1>(v);
  v += dpp_i<0x4E>(v);
  v += dpp_i<0x141>(v);
  v += dpp_i<0x140>(v);
  return (unsigned)(__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
                    __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
// double-double wavefront sum: plain FP64 wavefront sums of the high and of
// the low parts (the per-lane values are already compensated sums), then
// renormalised; compensation happens where the wavefronts are combined
RF_DEV void wave_dd_sum(double& hi, double& lo) {
  const double h = wave_sum(hi), l = wave_sum(lo);
  two_sum(h, l, hi, lo);
}

// ================================= Breit-Wigner (x) Crystal Ball, K-point ==
// S(x) = sum_k w_k CB(y_k) BW(x - y_k), (y_k, w_k) a Gauss-Legendre rule on
// the resolution window [ylo, yhi]; BW(u) = 1/((u - M)^2 + Gamma^2/4);
// CB(y) = exp(-z^2/2) for z = y/sigma > -alpha, else A (B - z)^-n with
// A = (n/alpha)^n exp(-alpha^2/2), B = n/alpha - alpha (mean 0, low tail).
// N_S = sum_k w_k CB(y_k) I_k with I_k the analytic BW integral over the
// range, so S/N_S is normalised exactly for the rule.  Inputs
// (M, Gamma, sigma, alpha, n).
//
// The prologue is block-wide: every thread builds table rows for nodes
// k = tid, tid + RF_BS, ... in LDS:
//   row k = [ (y_k + M)_hi, (y_k + M)_lo, c_k, dc_k/dsigma, dc_k/dalpha, dc_k/dn ]
// with c_k = w_k CB(y_k), and N_S and its five derivatives are reduced across
// the block in a fixed order.  The per-event sweep carries S, dS/dM, dS/dGamma
// and the three dS/d(CB parameter) sums (forward mode over the rule, so no
// second pass over the events is needed for the CB parameters).
enum { NUMCONV_NC = 8 };
template <typename TT> struct NumconvRow { enum { stride = sizeof(TT) == 4 ? 8 : 6 }; };

RF_DEV double cb_shape(double y, double s, double al, double n, double* d) {
  const double z = y / s;
  if (z > -al) {
    const double v = ::exp(-0.5 * z * z);
    d[0] = v * z * z / s; d[1] = 0.0; d[2] = 0.0;
    return v;
  }
  const double A = ::pow(n / al, n) * ::exp(-0.5 * al * al);
  const double B = n / al - al;
  const double r = B - z;
  const double v = A * ::pow(r, -n);
  d[0] = v * (-n * (z / s) / r);
  d[1] = v * (-n / al - al + n * (n / (al * al) + 1.0) / r);
  d[2] = v * (::log(n / al) + 1.0 - ::log(r) - n / (al * r));
  return v;
}

// block-wide; gl = [x_0..x_{K-1}, w_0..w_{K-1}] on the window (FP64)
template <int BS, typename TT>
__device__ void numconv_prologue(const double* in, double lo, double hi, int K, const double* gl,
                                 double* C, TT* tab, double* scratch /* [BS/64][6] */) {
  const double M = in[0], G = in[1], s = in[2], al = in[3], n = in[4];
  constexpr int ST = NumconvRow<TT>::stride;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < K; k += BS) {
    const double y = gl[k], w = gl[K + k];
    double dc[3];
    const double c = w * cb_shape(y, s, al, n, dc);
    for (int j = 0; j < 3; ++j) dc[j] *= w;
    const double yM = y + M;
    const TT hi_ = (TT)yM;
    TT* row = tab + (size_t)ST * k;
    row[0] = hi_;
    row[1] = (TT)(yM - (double)hi_);
    row[2] = (TT)c;
    row[3] = (TT)dc[0];
    row[4] = (TT)dc[1];
    row[5] = (TT)dc[2];
    double I, dIM, dIG;
    bw_norm(lo - y, hi - y, M, G, &I, &dIM, &dIG);
    acc[0] += c * I;
    acc[1] += c * dIM;
    acc[2] += c * dIG;
    acc[3] += dc[0] * I;
    acc[4] += dc[1] * I;
    acc[5] += dc[2] * I;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = 0; j < 6; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) scratch[wid * 6 + j] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[6];
    for (int j = 0; j < 6; ++j) {
      double h = 0.0, l = 0.0;
      for (int w = 0; w < BS / 64; ++w) dd_add(h, l, scratch[w * 6 + j], 0.0);
      t[j] = h + l;
    }
    C[0] = 1.0 / t[0];
    for (int j = 1; j < 6; ++j) C[j] = t[j] / t[0];
    C[6] = 0.25 * G * G;
    C[7] = 0.5 * G;
  }
}
template <typename T, typename TT> struct NumconvK {
  T invN, g2, hg;
  const TT* tab;
  RF_DEV NumconvK make(const double* C, const TT* tab) {
    NumconvK k;
    k.invN = (T)C[0];
    k.g2 = (T)C[6];
    k.hg = (T)C[7];
    k.tab = tab;
    return k;
  }
};
// d[0..4] = d log S / d(M, Gamma, sigma, alpha, n)
template <typename T, typename TT, int K> RF_DEV T numconv_eval(T x, const NumconvK<T, TT>& k, T* d) {
  constexpr int ST = NumconvRow<TT>::stride;
  constexpr int CH = 16;  // nodes per FP32 partial before it is added to FP64
  double S = 0, dM = 0, dG = 0, ds = 0, da = 0, dn = 0;
#pragma unroll 1
  for (int j0 = 0; j0 < K; j0 += CH) {
    T s1 = 0, m1 = 0, g1 = 0, s3 = 0, a3 = 0, n3 = 0;
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      const int j = j0 + jj;
      if (K % CH != 0 && j >= K) break;
      const TT* row = k.tab + ST * j;
      const T q = ((x - (T)row[0]) - (T)row[1]);
      const T b = RM<T>::rcp(fma(q, q, k.g2));
      const T cb = (T)row[2] * b;
      const T cb2 = cb * b;
      s1 += cb;
      m1 = fma(q, cb2, m1);
      g1 += cb2;
      s3 = fma((T)row[3], b, s3);
      a3 = fma((T)row[4], b, a3);
      n3 = fma((T)row[5], b, n3);
    }
    S += (double)s1; dM += (double)m1; dG += (double)g1;
    ds += (double)s3; da += (double)a3; dn += (double)n3;
  }
  const double iS = 1.0 / S;
  d[0] = (T)(2.0 * dM * iS);
  d[1] = (T)(-(double)k.hg * dG * iS);
  d[2] = (T)(ds * iS);
  d[3] = (T)(da * iS);
  d[4] = (T)(dn * iS);
  return (T)S;
}

