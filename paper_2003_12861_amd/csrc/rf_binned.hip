// rf_binned.hip -- binned template likelihood (HistFactory-like models,
// Section 3: per channel and sample a nominal histogram plus +-1 sigma
// histograms per systematic uncertainty, and a signal strength).
//
//   nu_csb = mu^[s=0] T_csb exp(sum_j |alpha_j| L^{sgn alpha_j}_csbj),
//            L^+- = log(T^+-/T)   (piecewise-exponential interpolation:
//            alpha = +-1 reproduces the +-1 sigma histogram exactly),
//   nu_cb  = sum_s nu_csb,
//   NLL    = sum_cb (nu_cb - n_cb log nu_cb) + sum_j alpha_j^2 / 2.
//
// One thread per (channel, bin, sample), the sample index fastest so that
// the FP32 interpolation tables -- stored as L[c][j][b][s] -- are read with
// fully coalesced loads; only the table of alpha_j's sign is read.  The 60
// exponent terms stay in registers and are reused by the adjoint:
//   dNLL/dalpha_j = sum_cb r_cb sum_s nu_csb dE_csb/dalpha_j + alpha_j,
//   r_cb = 1 - n_cb / nu_cb.
// Precision: the tables are FP32 in memory; the 60-term exponent, nu, r and
// every adjoint term are FP64 (FP64 FMA runs near the FP32 rate on CDNA4),
// because near the minimum r ~ 1/sqrt(n) cancels and an FP32 exponent (error
// ~5e-7) would be amplified ~50x in the gradient.
// Reduction (deterministic, in a fixed order): each lane holds its cell's 62
// terms (the Poisson term, d/dmu, d/dalpha_j); a transposed wavefront
// reduction (cross-half lane swaps, then an LDS pass) leaves one column per
// lane; the workgroup adds its four wavefronts and stores one row of 64
// columns (one coalesced store); the last workgroup of each group of BN_G
// adds its group's rows, and the last group the group rows, one column per
// lane -- all loads of a level in flight together.  (One level, the last
// workgroup adding every row, measured slower: 160 KB of rows through one
// compute unit take longer than the second ticket.)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "device/rf_dev.h"
#include "rf_internal.h"

#define BN_BSMAX 384  // workgroup size at most (chosen per model; its LDS stays under 64 KiB)
#define BN_MAXJ 64  // nuisance parameters at most (the kernel's arrays)
#define BN_G 16     // rows per reduction group
#define BN_G2 32    // group rows per pass of the last level
#define BN_RS 17    // LDS row stride (doubles) of a lane's 16 partial columns: conflict-free writes

namespace {

struct BinnedArgs {
  const float* T;      // [C][B][S]
  const float* nobs;   // [C][B]
  const float* L[BN_MAXJ];  // per nuisance parameter j: the table of its sign (alpha_j >= 0: L+, else L-),
                            // advanced to row j: element c J B S + b S + s of it is L_cbsj
  double absa[BN_MAXJ];     // |alpha_j|
  double* part;        // [nblk][64]: one row of column sums per workgroup
  double* gpart;       // [ngrp][64]: one row per group of BN_G workgroups
  unsigned* ticket;    // [0] global, [64 (1 + g)] group g
  double* out;         // [nll, grad[1+J]]
  double* hout;        // optional copy in mapped host memory, written word by word (or null)
  uint64_t neg;        // bit j set: alpha_j < 0
  double mu, cons;     // signal strength; sum_j alpha_j^2 / 2
  int32_t C, S, B, J;
  int32_t nblk, ngrp, logS, pad_;
  double alpha[BN_MAXJ];
};

// one double through a lane-swap builtin (two 32-bit halves)
__device__ __forceinline__ void swap32(double& x, double& y) {
  const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
  x = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
  y = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}
__device__ __forceinline__ void swap16(double& x, double& y) {
  const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
  x = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
  y = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}

template <int J>
__global__ __launch_bounds__(BN_BSMAX) void rf_binned_kernel(const BinnedArgs a) {
  constexpr int NS = 2 + J;  // NLL, mu, alpha_1..J: one column each
  static_assert(NS <= 64, "one lane per column");
  const int NW = (int)blockDim.x / 64;  // wavefronts of this workgroup
  // LDS (dynamic, sized by the host for this workgroup size): per wavefront
  // a [64][BN_RS] table of partial columns and a row of column sums; the
  // bins' totals when a bin spans wavefronts
  extern __shared__ double lds[];
  auto red = [&](int w) -> double* { return lds + (size_t)w * 64 * BN_RS; };
  auto wsum = [&](int w) -> double* { return lds + (size_t)NW * 64 * BN_RS + 64 * w; };
  double* const nu_s = lds + (size_t)NW * 64 * (BN_RS + 1);
  const int S = a.S;
  const uint32_t B = (uint32_t)a.B;
  // 32-bit cell indices (the host keeps C B S below 2^31); S is a power of
  // two (it divides the workgroup size)
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < (uint32_t)a.C * B * (uint32_t)S;
  const uint32_t tc = live ? t : 0u;
  const int s = (int)(tc & (uint32_t)(S - 1));
  const uint32_t cb = tc >> a.logS;  // c * B + b
  const uint32_t c = cb / B, b = cb - c * B;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;

  // every load of the thread is issued before any arithmetic, without a
  // branch: lanes past the end read cell 0 (their terms are zeroed through
  // r below).  Table addresses are a uniform 64-bit row base plus a 32-bit
  // per-lane byte offset (the host keeps the tables under 4 GiB).
  const uint32_t boff = 4u * ((c * (uint32_t)J * B + b) * (uint32_t)S + (uint32_t)s);
  float Tf = a.T[tc];  // T laid out [C][B][S] == thread order
  const float nf = a.nobs[cb];
  float Lv[J > 0 ? J : 1];
#pragma unroll
  for (int j = 0; j < J; ++j) Lv[j] = *(const float*)((const char*)a.L[j] + boff);
  // exponent E = sum_j |alpha_j| L^{sgn}_j in four independent FP64 chains
  double E;
  {
    double e4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < J; ++j) e4[j & 3] = fma(a.absa[j], (double)Lv[j], e4[j & 3]);
    E = (e4[0] + e4[1]) + (e4[2] + e4[3]);
  }
  const double base_nu = live ? (double)Tf * exp(E) : 0.0;  // nu without the signal strength
  const double nu = (s == 0) ? a.mu * base_nu : base_nu;
  // the bin's total over its S samples (consecutive lanes): a butterfly over
  // the lanes of the bin when it lies in one wavefront, every lane of the bin
  // ending with the same sum (additions commute exactly); through LDS
  // otherwise.  Then, in FP64, the Poisson term (on sample 0's lane) and
  // r = 1 - n/nu (on every lane of the bin).
  double tot = nu;
  if (S <= 64) {
    for (int h = 1; h < S; h <<= 1) tot += __shfl_xor(tot, h);
  } else {
    nu_s[threadIdx.x] = nu;
    __syncthreads();
    if (s == 0) {
      double t2 = 0.0;
      for (int q = 0; q < S; ++q) t2 += nu_s[threadIdx.x + q];
      nu_s[threadIdx.x] = t2;
    }
    __syncthreads();
    tot = nu_s[threadIdx.x - s];
  }
  const double n = (double)nf;
  // (the library's log where tot is zero, subnormal or not finite: such a
  // bin makes the NLL non-finite, as it must)
  const double lt = (tot >= 2.2250738585072014e-308 && tot < INFINITY) ? rf_log64(tot) : log(tot);
  const double nllt = (live && s == 0) ? tot - n * lt : 0.0;
  const double r = live ? 1.0 - n / tot : 0.0;
  const double rn = r * nu;  // zero past the end
  // the lane's terms, column k: 0 the Poisson term, 1 d/dmu (sample 0),
  // 2 + j: r nu L_j (the sign of alpha_j is applied to the column's total)
  auto term = [&](int k) -> double {
    if (k == 0) return nllt;
    if (k == 1) return s == 0 ? r * base_nu : 0.0;
    if (k < NS) return rn * (double)Lv[k - 2];
    return 0.0;
  };
  // Transposed reduction of the 64 columns.  Step 32: lanes 0-31 keep
  // columns 0-31 and lanes 32-63 columns 32-63, each adding its partner's
  // (lane ^ 32) copy of the half it keeps -- one cross-half swap per value
  // and one add, no selects.  Step 16 likewise with rows (lane ^ 16).  Lane
  // l then holds 16 columns (16 (l >> 4) + 0..15), each summed over the four
  // lanes with the same l mod 16; those go through LDS, where thread
  // (wave q, column c) adds the sixteen lanes of its column in wave q.  Fixed
  // order throughout, so the result is repeatable.
  double v[16];
  {
    double w32[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      double lo = term(k), hi = term(k + 32);
      swap32(lo, hi);
      w32[k] = lo + hi;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double lo = w32[k], hi = w32[k + 16];
      swap16(lo, hi);
      v[k] = lo + hi;
    }
  }
  {
    double* row = &red(wid)[lane * BN_RS];
#pragma unroll
    for (int k = 0; k < 16; ++k) row[k] = v[k];
  }
  // each wavefront reads back only its own rows: the LDS serves a
  // wavefront's accesses in order, so a wavefront-scope fence (no
  // reordering by the compiler) suffices
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  {
    // thread (wave wid, column lane): the sixteen lanes holding column lane
    const int g4 = lane >> 4, k = lane & 15;
    const double* col = &red(wid)[(16 * g4) * BN_RS + k];
    double h[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) h[i] = col[i * BN_RS];
#pragma unroll
    for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
      for (int i = 0; i < w; ++i) h[i] += h[i + w];
    wsum(wid)[lane] = h[0];
  }
  __syncthreads();
  if (wid != 0) return;
  // the workgroup's partial of column lane, wavefronts in a fixed order
  {
    double p = 0.0;
    for (int w = 0; w < NW; ++w) p += wsum(w)[lane];
    __hip_atomic_store(&a.part[(int64_t)blockIdx.x * 64 + lane], p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  rf_wait_stores();
  // level 1: the last workgroup of each group of BN_G adds the group's rows
  const int g = (int)blockIdx.x / BN_G, g0 = g * BN_G;
  const int gn = a.nblk - g0 < BN_G ? a.nblk - g0 : BN_G;
  {
    unsigned tk = lane == 0 ? rf_take_ticket(a.ticket + 64 * (1 + g)) : 0u;
    tk = (unsigned)__builtin_amdgcn_readfirstlane((int)tk);
    if (tk != (unsigned)(gn - 1)) return;
  }
  {
    double x[BN_G];
#pragma unroll
    for (int q = 0; q < BN_G; ++q)
      x[q] = __hip_atomic_load(&a.part[(int64_t)(g0 + (q < gn ? q : gn - 1)) * 64 + lane], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int q = 0; q < BN_G; ++q) x[q] = q < gn ? x[q] : 0.0;
#pragma unroll
    for (int w = BN_G / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int q = 0; q < w; ++q) x[q] += x[q + w];
    __hip_atomic_store(&a.gpart[(int64_t)g * 64 + lane], x[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  rf_wait_stores();
  {
    unsigned tk = 0u;
    if (lane == 0) {
      rf_reset_ticket(a.ticket + 64 * (1 + g));
      tk = rf_take_ticket(a.ticket);
    }
    tk = (unsigned)__builtin_amdgcn_readfirstlane((int)tk);
    if (tk != (unsigned)(a.ngrp - 1)) return;
  }
  // level 2: the group rows, BN_G2 at a time (all loads of a pass in
  // flight together), in a fixed order
  double fin = 0.0;
  for (int g1 = 0; g1 < a.ngrp; g1 += BN_G2) {
    double x[BN_G2];
#pragma unroll
    for (int q = 0; q < BN_G2; ++q) {
      const int gg = g1 + q < a.ngrp ? g1 + q : a.ngrp - 1;
      x[q] = __hip_atomic_load(&a.gpart[(int64_t)gg * 64 + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int q = 0; q < BN_G2; ++q) x[q] = g1 + q < a.ngrp ? x[q] : 0.0;
#pragma unroll
    for (int w = BN_G2 / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int q = 0; q < w; ++q) x[q] += x[q + w];
    fin += x[0];
  }
  // the result: column 0 plus the constraint sum_j alpha_j^2 / 2, column 1,
  // columns 2 + j times sgn(alpha_j) plus alpha_j; written by the wavefront
  // to the output and, word by word, to the host's mapped copy
  double res = fin;
  if (lane == 0) res = fin + a.cons;
  if (lane >= 2 && lane < NS) {
    const int j = lane - 2;
    res = (((a.neg >> j) & 1ull) ? -fin : fin) + a.alpha[j];
  }
  if (lane < NS) {
    a.out[lane] = res;
    if (a.hout) rf_store_host(a.hout + lane, res);
  }
  if (lane == 0) rf_reset_ticket(a.ticket);
}

// kernel instances: the number of nuisance parameters is a template
// argument so the table values stay in registers
using BinnedFn = void (*)(const BinnedArgs);
template <int J> BinnedFn pick() { return rf_binned_kernel<J>; }
BinnedFn kernel_for(int J) {
  switch (J) {
    case 0: return pick<0>();
    case 1: return pick<1>();
    case 2: return pick<2>();
    case 4: return pick<4>();
    case 8: return pick<8>();
    case 16: return pick<16>();
    case 32: return pick<32>();
    case 60: return pick<60>();
    case 62: return pick<62>();
  }
  return nullptr;
}
int padded_J(int J) {
  const int opts[] = {0, 1, 2, 4, 8, 16, 32, 60, 62};
  for (int o : opts)
    if (o >= J) return o;
  return -1;
}

}  // namespace

struct rf_binned {
  int C, S, B, J, Jp;  // Jp: compiled table depth (>= J, extra rows are zero)
  float *T = nullptr, *Lp = nullptr, *Lm = nullptr, *nobs = nullptr;
  double *part = nullptr, *gpart = nullptr, *out = nullptr;
  double *h_out = nullptr, *d_hout = nullptr;  // mapped result copy [2 + BN_MAXJ]
  unsigned* ticket = nullptr;
  int nblk = 0, ngrp = 0, bs = 256;  // workgroups, groups of BN_G, workgroup size
  void* last_stream = nullptr;        // stream of the previous launch (see order_launch)
  bool launched = false;
};

using namespace rf;

extern "C" {

void rf_binned_free(rf_binned* b) {
  if (!b) return;
  (void)hipFree(b->T);
  (void)hipFree(b->Lp);
  (void)hipFree(b->Lm);
  (void)hipFree(b->nobs);
  (void)hipFree(b->part);
  (void)hipFree(b->gpart);
  (void)hipFree(b->out);
  (void)hipFree(b->ticket);
  if (b->h_out) (void)hipHostFree(b->h_out);
  delete b;
}

int rf_binned_new(int32_t C, int32_t S, int32_t B, int32_t J, const double* T, const double* Tp,
                  const double* Tm, const double* nobs, void* stream, rf_binned** out) {
  if (!out || !T || !nobs || (J > 0 && (!Tp || !Tm))) return fail(RF_E_INVALID, "NULL argument");
  if (C < 1 || S < 1 || B < 1 || J < 0) return fail(RF_E_INVALID, "bad shape");
  if (256 % S != 0) return fail(RF_E_INVALID, "the number of samples must divide 256");
  const int Jp = padded_J(J);
  if (Jp < 0) return fail(RF_E_INVALID, "at most 62 nuisance parameters");
  const size_t nT = (size_t)C * S * B, nL = (size_t)C * Jp * B * S;
  if (nL >= ((size_t)1 << 30) || nT >= ((size_t)1 << 31))
    return fail(RF_E_INVALID, "tables too large (each +-1 sigma table must stay under 4 GiB)");
  std::vector<float> hT(nT), hLp(nL > 0 ? nL : 1, 0.f), hLm(nL > 0 ? nL : 1, 0.f), hn((size_t)C * B);
  for (int c = 0; c < C; ++c)
    for (int s = 0; s < S; ++s)
      for (int b = 0; b < B; ++b) {
        const double t = T[((size_t)c * S + s) * B + b];
        if (!(t > 0) || !std::isfinite(t)) return fail(RF_E_INVALID, "nominal yields must be finite and > 0");
        hT[((size_t)c * B + b) * S + s] = (float)t;
        for (int j = 0; j < J; ++j) {
          const size_t src = (((size_t)c * S + s) * J + j) * B + b;
          const size_t dst = (((size_t)c * Jp + j) * B + b) * S + s;
          if (!(Tp[src] > 0) || !(Tm[src] > 0)) return fail(RF_E_INVALID, "variation yields must be > 0");
          hLp[dst] = (float)std::log(Tp[src] / t);
          hLm[dst] = (float)std::log(Tm[src] / t);
        }
      }
  for (size_t i = 0; i < (size_t)C * B; ++i) {
    if (!(nobs[i] >= 0) || nobs[i] > 16777216.0) return fail(RF_E_INVALID, "observed counts must be in [0, 2^24]");
    hn[i] = (float)nobs[i];
  }
  rf_binned* bn = new rf_binned();
  bn->C = C; bn->S = S; bn->B = B; bn->J = J; bn->Jp = Jp;
  const int64_t threads = (int64_t)C * B * S;
  // workgroup size: enough threads that the workgroups fit the compute units
  // in one round (one each: no unit gets a second workgroup while others
  // idle), a multiple of 64 and of S (a bin never straddles two
  // workgroups), at most BN_BSMAX
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    const int unit = S > 64 ? S : 64;
    int64_t per = (threads + cus - 1) / cus;
    per = (per + unit - 1) / unit * unit;
    bn->bs = (int)(per < unit ? unit : (per > BN_BSMAX ? BN_BSMAX : per));
    if (bn->bs % unit) bn->bs = 256;  // (S = 256: 256 divides no larger size allowed)
  }
  bn->nblk = (int)((threads + bn->bs - 1) / bn->bs);
  hipError_t e;
  hipStream_t st = (hipStream_t)stream;
  auto up = [&](float** d, const std::vector<float>& h) -> hipError_t {
    hipError_t r = hipMalloc(d, sizeof(float) * h.size());
    if (r != hipSuccess) return r;
    return hipMemcpyAsync(*d, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st);
  };
  if ((e = up(&bn->T, hT)) != hipSuccess || (e = up(&bn->Lp, hLp)) != hipSuccess ||
      (e = up(&bn->Lm, hLm)) != hipSuccess || (e = up(&bn->nobs, hn)) != hipSuccess) {
    rf_binned_free(bn);
    return hip_fail(e, "binned upload");
  }
  bn->ngrp = (bn->nblk + BN_G - 1) / BN_G;
  const size_t NS = 64;  // one row of 64 columns per workgroup and group
  const size_t nticket = (size_t)64 * (1 + bn->ngrp);
  const size_t nhout = 2 + BN_MAXJ;
  if ((e = hipMalloc(&bn->part, sizeof(double) * NS * bn->nblk)) != hipSuccess ||
      (e = hipMalloc(&bn->gpart, sizeof(double) * NS * bn->ngrp)) != hipSuccess ||
      (e = hipMalloc(&bn->out, sizeof(double) * (2 + Jp))) != hipSuccess ||
      (e = hipMalloc(&bn->ticket, sizeof(unsigned) * nticket)) != hipSuccess ||
      (e = hipHostMalloc(&bn->h_out, sizeof(double) * nhout, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess ||
      (e = hipHostGetDevicePointer((void**)&bn->d_hout, bn->h_out, 0)) != hipSuccess ||
      (e = hipMemsetAsync(bn->ticket, 0, sizeof(unsigned) * nticket, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    rf_binned_free(bn);
    return hip_fail(e, "binned workspace");
  }
  memset(bn->h_out, 0, sizeof(double) * nhout);
  *out = bn;
  return RF_OK;
}

namespace {
int binned_launch(rf_binned* b, const double* theta, void* stream, double* hout) {
  if (!b || !theta) return fail(RF_E_INVALID, "NULL argument");
  for (int k = 0; k <= b->J; ++k)
    if (!std::isfinite(theta[k])) return fail(RF_E_DOMAIN, "theta must be finite");
  if (!(theta[0] >= 0)) return fail(RF_E_DOMAIN, "signal strength must be >= 0");
  if (int rc = order_launch(b->last_stream, b->launched, stream)) return rc;
  BinnedArgs a;
  memset(&a, 0, sizeof a);
  a.T = b->T; a.nobs = b->nobs;
  a.part = b->part; a.gpart = b->gpart; a.ticket = b->ticket; a.out = b->out;
  a.hout = hout;
  a.C = b->C; a.S = b->S; a.B = b->B; a.J = b->Jp; a.nblk = b->nblk; a.ngrp = b->ngrp;
  a.mu = theta[0];
  while ((1 << a.logS) < b->S) ++a.logS;
  const size_t row = (size_t)b->B * b->S;  // elements between the rows of two nuisance parameters
  for (int j = 0; j < b->Jp; ++j) {
    // padded rows: alpha = 0 (their table rows are zero)
    const double al = j < b->J ? theta[1 + j] : 0.0;
    a.alpha[j] = al;
    a.absa[j] = std::fabs(al);
    if (al < 0) a.neg |= 1ull << j;
    a.L[j] = (al >= 0 ? b->Lp : b->Lm) + (size_t)j * row;
    a.cons += 0.5 * al * al;
  }
  const size_t lds = sizeof(double) * ((size_t)(b->bs / 64) * 64 * (BN_RS + 1) + b->bs);
  hipLaunchKernelGGL(kernel_for(b->Jp), dim3(b->nblk), dim3(b->bs), lds, (hipStream_t)stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "binned launch");
  return RF_OK;
}
}  // namespace

int rf_binned_nll_grad_async(rf_binned* b, const double* theta, void* stream) {
  return binned_launch(b, theta, stream, nullptr);
}

int rf_binned_nll_grad(rf_binned* b, const double* theta, double* nll, double* grad, void* stream) {
  if (!nll || !grad) return fail(RF_E_INVALID, "NULL argument");
  if (!b) return fail(RF_E_INVALID, "NULL argument");
  // the last workgroup writes the result into mapped host memory, word by
  // word; this call polls the words
  arm_result(b->h_out, 2 + b->Jp);
  int rc = binned_launch(b, theta, stream, b->d_hout);
  if (rc) return rc;
  rc = wait_result(b->h_out, 2 + b->Jp, stream, nullptr);
  if (rc) return rc;
  *nll = b->h_out[0];
  for (int k = 0; k <= b->J; ++k) grad[k] = b->h_out[1 + k];
  if (!std::isfinite(*nll)) return fail(RF_E_NONFINITE, "non-finite NLL (a bin with nu <= 0)");
  return RF_OK;
}

const double* rf_binned_result(const rf_binned* b) { return b ? b->out : nullptr; }
}  // extern "C"

namespace rf {
int binned_n_params(const rf_binned* b) { return b ? 1 + b->J : 0; }
}  // namespace rf
