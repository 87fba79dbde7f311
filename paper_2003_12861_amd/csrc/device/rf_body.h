// rf_body.h -- generic body of a generated likelihood kernel.
//
// Included after the generated part, which defines:
//   RF_T, RF_NCOL, RF_NCST, RF_NSUM, RF_P, RF_BS, RF_PF, RF_TAIL64, RF_WAVE_UNIFORM
//   struct KS<T>                   per-event constants (loaded from the FP64 block)
//   rf_prologue(th, cst, a)        FP64 parameter-only branch (normalisations)
//   rf_eval<T, MODE>(x, k, acc, p, valid) one event: p, -log p and the adjoint sums
//   rf_epilogue<MODE>(S, cst, th, out, nbad)  final combination (one thread)
// MODE 0 = per-event values, 1 = NLL, 2 = NLL + gradient.
//
// Reduction (deterministic, no floating-point atomics): per-thread plain FP64
// sums -> wavefront butterfly (plain FP64) -> across wavefronts in fixed
// order with TwoSum into (hi, lo) -> one (hi, lo) partial per workgroup ->
// the last workgroup to finish (atomic ticket) adds all partials in a fixed
// order with double-double arithmetic and runs the epilogue.
#pragma once

template <typename T> RF_DEV T rf_ld(const void* col, int c, int64_t i) {
  return ((const T*)col)[i];
}

template <int MODE> RF_DEV void rf_body(const RfArgs& a) {
  constexpr int NSUM = (MODE == 2) ? RF_NSUM : 1;
  constexpr int NW = RF_BS / 64;
  __shared__ double cst[RF_NCST > 0 ? RF_NCST : 1];
  __shared__ double red[NW][NSUM];
  __shared__ unsigned redbad[NW];
  __shared__ double fin[NSUM];
  __shared__ int last;

#if RF_WAVE_UNIFORM
  // whole wavefronts step through the events together (wave-cooperative
  // leaves); lanes past the end evaluate a valid event and discard it
  const int64_t n = a.n;
  const int64_t step = (int64_t)gridDim.x * RF_BS;
  rf_prologue(a.theta, cst, a);
  __syncthreads();
  const KS<RF_T> k = KS<RF_T>::load(cst);
  double acc[NSUM];
#pragma unroll
  for (int j = 0; j < NSUM; ++j) acc[j] = 0.0;
  unsigned nbad = 0;
  const int lane0 = threadIdx.x & 63;
  for (int64_t wb = (int64_t)blockIdx.x * RF_BS + (threadIdx.x & ~63); wb < n; wb += step) {
    __asm__ volatile("" ::: "memory");
    const int64_t i = wb + lane0;
    const bool valid = i < n;
    RF_T x[RF_NCOL > 0 ? RF_NCOL : 1];
#pragma unroll
    for (int c = 0; c < RF_NCOL; ++c) x[c] = rf_ld<RF_T>(a.col[c], c, valid ? i : wb);
    RF_T p;
    const bool ok = rf_eval<RF_T, MODE>(x, k, acc, &p, valid);
    if (valid && !ok) ++nbad;
    if (MODE == 0 && valid) ((RF_T*)a.values)[i] = p;
  }
#else
  const int64_t n = a.n;
  const int64_t step = (int64_t)gridDim.x * RF_BS;
  const int64_t i0 = (int64_t)blockIdx.x * RF_BS + threadIdx.x;
  // Prefetch ring: the columns of events i, i+step, ..., i+(RF_PF-1)*step are
  // in flight while event i is computed (register rotation, no unrolling);
  // the first loads are issued before the prologue so that their latency
  // overlaps the FP64 normalisation work.
  RF_T xq[RF_PF][RF_NCOL > 0 ? RF_NCOL : 1];
#pragma unroll
  for (int q = 0; q < RF_PF; ++q) {
    const int64_t i = i0 + q * step;
#pragma unroll
    for (int c = 0; c < RF_NCOL; ++c) xq[q][c] = i < n ? rf_ld<RF_T>(a.col[c], c, i) : (RF_T)0;
  }

  rf_prologue(a.theta, cst, a);
  __syncthreads();
  const KS<RF_T> k = KS<RF_T>::load(cst);

  double acc[NSUM];
#pragma unroll
  for (int j = 0; j < NSUM; ++j) acc[j] = 0.0;
  unsigned nbad = 0;

  for (int64_t i = i0; i < n; i += step) {
    RF_T x[RF_NCOL > 0 ? RF_NCOL : 1];
#pragma unroll
    for (int c = 0; c < RF_NCOL; ++c) x[c] = xq[0][c];
#pragma unroll
    for (int q = 0; q + 1 < RF_PF; ++q)
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) xq[q][c] = xq[q + 1][c];
    {
      const int64_t in = i + RF_PF * step;
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) xq[RF_PF - 1][c] = in < n ? rf_ld<RF_T>(a.col[c], c, in) : (RF_T)0;
    }
    RF_T p;
    const bool ok = rf_eval<RF_T, MODE>(x, k, acc, &p, true);
    if (!ok) {
#if RF_TAIL64
      // FP32 result too small (or not finite): redo this event in FP64
      double xd[RF_NCOL > 0 ? RF_NCOL : 1];
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) xd[c] = (double)x[c];
      const KS<double> kd = KS<double>::load(cst);
      double pd;
      const bool okd = rf_eval<double, MODE>(xd, kd, acc, &pd, true);
      if (!okd) ++nbad;
      p = (RF_T)pd;
#else
      ++nbad;
#endif
    }
    if (MODE == 0) ((RF_T*)a.values)[i] = p;
  }
#endif
  if (MODE == 0) return;

  // ---- workgroup reduction ----
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NSUM; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[wid][j] = v;
  }
  const unsigned wb = wave_sum_u(nbad);
  if (lane == 0) redbad[wid] = wb;
  __syncthreads();
  const int nblk = a.nblk_max;
  for (int j = threadIdx.x; j < NSUM; j += RF_BS) {
    double hi = 0.0, lo = 0.0;
    for (int w = 0; w < NW; ++w) dd_add(hi, lo, red[w][j], 0.0);
    __hip_atomic_store(&a.part[(2 * j) * (int64_t)nblk + blockIdx.x], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&a.part[(2 * j + 1) * (int64_t)nblk + blockIdx.x], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) {
    unsigned t = 0;
    for (int w = 0; w < NW; ++w) t += redbad[w];
    __hip_atomic_store(&a.part_bad[blockIdx.x], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // release this workgroup's partials (only the storing wavefront fences)
  if ((int)threadIdx.x < NSUM || threadIdx.x == 0) __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(a.ticket, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();

  // ---- last workgroup: fixed-order double-double sum of all partials ----
  // Every thread owns the blocks b = tid, tid + RF_BS, ...; eight sums per
  // pass so that each thread has 16 independent loads in flight.  The
  // combination order (thread-local, then the wavefront butterfly, then the
  // wavefronts in index order) does not depend on timing: repeated calls give
  // bitwise identical results.
  __shared__ double rh[NW][8], rl[NW][8];
  const int nb = (int)gridDim.x;
  for (int j0 = 0; j0 < NSUM; j0 += 8) {
    double h[8], l[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { h[u] = 0.0; l[u] = 0.0; }
    for (int b = threadIdx.x; b < nb; b += RF_BS) {
      double ph[8], pl[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u < NSUM ? j0 + u : NSUM - 1;
        ph[u] = __hip_atomic_load(&a.part[(2 * j) * (int64_t)nblk + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pl[u] = __hip_atomic_load(&a.part[(2 * j + 1) * (int64_t)nblk + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) dd_add(h[u], l[u], ph[u], pl[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      wave_dd_sum(h[u], l[u]);
      if (lane == 0) { rh[wid][u] = h[u]; rl[wid][u] = l[u]; }
    }
    __syncthreads();
    if (threadIdx.x < 8 && j0 + (int)threadIdx.x < NSUM) {
      double H = 0.0, Lo = 0.0;
      for (int w = 0; w < NW; ++w) dd_add(H, Lo, rh[w][threadIdx.x], rl[w][threadIdx.x]);
      fin[j0 + threadIdx.x] = H + Lo;
    }
    __syncthreads();
  }
  if (wid == 0) {
    unsigned t = 0;
    for (int b = lane; b < nb; b += 64)
      t += __hip_atomic_load(&a.part_bad[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t = wave_sum_u(t);
    if (lane == 0) redbad[0] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    rf_epilogue<MODE>(fin, cst, a.theta, a.out, redbad[0]);
    *a.ticket = 0u;
  }
}

extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_values(const RfArgs a) { rf_body<0>(a); }
extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_nll(const RfArgs a) { rf_body<1>(a); }
extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_grad(const RfArgs a) { rf_body<2>(a); }
