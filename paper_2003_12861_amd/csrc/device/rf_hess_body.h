// rf_hess_body.h -- body of a generated Hessian kernel.
//
// Included after the generated part, which defines:
//   RF_T (column dtype), RF_NCOL, RF_NCST, RF_NHC, RF_NSH, RF_P, RF_BS,
//   rf_prologue(th, cst, a)      the fused kernels' FP64 prologue (N, dN)
//   rf_prologue_h(th, cst, hc)   leaf inputs and second derivatives of N
//   rf_eval_h(x, cst, hc, acc)   one event: log p, the slot gradient of
//                                log p and its slot Hessian (FP64), added to
//                                the RF_NSH sums; false if p is unusable
//   rf_epilogue_h(S, th, out, nbad)  contraction with the parameter
//                                functions' first and second derivatives
// The per-event work is FP64 whatever the columns' dtype.  Reduction as in the
// fused kernels, in a fixed order: per-thread FP64 sums -> wavefront sums ->
// one partial per workgroup -> the last workgroup (atomic ticket) adds the
// partials and writes [nll, grad[P], n_bad, hess[P * P]] to the output and,
// word by word with system-scope stores, to the host's mapped copy.
#pragma once

#define RF_NCOL1 (RF_NCOL > 0 ? RF_NCOL : 1)

extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_hess(const RfArgs a) {
  constexpr int NW = RF_BS / 64;
  constexpr int NS1 = RF_NSH + 1;  // the sums, then the bad-event count
  __shared__ double cst[RF_NCST > 0 ? RF_NCST : 1];
  __shared__ double hc[RF_NHC > 0 ? RF_NHC : 1];
  __shared__ double red[NW][NS1];
  __shared__ double fin[NS1];
  __shared__ int last;
  rf_prologue(a.theta, cst, a);
  __syncthreads();
  rf_prologue_h(a.theta, cst, hc);
  __syncthreads();
  double acc[RF_NSH];
#pragma unroll
  for (int j = 0; j < RF_NSH; ++j) acc[j] = 0.0;
  unsigned nbad = 0;
  const int64_t n = a.n, step = (int64_t)gridDim.x * RF_BS;
  for (int64_t i = (int64_t)blockIdx.x * RF_BS + threadIdx.x; i < n; i += step) {
    double x[RF_NCOL1];
#pragma unroll
    for (int c = 0; c < RF_NCOL; ++c) x[c] = (double)((const RF_T*)a.col[c])[i];
    if (!rf_eval_h(x, cst, hc, acc)) ++nbad;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < RF_NSH; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[wid][j] = v;
  }
  const unsigned wb = wave_sum_u(nbad);
  if (lane == 0) red[wid][RF_NSH] = (double)wb;
  __syncthreads();
  const bool solo = gridDim.x == 1;
  const int nblk = a.nblk_max;
  for (int j = threadIdx.x; j < NS1; j += RF_BS) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w][j];
    if (solo)
      fin[j] = s;
    else
      __hip_atomic_store(&a.part[j * (int64_t)nblk + blockIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!solo) {
    rf_wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) last = (rf_take_ticket(a.ticket) == gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    // the last workgroup: wavefront w adds sums w, w + NW, ... over all
    // workgroups in a fixed order (lane l takes workgroups l, l + 64, ...)
    const int nb = (int)gridDim.x;
    for (int j = wid; j < NS1; j += NW) {
      double h = 0.0;
      for (int b0 = 0; b0 < nb; b0 += 64) {
        const int b = b0 + lane;
        const double v =
            __hip_atomic_load(&a.part[j * (int64_t)nblk + (b < nb ? b : nb - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        h += b < nb ? v : 0.0;
      }
      h = wave_sum(h);
      if (lane == 0) fin[j] = h;
    }
  }
  __syncthreads();
  if (wid == 0) {
    constexpr int NOUT = RF_P + 2 + RF_P * RF_P;
    __shared__ double res[NOUT];
    for (int j = lane; j < NOUT; j += 64) res[j] = 0.0;
    if (lane == 0) rf_epilogue_h(fin, a.theta, res, (unsigned)fin[RF_NSH]);
    for (int j = lane; j < NOUT; j += 64) {
      const double v = res[j];
      a.out[j] = v;
      if (a.hout) rf_store_host(a.hout + j, v);
    }
    if (lane == 0) rf_reset_ticket(a.ticket);
  }
}
