// rf_body.h -- generic body of a generated likelihood kernel.
//
// Included after the generated part, which defines:
//   RF_T, RF_NCOL, RF_NCST, RF_NSUM, RF_P, RF_BS, RF_WAVE_UNIFORM, RF_TAIL64,
//   RF_EPT (events per lane and step: 16 bytes of each column, or 1)
//   struct KS<T>                   per-event constants (loaded from the FP64 block)
//   rf_prologue(th, cst, a)        FP64 parameter-only branch (normalisations)
//   rf_eval<T, MODE>(x, k, acc, &p) one event: p, log p and the adjoint sums;
//                                  false if p is unusable (adds nothing then)
//   rf_epilogue<MODE>(S, cst, th, out, nbad)  final combination (one thread)
// MODE 0 = per-event values, 1 = NLL, 2 = NLL + gradient.
//
// Event loop.  Each lane takes groups of RF_EPT consecutive events (4 in
// FP32, 2 in FP64: one 16-byte load per column; 1 for leaves whose per-event
// work hides any latency), with the next group's loads in flight while the
// current group is evaluated (consecutive lanes read
// consecutive 16-byte pieces, so every load instruction of a wavefront
// covers 1 KiB contiguously).  FP32 programs add each group's terms into
// FP32 partial sums that go into the per-thread FP64 sums once per group;
// an event whose FP32 probability is below 1e-30 or not finite adds nothing
// there and is evaluated again in FP64 (a branch taken only by wavefronts
// holding such an event).
//
// Reduction (deterministic, no floating-point atomics): per-thread FP64 sums
// -> wavefront butterfly (plain FP64) -> across wavefronts in fixed order
// with TwoSum into (hi, lo) -> one (hi, lo) partial per workgroup -> the last
// workgroup to finish (atomic ticket) adds all partials in a fixed order with
// double-double arithmetic and runs the epilogue.
#pragma once

#define RF_NCOL1 (RF_NCOL > 0 ? RF_NCOL : 1)

// E values of a column from event i on; one 16-byte load when E values make
// 16 bytes and the column is 16-byte aligned
template <typename T, int E> RF_DEV void rf_ldv(const T* p, int64_t i, bool vec, T (&v)[E]) {
  if constexpr (E * sizeof(T) == 16) {
    if (vec) {
      if constexpr (sizeof(T) == 4) {
        const float4 q = *(const float4*)(p + i);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
        const double2 q = *(const double2*)(p + i);
        v[0] = q.x; v[1] = q.y;
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = p[i + e];
}
template <typename T, int E> RF_DEV void rf_stv(T* p, int64_t i, bool vec, const T (&v)[E]) {
  if constexpr (E * sizeof(T) == 16) {
    if (vec) {
      if constexpr (sizeof(T) == 4) *(float4*)(p + i) = make_float4(v[0], v[1], v[2], v[3]);
      else *(double2*)(p + i) = make_double2(v[0], v[1]);
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) p[i + e] = v[e];
}

// E events (x[c][e]) starting at event index i0: evaluate, add to the FP64
// sums, redo unusable FP32 events in FP64, store values (MODE 0).
template <int MODE, int E>
RF_DEV void rf_group(const RF_T (&x)[RF_NCOL1][E], const KS<RF_T>& k, double* acc, unsigned& nbad,
                     const RfArgs& a, int64_t i0, bool vec, const double* cst) {
  constexpr int NSUM = (MODE == 2) ? RF_NSUM : 1;
  constexpr bool F32 = sizeof(RF_T) == 4;
  RF_T p[E];
  unsigned badm = 0;
  RF_T part[NSUM];
#pragma unroll
  for (int j = 0; j < NSUM; ++j) part[j] = (RF_T)0;
  RF_T* const sums = F32 ? part : (RF_T*)acc;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    RF_T xe[RF_NCOL1];
#pragma unroll
    for (int c = 0; c < RF_NCOL1; ++c) xe[c] = x[c][e];
    const bool ok = rf_eval<RF_T, MODE>(xe, k, sums, &p[e]);
    badm |= ok ? 0u : (1u << e);
  }
  if (F32 && MODE != 0) {
    acc[0] += RF_LN2 * (double)part[0];  // the FP32 terms are log2 p
#pragma unroll
    for (int j = 1; j < NSUM; ++j) acc[j] += (double)part[j];
  }
  if (badm) {
#if RF_TAIL64
    const KS<double> kd = KS<double>::load(cst);
    for (int e = 0; e < E; ++e) {
      if (!((badm >> e) & 1u)) continue;
      double xd[RF_NCOL1];
#pragma unroll
      for (int c = 0; c < RF_NCOL1; ++c) xd[c] = (double)x[c][e];
      double pd;
      if (!rf_eval<double, MODE>(xd, kd, acc, &pd)) ++nbad;
      p[e] = (RF_T)pd;
    }
#else
    nbad += __builtin_popcount(badm);
#endif
  }
  if (MODE == 0) rf_stv<RF_T, E>((RF_T*)a.values, i0, vec, p);
}

template <int MODE> RF_DEV void rf_body(const RfArgs& a) {
  constexpr int NSUM = (MODE == 2) ? RF_NSUM : 1;
  constexpr int NW = RF_BS / 64;
  __shared__ double cst[RF_NCST > 0 ? RF_NCST : 1];
  constexpr int NS2 = NSUM + 1;
  __shared__ double red[NW][NS2];
  __shared__ double fin[NS2];
  __shared__ int last;

  const int64_t n = a.n;
  double acc[NSUM];
#pragma unroll
  for (int j = 0; j < NSUM; ++j) acc[j] = 0.0;
  unsigned nbad = 0;
#if RF_WAVE_UNIFORM
  // whole wavefronts step through the events together (wave-cooperative
  // leaves); lanes past the end evaluate a valid event and discard it
  {
    const int64_t step = (int64_t)gridDim.x * RF_BS;
    rf_prologue(a.theta, cst, a);
    __syncthreads();
    const KS<RF_T> k = KS<RF_T>::load(cst);
    const int lane0 = threadIdx.x & 63;
    for (int64_t wb = (int64_t)blockIdx.x * RF_BS + (threadIdx.x & ~63); wb < n; wb += step) {
      __asm__ volatile("" ::: "memory");
      const int64_t i = wb + lane0;
      const bool valid = i < n;
      RF_T x[RF_NCOL1];
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) x[c] = ((const RF_T*)a.col[c])[valid ? i : wb];
      RF_T part[NSUM];
#pragma unroll
      for (int j = 0; j < NSUM; ++j) part[j] = (RF_T)0;
      RF_T p;
      const bool ok = rf_eval<RF_T, MODE>(x, k, part, &p);
      if (valid) {
        if (MODE != 0) {
          acc[0] += (sizeof(RF_T) == 4 ? RF_LN2 : 1.0) * (double)part[0];
#pragma unroll
          for (int j = 1; j < NSUM; ++j) acc[j] += (double)part[j];
        }
        if (!ok) ++nbad;
        if (MODE == 0) ((RF_T*)a.values)[i] = p;
      }
    }
  }
#else
  {
    const int64_t ng = n / RF_EPT;  // whole groups; the last n % 4 events follow
    const int64_t gstep = (int64_t)gridDim.x * RF_BS;
    const int64_t gid = (int64_t)blockIdx.x * RF_BS + threadIdx.x;
    const bool vec = a.vec != 0;
    // the first group's loads are issued before the prologue so that their
    // latency overlaps the FP64 normalisation work
    RF_T xc[RF_NCOL1][RF_EPT];
    if (gid < ng) {
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], gid * RF_EPT, vec, xc[c]);
    }
    rf_prologue(a.theta, cst, a);
    __syncthreads();
    const KS<RF_T> k = KS<RF_T>::load(cst);
    for (int64_t g = gid; g < ng; g += gstep) {
      // next group (clamped to the last one: always a valid address)
      const int64_t gn = g + gstep < ng ? g + gstep : ng - 1;
      RF_T xn[RF_NCOL1][RF_EPT];
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], gn * RF_EPT, vec, xn[c]);
      rf_group<MODE, RF_EPT>(xc, k, acc, nbad, a, g * RF_EPT, vec, cst);
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c)
#pragma unroll
        for (int e = 0; e < RF_EPT; ++e) xc[c][e] = xn[c][e];
    }
    const int64_t tail0 = ng * RF_EPT;
    if (gid < n - tail0) {
      RF_T x1[RF_NCOL1][1];
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) x1[c][0] = ((const RF_T*)a.col[c])[tail0 + gid];
      rf_group<MODE, 1>(x1, k, acc, nbad, a, tail0 + gid, false, cst);
    }
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
  // the bad-event count travels as sum NSUM (exact in FP64)
  const unsigned wb = wave_sum_u(nbad);
  if (lane == 0) red[wid][NSUM] = (double)wb;
  __syncthreads();
  const int nblk = a.nblk_max;
  for (int j = threadIdx.x; j < NS2; j += RF_BS) {
    double hi = 0.0, lo = 0.0;
    for (int w = 0; w < NW; ++w) dd_add(hi, lo, red[w][j], 0.0);
    __hip_atomic_store(&a.part[(2 * j) * (int64_t)nblk + blockIdx.x], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&a.part[(2 * j + 1) * (int64_t)nblk + blockIdx.x], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // publish this workgroup's partials, then take a ticket
  rf_wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) last = (rf_take_ticket(a.ticket) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;

  // ---- last workgroup: fixed-order double-double sum of all partials ----
  // Every thread owns the blocks b = tid, tid + RF_BS, ...; eight sums of
  // two blocks per step so that each thread has 32 independent loads in
  // flight (one memory round trip per step).  The
  // combination order (thread-local, then the wavefront butterfly, then the
  // wavefronts in index order) does not depend on timing: repeated calls give
  // bitwise identical results.
  __shared__ double rh[NW][8], rl[NW][8];
  const int nb = (int)gridDim.x;
  for (int j0 = 0; j0 < NS2; j0 += 8) {
    double h[8], l[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { h[u] = 0.0; l[u] = 0.0; }
    for (int b = threadIdx.x; b < nb; b += 2 * RF_BS) {
      const bool two = b + RF_BS < nb;
      const int bq[2] = {b, two ? b + RF_BS : b};  // second load clamped to a valid block
      double ph[2][8], pl[2][8];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = j0 + u < NS2 ? j0 + u : NS2 - 1;
          ph[q][u] = __hip_atomic_load(&a.part[(2 * j) * (int64_t)nblk + bq[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          pl[q][u] = __hip_atomic_load(&a.part[(2 * j + 1) * (int64_t)nblk + bq[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
      for (int u = 0; u < 8; ++u) dd_add(h[u], l[u], ph[0][u], pl[0][u]);
      if (two) {
#pragma unroll
        for (int u = 0; u < 8; ++u) dd_add(h[u], l[u], ph[1][u], pl[1][u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      wave_dd_sum(h[u], l[u]);
      if (lane == 0) { rh[wid][u] = h[u]; rl[wid][u] = l[u]; }
    }
    __syncthreads();
    if (threadIdx.x < 8 && j0 + (int)threadIdx.x < NS2) {
      double H = 0.0, Lo = 0.0;
      for (int w = 0; w < NW; ++w) dd_add(H, Lo, rh[w][threadIdx.x], rl[w][threadIdx.x]);
      fin[j0 + threadIdx.x] = H + Lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rf_epilogue<MODE>(fin, cst, a.theta, a.out, (unsigned)fin[NSUM]);
    rf_reset_ticket(a.ticket);
    if (a.hout) {
      // host copy, then the completion word the host polls for
      for (int j = 0; j < RF_P + 2 + NSUM; ++j) a.hout[j] = a.out[j];
      __threadfence_system();
      __hip_atomic_store((uint64_t*)(a.hout + RF_P + 2 + RF_NSUM), a.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_values(const RfArgs a) { rf_body<0>(a); }
extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_nll(const RfArgs a) { rf_body<1>(a); }
extern "C" __global__ __launch_bounds__(RF_BS) void rf_k_grad(const RfArgs a) { rf_body<2>(a); }
