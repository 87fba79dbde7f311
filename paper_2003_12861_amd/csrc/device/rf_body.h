// rf_body.h -- generic body of a generated likelihood kernel.
//
// Included after the generated part, which defines:
//   RF_T, RF_NCOL, RF_NCST, RF_NSUM, RF_P, RF_BS, RF_WAVE_UNIFORM, RF_TAIL64,
//   RF_EPT (events per lane and step: 16 bytes of each column, or 1),
//   RF_PFD (groups in flight per lane: depth of the load ring),
//   RF_TG (ticket groups: 1 = one counter)
//   struct KS<T>                   per-event constants (loaded from the FP64 block)
//   rf_prologue(th, cst, a)        FP64 parameter-only branch (normalisations)
//   rf_eval<T, MODE>(x, k, acc, &p) one event: p, log p and the adjoint sums;
//                                  false if p is unusable (adds nothing then)
//   rf_epilogue<MODE>(S, cst, th, out, nbad)  final combination (one thread)
// MODE 0 = per-event values, 1 = NLL, 2 = NLL + gradient.
//
// Event loop.  Each lane takes groups of RF_EPT consecutive events (4 in
// FP32, 2 in FP64: one 16-byte load per column; 1 for leaves whose per-event
// work hides any latency), with the loads of the next RF_PFD - 1 groups in
// flight while a group is evaluated (a ring of RF_PFD register slots; the
// loop is unrolled over the ring, so a slot is refilled right after it is
// used and no register moves wait on a load; consecutive lanes read
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

// E values of a column from event i on: one 16-byte load when E values make
// 16 bytes.  The vector types only claim the element's alignment (global
// memory accesses need no more on this target), so any column works and an
// aligned one gets full-width loads.
typedef float rf_f4 __attribute__((ext_vector_type(4), aligned(4)));
typedef double rf_d2 __attribute__((ext_vector_type(2), aligned(8)));
template <typename T, int E> RF_DEV void rf_ldv(const T* p, int64_t i, T (&v)[E]) {
  if constexpr (E == 4 && sizeof(T) == 4) {
    const rf_f4 q = *(const rf_f4*)(p + i);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else if constexpr (E == 2 && sizeof(T) == 8) {
    const rf_d2 q = *(const rf_d2*)(p + i);
    v[0] = q.x; v[1] = q.y;
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = p[i + e];
  }
}
template <typename T, int E> RF_DEV void rf_stv(T* p, int64_t i, const T (&v)[E]) {
  if constexpr (E == 4 && sizeof(T) == 4) {
    *(rf_f4*)(p + i) = rf_f4{v[0], v[1], v[2], v[3]};
  } else if constexpr (E == 2 && sizeof(T) == 8) {
    *(rf_d2*)(p + i) = rf_d2{v[0], v[1]};
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) p[i + e] = v[e];
  }
}

// FP32 programs add a group's per-event terms into FP32 partial sums, then
// into the per-thread FP64 sums; FP64 programs add them to the FP64 sums
// directly.  (Partials kept across groups let the compiler overlap groups at
// a higher register count.)
template <int NSUM> RF_DEV void rf_flush(RF_T* part, double* acc) {
  if constexpr (sizeof(RF_T) == 4) {
    acc[0] += RF_LN2 * (double)part[0];  // the FP32 terms are log2 p
#pragma unroll
    for (int j = 1; j < NSUM; ++j) acc[j] += (double)part[j];
#pragma unroll
    for (int j = 0; j < NSUM; ++j) part[j] = (RF_T)0;
  }
}

// E events (x[c][e]) starting at event index i0: evaluate, add to the FP64
// sums, redo unusable FP32 events in FP64, store values (MODE 0).
template <int MODE, int E>
RF_DEV void rf_group(const RF_T (&x)[RF_NCOL1][E], const KS<RF_T>& k, double* acc, unsigned& nbad,
                     const RfArgs& a, int64_t i0, const double* cst) {
  constexpr int NSUM = (MODE == 2) ? RF_NSUM : 1;
  RF_T p[E];
  unsigned badm = 0;
  RF_T part[NSUM];
#pragma unroll
  for (int j = 0; j < NSUM; ++j) part[j] = (RF_T)0;
  RF_T* const sums = sizeof(RF_T) == 4 ? part : (RF_T*)acc;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    RF_T xe[RF_NCOL1];
#pragma unroll
    for (int c = 0; c < RF_NCOL1; ++c) xe[c] = x[c][e];
    const bool ok = rf_eval<RF_T, MODE>(xe, k, sums, &p[e]);
    badm |= ok ? 0u : (1u << e);
  }
  if (MODE != 0) rf_flush<NSUM>(part, acc);
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
  if (MODE == 0) rf_stv<RF_T, E>((RF_T*)a.values, i0, p);
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
      RF_T pe[NSUM];
#pragma unroll
      for (int j = 0; j < NSUM; ++j) pe[j] = (RF_T)0;
      RF_T p;
      const bool ok = rf_eval<RF_T, MODE>(x, k, pe, &p);
      if (valid) {
        if (MODE != 0) {
          acc[0] += (sizeof(RF_T) == 4 ? RF_LN2 : 1.0) * (double)pe[0];
#pragma unroll
          for (int j = 1; j < NSUM; ++j) acc[j] += (double)pe[j];
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
    constexpr int D = RF_PFD;
    // group indices past the end are clamped to the last group: every load
    // address is valid (only used when ng > 0)
    auto clampg = [ng](int64_t g) { return g < ng ? g : ng - 1; };
    // the ring's first loads are issued before the prologue so that their
    // latency overlaps the FP64 normalisation work
    RF_T xb[D][RF_NCOL1][RF_EPT];
    if (ng > 0) {
#pragma unroll
      for (int u = 0; u < D; ++u)
#pragma unroll
        for (int c = 0; c < RF_NCOL; ++c)
          rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], clampg(gid + u * gstep) * RF_EPT, xb[u][c]);
    }
    rf_prologue(a.theta, cst, a);
    __syncthreads();
    const KS<RF_T> k = KS<RF_T>::load(cst);
    for (int64_t g = gid; g < ng; g += D * gstep) {
#pragma unroll
      for (int u = 0; u < D; ++u) {
        const int64_t gu = g + u * gstep;
        if (gu < ng) rf_group<MODE, RF_EPT>(xb[u], k, acc, nbad, a, gu * RF_EPT, cst);
        if (D > 1 || gu + gstep < ng) {
#pragma unroll
          for (int c = 0; c < RF_NCOL; ++c)
            rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], clampg(gu + D * gstep) * RF_EPT, xb[u][c]);
        }
      }
    }
    const int64_t tail0 = ng * RF_EPT;
    if (gid < n - tail0) {
      RF_T x1[RF_NCOL1][1];
#pragma unroll
      for (int c = 0; c < RF_NCOL; ++c) x1[c][0] = ((const RF_T*)a.col[c])[tail0 + gid];
      rf_group<MODE, 1>(x1, k, acc, nbad, a, tail0 + gid, cst);
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
  // one compensated value per sum: the wavefront sums added with TwoSum,
  // rounded once
  for (int j = threadIdx.x; j < NS2; j += RF_BS) {
    double hi = 0.0, lo = 0.0;
    for (int w = 0; w < NW; ++w) dd_add(hi, lo, red[w][j], 0.0);
    __hip_atomic_store(&a.part[j * (int64_t)nblk + blockIdx.x], hi + lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // publish this workgroup's partials, then take a ticket
  rf_wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (RF_TG == 1) {
      last = (rf_take_ticket(a.ticket) == gridDim.x - 1);
    } else {
      // two levels: RF_TG group counters (256 bytes apart), then the global
      // counter for the last workgroup of each group -- spreads the
      // end-of-kernel atomics over several addresses
      const unsigned g = blockIdx.x % RF_TG;
      const unsigned gsize = gridDim.x / RF_TG + (g < gridDim.x % RF_TG ? 1u : 0u);
      const unsigned ngroups = gridDim.x < RF_TG ? gridDim.x : RF_TG;
      last = 0;
      if (rf_take_ticket(a.ticket + 64 * (1 + g)) == gsize - 1) {
        rf_reset_ticket(a.ticket + 64 * (1 + g));
        last = (rf_take_ticket(a.ticket) == ngroups - 1);
      }
    }
  }
  __syncthreads();
  if (!last) return;

  // ---- last workgroup: fixed-order double-double sum of all partials ----
  // Every thread owns the blocks b = tid, tid + RF_BS, ...; eight sums of
  // two blocks per step, 16 independent loads in flight (one memory round
  // trip per step and 2 RF_BS workgroups; more would raise the register
  // count of the whole kernel).  The combination order (thread-local, then the wavefront
  // sums, then the wavefronts in index order) does not depend on timing:
  // repeated calls give bitwise identical results.
  __shared__ double rh[NW][8], rl[NW][8];
  const int nb = (int)gridDim.x;
  for (int j0 = 0; j0 < NS2; j0 += 8) {
    double h[8], l[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { h[u] = 0.0; l[u] = 0.0; }
    for (int b = threadIdx.x; b < nb; b += 2 * RF_BS) {
      // loads past the last workgroup are clamped to a valid one and skipped
      int bq[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) bq[q] = b + q * RF_BS < nb ? b + q * RF_BS : b;
      double pv[2][8];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = j0 + u < NS2 ? j0 + u : NS2 - 1;
          pv[q][u] = __hip_atomic_load(&a.part[j * (int64_t)nblk + bq[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (b + q * RF_BS < nb) {
#pragma unroll
          for (int u = 0; u < 8; ++u) dd_add(h[u], l[u], pv[q][u], 0.0);
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

// entry points, named by precision form: rf_k_{values,nll,grad}_{f32,f64}
#define RF_CAT2(x, y) x##y
#define RF_CAT(x, y) RF_CAT2(x, y)
extern "C" __global__ __launch_bounds__(RF_BS) void RF_CAT(rf_k_values_, RF_PREC)(const RfArgs a) { rf_body<0>(a); }
extern "C" __global__ __launch_bounds__(RF_BS) void RF_CAT(rf_k_nll_, RF_PREC)(const RfArgs a) { rf_body<1>(a); }
extern "C" __global__ __launch_bounds__(RF_BS) void RF_CAT(rf_k_grad_, RF_PREC)(const RfArgs a) { rf_body<2>(a); }
