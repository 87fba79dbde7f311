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
// with TwoSum, rounded once -> one FP64 partial per workgroup -> the last
// workgroup to finish (atomic ticket) adds all partials in a fixed order and
// runs the epilogue.
#pragma once

#define RF_NCOL1 (RF_NCOL > 0 ? RF_NCOL : 1)

// E values of a column from event i on: one 16-byte load when E values make
// 16 bytes.  The vector types only claim the element's alignment (global
// memory accesses need no more on this target), so any column works and an
// aligned one gets full-width loads.  FP32 columns are read with non-temporal
// loads (each event is read once per evaluation, and the streamed columns
// then do not displace the kernel's code and constants from the caches).
// Measured at 1e7 events: one column, after a cache eviction 20.3 us against
// 23.4-23.7, back to back unchanged, synchronous step about 0.3 us lower; two
// columns (80 MB, which the Infinity Cache would otherwise keep between
// evaluations), after a cache eviction 11-13 us faster, back to back 0.6-0.8
// us slower; the 2-D model at 5e7 events, 241 against 244 us.  FP64 columns
// keep ordinary loads: with non-temporal ones the 1e7-event FP64 kernel ran
// 41.4-42.6 us back to back against 39.6.
typedef float rf_f4 __attribute__((ext_vector_type(4), aligned(4)));
typedef double rf_d2 __attribute__((ext_vector_type(2), aligned(8)));
template <typename T, int E> RF_DEV void rf_ldv(const T* p, int64_t i, T (&v)[E]) {
  if constexpr (E == 4 && sizeof(T) == 4) {
    const rf_f4 q = __builtin_nontemporal_load((const rf_f4*)(p + i));
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else if constexpr (E == 2 && sizeof(T) == 8) {
    const rf_d2 q = *(const rf_d2*)(p + i);
    v[0] = q.x; v[1] = q.y;
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = __builtin_nontemporal_load(p + i + e);
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

// FP32 programs, NLL modes, full tiles: the events of a ring round (up to
// RF_PFD groups) are evaluated without per-event checks into one set of FP32
// partial sums, keeping the smallest probability.  The round is then checked
// as a whole: it is usable when that minimum is above the tail threshold and
// the sum of log2 p is finite (a probability that is infinite or NaN makes it
// infinite or NaN).  A usable round goes into the FP64 sums; an unusable one
// (rare: an event in a far tail) is dropped, and each of its events is read
// again and evaluated in FP64 with its own check, as in rf_group.
template <int MODE, int E>
RF_DEV void rf_group_unchecked(const RF_T (&x)[RF_NCOL1][E], const KS<RF_T>& k, RF_T* part, RF_T& pmin) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    RF_T xe[RF_NCOL1];
#pragma unroll
    for (int c = 0; c < RF_NCOL1; ++c) xe[c] = x[c][e];
    RF_T p;
    (void)rf_eval<RF_T, MODE, 0>(xe, k, part, &p);
    pmin = fminf(pmin, p);
  }
}
template <int MODE>
RF_DEV void rf_round_fp64(const RfArgs& a, int64_t g0, const double* cst, double* acc, unsigned& nbad) {
  const KS<double> kd = KS<double>::load(cst);
  // one event at a time (rolled loops): this path must not raise the
  // kernel's register count, which the unrolled FP64 events would
#pragma clang loop unroll(disable)
  for (int e = 0; e < RF_EPT; ++e) {
    double xd[RF_NCOL1];
#pragma unroll
    for (int c = 0; c < RF_NCOL; ++c) xd[c] = (double)((const RF_T*)a.col[c])[g0 * RF_EPT + e];
    double pd;
    if (!rf_eval<double, MODE>(xd, kd, acc, &pd)) ++nbad;
  }
}

// Issue priority of the wavefronts by the work left.  The arbiter of a SIMD
// issues from the wave of highest priority first, and among equals from the
// oldest: without this, the workgroups that reach a CU first run ahead and
// the last ones finish their share alone, with too few waves to hide
// latency.  Lowering the priority of waves that are near the end of their
// share (fixed share; the summation order does not change) lets the others
// catch up, so that the workgroups of a CU finish together.
RF_DEV void rf_prio_remaining(int64_t r, int64_t total) {
#if RF_PRIO == 1
  // by positions left: the last three are graded
  if (r >= 4) __builtin_amdgcn_s_setprio(3);
  else if (r == 3) __builtin_amdgcn_s_setprio(2);
  else if (r == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
#else
  // by quarters of the share done
  const int64_t q = (4 * (total - r)) / (total > 0 ? total : 1);
  if (q <= 0) __builtin_amdgcn_s_setprio(3);
  else if (q == 1) __builtin_amdgcn_s_setprio(2);
  else if (q == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
#endif
}

template <int MODE> RF_DEV void rf_body(const RfArgs& a) {
  constexpr int NSUM = (MODE == 2) ? RF_NSUM : 1;
  constexpr int NW = RF_BS / 64;
  __shared__ double cst[RF_NCST > 0 ? RF_NCST : 1];
  constexpr int NS2 = NSUM + 1;
#if !RF_LDSRED
  __shared__ double red[NW][NS2];
#endif
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
    const int64_t ng = n / RF_EPT;  // whole groups; the last n % RF_EPT events follow
    const int64_t gstep = (int64_t)gridDim.x * RF_BS;
    const int64_t base0 = (int64_t)blockIdx.x * RF_BS;  // thread 0's group at position 0
    constexpr int D = RF_PFD;
    // Fixed assignment: at position m the workgroup takes the tile of groups
    // base0 + m gstep + [0, RF_BS), one per thread (consecutive threads,
    // consecutive groups), which keeps the summation order, and so the
    // result, identical from call to call.  The main loop runs the MB full
    // tiles, where every lane is in range: no lane checks, and a refill
    // past the last full tile re-reads that tile (its base is clamped in
    // scalar registers) -- so every ring slot is refilled unconditionally
    // and the compiler waits for one slot at a time.  The one partial tile
    // and the last n % RF_EPT events follow with lane checks.
    const int64_t MB = ng >= base0 + RF_BS ? (ng - base0 - RF_BS) / gstep + 1 : 0;
    auto tile = [&](int64_t m) { return base0 + (m < MB ? m : MB - 1) * gstep; };  // uniform
    RF_T xb[D][RF_NCOL1][RF_EPT];
#if RF_PRIO
    // the prologue at the highest issue priority: the waves of the
    // workgroups already in their event loops run at it too (see
    // rf_prio_remaining), and a later workgroup's prologue at the default
    // priority waited behind them for up to 9 us
    __builtin_amdgcn_s_setprio(3);
#endif
    // the ring's first loads are issued before the prologue so that their
    // latency overlaps the FP64 normalisation work
    if (MB > 0) {
#pragma unroll
      for (int u = 0; u < D; ++u)
#pragma unroll
        for (int c = 0; c < RF_NCOL; ++c)
          rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], (tile(u) + threadIdx.x) * RF_EPT, xb[u][c]);
    }
    rf_prologue(a.theta, cst, a);
    __syncthreads();
    const KS<RF_T> k = KS<RF_T>::load(cst);
    // (leaves with one event per step do enough work per event that the
    // per-event check costs nothing; they keep rf_group)
    constexpr bool ROUNDS = sizeof(RF_T) == 4 && MODE != 0 && RF_TAIL64 && RF_EPT > 1;
    for (int64_t m0 = 0; m0 < MB; m0 += D) {
      RF_T part[NSUM];
#pragma unroll
      for (int j = 0; j < NSUM; ++j) part[j] = (RF_T)0;
      RF_T pmin = (RF_T)INFINITY;
#pragma unroll
      for (int u = 0; u < D; ++u) {
#if RF_PRIO
        rf_prio_remaining(MB - (m0 + u), MB);
#endif
        // the last ring round may hold fewer than D full tiles (uniform test)
        if (m0 + u < MB) {
          if constexpr (ROUNDS)
            rf_group_unchecked<MODE, RF_EPT>(xb[u], k, part, pmin);
          else
            rf_group<MODE, RF_EPT>(xb[u], k, acc, nbad, a, (base0 + (m0 + u) * gstep + threadIdx.x) * RF_EPT, cst);
        }
#pragma unroll
        for (int c = 0; c < RF_NCOL; ++c)
          rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], (tile(m0 + u + D) + threadIdx.x) * RF_EPT, xb[u][c]);
      }
      if constexpr (ROUNDS) {
        if (pmin > RM<RF_T>::tiny() && __builtin_isfinite(part[0])) {
          rf_flush<NSUM>(part, acc);
        } else {
#pragma clang loop unroll(disable)
          for (int u = 0; u < D; ++u)
            if (m0 + u < MB) rf_round_fp64<MODE>(a, base0 + (m0 + u) * gstep + threadIdx.x, cst, acc, nbad);
        }
      }
    }
    // the partial tile (at most one per workgroup: the next one starts past ng)
    {
      const int64_t gp = base0 + MB * gstep + threadIdx.x;
      if (gp < ng) {
        RF_T xp[RF_NCOL1][RF_EPT];
#pragma unroll
        for (int c = 0; c < RF_NCOL; ++c) rf_ldv<RF_T, RF_EPT>((const RF_T*)a.col[c], gp * RF_EPT, xp[c]);
        rf_group<MODE, RF_EPT>(xp, k, acc, nbad, a, gp * RF_EPT, cst);
      }
    }
#if RF_PRIO
    __builtin_amdgcn_s_setprio(3);  // the hand-off that follows is on the critical path
#endif
    const int64_t tail0 = ng * RF_EPT;
    const int64_t gid = base0 + threadIdx.x;
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
  const int nblk = a.nblk_max;
  // a single workgroup keeps its sums in LDS and goes straight to the
  // epilogue: no partials to publish, no ticket, no second pass (the result
  // is the one the multi-workgroup path computes, which only adds zeros)
  const bool solo = gridDim.x == 1;
#if RF_LDSRED
  // Through LDS: every thread writes its sums (and its bad-event count, as
  // the last sum: exact in FP64); in round r, the RF_BS / 8 threads of sum
  // 8 r + t / (RF_BS / 8) each add eight consecutive values pairwise, the
  // sixteen lanes of a row by DPP and the rows by readlane -- a fixed order,
  // and a few VALU instructions per sum instead of a butterfly per sum and
  // wavefront.
  static_assert(RF_BS == 256 || RF_BS == 512, "the LDS reduction takes RF_BS / 8 lanes per sum");
  constexpr int TPS = RF_BS / 8;
  __shared__ double sred[NS2][RF_BS];
#pragma unroll
  for (int j = 0; j < NSUM; ++j) sred[j][threadIdx.x] = acc[j];
  sred[NSUM][threadIdx.x] = (double)nbad;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < (NS2 + 7) / 8; ++r) {
    const int j = r * 8 + (int)threadIdx.x / TPS;
    const double* row = &sred[j < NS2 ? j : NS2 - 1][((int)threadIdx.x % TPS) * 8];
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = row[q];
#pragma unroll
    for (int w = 4; w >= 1; w >>= 1)
#pragma unroll
      for (int q = 0; q < w; ++q) v[q] += v[q + w];
    const double rs = row_sum(v[0]);
    const double h0 = lane_d(rs, 0) + lane_d(rs, 16);
    const double h1 = lane_d(rs, 32) + lane_d(rs, 48);
    if (lane == 0) {
      if constexpr (TPS == 32) {  // a sum per half-wavefront
        const int ja = r * 8 + 2 * wid;
        if (solo) {
          if (ja < NS2) fin[ja] = h0;
          if (ja + 1 < NS2) fin[ja + 1] = h1;
        } else {
          if (ja < NS2)
            __hip_atomic_store(&a.part[ja * (int64_t)nblk + blockIdx.x], h0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (ja + 1 < NS2)
            __hip_atomic_store(&a.part[(ja + 1) * (int64_t)nblk + blockIdx.x], h1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      } else {  // a sum per wavefront
        const int ja = r * 8 + wid;
        if (ja < NS2) {
          if (solo)
            fin[ja] = h0 + h1;
          else
            __hip_atomic_store(&a.part[ja * (int64_t)nblk + blockIdx.x], h0 + h1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
#else
#pragma unroll
  for (int j = 0; j < NSUM; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[wid][j] = v;
  }
  // the bad-event count travels as sum NSUM (exact in FP64)
  const unsigned wb = wave_sum_u(nbad);
  if (lane == 0) red[wid][NSUM] = (double)wb;
  __syncthreads();
  // one compensated value per sum: the wavefront sums added with TwoSum,
  // rounded once
  for (int j = threadIdx.x; j < NS2; j += RF_BS) {
    double hi = 0.0, lo = 0.0;
    for (int w = 0; w < NW; ++w) dd_add(hi, lo, red[w][j], 0.0);
    if (solo)
      fin[j] = hi + lo;
    else
      __hip_atomic_store(&a.part[j * (int64_t)nblk + blockIdx.x], hi + lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#endif
  if (!solo) {
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

    // ---- last workgroup: sum of all partials in a fixed order ----
    // Wavefront w adds sums w, w + NW, ... two at a time: each lane reads the
    // partials of workgroups lane, lane + 64, ... (sixteen per sum and pass,
    // all loads of a pass in flight together; consecutive lanes read
    // consecutive words), adds them pairwise, and a wavefront sum completes
    // the total.  The order depends only on the workgroup count, so repeated
    // calls give bitwise identical results; the rounding error is a few units
    // of 2^-53 times the sum of magnitudes of the partials.
    const int nb = (int)gridDim.x;
    for (int j0 = wid; j0 < NS2; j0 += 2 * NW) {
      const int j1 = j0 + NW < NS2 ? j0 + NW : j0;  // second sum (a repeat of the first if none)
      double h0 = 0.0, h1 = 0.0;
      for (int b0 = 0; b0 < nb; b0 += 16 * 64) {
        double v0[16], v1[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int b = b0 + q * 64 + lane;
          const int bc = b < nb ? b : nb - 1;  // a valid address; the value is dropped
          v0[q] = __hip_atomic_load(&a.part[j0 * (int64_t)nblk + bc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          v1[q] = __hip_atomic_load(&a.part[j1 * (int64_t)nblk + bc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (b0 + q * 64 + lane >= nb) { v0[q] = 0.0; v1[q] = 0.0; }
#pragma unroll
        for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
          for (int q = 0; q < w; ++q) { v0[q] += v0[q + w]; v1[q] += v1[q + w]; }
        h0 += v0[0];
        h1 += v1[0];
      }
      h0 = wave_sum(h0);
      h1 = wave_sum(h1);
      if (lane == 0) { fin[j0] = h0; fin[j1] = h1; }
    }
  }  // !solo
  __syncthreads();
  if (wid == 0) {
    // the epilogue (one lane) writes the result into LDS; the wavefront
    // copies it to the output and to the host's mapped copy
    constexpr int NOUT = RF_P + 2 + RF_NSUM;
    __shared__ double res[NOUT];
    for (int j = lane; j < NOUT; j += 64) res[j] = 0.0;
    if (lane == 0) rf_epilogue<MODE>(fin, cst, a.theta, res, (unsigned)fin[NSUM]);
    // each word of the host's copy by a system-scope store: the host polls
    // the words themselves (it armed them with a pattern no result has)
    for (int j = lane; j < NOUT; j += 64) {
      const double v = res[j];
      a.out[j] = v;
      if (a.hout) rf_store_host(a.hout + j, v);
    }
    if (lane == 0) rf_reset_ticket(a.ticket);
  }
}

// entry points, named by precision form: rf_k_{values,nll,grad}_{f32,f64}
#define RF_CAT2(x, y) x##y
#define RF_CAT(x, y) RF_CAT2(x, y)
// RF_WPE: wavefronts per SIMD the register allocation must allow (0: the
// compiler's choice)
#if RF_WPE > 0
#define RF_LB __launch_bounds__(RF_BS, RF_WPE)
#else
#define RF_LB __launch_bounds__(RF_BS)
#endif
extern "C" __global__ RF_LB void RF_CAT(rf_k_values_, RF_PREC)(const RfArgs a) { rf_body<0>(a); }
extern "C" __global__ RF_LB void RF_CAT(rf_k_nll_, RF_PREC)(const RfArgs a) { rf_body<1>(a); }
extern "C" __global__ RF_LB void RF_CAT(rf_k_grad_, RF_PREC)(const RfArgs a) { rf_body<2>(a); }
