// rf_mlp_dev.h -- wave-level engine of the 6-64-64-64-1 tanh MLP (BF16
// weights, FP32 accumulation) used by the surrogate PDF leaf, its
// normalisation kernel and the training kernels.  Requires rf_dev.h.
//
// Tiles.  A wavefront handles 64 rows (events or training samples) at once;
// row r belongs to lane r.  A hidden activation tile (64 features x 64 rows)
// lives in registers in the 32x32 MFMA accumulator layout (the same for the
// K = 8 and K = 16 bf16 forms): element v of lane l in block (mb, eb) holds
//     feature 32 mb + 8 (v/4) + 4 (l/32) + v%4,   row 32 eb + l%32,
// stored at h[(2 mb + eb) * 16 + v].  For out = W h the A operand is a
// fragment of W read from LDS and the B operand is a run of 8 registers of h.
// The 64x64 products use v_mfma_f32_32x32x16_bf16 (K = 16 per instruction).
// The sum over K does not depend on how the 16 features of a K-step are
// ordered, as long as A and B order them alike; K-step t takes, in lane half
// hl = l/32, the eight features 16 t + 4 hl + {0..3} and 16 t + 8 + 4 hl +
// {0..3}, which are exactly h[(2 (t/2) + eb) * 16 + 8 (t%2) + 0..7] -- the
// layer output is already the next layer's input layout, so nothing moves
// between layers.
//
// Precision.  Weights are exact in bf16.  FP32 activations enter the MFMA
// as NSPLIT bf16 parts h = h1 + h2 (+ h3) (each part the round-to-nearest
// bf16 of the remaining residual); every bf16 x bf16 product is exact in
// FP32 and the accumulation is FP32, so with NSPLIT = 3 a layer matches an
// FP32 matrix product (residual below 2^-24 |h|).
#pragma once

typedef short rf_bf16x4 __attribute__((ext_vector_type(4)));
typedef short rf_bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 rf_bf16v8 __attribute__((ext_vector_type(8)));  // MFMA operand type
typedef float rf_f32x16 __attribute__((ext_vector_type(16)));

// Compiler barrier (memory clobber) between the engine's phases and at the top
// of tile loops: the per-lane weight values stay in LDS and are read where they
// are used, instead of being hoisted early (or out of loops) into registers,
// which would spill.
#define MLP_TILE_BARRIER() __asm__ volatile("" ::: "memory")

#define MLP_NW 8833
#define MLP_RS 68  // LDS row stride (bf16 elements) of the 64x64 matrices
enum { MLP_OW1 = 0, MLP_OB1 = 384, MLP_OW2 = 448, MLP_OB2 = 4544, MLP_OW3 = 4608,
       MLP_OB3 = 8704, MLP_OW4 = 8768, MLP_OB4 = 8832 };

// Per-feature float arrays start on 16-byte boundaries: a lane reads the
// coefficients of its four consecutive features (mlp_c4) in one LDS access.
struct __attribute__((aligned(16))) MlpLds {
  unsigned short W2[64 * MLP_RS], W3[64 * MLP_RS];    // [out][in]
  unsigned short W2T[64 * MLP_RS], W3T[64 * MLP_RS];  // [in][out]
  float W1[64 * 6], b1[64], b2[64], b3[64], W4[64];
  // the surrogate leaf's layer 1, scaled by MLP_TANH_K: pre-activation
  // = (w10 u0 + c1) / MLP_TANH_K
  float w10[64];    // column 0 of W1 (the per-row input u0)
  float c1[64];     // the part from the row-independent inputs and the bias
  float gq[5][64];  // d(layer-1 pre-activation o)/d q_j of the surrogate leaf
  float b4;
};

RF_DEV float bf16_bits_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// block-wide: weights (8833 bf16) -> LDS
RF_DEV void mlp_load(const unsigned short* __restrict__ w, MlpLds& s) {
  for (int t = threadIdx.x; t < 4096; t += blockDim.x) {
    const int o = t >> 6, i = t & 63;
    const unsigned short v2 = w[MLP_OW2 + t], v3 = w[MLP_OW3 + t];
    s.W2[o * MLP_RS + i] = v2;
    s.W2T[i * MLP_RS + o] = v2;
    s.W3[o * MLP_RS + i] = v3;
    s.W3T[i * MLP_RS + o] = v3;
  }
  for (int t = threadIdx.x; t < 384; t += blockDim.x) s.W1[t] = bf16_bits_to_f32(w[MLP_OW1 + t]);
  for (int t = threadIdx.x; t < 64; t += blockDim.x) {
    s.b1[t] = bf16_bits_to_f32(w[MLP_OB1 + t]);
    s.b2[t] = bf16_bits_to_f32(w[MLP_OB2 + t]);
    s.b3[t] = bf16_bits_to_f32(w[MLP_OB3 + t]);
    s.W4[t] = bf16_bits_to_f32(w[MLP_OW4 + t]);
  }
  if (threadIdx.x == 0) s.b4 = bf16_bits_to_f32(w[MLP_OB4]);
}

RF_DEV int mlp_feat(int mb, int v, int hl) { return 32 * mb + 8 * (v >> 2) + 4 * hl + (v & 3); }

// c[mlp_feat(mb, 4 vq + 0..3, hl)] of a 16-byte aligned per-feature LDS array
RF_DEV float4 mlp_c4(const float* c, int mb, int vq, int hl) {
  return *(const float4*)&c[32 * mb + 8 * vq + 4 * hl];
}
RF_DEV float f4at(const float4& f, int i) { return i == 0 ? f.x : i == 1 ? f.y : i == 2 ? f.z : f.w; }

// tanh(x) = sign(x) (1 - t) / (1 + t), t = exp(-2|x|) = 2^(-|y|), y = 2 log2(e) x;
// with q = 1/(1 + t) the quotient is q - t q, one fused multiply-add.
// mlp_tanh_y takes y (inputs already scaled by 2 log2(e)).
#define MLP_TANH_K 2.8853900817779268f
RF_DEV float mlp_tanh_y(float y) {
  const float t = __builtin_amdgcn_exp2f(-fabsf(y));
  const float q = __builtin_amdgcn_rcpf(1.0f + t);
  return copysignf(fmaf(-t, q, q), y);
}
RF_DEV float mlp_tanh(float x) { return mlp_tanh_y(MLP_TANH_K * x); }

// Split 2 K consecutive activations into NS bf16 parts, packed as MFMA
// operands.  Pairs are converted together (one v_cvt_pk_bf16_f32, round to
// nearest even) and only whole packed words are reinterpreted: element 2 k of
// an operand is the low half of word k.
typedef float rf_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 rf_bf16v2 __attribute__((ext_vector_type(2)));
typedef unsigned rf_u32x4 __attribute__((ext_vector_type(4)));
RF_DEV unsigned bf16_pack2(float a, float b) {
  const rf_f32x2 f = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f, rf_bf16v2));
}
template <int NS, int K>
RF_DEV void mlp_split_words(const float* h, unsigned (&w)[NS][K]) {
  float r[2 * K];
#pragma unroll
  for (int i = 0; i < 2 * K; ++i) r[i] = h[i];
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      w[q][k] = bf16_pack2(r[2 * k], r[2 * k + 1]);
      if (q + 1 < NS) {  // residuals: exact in FP32
        r[2 * k] -= __uint_as_float(w[q][k] << 16);
        r[2 * k + 1] -= __uint_as_float(w[q][k] & 0xffff0000u);
      }
    }
}
template <int NS>
RF_DEV void mlp_split8(const float* h, rf_bf16v8* part) {
  unsigned w[NS][4];
  mlp_split_words<NS, 4>(h, w);
#pragma unroll
  for (int q = 0; q < NS; ++q)
    part[q] = __builtin_bit_cast(rf_bf16v8, (rf_u32x4){w[q][0], w[q][1], w[q][2], w[q][3]});
}

// Event blocks.  A call processes NEB blocks of 32 rows starting at block
// eb0 (NEB = 2, eb0 = 0: the whole 64-row tile; NEB = 1: one half, which
// halves the registers holding activations).  Tile storage of a layer:
// h[(NEB mb + e) * 16 + v] for e < NEB, row 32 (eb0 + e) + l%32.

// One 64x64 layer, W a 64x64 LDS matrix (row stride MLP_RS):
//   MODE 0 (forward):  out = tanh(W in + b)
//   MODE 1 (backward): out = (W in) * (1 - out^2)   (out holds h on entry)
//   MODE 2 (backward): out = (W in) * fac, fac[i] = b[i * 64 + lane] (LDS)
template <int NS, int MODE, int NEB>
RF_DEV void mlp_layer(const unsigned short* W, const float* b, const float* in, float* out) {
  MLP_TILE_BARRIER();  // phase boundary: keep this layer's LDS reads inside it
  const int l = threadIdx.x & 63, hl = l >> 5, lr = l & 31;
  rf_f32x16 acc[2][NEB];
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int vq = 0; vq < 4; ++vq) {
      const float4 b4 = MODE == 0 ? mlp_c4(b, mo, vq, hl) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < NEB; ++e) acc[mo][e][4 * vq + i] = f4at(b4, i);
    }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    rf_bf16v8 Bq[NEB][NS];
#pragma unroll
    for (int e = 0; e < NEB; ++e) mlp_split8<NS>(in + (NEB * (t >> 1) + e) * 16 + 8 * (t & 1), Bq[e]);
#pragma unroll
    for (int mo = 0; mo < 2; ++mo) {
      const unsigned short* wr = &W[(32 * mo + lr) * MLP_RS + 16 * t + 4 * hl];
      const rf_bf16x8 a8 = __builtin_shufflevector(*(const rf_bf16x4*)wr, *(const rf_bf16x4*)(wr + 8), 0, 1, 2, 3,
                                                   4, 5, 6, 7);
      const rf_bf16v8 A = __builtin_bit_cast(rf_bf16v8, a8);
#pragma unroll
      for (int q = NS - 1; q >= 0; --q)  // small parts first
#pragma unroll
        for (int e = 0; e < NEB; ++e)
          acc[mo][e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bq[e][q], acc[mo][e], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mo = 0; mo < 2; ++mo)
#pragma unroll
    for (int e = 0; e < NEB; ++e)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int idx = (NEB * mo + e) * 16 + v;
        float& o = out[idx];
        if (MODE == 0) o = mlp_tanh(acc[mo][e][v]);
        else if (MODE == 1) o = acc[mo][e][v] * (1.0f - o * o);
        else o = acc[mo][e][v] * b[idx * 64 + l];
      }
  MLP_TILE_BARRIER();
}

// the value of row (32 eb + l%32), owned by lane 32 eb + l%32
RF_DEV float mlp_rowval(float own, int eb) {
  const int hl = (threadIdx.x & 63) >> 5;
  const float other = __shfl_xor(own, 32, 64);
  return eb == hl ? own : other;
}

// layer 1 when only input 0 varies per row: a = W1[:,0] u0 + c (w10, c1 hold
// MLP_TANH_K times these coefficients)
template <int NEB>
RF_DEV void mlp_layer1_u0(const MlpLds& s, float u0, float* h1, int eb0) {
  MLP_TILE_BARRIER();
  const int hl = (threadIdx.x & 63) >> 5;
  float ue[NEB];
#pragma unroll
  for (int e = 0; e < NEB; ++e) ue[e] = mlp_rowval(u0, eb0 + e);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int vq = 0; vq < 4; ++vq) {
      const float4 w4 = mlp_c4(s.w10, mb, vq, hl), c4 = mlp_c4(s.c1, mb, vq, hl);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < NEB; ++e)
          h1[(NEB * mb + e) * 16 + 4 * vq + i] = mlp_tanh_y(fmaf(f4at(w4, i), ue[e], f4at(c4, i)));
    }
}

// layer 1 with all six inputs per row (training; whole tile)
RF_DEV void mlp_layer1_full(const MlpLds& s, const float* u, float* h1) {
  const int hl = (threadIdx.x & 63) >> 5;
  float ue[2][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    ue[0][j] = mlp_rowval(u[j], 0);
    ue[1][j] = mlp_rowval(u[j], 1);
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int o = mlp_feat(mb, v, hl);
#pragma unroll
      for (int eb = 0; eb < 2; ++eb) {
        float a = s.b1[o];
#pragma unroll
        for (int j = 0; j < 6; ++j) a = fmaf(s.W1[o * 6 + j], ue[eb][j], a);
        h1[(2 * mb + eb) * 16 + v] = mlp_tanh(a);
      }
    }
}

// NJ row sums in one pass over the tile: out[j] = sum over features f of
// coef[j * jstride + f] * t[f][row] for this lane's own row, valid on lanes
// whose row lies in the call's blocks (l/32 in [eb0, eb0 + NEB)); each
// coefficient array is contiguous in f and 16-byte aligned, so four
// features' coefficients come in one LDS access
template <int NEB, int NJ>
RF_DEV void mlp_rowdots(const float* coef, int jstride, const float* t, int eb0, float* out) {
  MLP_TILE_BARRIER();
  const int hl = (threadIdx.x & 63) >> 5;
  float p[NJ][NEB];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int e = 0; e < NEB; ++e) p[j][e] = 0.f;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int vq = 0; vq < 4; ++vq) {
      float4 c[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) c[j] = mlp_c4(coef + j * jstride, mb, vq, hl);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int e = 0; e < NEB; ++e)
            p[j][e] = fmaf(f4at(c[j], i), t[(NEB * mb + e) * 16 + 4 * vq + i], p[j][e]);
    }
  // the partner lane (l ^ 32) holds the other half of the features of the
  // same rows; it needs the block of its own row, 1 - hl
  const int ep = 1 - hl - eb0, eo = hl - eb0;
  float send[NJ], mine[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    send[j] = 0.f;
    mine[j] = 0.f;
#pragma unroll
    for (int e = 0; e < NEB; ++e) {
      if (e == ep) send[j] = p[j][e];
      if (e == eo) mine[j] = p[j][e];
    }
  }
  MLP_TILE_BARRIER();
#pragma unroll
  for (int j = 0; j < NJ; ++j) out[j] = mine[j] + __shfl_xor(send[j], 32, 64);
}

// ---- 32-row tiles for training: one wavefront per 32 rows, lanes l and
// l + 32 hold the two halves of the features of the same row l % 32 (the
// NEB = 1 tile layout).  Per element the arithmetic is that of the 64-row
// functions above, in the same order.

// sum over features of coef[f * stride] * t[f] for the lane's row, on both
// lanes of the row
template <int STRIDE>
RF_DEV float mlp_rowdot_pair(const float* coef, const float* t) {
  MLP_TILE_BARRIER();
  const int hl = (threadIdx.x & 63) >> 5;
  float p = 0.f;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int vq = 0; vq < 4; ++vq) {
      float c[4];
      if (STRIDE == 1) {
        const float4 c4 = mlp_c4(coef, mb, vq, hl);
        c[0] = c4.x; c[1] = c4.y; c[2] = c4.z; c[3] = c4.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = coef[mlp_feat(mb, 4 * vq + i, hl) * STRIDE];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) p = fmaf(c[i], t[mb * 16 + 4 * vq + i], p);
    }
  MLP_TILE_BARRIER();
  return p + __shfl_xor(p, 32, 64);
}

// layer 1 with all six inputs of the lane's own row
RF_DEV void mlp_layer1_pair(const MlpLds& s, const float* u, float* h1) {
  const int hl = (threadIdx.x & 63) >> 5;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int o = mlp_feat(mb, v, hl);
      float a = s.b1[o];
#pragma unroll
      for (int j = 0; j < 6; ++j) a = fmaf(s.W1[o * 6 + j], u[j], a);
      h1[mb * 16 + v] = mlp_tanh(a);
    }
}

template <int NS>
RF_DEV float mlp_forward_pair(const MlpLds& s, const float* u, float* h1, float* h2, float* h3) {
  mlp_layer1_pair(s, u, h1);
  mlp_layer<NS, 0, 1>(s.W2, s.b2, h1, h2);
  mlp_layer<NS, 0, 1>(s.W3, s.b3, h2, h3);
  return mlp_rowdot_pair<1>(s.W4, h3) + s.b4;
}

// backward from the row's output cotangent g: d1, d2, d3 replace h1, h2, h3
template <int NS>
RF_DEV void mlp_backward_pair(const MlpLds& s, float g, float* h1, float* h2, float* h3) {
  const int hl = (threadIdx.x & 63) >> 5;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int vq = 0; vq < 4; ++vq) {
      const float4 w4 = mlp_c4(s.W4, mb, vq, hl);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float& t = h3[mb * 16 + 4 * vq + i];
        t = g * f4at(w4, i) * (1.0f - t * t);
      }
    }
  mlp_layer<NS, 1, 1>(s.W3T, nullptr, h3, h2);
  mlp_layer<NS, 1, 1>(s.W2T, nullptr, h2, h1);
}

// Half-tile forward/backward for the surrogate leaf (NEB = 1, block eb0):
// layer 1's derivative factor (1 - h1^2) is parked in the wavefront's LDS
// tile sav[32 * 64] (lane-contiguous) instead of registers.
template <int NS>
RF_DEV float mlp_forward_half(const MlpLds& s, float u0, int eb0, float* sav, float* h2, float* h3) {
  const int l = threadIdx.x & 63;
  float h1[32];
  mlp_layer1_u0<1>(s, u0, h1, eb0);
  mlp_layer<NS, 0, 1>(s.W2, s.b2, h1, h2);
#pragma unroll
  for (int i = 0; i < 32; ++i) sav[i * 64 + l] = 1.0f - h1[i] * h1[i];
  mlp_layer<NS, 0, 1>(s.W3, s.b3, h2, h3);
  float o;
  mlp_rowdots<1, 1>(s.W4, 0, h3, eb0, &o);
  return o + s.b4;
}
template <int NS>
RF_DEV void mlp_backward_half(const MlpLds& s, int eb0, const float* sav, float* d1, float* h2, float* h3) {
  const int hl = (threadIdx.x & 63) >> 5;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int vq = 0; vq < 4; ++vq) {
      const float4 w4 = mlp_c4(s.W4, mb, vq, hl);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float& t = h3[mb * 16 + 4 * vq + i];
        t = f4at(w4, i) * (1.0f - t * t);  // cotangent 1 per row
      }
    }
  mlp_layer<NS, 1, 1>(s.W3T, nullptr, h3, h2);
  mlp_layer<NS, 2, 1>(s.W2T, sav, h2, d1);
}

// s and ds/dq_j (GRAD) of the lane's own row, two half-tile passes
template <int NS, bool GRAD>
RF_DEV float mlp_eval_u0(const MlpLds& s, float u0, float* sav, float* dq) {
  const int hl = (threadIdx.x & 63) >> 5;
  float out = 0.f;
#pragma unroll
  for (int j = 0; j < 5; ++j) dq[j] = 0.f;
#pragma unroll 1
  for (int eb0 = 0; eb0 < 2; ++eb0) {  // not unrolled: one half's state at a time
    MLP_TILE_BARRIER();
    float h2[32], h3[32];
    const float sv = mlp_forward_half<NS>(s, u0, eb0, sav, h2, h3);
    if (hl == eb0) out = sv;
    if (GRAD) {
      float d1[32];
      mlp_backward_half<NS>(s, eb0, sav, d1, h2, h3);
      float gj[5];
      mlp_rowdots<1, 5>(&s.gq[0][0], 64, d1, eb0, gj);
#pragma unroll
      for (int j = 0; j < 5; ++j)
        if (hl == eb0) dq[j] = gj[j];
    }
  }
  return out;
}

// ------------------------------------------------------ surrogate PDF leaf --
// u(x; q) = exp(s(u0, u1..u5)), u_j = 2 (r_j - lo_j)/(hi_j - lo_j) - 1 with
// r = (x - q1, q1..q5) (the first input is the position relative to q1, the
// Breit-Wigner mass); normalised by Nhat(q) = sum_g w_g exp(s(x_g, q)) over a
// Gauss-Legendre grid on x's range (computed by rf_mlp_renorm before the
// likelihood kernel, delivered as [Nhat, dNhat/dq1..5] in the aux block).
// Constant block: C[0] = 1/Nhat, C[1..5] = d log Nhat / dq_j.
enum { MLP_NC = 8 };

// block-wide: weights -> LDS, layer-1 constant of the five row-independent
// inputs q (raw values, box = 6 (lo, hi) pairs, x first), and the scale
// factors du_j/dq_j
template <int BS>
__device__ void mlp_setup(const double* q, const double* box, const unsigned short* w, MlpLds& s, float* qs) {
  mlp_load(w, s);
  __syncthreads();
  for (int o = threadIdx.x; o < 64; o += BS) {
    float c = s.b1[o];
    for (int j = 1; j < 6; ++j) {
      const double u = 2.0 * (q[j - 1] - box[2 * j]) / (box[2 * j + 1] - box[2 * j]) - 1.0;
      c = fmaf(s.W1[o * 6 + j], (float)u, c);
    }
    s.c1[o] = MLP_TANH_K * c;
    s.w10[o] = MLP_TANH_K * s.W1[o * 6];
  }
  if (threadIdx.x < 5) qs[threadIdx.x] = (float)(2.0 / (box[2 * threadIdx.x + 3] - box[2 * threadIdx.x + 2]));
  // u0 = map of (x - q1): q1 enters layer 1 through u0 as well
  const double s0 = 2.0 / (box[1] - box[0]);
  for (int t = threadIdx.x; t < 5 * 64; t += BS) {
    const int j = t / 64, o = t % 64;
    double g = (double)s.W1[o * 6 + j + 1] * 2.0 / (box[2 * j + 3] - box[2 * j + 2]);
    if (j == 0) g -= (double)s.W1[o * 6] * s0;
    s.gq[j][o] = (float)g;
  }
}

// ---- analytic base of the surrogate --------------------------------------
// The network learns the residual r = log p_sig - log b over an analytic
// base b(d = x - M; Gamma, sigma, alpha, n): a pseudo-Voigt -- the mixture of
// a Lorentzian and a Gaussian of common full width f with weight eta, by
// Thompson, Cox & Hastings (J. Appl. Cryst. 20 (1987) 79), f_G = 2 sigma
// sqrt(2 ln 2), f_L = Gamma -- whose Gaussian part carries the Crystal Ball's
// power-law tail below z = -alpha (z in units of the component's width
// s_e = f / (2 sqrt(2 ln 2))):
//   b = eta L(d) + (1 - eta) C(d / s_e) / (s_e sqrt(2 pi)),
//   L(d) = (h / pi) / (d^2 + h^2), h = f / 2,
//   C(z) = exp(-z^2/2) (z > -alpha), exp(log A - n log(B - z)) otherwise,
//   A = (n/alpha)^n exp(-alpha^2/2), B = n/alpha - alpha.
// The base carries most of log p_sig's variation (the residual's spread is
// ~20x smaller), so the same network is far more accurate.  Parameter-only
// constants, FP64, layout MB_* below (offsets inside the leaf's block).
enum { MB_H = 8, MB_CL, MB_ISE, MB_CG, MB_ETA, MB_AL, MB_N, MB_LOGA, MB_B, MB_DFG, MB_DFS, MB_DEG, MB_DES, MB_INVC0,
       MB_M, MB_END };
RF_DEV void mlp_base_constants(const double* q, double* C) {
  const double G = q[1], sg = q[2], al = q[3], n = q[4];
  const double c0 = 2.0 * ::sqrt(2.0 * ::log(2.0));
  const double fg = c0 * sg, fl = G;
  const double P = fg * fg * fg * fg * fg + 2.69269 * fg * fg * fg * fg * fl + 2.42843 * fg * fg * fg * fl * fl +
                   4.47163 * fg * fg * fl * fl * fl + 0.07842 * fg * fl * fl * fl * fl + fl * fl * fl * fl * fl;
  const double dPg = 5 * fg * fg * fg * fg + 4 * 2.69269 * fg * fg * fg * fl + 3 * 2.42843 * fg * fg * fl * fl +
                     2 * 4.47163 * fg * fl * fl * fl + 0.07842 * fl * fl * fl * fl;
  const double dPl = 2.69269 * fg * fg * fg * fg + 2 * 2.42843 * fg * fg * fg * fl + 3 * 4.47163 * fg * fg * fl * fl +
                     4 * 0.07842 * fg * fl * fl * fl + 5 * fl * fl * fl * fl;
  const double f = ::pow(P, 0.2);
  const double df_dP = 0.2 * f / P;
  const double dfG = df_dP * dPl, dfS = df_dP * dPg * c0;  // df/dGamma, df/dsigma
  const double r = fl / f;
  const double eta = 1.36603 * r - 0.47719 * r * r + 0.11116 * r * r * r;
  const double deta_dr = 1.36603 - 2 * 0.47719 * r + 3 * 0.11116 * r * r;
  const double se = f / c0;
  C[MB_H] = 0.5 * f;
  C[MB_CL] = 0.5 * f / RF_PI;
  C[MB_ISE] = 1.0 / se;
  C[MB_CG] = 1.0 / (se * RF_SQRT2PI);
  C[MB_ETA] = eta;
  C[MB_AL] = al;
  C[MB_N] = n;
  C[MB_LOGA] = n * ::log(n / al) - 0.5 * al * al;
  C[MB_B] = n / al - al;
  C[MB_DFG] = dfG;
  C[MB_DFS] = dfS;
  C[MB_DEG] = deta_dr * (1.0 / f - fl * dfG / (f * f));
  C[MB_DES] = deta_dr * (-fl * dfS / (f * f));
  C[MB_INVC0] = 1.0 / c0;
  C[MB_M] = q[0];
}
struct MlpBase {
  Loc<float> M;
  float h, cl, ise, cg, eta, al, n, logA, B, dfG, dfS, deG, deS, ic0;
  RF_DEV MlpBase make(const double* C) {
    MlpBase b;
    b.M = Loc<float>::make(C[MB_M]);
    b.h = (float)C[MB_H]; b.cl = (float)C[MB_CL]; b.ise = (float)C[MB_ISE]; b.cg = (float)C[MB_CG];
    b.eta = (float)C[MB_ETA]; b.al = (float)C[MB_AL]; b.n = (float)C[MB_N]; b.logA = (float)C[MB_LOGA];
    b.B = (float)C[MB_B]; b.dfG = (float)C[MB_DFG]; b.dfS = (float)C[MB_DFS]; b.deG = (float)C[MB_DEG];
    b.deS = (float)C[MB_DES]; b.ic0 = (float)C[MB_INVC0];
    return b;
  }
};
// base value b at x; with GRAD, db[j] = d log b / d q_{j+1}, q = (M, Gamma, sigma, alpha, n)
template <bool GRAD> RF_DEV float mlp_base(float x, const MlpBase& B, float* db) {
  const float d = B.M.sub(x);
  const float iD = __builtin_amdgcn_rcpf(fmaf(d, d, B.h * B.h));
  const float L = B.cl * iD;
  const float z = d * B.ise;
  const bool core = z > -B.al;
  float g, C, ga = 0.f, gn = 0.f;  // g = d log C / dz; ga, gn = d log C / d(alpha, n)
  if (core) {
    C = __expf(-0.5f * z * z);
    g = -z;
  } else {
    const float t = B.B - z, it = __builtin_amdgcn_rcpf(t), lt = __logf(t);
    C = __expf(B.logA - B.n * lt);
    g = B.n * it;
    ga = (-B.n / B.al - B.al) + B.n * (B.n / (B.al * B.al) + 1.f) * it;
    gn = (__logf(B.n / B.al) + 1.f) - lt - (B.n / B.al) * it;
  }
  const float Gn = B.cg * C;
  const float pv = fmaf(B.eta, L - Gn, Gn);
  if (GRAD) {
    const float ip = __builtin_amdgcn_rcpf(pv);
    const float omE = 1.f - B.eta;
    const float dLd = -2.f * d * L * iD, dGd = Gn * g * B.ise;
    const float dLf = 0.5f * L * (1.f / B.h - 2.f * B.h * iD);
    const float dGf = -Gn * (1.f + g * z) * B.ise * B.ic0;
    const float dpf = fmaf(B.eta, dLf, omE * dGf), dpe = L - Gn;
    db[0] = -ip * fmaf(B.eta, dLd, omE * dGd);
    db[1] = ip * fmaf(dpf, B.dfG, dpe * B.deG);
    db[2] = ip * fmaf(dpf, B.dfS, dpe * B.deS);
    db[3] = ip * omE * Gn * ga;
    db[4] = ip * omE * Gn * gn;
  }
  return pv;
}

template <int BS>
__device__ void mlp_prologue(const double* q, const double* box, const double* nh, int nrow,
                             const unsigned short* w, double* C, MlpLds& s, float* qs) {
  mlp_setup<BS>(q, box, w, s, qs);
  if (threadIdx.x == 0) {
    // nh: nrow rows [Nhat, dNhat/dq1..5], one per workgroup of the
    // normalisation kernel, added in row order
    double t[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < nrow; ++r)
      for (int j = 0; j < 6; ++j) t[j] += nh[r * 6 + j];
    C[0] = 1.0 / t[0];
    for (int j = 0; j < 5; ++j) C[1 + j] = t[1 + j] / t[0];
    C[6] = 2.0 / (box[1] - box[0]);               // du0/dx
    C[7] = -(q[0] + box[0]) * C[6] - 1.0;          // u0 = x C[6] + C[7]
    mlp_base_constants(q, C);
  }
}

template <typename T> struct MlpK {
  T invN;
  float xs, xo;
  const MlpLds* s;
  float* sav;  // this wavefront's LDS tile for (1 - h1^2) of a half tile
  MlpBase base;
  RF_DEV MlpK make(const double* C, const MlpLds* s, float* sav_base) {
    MlpK k;
    k.invN = (T)C[0];
    k.xs = (float)C[6];
    k.xo = (float)C[7];
    k.s = s;
    k.sav = sav_base + (threadIdx.x >> 6) * 32 * 64;
    k.base = MlpBase::make(C);
    return k;
  }
};

// wave-cooperative: every lane of the wavefront must call it together.
// Returns exp(s) b(x) for the lane's event; with GRAD, d[j] = d(s + log b)/dq_{j+1}.
template <typename T, int NS, bool GRAD>
RF_DEV T mlp_leaf_eval(T x, const MlpK<T>& k, T* d) {
  const float u0 = fmaf((float)x, k.xs, k.xo);
  float dq[5], db[5];
  const float sv = mlp_eval_u0<NS, GRAD>(*k.s, u0, k.sav, dq);
  const float bv = mlp_base<GRAD>((float)x, k.base, db);
  if (GRAD)
#pragma unroll
    for (int j = 0; j < 5; ++j) d[j] = (T)(dq[j] + db[j]);
  return (T)(expf(sv) * bv);
}
