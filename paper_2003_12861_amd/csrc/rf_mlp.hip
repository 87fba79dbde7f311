// rf_mlp.hip -- kernels of the learned surrogate: the normalisation of the
// surrogate PDF, training forward/backward/Adam, and the exact convolution
// targets it is trained on.
//
// The surrogate replaces the expensive numerically convolved signal PDF
// (Breit-Wigner (x) Crystal Ball by a K-point rule) with a 6-64-64-64-1 tanh
// MLP s(x, M, Gamma, sigma, alpha, n) ~ log p_sig, BF16 weights and FP32
// accumulation on the matrix cores (see device/rf_mlp_dev.h for the tile
// layout).  Training uses the project's own kernels end to end:
//   targets  rf_bwcb_logpdf   exact log p_sig at per-sample parameters (FP64)
//   forward  rf_mlp_forward   MFMA forward of 64-row tiles per wavefront
//   loss     rf_mse_grad      dL/ds for a mean-squared-error loss
//   backward rf_mlp_backward  MFMA backward of the activations; weight
//                             gradients from LDS-staged tiles, one private
//                             partial per workgroup, summed in a fixed order
//   update   rf_adam_step     Adam on FP32 master weights, BF16 copy (RNE)
//   step     rf_mlp_train_step  one optimiser step in two launches: the
//                             backward kernel gathers its batch rows by index
//                             and forms the loss cotangent from the forward
//                             pass it runs anyway; Adam runs inside the
//                             reduction of the weight gradients
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "device/rf_dev.h"
#include "device/rf_mlp_dev.h"
#include "rf_internal.h"

#define MLP_SPLIT 3

namespace {

// ---------------------------------------------------------- normalisation --
struct RenormArgs {
  const unsigned short* w;
  const double* grid;  // [x_0..x_{K-1}, w_0..w_{K-1}] on x's range
  double* out;         // per workgroup: [Nhat, dNhat/dq1..5] of its tiles
  int K;
  int pad_;
  double q[5];
  double box[12];
};

// workgroups of four wavefronts, one 64-point tile of the rule per
// wavefront (MLP_RN_TILES tiles per workgroup); each workgroup writes its six
// sums, which the fused kernel's prologue adds in workgroup order
#define RN_W 4
__global__ __launch_bounds__(64 * RN_W) void mlp_renorm_kernel(const RenormArgs a) {
  __shared__ MlpLds s;
  __shared__ float qs[5];
  __shared__ double red[RN_W][6];
  __shared__ float sav[RN_W * 32 * 64];
  __shared__ double bc[MB_END];
  mlp_setup<64 * RN_W>(a.q, a.box, a.w, s, qs);
  if (threadIdx.x == 0) mlp_base_constants(a.q, bc);
  __syncthreads();
  const MlpBase B = MlpBase::make(bc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const double xsd = 2.0 / (a.box[1] - a.box[0]);
  const float xs = (float)xsd;
  const float xo = (float)(-(a.q[0] + a.box[0]) * xsd - 1.0);  // u0 = map of (x - q1)
  for (int t = blockIdx.x * RN_W + wid; t * 64 < a.K; t += gridDim.x * RN_W) {  // wave-uniform loop
    MLP_TILE_BARRIER();
    const int g = t * 64 + lane;
    const bool valid = g < a.K;
    const double xg = a.grid[valid ? g : 0];
    const double wg = valid ? a.grid[a.K + g] : 0.0;
    const float u0 = fmaf((float)xg, xs, xo);
    float dq[5], db[5];
    const float sv = mlp_eval_u0<MLP_SPLIT, true>(s, u0, sav + wid * 32 * 64, dq);
    const float bv = mlp_base<true>((float)xg, B, db);
    const double e = wg * exp((double)sv) * (double)bv;
    acc[0] += e;
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[1 + j] += e * (double)(dq[j] + db[j]);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[wid][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double h = 0.0, l = 0.0;
    for (int w = 0; w < RN_W; ++w) dd_add(h, l, red[w][threadIdx.x], 0.0);
    a.out[blockIdx.x * 6 + threadIdx.x] = h + l;
  }
}

// ----------------------------------------------------------------- forward --
// act (optional): per row the three hidden layers [h1 | h2 | h3], stored as
// each layer completes so that no more than two layers are live at a time
RF_DEV void mlp_store_act(float* act, int64_t t, int64_t n, int L, const float* h) {
  const int lane = threadIdx.x & 63, hl = lane >> 5, lr = lane & 31;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int eb = 0; eb < 2; ++eb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = t * 64 + 32 * eb + lr;
        if (r < n) act[r * 192 + 64 * L + mlp_feat(mb, v, hl)] = h[(2 * mb + eb) * 16 + v];
      }
}

template <bool ACT>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const unsigned short* w, const float* in, int64_t n,
                                                      float* out, float* act) {
  __shared__ MlpLds s;
  mlp_load(w, s);
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t ntile = (n + 63) / 64;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wid; t < ntile; t += (int64_t)gridDim.x * 4) {
    MLP_TILE_BARRIER();
    const int64_t row = t * 64 + lane;
    const bool valid = row < n;
    float u[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) u[j] = valid ? in[row * 6 + j] : 0.0f;
    float ha[64], hb[64];
    mlp_layer1_full(s, u, ha);
    if (ACT) mlp_store_act(act, t, n, 0, ha);
    mlp_layer<MLP_SPLIT, 0, 2>(s.W2, s.b2, ha, hb);
    if (ACT) mlp_store_act(act, t, n, 1, hb);
    mlp_layer<MLP_SPLIT, 0, 2>(s.W3, s.b3, hb, ha);
    if (ACT) mlp_store_act(act, t, n, 2, ha);
    float sv;
    mlp_rowdots<2, 1>(s.W4, 0, ha, 0, &sv);
    sv += s.b4;
    if (valid) out[row] = sv;
  }
}

// ---------------------------------------------------------------- backward --
#define TS 65  // LDS row stride of the staged [row][feature] tiles
struct BwdLds {
  float HT[3][64 * TS];  // forward activations h1, h2, h3
  float DT[3][64 * TS];  // dL/d(pre-activation) d1, d2, d3
  float UT[64 * 6];
  float G[64];
};

// dW[o][i] += sum over the tile's 64 rows r of D[o][r] H[i][r] on MFMA
// (v_mfma_f32_32x32x16_bf16): M = o, N = i, K = r.  The operands come from
// the staged [row][feature] tiles: in K-step t, lane l provides rows 16 t +
// 8 (l/32) + 0..7 of D[32 mo + l%32][.] (A) and of H[32 ni + l%32][.] (B);
// both operands order the 16 rows of a step alike.  Both are FP32 and enter
// as three bf16 parts each; the six products of parts whose orders add up to
// at most two are accumulated (small ones first), which matches an FP32
// product to about 2^-24.  acc[m][ni][v] = dW[mlp_feat(mo0 + m, v, l/32)][32 ni + l%32]
// for the NM output row blocks mo0 .. mo0 + NM - 1.
template <int NM>
RF_DEV void mlp_dw_mfma(const float* D, const float* H, int mo0, rf_f32x16 (&acc)[NM][2]) {
  const int l = threadIdx.x & 63, hl = l >> 5, lr = l & 31;
#pragma unroll 1  // one K-step at a time: unrolling spills
  for (int t = 0; t < 4; ++t) {
    rf_bf16v8 Ap[NM][3], Bp[2][3];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      float a8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) a8[j] = D[(16 * t + 8 * hl + j) * TS + 32 * (mo0 + m) + lr];
      mlp_split8<3>(a8, Ap[m]);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float b8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) b8[j] = H[(16 * t + 8 * hl + j) * TS + 32 * m + lr];
      mlp_split8<3>(b8, Bp[m]);
    }
#pragma unroll
    for (int ord = 2; ord >= 0; --ord)
#pragma unroll
      for (int qa = 0; qa <= ord; ++qa)
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
            acc[m][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ap[m][qa], Bp[ni][ord - qa], acc[m][ni], 0, 0, 0);
  }
}

// Cotangent source of the backward kernel: given per row (dout), or the
// mean-squared-error gradient scale (s - target[src]) of the forward output s
// (target != nullptr); rows are in[src], src = idx ? idx[row] : row, an index
// clamped into [0, nsrc) (rows of in and target) so that no read leaves them.
struct BwdRows {
  const float* dout;
  const int64_t* idx;
  const float* target;
  float scale;
  int64_t nsrc;
};

// A workgroup of two wavefronts takes a 64-row tile: wavefront wv runs the
// forward and backward passes of rows 32 wv .. 32 wv + 31 (32-row tiles),
// both stage their activations and cotangents in LDS, then wavefront wv
// forms the weight-gradient rows 32 wv .. 32 wv + 31 of the two hidden
// layers and one share of the per-unit sums.
#define BWD_W 2
template <bool FUSED>
__global__ __launch_bounds__(64 * BWD_W) void mlp_bwd_kernel(const unsigned short* w, const float* in, const BwdRows r,
                                                             int64_t n, float* part, float* din) {
  __shared__ MlpLds s;
  __shared__ BwdLds b;
  mlp_load(w, s);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, hl = lane >> 5, lr = lane & 31;
  const int er = 32 * wv + lr;  // the lane's row in the tile
  float* P = part + (size_t)blockIdx.x * MLP_NW;
  __syncthreads();
  const int64_t ntile = (n + 63) / 64;
  for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
    MLP_TILE_BARRIER();
    const int64_t row = t * 64 + er;
    const bool valid = row < n;
    int64_t src = !valid ? 0 : (FUSED && r.idx) ? r.idx[row] : row;
    src = src < 0 ? 0 : (src >= r.nsrc ? r.nsrc - 1 : src);
    float u[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) u[j] = valid ? in[src * 6 + j] : 0.0f;
    // the row's target (or cotangent) is read before the forward pass, so its
    // latency overlaps the network
    const float gin = !valid ? 0.0f : FUSED ? r.target[src] : r.dout[row];
    float h[3][32];
    const float sv = mlp_forward_pair<MLP_SPLIT>(s, u, h[0], h[1], h[2]);
    const float g = FUSED && valid ? r.scale * (sv - gin) : gin;
    // stage forward activations, inputs and output cotangents
#pragma unroll
    for (int L = 0; L < 3; ++L)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int v = 0; v < 16; ++v) b.HT[L][er * TS + mlp_feat(mb, v, hl)] = h[L][mb * 16 + v];
    if (hl == 0) {
#pragma unroll
      for (int j = 0; j < 6; ++j) b.UT[er * 6 + j] = u[j];
      b.G[er] = g;
    }
    mlp_backward_pair<MLP_SPLIT>(s, g, h[0], h[1], h[2]);
#pragma unroll
    for (int L = 0; L < 3; ++L)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int v = 0; v < 16; ++v) b.DT[L][er * TS + mlp_feat(mb, v, hl)] = h[L][mb * 16 + v];
    if (din) {  // uniform: every lane takes part in the cross-lane sums
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const float gj = mlp_rowdot_pair<6>(s.W1 + j, h[0]);
        if (valid && hl == 0) din[row * 6 + j] = gj;
      }
    }
    __syncthreads();
    // weight gradients, summed over the 64 rows of the tile; the block's
    // first tile writes its partial, later ones add to it
    const bool first = t == (int64_t)blockIdx.x;
    auto put = [&](int k, float v) { P[k] = first ? v : P[k] + v; };
    // layers 3 (d3 x h2) and 2 (d2 x h1) on MFMA (one layer at a time),
    // output rows 32 wv .. 32 wv + 31
#pragma unroll 1
    for (int L = 2; L >= 1; --L) {
      rf_f32x16 acc[1][2];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[0][ni][v] = 0.0f;
      mlp_dw_mfma<1>(b.DT[L], b.HT[L - 1], wv, acc);
      const int ow = L == 2 ? MLP_OW3 : MLP_OW2;
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int v = 0; v < 16; ++v) put(ow + mlp_feat(wv, v, hl) * 64 + 32 * ni + lr, acc[0][ni][v]);
    }
    // per-unit sums over the rows (lane = unit o): wavefront 0 the biases of
    // layers 2 and 3 and the output layer (g x h3), wavefront 1 layer 1
    // (d1 x u) and its bias
    {
      const int o = lane;
      if (wv == 0) {
        float bb2 = 0.0f, bb3 = 0.0f, acc4 = 0.0f, accg = 0.0f;
#pragma unroll 1
        for (int e0 = 0; e0 < 64; e0 += 8) {  // eight rows' LDS reads issued together
          float d3[8], d2[8], h3[8], gg[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int e = e0 + q;
            d3[q] = b.DT[2][e * TS + o];
            d2[q] = b.DT[1][e * TS + o];
            h3[q] = b.HT[2][e * TS + o];
            gg[q] = b.G[e];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            bb3 += d3[q];
            bb2 += d2[q];
            acc4 = fmaf(gg[q], h3[q], acc4);
            accg += gg[q];
          }
        }
        put(MLP_OB3 + o, bb3);
        put(MLP_OB2 + o, bb2);
        put(MLP_OW4 + o, acc4);
        if (o == 0) put(MLP_OB4, accg);
      } else {
        float acc1[6] = {0, 0, 0, 0, 0, 0}, bb1 = 0.0f;
#pragma unroll 1
        for (int e0 = 0; e0 < 64; e0 += 8) {
          float d1[8], uu[8][6];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int e = e0 + q;
            d1[q] = b.DT[0][e * TS + o];
#pragma unroll
            for (int j = 0; j < 6; ++j) uu[q][j] = b.UT[e * 6 + j];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            bb1 += d1[q];
#pragma unroll
            for (int j = 0; j < 6; ++j) acc1[j] = fmaf(d1[q], uu[q][j], acc1[j]);
          }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) put(MLP_OW1 + o * 6 + j, acc1[j]);
        put(MLP_OB1 + o, bb1);
      }
    }
    __syncthreads();
  }
}

// dw[k] = sum over the blocks' partials, in a fixed order: wavefront w of a
// 256-thread block adds partial rows w, w + 4, ... for 64 consecutive k (16
// loads in flight per lane, pairwise), the four wavefront sums are added in
// order
struct AdamArgs {
  float* w32;
  unsigned short* wbf;
  float *m, *v;
  float lr, b1, b2, eps, c1, c2;
};
// Adam update of weight i with gradient gi from its current state (m0, v0,
// w0); writes the state and refreshes the BF16 copy
__device__ __forceinline__ void adam_update(const AdamArgs& a, int64_t i, float gi, float m0, float v0, float w0) {
  const float mi = a.b1 * m0 + (1.0f - a.b1) * gi;
  const float vi = a.b2 * v0 + (1.0f - a.b2) * gi * gi;
  a.m[i] = mi;
  a.v[i] = vi;
  const float wi = w0 - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
  a.w32[i] = wi;
  const __bf16 hb = (__bf16)wi;  // round to nearest even
  a.wbf[i] = __builtin_bit_cast(unsigned short, hb);
}

template <bool ADAM>
__global__ __launch_bounds__(256) void mlp_dw_reduce_kernel(const float* part, int nblk, float* dw, const AdamArgs ad) {
  __shared__ double ws[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const int kc = k < MLP_NW ? k : MLP_NW - 1;
  // the optimiser state is read up front, overlapping the partials' loads
  float m0 = 0.f, v0 = 0.f, w0 = 0.f;
  if (ADAM && w == 0) {
    m0 = ad.m[kc];
    v0 = ad.v[kc];
    w0 = ad.w32[kc];
  }
  double h = 0.0;
  for (int b0 = w; b0 < nblk; b0 += 4 * 16) {
    float v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int b = b0 + 4 * q;
      v[q] = part[(size_t)(b < nblk ? b : w) * MLP_NW + kc];
    }
    double d[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) d[q] = b0 + 4 * q < nblk ? (double)v[q] : 0.0;
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1)
#pragma unroll
      for (int q = 0; q < m; ++q) d[q] += d[q + m];
    h += d[0];
  }
  ws[w][lane] = h;
  __syncthreads();
  if (w == 0 && k < MLP_NW) {
    const float gk = (float)((ws[0][lane] + ws[1][lane]) + (ws[2][lane] + ws[3][lane]));
    if (dw) dw[k] = gk;
    if (ADAM) adam_update(ad, k, gk, m0, v0, w0);
  }
}

__global__ void adam_kernel(const AdamArgs a, const float* g, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) adam_update(a, i, g[i], a.m[i], a.v[i], a.w32[i]);
}

__global__ void mse_grad_kernel(const float* out, const float* y, int64_t n, float scale, float* dout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dout[i] = scale * (out[i] - y[i]);
}

// exact log p_sig(x; M, Gamma, sigma, alpha, n) per sample (FP64): the same
// rule as the convolution leaf, with per-sample parameters
// RESID = false: out (double) = log p_sig; true: out (float) = log p_sig -
// log b, b the surrogate leaf's analytic base exactly as the leaf evaluates it
// (its FP64 constants, its FP32 value), the residual the network learns
template <bool RESID>
__global__ void bwcb_logpdf_kernel(const double* xq, int64_t n, const double* gl, int K, double lo, double hi,
                                   void* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = xq[i * 6], M = xq[i * 6 + 1], G = xq[i * 6 + 2];
  const double sg = xq[i * 6 + 3], al = xq[i * 6 + 4], nn = xq[i * 6 + 5];
  double S = 0.0, N = 0.0;
  for (int k = 0; k < K; ++k) {
    const double y = gl[k], wk = gl[K + k];
    double dc[3];
    const double c = wk * cb_shape(y, sg, al, nn, dc);
    const double q = x - y - M;
    S += c / (q * q + 0.25 * G * G);
    double I, dIM, dIG;
    bw_norm(lo - y, hi - y, M, G, &I, &dIM, &dIG);
    N += c * I;
  }
  const double lp = log(S / N);
  if (RESID) {
    double C[MB_END];
    const double q[5] = {M, G, sg, al, nn};
    mlp_base_constants(q, C);
    const MlpBase B = MlpBase::make(C);
    ((float*)out)[i] = (float)(lp - (double)logf(mlp_base<false>((float)x, B, nullptr)));
  } else {
    ((double*)out)[i] = lp;
  }
}

int launch_err(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RF_OK : rf::hip_fail(e, what);
}

std::mutex g_ws_mu;
// per-workgroup partial weight gradients of the backward kernel: one buffer
// per (device, stream), so that calls on different streams never share one
// (calls on one stream are ordered by the stream)
struct PartWs {
  int dev;
  void* stream;
  float* p;
  size_t n;
};
std::vector<PartWs> g_parts;
double* g_gl = nullptr;
int g_gl_K = 0;
double g_gl_lo = 0, g_gl_hi = 0;

}  // namespace

namespace rf {
int mlp_renorm_launch(const void* w, const double* q5, const double* box12, const double* grid, int K, double* out,
                      void* stream) {
  RenormArgs a;
  memset(&a, 0, sizeof a);
  a.w = (const unsigned short*)w;
  a.grid = grid;
  a.out = out;
  a.K = K;
  for (int j = 0; j < 5; ++j) a.q[j] = q5[j];
  for (int j = 0; j < 12; ++j) a.box[j] = box12[j];
  hipLaunchKernelGGL(mlp_renorm_kernel, dim3(mlp_renorm_blocks(K)), dim3(64 * RN_W), 0, (hipStream_t)stream, a);
  return launch_err("mlp_renorm");
}
}  // namespace rf

namespace {
using namespace rf;
AdamArgs adam_args(float* w32, void* wbf, float* m, float* v, float lr, float beta1, float beta2, float eps,
                   int32_t step) {
  AdamArgs a;
  a.w32 = w32;
  a.wbf = (unsigned short*)wbf;
  a.m = m;
  a.v = v;
  a.lr = lr;
  a.b1 = beta1;
  a.b2 = beta2;
  a.eps = eps;
  a.c1 = 1.0f - powf(beta1, (float)step);
  a.c2 = 1.0f - powf(beta2, (float)step);
  return a;
}

// backward over n rows + the ordered reduction of the per-workgroup partials
// (with Adam applied to the summed gradient when ad is given)
int backward_launch(const void* w, const float* in, const BwdRows& r, int64_t n, float* dw, float* din,
                    const AdamArgs* ad, void* stream) {
  const int64_t ntile = (n + 63) / 64;
  int nblk = (int)(ntile < 512 ? ntile : 512);
  int dev = 0;
  hipError_t de = hipGetDevice(&dev);
  if (de != hipSuccess) return hip_fail(de, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  PartWs* ws = nullptr;
  for (PartWs& q : g_parts)
    if (q.dev == dev && q.stream == stream) ws = &q;
  if (!ws) {
    g_parts.push_back(PartWs{dev, stream, nullptr, 0});
    ws = &g_parts.back();
  }
  if (ws->n < (size_t)nblk * MLP_NW) {
    if (ws->p) (void)hipFree(ws->p);
    ws->p = nullptr;
    ws->n = 0;
    hipError_t e = hipMalloc(&ws->p, sizeof(float) * (size_t)nblk * MLP_NW);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc mlp partials");
    ws->n = (size_t)nblk * MLP_NW;
  }
  float* const g_part = ws->p;
  if (ntile == 0) {
    nblk = 0;  // no partials: the reduction writes zeros
  } else {
    // every block takes at least one tile (nblk <= ntile): its first tile
    // writes the block's partial
    if (r.target)
      hipLaunchKernelGGL(mlp_bwd_kernel<true>, dim3(nblk), dim3(64 * BWD_W), 0, (hipStream_t)stream, (const unsigned short*)w,
                         in, r, n, g_part, din);
    else
      hipLaunchKernelGGL(mlp_bwd_kernel<false>, dim3(nblk), dim3(64 * BWD_W), 0, (hipStream_t)stream, (const unsigned short*)w,
                         in, r, n, g_part, din);
    int rc = launch_err("mlp_backward");
    if (rc) return rc;
  }
  if (ad)
    hipLaunchKernelGGL(mlp_dw_reduce_kernel<true>, dim3((MLP_NW + 63) / 64), dim3(256), 0, (hipStream_t)stream, g_part,
                       nblk, dw, *ad);
  else
    hipLaunchKernelGGL(mlp_dw_reduce_kernel<false>, dim3((MLP_NW + 63) / 64), dim3(256), 0, (hipStream_t)stream,
                       g_part, nblk, dw, AdamArgs{});
  return launch_err("mlp_dw_reduce");
}
}  // namespace

using namespace rf;

extern "C" {

int rf_mlp_forward(const void* w, const float* in, int64_t n, float* out, float* act, void* stream) {
  if (!w || (n > 0 && (!in || !out)) || n < 0) return fail(RF_E_INVALID, "bad arguments");
  if (n == 0) return RF_OK;
  const int64_t ntile = (n + 63) / 64;
  int blocks = (int)((ntile + 3) / 4);
  if (blocks > 2048) blocks = 2048;
  if (act)
    hipLaunchKernelGGL(mlp_fwd_kernel<true>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const unsigned short*)w,
                       in, n, out, act);
  else
    hipLaunchKernelGGL(mlp_fwd_kernel<false>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const unsigned short*)w, in, n, out, act);
  return launch_err("mlp_forward");
}


int rf_mlp_backward(const void* w, const float* in, const float* act, const float* dout, int64_t n, float* dw,
                    float* din, void* stream) {
  (void)act;  // activations are recomputed from the inputs (cheaper than reading them back)
  if (!w || !dw || n < 0 || (n > 0 && (!in || !dout))) return fail(RF_E_INVALID, "bad arguments");
  BwdRows r{dout, nullptr, nullptr, 0.0f, n};
  return backward_launch(w, in, r, n, dw, din, nullptr, stream);
}

int rf_mlp_train_step(void* w, float* w32, float* m, float* v, const float* in, const float* target,
                      const int64_t* idx, int64_t batch, int64_t n_rows, uint32_t flags, float lr, float beta1,
                      float beta2, float eps, int32_t step, float* dw, void* stream) {
  if (!w || !w32 || !m || !v || !in || !target || batch < 1 || step < 1)
    return fail(RF_E_INVALID, "bad arguments");
  if (idx ? n_rows < 1 : n_rows < batch) return fail(RF_E_INVALID, "n_rows: fewer rows than the batch reads");
  if (idx && (flags & RF_VALIDATE)) {
    // the indices on the host: every one must name a row of the arrays
    std::vector<int64_t> h((size_t)batch);
    hipError_t e = hipMemcpyAsync(h.data(), idx, sizeof(int64_t) * (size_t)batch, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "reading the batch indices");
    int64_t bad = 0;
    for (int64_t i : h) bad += (i < 0 || i >= n_rows) ? 1 : 0;
    if (bad) return fail(RF_E_INVALID, std::to_string(bad) + " batch indices outside [0, n_rows)");
  }
  BwdRows r{nullptr, idx, target, 2.0f / (float)batch, idx ? n_rows : batch};
  const AdamArgs ad = adam_args(w32, w, m, v, lr, beta1, beta2, eps, step);
  return backward_launch(w, in, r, batch, dw, nullptr, &ad, stream);
}

int rf_adam_step(float* w32, void* wbf, float* m, float* v, const float* g, int64_t n, float lr, float beta1,
                 float beta2, float eps, int32_t step, void* stream) {
  if (!w32 || !wbf || !m || !v || !g || n < 0 || step < 1) return fail(RF_E_INVALID, "bad arguments");
  if (n == 0) return RF_OK;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     adam_args(w32, wbf, m, v, lr, beta1, beta2, eps, step), g, n);
  return launch_err("adam");
}

int rf_mse_grad(const float* out, const float* target, int64_t n, float scale, float* dout, void* stream) {
  if (n < 0 || (n > 0 && (!out || !target || !dout))) return fail(RF_E_INVALID, "bad arguments");
  if (n == 0) return RF_OK;
  hipLaunchKernelGGL(mse_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, out, target,
                     n, scale, dout);
  return launch_err("mse_grad");
}

static int bwcb_launch(const double* xq, int64_t n, int32_t K, double ylo, double yhi, double lo, double hi, void* out,
                       bool resid, void* stream) {
  if (n < 0 || K < 2 || K > 4096 || !(ylo < yhi) || !(lo < hi) || (n > 0 && (!xq || !out)))
    return fail(RF_E_INVALID, "bad arguments");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (!g_gl || g_gl_K != K || g_gl_lo != ylo || g_gl_hi != yhi) {
    if (g_gl) (void)hipFree(g_gl);
    g_gl = nullptr;
    std::vector<double> h(2 * K);
    gauss_legendre(K, ylo, yhi, h.data(), h.data() + K);
    hipError_t e = hipMalloc(&g_gl, sizeof(double) * 2 * K);
    if (e == hipSuccess) e = hipMemcpy(g_gl, h.data(), sizeof(double) * 2 * K, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "bwcb rule upload");
    g_gl_K = K;
    g_gl_lo = ylo;
    g_gl_hi = yhi;
  }
  if (n == 0) return RF_OK;
  if (resid)
    hipLaunchKernelGGL(bwcb_logpdf_kernel<true>, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, (hipStream_t)stream,
                       xq, n, g_gl, K, lo, hi, out);
  else
    hipLaunchKernelGGL(bwcb_logpdf_kernel<false>, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, (hipStream_t)stream,
                       xq, n, g_gl, K, lo, hi, out);
  return launch_err("bwcb_logpdf");
}

int rf_bwcb_logpdf(const double* xq, int64_t n, int32_t K, double ylo, double yhi, double lo, double hi, double* out,
                   void* stream) {
  return bwcb_launch(xq, n, K, ylo, yhi, lo, hi, out, false, stream);
}

int rf_mlp_targets(const double* xq, int64_t n, int32_t K, double ylo, double yhi, double lo, double hi, float* out,
                   void* stream) {
  return bwcb_launch(xq, n, K, ylo, yhi, lo, hi, out, true, stream);
}

}  // extern "C"
