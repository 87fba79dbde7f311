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

// dW[o][i] += sum over the tile's 64 rows r of D[o][r] H[i][r] on MFMA:
// M = o, N = i, K = r.  The operands come from the staged [row][feature]
// tiles: lane l of K-step s provides D[32 mo + l%32][8 s + 4 (l/32) + 0..3]
// (A) and H[32 ni + l%32][same rows] (B).  Both are FP32 and enter as three
// bf16 parts each; the six products of parts whose orders add up to at most
// two are accumulated (small ones first), which matches an FP32 product to
// about 2^-24.  acc[mo][ni][v] = dW[mlp_feat(mo, v, l/32)][32 ni + l%32].
RF_DEV void mlp_dw_mfma(const float* D, const float* H, rf_f32x16 (&acc)[2][2]) {
  const int l = threadIdx.x & 63, hl = l >> 5, lr = l & 31;
#pragma unroll 1  // one K-step at a time: unrolling spills
  for (int s = 0; s < 8; ++s) {
    rf_bf16x4 Ap[2][3], Bp[2][3];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float a4[4], b4[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a4[j] = D[(8 * s + 4 * hl + j) * TS + 32 * m + lr];
        b4[j] = H[(8 * s + 4 * hl + j) * TS + 32 * m + lr];
      }
      mlp_split4<3>(a4, Ap[m]);
      mlp_split4<3>(b4, Bp[m]);
    }
#pragma unroll
    for (int ord = 2; ord >= 0; --ord)
#pragma unroll
      for (int qa = 0; qa <= ord; ++qa)
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
            acc[mo][ni] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(Ap[mo][qa], Bp[ni][ord - qa], acc[mo][ni], 0, 0, 0);
  }
}

__global__ __launch_bounds__(64) void mlp_bwd_kernel(const unsigned short* w, const float* in, const float* dout,
                                                     int64_t n, float* part, float* din) {
  __shared__ MlpLds s;
  __shared__ BwdLds b;
  mlp_load(w, s);
  const int lane = threadIdx.x, hl = lane >> 5, lr = lane & 31;
  float* P = part + (size_t)blockIdx.x * MLP_NW;
  __syncthreads();
  const int64_t ntile = (n + 63) / 64;
  for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
    MLP_TILE_BARRIER();
    const int64_t row = t * 64 + lane;
    const bool valid = row < n;
    float u[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) u[j] = valid ? in[row * 6 + j] : 0.0f;
    const float g = valid ? dout[row] : 0.0f;
    float h[3][64];
    (void)mlp_forward_full<MLP_SPLIT>(s, u, h[0], h[1], h[2]);
    // stage forward activations, inputs and output cotangents
#pragma unroll
    for (int L = 0; L < 3; ++L)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int eb = 0; eb < 2; ++eb)
#pragma unroll
          for (int v = 0; v < 16; ++v) b.HT[L][(32 * eb + lr) * TS + mlp_feat(mb, v, hl)] = h[L][(2 * mb + eb) * 16 + v];
#pragma unroll
    for (int j = 0; j < 6; ++j) b.UT[lane * 6 + j] = u[j];
    b.G[lane] = g;
    mlp_backward<MLP_SPLIT>(s, g, h[0], h[1], h[2]);
#pragma unroll
    for (int L = 0; L < 3; ++L)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int eb = 0; eb < 2; ++eb)
#pragma unroll
          for (int v = 0; v < 16; ++v) b.DT[L][(32 * eb + lr) * TS + mlp_feat(mb, v, hl)] = h[L][(2 * mb + eb) * 16 + v];
    if (din) {  // uniform: every lane takes part in the cross-lane sums
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const float gj = mlp_input_grad(s, h[0], j);
        if (valid) din[row * 6 + j] = gj;
      }
    }
    __syncthreads();
    // weight gradients, summed over the 64 rows of the tile; the block's
    // first tile writes its partial, later ones add to it
    const bool first = t == (int64_t)blockIdx.x;
    auto put = [&](int k, float v) { P[k] = first ? v : P[k] + v; };
    // layers 3 (d3 x h2) and 2 (d2 x h1) on MFMA (one layer at a time)
#pragma unroll 1
    for (int L = 2; L >= 1; --L) {
      rf_f32x16 acc[2][2];
#pragma unroll
      for (int mo = 0; mo < 2; ++mo)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[mo][ni][v] = 0.0f;
      mlp_dw_mfma(b.DT[L], b.HT[L - 1], acc);
      const int ow = L == 2 ? MLP_OW3 : MLP_OW2;
#pragma unroll
      for (int mo = 0; mo < 2; ++mo)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
          for (int v = 0; v < 16; ++v) put(ow + mlp_feat(mo, v, hl) * 64 + 32 * ni + lr, acc[mo][ni][v]);
    }
    // biases of layers 2 and 3, layer 1 (d1 x u) and the output layer (g x
    // h3): lane = unit o
    {
      const int o = lane;
      float bb2 = 0.0f, bb3 = 0.0f, acc1[6] = {0, 0, 0, 0, 0, 0}, bb1 = 0.0f, acc4 = 0.0f, accg = 0.0f;
      for (int e = 0; e < 64; ++e) {
        bb3 += b.DT[2][e * TS + o];
        bb2 += b.DT[1][e * TS + o];
        const float d = b.DT[0][e * TS + o];
        bb1 += d;
#pragma unroll
        for (int j = 0; j < 6; ++j) acc1[j] = fmaf(d, b.UT[e * 6 + j], acc1[j]);
        acc4 = fmaf(b.G[e], b.HT[2][e * TS + o], acc4);
        accg += b.G[e];
      }
      put(MLP_OB3 + o, bb3);
      put(MLP_OB2 + o, bb2);
#pragma unroll
      for (int j = 0; j < 6; ++j) put(MLP_OW1 + o * 6 + j, acc1[j]);
      put(MLP_OB1 + o, bb1);
      put(MLP_OW4 + o, acc4);
      if (o == 0) put(MLP_OB4, accg);
    }
    __syncthreads();
  }
}

// dw[k] = sum over the blocks' partials, in a fixed order: wavefront w of a
// 256-thread block adds partial rows w, w + 4, ... for 64 consecutive k (16
// loads in flight per lane, pairwise), the four wavefront sums are added in
// order
__global__ __launch_bounds__(256) void mlp_dw_reduce_kernel(const float* part, int nblk, float* dw) {
  __shared__ double ws[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const int kc = k < MLP_NW ? k : MLP_NW - 1;
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
  if (w == 0 && k < MLP_NW) dw[k] = (float)((ws[0][lane] + ws[1][lane]) + (ws[2][lane] + ws[3][lane]));
}

__global__ void adam_kernel(float* w32, unsigned short* wbf, float* m, float* v, const float* g, int64_t n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w32[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w32[i] = wi;
  const __bf16 hb = (__bf16)wi;  // round to nearest even
  wbf[i] = __builtin_bit_cast(unsigned short, hb);
}

__global__ void mse_grad_kernel(const float* out, const float* y, int64_t n, float scale, float* dout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dout[i] = scale * (out[i] - y[i]);
}

// exact log p_sig(x; M, Gamma, sigma, alpha, n) per sample (FP64): the same
// rule as the convolution leaf, with per-sample parameters
__global__ void bwcb_logpdf_kernel(const double* xq, int64_t n, const double* gl, int K, double lo, double hi,
                                   double* out) {
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
  out[i] = log(S / N);
}

int launch_err(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RF_OK : rf::hip_fail(e, what);
}

std::mutex g_ws_mu;
float* g_part = nullptr;
size_t g_part_n = 0;
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
  const int64_t ntile = (n + 63) / 64;
  int nblk = (int)(ntile < 512 ? ntile : 512);
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (g_part_n < (size_t)nblk * MLP_NW) {
    if (g_part) (void)hipFree(g_part);
    g_part = nullptr;
    g_part_n = 0;
    hipError_t e = hipMalloc(&g_part, sizeof(float) * (size_t)nblk * MLP_NW);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc mlp partials");
    g_part_n = (size_t)nblk * MLP_NW;
  }
  if (ntile == 0) {
    nblk = 0;  // no partials: the reduction writes zeros
  } else {
    // every block takes at least one tile (nblk <= ntile): its first tile
    // writes the block's partial
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3(nblk), dim3(64), 0, (hipStream_t)stream, (const unsigned short*)w, in, dout,
                       n, g_part, din);
    int rc = launch_err("mlp_backward");
    if (rc) return rc;
  }
  hipLaunchKernelGGL(mlp_dw_reduce_kernel, dim3((MLP_NW + 63) / 64), dim3(256), 0, (hipStream_t)stream, g_part, nblk,
                     dw);
  return launch_err("mlp_dw_reduce");
}

int rf_adam_step(float* w32, void* wbf, float* m, float* v, const float* g, int64_t n, float lr, float beta1,
                 float beta2, float eps, int32_t step, void* stream) {
  if (!w32 || !wbf || !m || !v || !g || n < 0 || step < 1) return fail(RF_E_INVALID, "bad arguments");
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w32,
                     (unsigned short*)wbf, m, v, g, n, lr, beta1, beta2, eps, c1, c2);
  return launch_err("adam");
}

int rf_mse_grad(const float* out, const float* target, int64_t n, float scale, float* dout, void* stream) {
  if (n < 0 || (n > 0 && (!out || !target || !dout))) return fail(RF_E_INVALID, "bad arguments");
  if (n == 0) return RF_OK;
  hipLaunchKernelGGL(mse_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, out, target,
                     n, scale, dout);
  return launch_err("mse_grad");
}

int rf_bwcb_logpdf(const double* xq, int64_t n, int32_t K, double ylo, double yhi, double lo, double hi, double* out,
                   void* stream) {
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
  hipLaunchKernelGGL(bwcb_logpdf_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, (hipStream_t)stream, xq, n,
                     g_gl, K, lo, hi, out);
  return launch_err("bwcb_logpdf");
}

}  // extern "C"
