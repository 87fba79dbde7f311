// rf_peaks.hip -- microbenchmarks of the issue rates and the bandwidth that
// bound the likelihood kernels, measured on the device they run on (the
// rooflines' ceilings; the datasheet's figures are derived from unit counts
// and assume instruction mixes these kernels do not have).
//
// Every VALU kernel runs one long loop per lane over independent dependency
// chains (eight accumulators, so that issue, not latency, limits it) on a grid
// that fills the device several times over, and stores its accumulators at
// the end so that nothing is optimised away.  The rate is the number of
// operations of the kind named over the kernel's duration (HIP events).
//   kind 0  FP32 FMA                          lane-FMA/s
//   kind 1  FP64 FMA                          lane-FMA/s
//   kind 2  FP32 hardware exp2                lane-ops/s
//   kind 3  FP32 mix: 14 FMA + 1 transcendental (exp2, log2, rcp in turn), the
//           1-D likelihood kernel's ratio     lane-slots/s (FMA 1, trans 4)
//   kind 4  FP32 mix: 12 FMA + 1 rcp, the exact convolution's inner loop
//                                             lane-slots/s (FMA 1, rcp 4)
//   kind 5  FP64 exp (the device library's)   lane-calls/s
//   kind 6  FP64 log (the device library's)   lane-calls/s
//   kind 7  FP64 reciprocal: hardware estimate + one Newton step
//                                             lane-calls/s
//   kind 8  streaming read, 16-byte loads     bytes/s
//   kind 9  FP64 log of the event loop (rf_log64) lane-calls/s
#include <hip/hip_runtime.h>

#include <cmath>

#include "device/rf_dev.h"
#include "rf_internal.h"

namespace {

// the library's own device math functions, element by element (for tests
// against the host's libm): fn 0 = rf_log64
__global__ __launch_bounds__(256) void math_kernel(int fn, const double* in, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (fn == 0) out[i] = rf_log64(in[i]);
  else out[i] = rf_exp2_neg(in[i]);
}

constexpr int kBS = 256;

template <int KIND>
__global__ __launch_bounds__(kBS) void peak_valu(float* outf, double* outd, int iters, float s) {
  const int tid = blockIdx.x * kBS + threadIdx.x;
  if (KIND == 1 || KIND >= 5) {
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 1.0 + 1e-3 * (k + 1) + 1e-9 * tid;
    const double b = 0.999999 + 1e-12 * s, c = 1e-7 * s;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (KIND == 1) a[k] = fma(a[k], b, c);
        if (KIND == 5) a[k] = ::exp(a[k] * 1e-3) + c;
        if (KIND == 6) a[k] = ::log(a[k] + 1.5) + c;
        if (KIND == 9) a[k] = rf_log64(a[k] + 1.5) + c;
        if (KIND == 7) {
          const double r = __builtin_amdgcn_rcp(a[k]);
          a[k] = fma(r, fma(-a[k], r, 1.0), r) + 1.5;
        }
      }
    }
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += a[k];
    outd[tid] = t;
    return;
  }
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.0f + 1e-3f * (k + 1) + 1e-7f * (tid & 1023);
  const float b = 0.9999f + 1e-9f * s, c = 1e-6f * s;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (KIND == 0) a[k] = fmaf(a[k], b, c);
      if (KIND == 2) a[k] = __builtin_amdgcn_exp2f(a[k] * -0.5f);
      if (KIND == 3) {
#pragma unroll
        for (int m = 0; m < 14; ++m) a[k] = fmaf(a[k], b, c);
        const int t = k % 3;
        a[k] = t == 0 ? __builtin_amdgcn_exp2f(a[k] * -0.5f)
                      : (t == 1 ? __builtin_amdgcn_logf(a[k] + 2.0f) : __builtin_amdgcn_rcpf(a[k] + 1.5f));
      }
      if (KIND == 4) {
#pragma unroll
        for (int m = 0; m < 12; ++m) a[k] = fmaf(a[k], b, c);
        a[k] = __builtin_amdgcn_rcpf(a[k] + 1.5f);
      }
    }
  }
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) t += a[k];
  outf[tid] = t;
}

typedef float f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBS) void peak_stream(const f4* in, int64_t n4, float* out) {
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  const int64_t stride = (int64_t)gridDim.x * kBS;
  int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
  // four loads in flight per lane
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const f4 x0 = in[i], x1 = in[i + stride], x2 = in[i + 2 * stride], x3 = in[i + 3 * stride];
    acc += x0 + x1 + x2 + x3;
  }
  for (; i < n4; i += stride) acc += in[i];
  out[(int64_t)blockIdx.x * kBS + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

// ops per lane and loop iteration of each kind (in its unit)
static double ops_per_iter(int kind) {
  switch (kind) {
    case 0: case 1: case 2: case 5: case 6: case 7: case 9: return 8.0;
    case 3: return 8.0 * (14.0 + 4.0);
    case 4: return 8.0 * (12.0 + 4.0);
  }
  return 0.0;
}

extern "C" int rf_peak(int32_t kind, int32_t iters, int64_t stream_bytes, double* rate, double* seconds) {
  if (!rate || kind < 0 || kind > 9 || iters < 1) return rf::fail(RF_E_INVALID, "bad arguments");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return rf::hip_fail(e, "device query");
  const int blocks = cus * 32;  // eight waves per SIMD, four times over
  const int64_t threads = (int64_t)blocks * kBS;
  float* of = nullptr;
  double* od = nullptr;
  void* buf = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto cleanup = [&]() {
    if (of) (void)hipFree(of);
    if (od) (void)hipFree(od);
    if (buf) (void)hipFree(buf);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  if ((e = hipMalloc(&of, sizeof(float) * threads)) != hipSuccess ||
      (e = hipMalloc(&od, sizeof(double) * threads)) != hipSuccess || (e = hipEventCreate(&t0)) != hipSuccess ||
      (e = hipEventCreate(&t1)) != hipSuccess) {
    cleanup();
    return rf::hip_fail(e, "peak setup");
  }
  int64_t n4 = 0;
  if (kind == 8) {
    n4 = (stream_bytes > 0 ? stream_bytes : ((int64_t)1 << 30)) / 16;
    if ((e = hipMalloc(&buf, 16 * n4)) != hipSuccess || (e = hipMemset(buf, 0, 16 * n4)) != hipSuccess) {
      cleanup();
      return rf::hip_fail(e, "peak stream buffer");
    }
  }
  auto launch = [&]() {
    switch (kind) {
      case 0: hipLaunchKernelGGL(peak_valu<0>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 1: hipLaunchKernelGGL(peak_valu<1>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 2: hipLaunchKernelGGL(peak_valu<2>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 3: hipLaunchKernelGGL(peak_valu<3>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 4: hipLaunchKernelGGL(peak_valu<4>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 5: hipLaunchKernelGGL(peak_valu<5>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 6: hipLaunchKernelGGL(peak_valu<6>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 7: hipLaunchKernelGGL(peak_valu<7>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
      case 8: hipLaunchKernelGGL(peak_stream, dim3(blocks), dim3(kBS), 0, 0, (const f4*)buf, n4, of); break;
      case 9: hipLaunchKernelGGL(peak_valu<9>, dim3(blocks), dim3(kBS), 0, 0, of, od, iters, 1.0f); break;
    }
  };
  launch();  // warm-up (code load, clocks)
  e = hipEventRecord(t0, 0);
  const int reps = 5;
  for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(t1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  if (e != hipSuccess) {
    cleanup();
    return rf::hip_fail(e, "peak run");
  }
  const double s = ms * 1e-3 / reps;
  const double work = kind == 8 ? 16.0 * (double)n4 : (double)threads * iters * ops_per_iter(kind);
  *rate = work / s;
  if (seconds) *seconds = s;
  cleanup();
  return RF_OK;
}

extern "C" int rf_eval_math(int32_t fn, const double* dev_in, int64_t n, double* dev_out, void* stream) {
  if (fn < 0 || fn > 1 || n < 0 || (n > 0 && (!dev_in || !dev_out))) return rf::fail(RF_E_INVALID, "bad arguments");
  if (n == 0) return RF_OK;
  hipLaunchKernelGGL(math_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, fn, dev_in, n,
                     dev_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RF_OK : rf::hip_fail(e, "math_kernel");
}
