// rf_validate.hip -- the RF_VALIDATE pass of rf_bind_columns: one read of
// every bound column, counting events outside their observable's range (or
// not finite, or not an integer where the observable is a count) and event
// weights that are not finite.  A count, so the order
// of the atomic additions does not matter.
#include <hip/hip_runtime.h>

#include <cstring>

#include "rf_internal.h"

namespace {

#define VAL_MAXC 8
struct ValArgs {
  const void* col[VAL_MAXC];
  double lo[VAL_MAXC], hi[VAL_MAXC];
  int n_cols, n_range;
  unsigned int_mask;  // columns whose values must be integers
  int64_t n;
  unsigned long long* bad;
};

template <typename T>
__global__ __launch_bounds__(256) void validate_kernel(const ValArgs a) {
  unsigned cnt = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < a.n_cols; ++c) {
    const T* x = (const T*)a.col[c];
    const bool range = c < a.n_range;
    const double lo = a.lo[c], hi = a.hi[c];
    const bool integer = (a.int_mask >> c) & 1u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
      const double v = (double)x[i];
      bool ok = range ? (v >= lo && v <= hi) : isfinite(v);  // NaN fails both
      if (integer) ok = ok && v == floor(v);
      cnt += ok ? 0u : 1u;
    }
  }
  // wavefront sum, one atomic per wavefront with a non-zero count
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(a.bad, (unsigned long long)cnt);
}

}  // namespace

namespace rf {
int validate_columns(const void* const* cols, int n_cols, int n_range, const double* lo, const double* hi,
                     unsigned int_mask, int64_t n, bool f32, void* stream, int64_t* n_bad) {
  *n_bad = 0;
  if (n <= 0 || n_cols <= 0) return RF_OK;
  if (n_cols > VAL_MAXC) return fail(RF_E_INVALID, "too many columns to validate");
  ValArgs a;
  memset(&a, 0, sizeof a);
  for (int c = 0; c < n_cols; ++c) {
    a.col[c] = cols[c];
    a.lo[c] = c < n_range ? lo[c] : 0.0;
    a.hi[c] = c < n_range ? hi[c] : 0.0;
  }
  a.n_cols = n_cols;
  a.n_range = n_range;
  a.int_mask = int_mask;
  a.n = n;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, sizeof(unsigned long long));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (validation counter)");
  unsigned long long h = 0;
  a.bad = d;
  const int64_t want = (n + 255) / 256;
  const int blocks = (int)(want < 2048 ? want : 2048);
  if ((e = hipMemsetAsync(d, 0, sizeof h, st)) == hipSuccess) {
    if (f32)
      hipLaunchKernelGGL(validate_kernel<float>, dim3(blocks), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(validate_kernel<double>, dim3(blocks), dim3(256), 0, st, a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const hipError_t ef = hipFree(d);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) return hip_fail(e, "column validation");
  *n_bad = (int64_t)h;
  return RF_OK;
}
}  // namespace rf
