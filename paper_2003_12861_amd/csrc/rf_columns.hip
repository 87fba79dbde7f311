// rf_columns.hip -- event columns given with a stride or in the other
// floating-point type, made contiguous in the program's type on the device
// (one array per observable is the layout the batch interface reads,
// Section 4.1), then bound as rf_bind_columns binds contiguous ones.
#include <hip/hip_runtime.h>

#include <vector>

#include "rf_internal.h"

namespace {

// dst[i] = src[i * stride] converted to T (round to nearest); HBM-bound: the
// reads are as scattered as the stride, the writes are contiguous
template <typename S, typename T>
__global__ __launch_bounds__(256) void gather_column(const S* __restrict__ src, int64_t stride, int64_t n,
                                                     T* __restrict__ dst) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) dst[i] = (T)src[i * stride];
}

}  // namespace

using namespace rf;

extern "C" int rf_bind_columns_strided(rf_program* p, const void* const* dev_cols, const int64_t* strides,
                                       const int32_t* dtypes, int32_t n_cols, int64_t n_events, void* stream) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (!p->loaded) return fail(RF_E_STATE, "program was compiled without loading");
  if (n_cols != p->L.n_cols + p->L.weighted || n_cols > RF_MAX_COLS)
    return fail(RF_E_INVALID, "number of columns differs from the program's");
  if (n_events < 0) return fail(RF_E_INVALID, "n_events < 0");
  if (n_events > 0 && n_cols > 0 && (!dev_cols || !strides || !dtypes))
    return fail(RF_E_INVALID, "columns, strides or dtypes are NULL");
  const bool f32 = p->L.precision == RF_FP32_COMP;
  const int want = f32 ? RF_COL_F32 : RF_COL_F64;
  std::vector<const void*> cols(n_cols > 0 ? n_cols : 1, nullptr);
  for (int c = 0; c < n_cols && n_events > 0; ++c) {
    if (!dev_cols[c]) return fail(RF_E_INVALID, "column pointer is NULL");
    if (dtypes[c] != RF_COL_F32 && dtypes[c] != RF_COL_F64) return fail(RF_E_INVALID, "unknown column dtype");
    if (strides[c] < 1) return fail(RF_E_INVALID, "column strides must be >= 1");
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device) return fail(RF_E_STATE, "current device differs from the one the program was loaded on");
  bool copied = false;
  for (int c = 0; c < n_cols; ++c) {
    if (n_events == 0 || (dtypes[c] == want && strides[c] == 1)) {  // bound in place
      cols[c] = n_events == 0 ? nullptr : dev_cols[c];
      continue;
    }
    const size_t bytes = (size_t)n_events * (f32 ? sizeof(float) : sizeof(double));
    if (p->owned_bytes[c] < bytes) {
      if (p->owned[c]) {
        // an evaluation in flight may still read the old copy
        if (p->launched && (e = hipStreamSynchronize((hipStream_t)p->last_stream)) != hipSuccess)
          return hip_fail(e, "hipStreamSynchronize (previous stream)");
        (void)hipFree(p->owned[c]);
        p->owned[c] = nullptr;
        p->owned_bytes[c] = 0;
      }
      if ((e = hipMalloc(&p->owned[c], bytes)) != hipSuccess) return hip_fail(e, "hipMalloc (column copy)");
      p->owned_bytes[c] = bytes;
    }
    int64_t blocks = (n_events + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    const dim3 grid((unsigned)blocks), block(256);
    const hipStream_t st = (hipStream_t)stream;
    if (dtypes[c] == RF_COL_F32 && f32)
      hipLaunchKernelGGL((gather_column<float, float>), grid, block, 0, st, (const float*)dev_cols[c], strides[c],
                         n_events, (float*)p->owned[c]);
    else if (dtypes[c] == RF_COL_F32)
      hipLaunchKernelGGL((gather_column<float, double>), grid, block, 0, st, (const float*)dev_cols[c], strides[c],
                         n_events, (double*)p->owned[c]);
    else if (f32)
      hipLaunchKernelGGL((gather_column<double, float>), grid, block, 0, st, (const double*)dev_cols[c], strides[c],
                         n_events, (float*)p->owned[c]);
    else
      hipLaunchKernelGGL((gather_column<double, double>), grid, block, 0, st, (const double*)dev_cols[c], strides[c],
                         n_events, (double*)p->owned[c]);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "column copy launch");
    cols[c] = p->owned[c];
    copied = true;
  }
  // later evaluations on another stream wait for the copies (see order_launch)
  if (copied && (e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess)
    return hip_fail(e, "hipStreamSynchronize (column copies)");
  return rf_bind_columns(p, cols.data(), n_cols, n_events, stream);
}
