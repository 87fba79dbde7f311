// rf_static.hip -- NLL+gradient evaluation that allocates nothing.
//
// rf_nll_grad_noalloc runs the same fused gradient kernel as
// rf_nll_grad_async, but the kernel's cross-workgroup scratch (the ticket
// words of the end-of-kernel hand-off and the per-workgroup partial sums)
// lives in one file-scope device array of fixed size instead of the program's
// bind-time workspace, and the result block goes to a buffer the caller
// passes.  No call here allocates or frees memory, so it can be used where
// allocation is not allowed (stream capture into a graph, serving loops).
//
// Each device holds its own copy of the array until the process ends; its
// device address is looked up once per device (hipGetSymbolAddress with that
// device current) and only that address is handed to kernels.  Every call on
// a device shares the array: calls that overlap on one device race.
#include <mutex>

#include "rf_internal.h"

// the scratch array: ticket words first (one 256-byte-aligned block), then
// the partial sums, (n_sums + 1) rows of one double per workgroup
#define RF_SCRATCH_BYTES (256u * 1024u)  // 256 KiB per device
static __device__ __align__(256) unsigned char scratch[RF_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = RF_SCRATCH_BYTES;
constexpr size_t kTicketBytes = 256 * ((sizeof(unsigned) * RF_TICKET_WORDS + 255) / 256);
static_assert(kTicketBytes < kScratchBytes, "the ticket words fit the scratch array");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up on first use)
int scratch_ptr(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return rf::fail(RF_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return rf::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return rf::fail(RF_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[dev] = ptr;
  }
  *out = (unsigned char*)g_ptr[dev];
  return RF_OK;
}

// the ticket words must be zero when a gradient kernel starts; a fill kernel
// (not a memset node) keeps the call capturable into a graph
__global__ __launch_bounds__(256) void clear_words(unsigned* w, int n) {
  for (int i = threadIdx.x; i < n; i += 256) w[i] = 0u;
}

}  // namespace

extern "C" int rf_nll_grad_noalloc(rf_program* p, const double* theta, double* dev_result, void* stream) {
  if (!p) return rf::fail(RF_E_INVALID, "program is NULL");
  if (!p->loaded) return rf::fail(RF_E_STATE, "program was compiled without loading (RF_COMPILE_NO_LOAD)");
  if (p->n < 0) return rf::fail(RF_E_STATE, "columns are not bound");
  if (!dev_result) return rf::fail(RF_E_INVALID, "dev_result is NULL");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rf::hip_fail(e, "hipGetDevice");
  if (dev != p->device) return rf::fail(RF_E_STATE, "current device differs from the one the program was loaded on");
  const size_t rows = (size_t)p->L.n_sums + 1;  // sums, then the bad-event count
  const size_t need = kTicketBytes + sizeof(double) * rows * (size_t)p->nblk;
  if (need > kScratchBytes)
    return rf::fail(RF_E_INVALID, "rf_nll_grad_noalloc: " + std::to_string(rows) + " sums x " +
                                      std::to_string(p->nblk) + " workgroups need " + std::to_string(need) +
                                      " bytes of scratch, more than its fixed " + std::to_string(kScratchBytes) +
                                      " (lower the workgroup count with rf_set_launch)");
  unsigned char* base = nullptr;
  int rc = scratch_ptr(dev, &base);
  if (rc) return rc;
  unsigned* ticket = (unsigned*)base;
  double* part = (double*)(base + kTicketBytes);
  hipLaunchKernelGGL(clear_words, dim3(1), dim3(256), 0, (hipStream_t)stream, ticket, (int)RF_TICKET_WORDS);
  e = hipGetLastError();
  if (e != hipSuccess) return rf::hip_fail(e, "clear_words launch");
  return rf::enqueue_grad_on(p, theta, part, p->nblk > 0 ? p->nblk : 1, ticket, dev_result, stream);
}
