// rf_capi.cpp -- programs: compile, bind, launch, read back.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include <fstream>
#include <iterator>

#include "rf_internal.h"

using namespace rf;

namespace {

int cu_count(int dev) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
  return n;
}

void free_workspace(rf_program* p) {  // release errors are not actionable here
  if (p->d_part) (void)hipFree(p->d_part);
  if (p->d_ticket) (void)hipFree(p->d_ticket);
  if (p->d_out) (void)hipFree(p->d_out);
  if (p->h_out) (void)hipHostFree(p->h_out);
  if (p->d_aux) (void)hipFree(p->d_aux);
  p->d_part = nullptr;
  p->d_ticket = nullptr;
  p->d_out = nullptr;
  p->h_out = nullptr;
  p->d_hout = nullptr;
  p->d_aux = nullptr;
}

int out_len(const rf_program* p) { return p->L.n_params + 2 + p->L.n_sums; }

// events per lane and step: 16 bytes of a column (4 in FP32, 2 in FP64); one
// for the convolution leaf, whose per-event loop hides the load latency
int choose_ept(const Lowered& L) {
  int ept = L.has_numconv ? 1 : (L.precision == RF_FP32_COMP ? 4 : 2);
  if (const char* e = getenv("RFGPU_EPT")) {  // tuning override
    const int v = atoi(e);
    if (v == 1 || v == 2 || v == 4) ept = v;
  }
  return ept;
}

// load ring depth: three groups in flight when a group is one 16-byte load;
// two for several columns (more registers per group); none beyond the
// current event for the convolution leaf
int choose_pfd(const Lowered& L, int ept) {
  int d = L.has_numconv ? 1 : (L.n_cols + L.weighted <= 1 ? 3 : 2);
  (void)ept;
  if (const char* e = getenv("RFGPU_PFD")) {  // tuning override
    const int v = atoi(e);
    if (v >= 1 && v <= 4) d = v;
  }
  return d;
}

int choose_blocks(const rf_program* p) {
  if (p->blocks_override > 0) return p->blocks_override;
  // about 8 steps per lane, at most as many workgroups as the CUs hold at
  // once (and at most 4 per CU): enough waves to hide the load latency, no
  // second round of workgroups behind the first, and few partials for the
  // last workgroup to add
  const int64_t per = (int64_t)p->block * p->ept * 8;
  int64_t b = (p->n + per - 1) / per;
  int bpc = 4;
  if (const char* e = getenv("RFGPU_BPC")) {  // tuning override of the per-CU cap
    const int v = atoi(e);
    if (v >= 1 && v <= 32) bpc = v;
  }
  const int64_t cap = (int64_t)cu_count(p->device) * (p->resident < bpc ? p->resident : bpc);
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

void fill_args(const rf_program* p, const double* theta, RfArgs& a) {
  memset(&a, 0, sizeof a);
  for (int c = 0; c < RF_MAX_COLS; ++c) a.col[c] = p->cols[c];
  a.n = p->n;
  a.part = p->d_part;
  a.ticket = p->d_ticket;
  a.out = p->d_out;
  a.aux = p->d_aux;
  a.weights = p->d_weights;
  a.nblk_max = p->nblk_max;
  a.hout = nullptr;
  for (int k = 0; k < p->L.n_params; ++k) a.theta[k] = theta[k];
  if (p->L.ext_nu >= 0) a.theta[p->L.n_params] = (double)p->n;  // N of the extended term
}

// parameter-dependent pre-pass: the surrogate leaves' normalisation
int pre_launch(rf_program* p, const double* theta, void* stream) {
  if (!p->L.has_mlp) return RF_OK;
  std::vector<double> pv;
  eval_paramlike(p->L, theta, pv);
  for (int id : p->L.mlp_nodes) {
    const Node& n = p->L.nodes[id];
    double q[5];
    for (int j = 0; j < 5; ++j) q[j] = pv[n.in[1 + j]];
    const int K = (int)n.attrs[12];
    const double* grid = p->d_aux + p->L.aux_off[id];
    int rc = mlp_renorm_launch(p->d_weights, q, n.attrs.data(), grid, K, p->d_aux + p->L.aux_off[id] + 2 * K, stream);
    if (rc) return rc;
  }
  return RF_OK;
}

int launch(rf_program* p, hipFunction_t f, RfArgs& a, void* stream) {
  int rc = order_launch(p->last_stream, p->launched, stream);
  if (rc) return rc;
  rc = pre_launch(p, a.theta, stream);
  if (rc) return rc;
  size_t sz = sizeof(RfArgs);
  void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &a, HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz, HIP_LAUNCH_PARAM_END};
  hipError_t e = hipModuleLaunchKernel(f, p->nblk, 1, 1, p->block, 1, 1, 0, (hipStream_t)stream, nullptr, cfg);
  if (e != hipSuccess) return hip_fail(e, "hipModuleLaunchKernel");
  return RF_OK;
}

int ready(rf_program* p, const double* theta) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (!p->loaded) return fail(RF_E_STATE, "program was compiled without loading (RF_COMPILE_NO_LOAD)");
  if (p->n < 0) return fail(RF_E_STATE, "columns are not bound");
  for (int id : p->L.mlp_nodes) {
    (void)id;
    if (!p->d_weights) return fail(RF_E_STATE, "MLP weights are not bound");
  }
  if (p->L.n_params && !theta) return fail(RF_E_INVALID, "theta is NULL");
  return check_theta(p->L, theta);
}

int run_sync(rf_program* p, hipFunction_t f, const double* theta, void* stream) {
  RfArgs a;
  fill_args(p, theta, a);
  // the last workgroup also writes the result into the mapped host buffer:
  // poll it (a short call returns as soon as the kernel's last workgroup is
  // done), falling back to a stream synchronisation after 20 ms
  a.hout = p->d_hout;
  arm_result(p->h_out, out_len(p));
  int rc = launch(p, f, a, stream);
  if (rc) return rc;
  p->n_sync++;
  return wait_result(p->h_out, out_len(p), stream, &p->n_slow);
}

}  // namespace

namespace rf {
int order_launch(void*& last, bool& launched, void* stream) {
  if (launched && last != stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)last);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize (previous stream)");
  }
  last = stream;
  launched = true;
  return RF_OK;
}

void arm_result(double* h, int n) {
  volatile uint64_t* w = (volatile uint64_t*)h;
  for (int j = 0; j < n; ++j) w[j] = RF_SENTINEL;
  std::atomic_thread_fence(std::memory_order_release);
}

int wait_result(const double* h, int n, void* stream, int64_t* slow) {
  volatile const uint64_t* w = (volatile const uint64_t*)h;
  auto arrived = [&]() {
    for (int j = n - 1; j >= 0; --j)
      if (w[j] == RF_SENTINEL) return false;
    return true;
  };
  const auto t0 = std::chrono::steady_clock::now();
  while (!arrived()) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
      if (slow) ++*slow;
      hipError_t e = hipStreamSynchronize((hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      if (!arrived()) return fail(RF_E_DEVICE, "kernel completed without writing its result");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return RF_OK;
}
}  // namespace rf

extern "C" {

const char* rf_version(void) { return "rfgpu-0.1"; }

int rf_compile(const rf_graph* g, int32_t top, int32_t precision, uint32_t flags, rf_program** out) {
  if (!g || !out) return fail(RF_E_INVALID, "NULL argument");
  *out = nullptr;
  rf_program* p = new rf_program();
  int rc = lower(g->nodes, top, precision, p->L);
  if (rc) { delete p; return rc; }
  p->flags = flags;
  p->L.weighted = (flags & RF_COMPILE_WEIGHTED) ? 1 : 0;
  if (p->L.ext_nu >= 0 && p->L.n_params >= RF_MAX_PARAMS) {
    delete p;
    return fail(RF_E_INVALID, "an extended program has at most 63 parameters");
  }
  // weighted extended likelihood: N of the extended term is the sum of the
  // weights, accumulated by the kernel as one more sum
  if (p->L.ext_nu >= 0 && p->L.weighted) p->L.wsum = p->L.n_sums++;
  if (p->L.n_cols + p->L.weighted > RF_MAX_COLS) {
    delete p;
    return fail(RF_E_INVALID, "a weighted program takes at most 7 observables");
  }
  if (const char* e = getenv("RFGPU_BS")) {  // tuning override of the workgroup size
    const int v = atoi(e);
    if (v >= 64 && v <= 1024 && v % 64 == 0) p->block = v;
  }
  p->ept = choose_ept(p->L);
  p->pfd = choose_pfd(p->L, p->ept);
  if (const char* e = getenv("RFGPU_TG")) {  // tuning override
    const int v = atoi(e);
    if (v >= 1 && v <= RF_TGMAX) p->tg = v;
  }
  if (const char* e = getenv("RFGPU_PRIO")) {  // tuning override of the issue-priority policy
    const int v = atoi(e);
    if (v >= 0 && v <= 2) p->prio = v;
  }
  p->source = generate_source(p->L, p->block, p->ept, p->pfd, p->tg, p->prio);
  rc = build_code_object(p->source, p->co_path);
  if (rc) { delete p; return rc; }
  if (!(flags & RF_COMPILE_NO_LOAD)) {
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
    rc = load_module(p->co_path, p->L.precision == RF_FP32_COMP, p->m);
    if (rc) { delete p; return rc; }
    int nb = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, p->m.k_grad, p->block, 0) == hipSuccess && nb > 0)
      p->resident = nb;
    p->loaded = true;
  }
  *out = p;
  return RF_OK;
}

void rf_program_free(rf_program* p) {
  if (!p) return;
  free_workspace(p);
  for (void* o : p->owned)
    if (o) (void)hipFree(o);
  if (p->unf.vals) (void)hipFree(p->unf.vals);
  if (p->unf.part) (void)hipFree(p->unf.part);
  if (p->unf.out) (void)hipFree(p->unf.out);
  if (p->unf.mod) (void)hipModuleUnload(p->unf.mod);
  if (p->hes.part) (void)hipFree(p->hes.part);
  if (p->hes.ticket) (void)hipFree(p->hes.ticket);
  if (p->hes.out) (void)hipFree(p->hes.out);
  if (p->hes.h_out) (void)hipHostFree(p->hes.h_out);
  if (p->hes.mod) (void)hipModuleUnload(p->hes.mod);
  if (p->m.mod) (void)hipModuleUnload(p->m.mod);
  delete p;
}

int rf_program_info(const rf_program* p, int32_t* n_params, int32_t* n_columns, int32_t* n_sums) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (n_params) *n_params = p->L.n_params;
  if (n_columns) *n_columns = p->L.n_cols + p->L.weighted;
  if (n_sums) *n_sums = p->L.n_sums;
  return RF_OK;
}

const char* rf_program_source(const rf_program* p) { return p ? p->source.c_str() : ""; }

int rf_program_stats(const rf_program* p, int64_t* sync_calls, int64_t* slow_waits) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (sync_calls) *sync_calls = p->n_sync;
  if (slow_waits) *slow_waits = p->n_slow;
  return RF_OK;
}

int rf_set_launch(rf_program* p, int32_t blocks, int32_t threads) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (blocks < 0) return fail(RF_E_INVALID, "blocks < 0");
  if (threads != 0 && threads != p->block) return fail(RF_E_INVALID, "threads per block is fixed at compile time");
  if (p->n >= 0 && blocks > p->nblk_max) return fail(RF_E_INVALID, "blocks exceeds the workspace sized at bind time");
  p->blocks_override = blocks;
  if (p->n >= 0) p->nblk = choose_blocks(p);
  return RF_OK;
}

int rf_bind_columns(rf_program* p, const void* const* dev_cols, int32_t n_cols, int64_t n_events, void* stream) {
  (void)stream;
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (!p->loaded) return fail(RF_E_STATE, "program was compiled without loading");
  if (n_cols != p->L.n_cols + p->L.weighted)
    return fail(RF_E_INVALID, p->L.weighted ? "a weighted program takes the observables' columns and one weight column"
                                            : "number of columns differs from the number of observables");
  if (n_events < 0) return fail(RF_E_INVALID, "n_events < 0");
  if (n_events > 0 && n_cols > 0 && !dev_cols) return fail(RF_E_INVALID, "columns are NULL");
  for (int c = 0; c < n_cols; ++c) {
    if (n_events > 0 && !dev_cols[c]) return fail(RF_E_INVALID, "column pointer is NULL");
    p->cols[c] = dev_cols ? dev_cols[c] : nullptr;
  }
  int dev = 0;
  hipError_t de = hipGetDevice(&dev);
  if (de != hipSuccess) return hip_fail(de, "hipGetDevice");
  if (dev != p->device) return fail(RF_E_STATE, "current device differs from the one the program was loaded on");
  p->n = n_events;
  const int saved = p->blocks_override;
  p->blocks_override = 0;
  const int need = choose_blocks(p);
  p->blocks_override = saved;
  const int cap = cu_count(dev) * 8;
  const int nmax = need > cap ? need : cap;
  if (!p->d_out || nmax > p->nblk_max) {
    // a failed allocation leaves the program unbound (no evaluation can run
    // on a partial workspace)
    auto unbind = [&](int rc) {
      free_workspace(p);
      p->n = -1;
      p->nblk_max = 0;
      return rc;
    };
    free_workspace(p);
    hipError_t e;
    const size_t np = (size_t)(p->L.n_sums + 1) * nmax;  // sums + bad-event count
    if ((e = hipMalloc(&p->d_part, sizeof(double) * np)) != hipSuccess) return unbind(hip_fail(e, "hipMalloc partials"));
    if ((e = hipMalloc(&p->d_ticket, sizeof(unsigned) * RF_TICKET_WORDS)) != hipSuccess) return unbind(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&p->d_out, sizeof(double) * out_len(p))) != hipSuccess) return unbind(hip_fail(e, "hipMalloc"));
    // mapped host copy of the result
    if ((e = hipHostMalloc(&p->h_out, sizeof(double) * out_len(p), hipHostMallocMapped | hipHostMallocCoherent)) !=
        hipSuccess)
      return unbind(hip_fail(e, "hipHostMalloc"));
    memset(p->h_out, 0, sizeof(double) * out_len(p));
    if ((e = hipHostGetDevicePointer((void**)&p->d_hout, p->h_out, 0)) != hipSuccess)
      return unbind(hip_fail(e, "hipHostGetDevicePointer"));
    if ((e = hipMemset(p->d_ticket, 0, sizeof(unsigned) * RF_TICKET_WORDS)) != hipSuccess) return unbind(hip_fail(e, "hipMemset"));
    if (!p->L.aux.empty()) {
      if ((e = hipMalloc(&p->d_aux, sizeof(double) * p->L.aux.size())) != hipSuccess) return unbind(hip_fail(e, "hipMalloc aux"));
      if ((e = hipMemcpy(p->d_aux, p->L.aux.data(), sizeof(double) * p->L.aux.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return unbind(hip_fail(e, "hipMemcpy aux"));
    }
    p->nblk_max = nmax;
  }
  p->nblk = choose_blocks(p);
  if (p->nblk > p->nblk_max) p->nblk = p->nblk_max;
  if (p->flags & RF_VALIDATE) {
    // observable ranges by column; the weight column (if any) must be finite
    double lo[RF_MAX_COLS] = {}, hi[RF_MAX_COLS] = {};
    for (const Node& nd : p->L.nodes)
      if (nd.op == K_OBS && nd.index >= 0 && nd.index < p->L.n_cols) {
        lo[nd.index] = nd.lo;
        hi[nd.index] = nd.hi;
      }
    int64_t bad = 0;
    unsigned int_mask = 0;  // the observables of Poisson leaves hold counts
    for (size_t id = 0; id < p->L.nodes.size(); ++id)
      if (p->L.reach[id] && p->L.nodes[id].op == RF_OP_POISSON)
        int_mask |= 1u << p->L.nodes[p->L.nodes[id].in[0]].index;
    int rc = validate_columns(p->cols, n_cols, p->L.n_cols, lo, hi, int_mask, n_events,
                              p->L.precision == RF_FP32_COMP, stream, &bad);
    if (rc) {
      p->n = -1;
      return rc;
    }
    if (bad) {
      p->n = -1;  // not bound
      return fail(RF_E_INVALID, std::to_string(bad) +
                                    " event values outside their observable's range, not finite, or not an integer count");
    }
  }
  return RF_OK;
}

int rf_bind_weights(rf_program* p, int32_t node, const void* dev_bf16, void* stream) {
  (void)stream;
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  bool found = false;
  for (int id : p->L.mlp_nodes) found |= (p->L.orig.empty() ? id : p->L.orig[id]) == node;
  if (!found) return fail(RF_E_INVALID, "node is not an MLP leaf of this program");
  if (!dev_bf16) return fail(RF_E_INVALID, "weights are NULL");
  p->d_weights = dev_bf16;
  return RF_OK;
}

int rf_eval_values(rf_program* p, const double* theta, void* dev_out, void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  if (p->n > 0 && !dev_out) return fail(RF_E_INVALID, "dev_out is NULL");
  RfArgs a;
  fill_args(p, theta, a);
  a.values = dev_out;
  return launch(p, p->m.k_values, a, stream);
}

int rf_nll(rf_program* p, const double* theta, double* nll, int64_t* n_bad, void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  if (!nll) return fail(RF_E_INVALID, "nll is NULL");
  // a weighted extended NLL needs the sum of the weights, which only the
  // gradient kernel accumulates; its result block has the NLL in the same place
  rc = run_sync(p, p->L.wsum >= 0 ? p->m.k_grad : p->m.k_nll, theta, stream);
  if (rc) return rc;
  const int64_t bad = (int64_t)p->h_out[p->L.n_params + 1];
  if (n_bad) *n_bad = bad;
  *nll = bad ? INFINITY : p->h_out[0];
  if (bad) return fail(RF_E_NONFINITE, std::to_string(bad) + " events with p <= 0 or non-finite p");
  return RF_OK;
}

int rf_nll_grad(rf_program* p, const double* theta, double* nll, double* grad, int64_t* n_bad, void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  if (!nll || (p->L.n_params && !grad)) return fail(RF_E_INVALID, "nll or grad is NULL");
  rc = run_sync(p, p->m.k_grad, theta, stream);
  if (rc) return rc;
  const int P = p->L.n_params;
  const int64_t bad = (int64_t)p->h_out[P + 1];
  if (n_bad) *n_bad = bad;
  *nll = bad ? INFINITY : p->h_out[0];
  for (int k = 0; k < P; ++k) grad[k] = bad ? NAN : p->h_out[1 + k];
  if (bad) return fail(RF_E_NONFINITE, std::to_string(bad) + " events with p <= 0 or non-finite p");
  return RF_OK;
}

int rf_nll_grad_async(rf_program* p, const double* theta, void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  RfArgs a;
  fill_args(p, theta, a);
  return launch(p, p->m.k_grad, a, stream);
}

}  // extern "C"

namespace rf {
int enqueue_grad_on(rf_program* p, const double* theta, double* part, int32_t part_stride, unsigned* ticket,
                    double* out, void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  if (part_stride < p->nblk) return fail(RF_E_INVALID, "partial stride below the workgroup count");
  RfArgs a;
  fill_args(p, theta, a);
  a.part = part;
  a.nblk_max = part_stride;
  a.ticket = ticket;
  a.out = out;
  return launch(p, p->m.k_grad, a, stream);
}
}  // namespace rf

extern "C" {

const double* rf_program_result(const rf_program* p) { return p ? p->d_out : nullptr; }

int rf_unfused_build(const rf_program* p) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  if (p->L.has_mlp) return fail(RF_E_INVALID, "the unfused mode takes programs without MLP leaves");
  std::string path;
  return build_code_object(generate_source(p->L, p->block, p->ept, p->pfd, p->tg, p->prio, true), path);
}

int rf_nll_unfused(rf_program* p, const double* theta, double* nll, int64_t* n_bad, void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  if (!nll) return fail(RF_E_INVALID, "nll is NULL");
  if (p->L.has_mlp) return fail(RF_E_INVALID, "the unfused mode takes programs without MLP leaves");
  rf_program::Unfused& u = p->unf;
  hipError_t e;
  if (!u.mod) {
    const std::string src = generate_source(p->L, p->block, p->ept, p->pfd, p->tg, p->prio, true);
    std::string path;
    if ((rc = build_code_object(src, path))) return rc;
    std::ifstream f(path, std::ios::binary);
    std::vector<char> bytes((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    if (bytes.empty()) return fail(RF_E_DEVICE, "empty code object " + path);
    if ((e = hipModuleLoadData(&u.mod, bytes.data())) != hipSuccess) return hip_fail(e, "hipModuleLoadData");
    const std::vector<int> slot = unfused_slots(p->L);
    std::vector<hipFunction_t> fns;
    for (size_t id = 0; id < slot.size(); ++id) {
      if (slot[id] < 0) continue;
      hipFunction_t fn;
      const std::string name = "rf_u" + std::to_string(id);
      if ((e = hipModuleGetFunction(&fn, u.mod, name.c_str())) != hipSuccess) return hip_fail(e, name.c_str());
      fns.push_back(fn);
    }
    if ((e = hipModuleGetFunction(&u.k_nll, u.mod, "rf_u_nll")) != hipSuccess) return hip_fail(e, "rf_u_nll");
    if ((e = hipModuleGetFunction(&u.k_sum, u.mod, "rf_u_sum")) != hipSuccess) return hip_fail(e, "rf_u_sum");
    u.nodes = fns;
  }
  const int64_t n = p->n;
  const size_t es = p->L.precision == RF_FP32_COMP ? 4 : 8;
  const size_t need = es * u.nodes.size() * (size_t)(n > 0 ? n : 1);
  if (need > u.vals_bytes) {
    if (u.vals) (void)hipFree(u.vals);
    u.vals = nullptr;
    u.vals_bytes = 0;
    if ((e = hipMalloc(&u.vals, need)) != hipSuccess) return hip_fail(e, "hipMalloc (node arrays)");
    u.vals_bytes = need;
  }
  int64_t G = (n + p->block - 1) / p->block;
  const int64_t gcap = (int64_t)cu_count(p->device) * 8;
  G = G < 1 ? 1 : (G > gcap ? gcap : G);
  if (G > u.part_n) {
    if (u.part) (void)hipFree(u.part);
    u.part = nullptr;
    u.part_n = 0;
    if ((e = hipMalloc(&u.part, sizeof(double) * 3 * G)) != hipSuccess) return hip_fail(e, "hipMalloc (partials)");
    u.part_n = (int)G;
  }
  if (!u.out && (e = hipMalloc(&u.out, sizeof(double) * 2)) != hipSuccess) return hip_fail(e, "hipMalloc");
  RfArgs a;
  fill_args(p, theta, a);
  a.values = u.vals;
  a.part = u.part;
  a.nblk_max = u.part_n;
  a.out = u.out;
  hipStream_t st = (hipStream_t)stream;
  void* args1[] = {&a};
  for (hipFunction_t fn : u.nodes)
    if ((e = hipModuleLaunchKernel(fn, (unsigned)G, 1, 1, p->block, 1, 1, 0, st, args1, nullptr)) != hipSuccess)
      return hip_fail(e, "unfused node kernel");
  if ((e = hipModuleLaunchKernel(u.k_nll, (unsigned)G, 1, 1, p->block, 1, 1, 0, st, args1, nullptr)) != hipSuccess)
    return hip_fail(e, "rf_u_nll");
  int nb = (int)G;
  void* args2[] = {&a, &nb};
  if ((e = hipModuleLaunchKernel(u.k_sum, 1, 1, 1, p->block, 1, 1, 0, st, args2, nullptr)) != hipSuccess)
    return hip_fail(e, "rf_u_sum");
  double h[2] = {0, 0};
  if ((e = hipMemcpyAsync(h, u.out, sizeof h, hipMemcpyDeviceToHost, st)) != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  const int64_t bad = (int64_t)h[1];
  if (n_bad) *n_bad = bad;
  *nll = bad ? INFINITY : h[0];
  if (bad) return fail(RF_E_NONFINITE, std::to_string(bad) + " events with p <= 0 or non-finite p");
  return RF_OK;
}

int rf_hess_build(const rf_program* p) {
  if (!p) return fail(RF_E_INVALID, "program is NULL");
  std::string why;
  if (!hess_supported(p->L, &why)) return fail(RF_E_INVALID, why);
  std::string path;
  return build_code_object(generate_hess_source(p->L, p->block), path);
}

int rf_nll_grad_hess(rf_program* p, const double* theta, double* nll, double* grad, double* hess, int64_t* n_bad,
                     void* stream) {
  int rc = ready(p, theta);
  if (rc) return rc;
  const int P = p->L.n_params;
  if (!nll || (P && (!grad || !hess))) return fail(RF_E_INVALID, "nll, grad or hess is NULL");
  std::string why;
  if (!hess_supported(p->L, &why)) return fail(RF_E_INVALID, why);
  rf_program::Hess& h = p->hes;
  hipError_t e;
  const int nout = P + 2 + P * P;
  if (!h.mod) {
    std::string path;
    if ((rc = build_code_object(generate_hess_source(p->L, p->block), path))) return rc;
    std::ifstream f(path, std::ios::binary);
    std::vector<char> bytes((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    if (bytes.empty()) return fail(RF_E_DEVICE, "empty code object " + path);
    if ((e = hipModuleLoadData(&h.mod, bytes.data())) != hipSuccess) return hip_fail(e, "hipModuleLoadData");
    if ((e = hipModuleGetFunction(&h.k, h.mod, "rf_k_hess")) != hipSuccess) return hip_fail(e, "rf_k_hess");
    if ((e = hipMalloc(&h.ticket, sizeof(unsigned) * RF_TICKET_WORDS)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMemset(h.ticket, 0, sizeof(unsigned) * RF_TICKET_WORDS)) != hipSuccess) return hip_fail(e, "hipMemset");
    if ((e = hipMalloc(&h.out, sizeof(double) * nout)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipHostMalloc(&h.h_out, sizeof(double) * nout, hipHostMallocMapped | hipHostMallocCoherent)) !=
        hipSuccess)
      return hip_fail(e, "hipHostMalloc");
    memset(h.h_out, 0, sizeof(double) * nout);
    if ((e = hipHostGetDevicePointer((void**)&h.d_hout, h.h_out, 0)) != hipSuccess)
      return hip_fail(e, "hipHostGetDevicePointer");
  }
  // one workgroup per 1024 events (four per lane), at most two per CU
  int64_t G = (p->n + 4 * (int64_t)p->block - 1) / (4 * (int64_t)p->block);
  const int64_t gcap = (int64_t)cu_count(p->device) * 2;
  G = G < 1 ? 1 : (G > gcap ? gcap : G);
  const int ns1 = hess_nsums(p->L) + 1;
  if (G > h.part_n) {
    if (h.part) (void)hipFree(h.part);
    h.part = nullptr;
    h.part_n = 0;
    if ((e = hipMalloc(&h.part, sizeof(double) * ns1 * G)) != hipSuccess) return hip_fail(e, "hipMalloc (partials)");
    h.part_n = (int)G;
  }
  RfArgs a;
  fill_args(p, theta, a);
  a.part = h.part;
  a.nblk_max = h.part_n;
  a.ticket = h.ticket;
  a.out = h.out;
  a.hout = h.d_hout;
  if ((rc = order_launch(p->last_stream, p->launched, stream))) return rc;
  arm_result(h.h_out, nout);
  size_t sz = sizeof(RfArgs);
  void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &a, HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz, HIP_LAUNCH_PARAM_END};
  if ((e = hipModuleLaunchKernel(h.k, (unsigned)G, 1, 1, p->block, 1, 1, 0, (hipStream_t)stream, nullptr, cfg)) !=
      hipSuccess)
    return hip_fail(e, "rf_k_hess launch");
  if ((rc = wait_result(h.h_out, nout, stream, nullptr))) return rc;
  const int64_t bad = (int64_t)h.h_out[P + 1];
  if (n_bad) *n_bad = bad;
  *nll = bad ? INFINITY : h.h_out[0];
  for (int k = 0; k < P; ++k) grad[k] = bad ? NAN : h.h_out[1 + k];
  for (int k = 0; k < P * P; ++k) hess[k] = bad ? NAN : h.h_out[P + 2 + k];
  if (bad) return fail(RF_E_NONFINITE, std::to_string(bad) + " events with p <= 0 or non-finite p");
  return RF_OK;
}

int rf_gauss_legendre(int32_t K, double lo, double hi, double* x, double* w) {
  if (K < 1 || !x || !w) return fail(RF_E_INVALID, "bad arguments");
  rf::gauss_legendre(K, lo, hi, x, w);
  return RF_OK;
}

}  // extern "C"
