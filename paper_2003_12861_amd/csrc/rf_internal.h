// rf_internal.h -- host-side structures of the likelihood library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/rfgpu.h"
#include "device/rf_kabi.h"

struct rf_program;
struct rf_binned;

namespace rf {

// node kinds beyond the public ops
enum { K_OBS = 100, K_PARAM = 101, K_CONST = 102 };

struct Node {
  int32_t op = 0;
  std::string name;
  std::vector<int32_t> in;
  std::vector<double> attrs;
  double lo = 0, hi = 0;  // OBS range / PARAM bounds
  double value = 0;       // CONST value
  int32_t index = -1;     // OBS column / PARAM theta index
};

bool is_leaf(int op);
bool is_paramlike(int op);
bool is_pdf(int op);
int leaf_n_shape(const Node& n);  // number of shape inputs of a leaf

// error reporting (thread-local message)
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// ---- lowered program ------------------------------------------------------
struct Slot {          // a shape/fraction input whose value depends on theta
  int node;            // leaf or ADD node
  int j;               // input position among its shape inputs (ADD: fraction j)
  int pl;              // parameter-like node feeding it
  int sum;             // leaf: index of its event sum D; ADD: -1 (uses Y sums)
};

struct Lowered {
  std::vector<Node> nodes;         // copy of the graph (expanded into a tree if PDF nodes were shared)
  std::vector<int> orig;           // after an expansion: the graph's id of each node (else empty)
  int top = -1;
  int precision = RF_FP64;
  int n_params = 0, n_cols = 0;    // n_cols: observables
  int weighted = 0;                // one more column: per-event weights
  int ext_nu = -1;                 // extended likelihood: node of nu (-1: not extended)
  int wsum = -1;                   // weighted extended likelihood: index of the sum of weights
  std::vector<double> plo, phi;    // parameter bounds
  std::vector<char> reach;
  std::vector<int> cst_off;        // per node: offset of its FP64 constant block
  int n_cst = 0;
  // PDF tree (every PDF node feeds one sum or product).  For each PDF node
  // c, beta_c is its per-event adjoint without parameter-only factors;
  // Y_c = sum_i beta_c u_c is accumulated for "canonical" nodes (the top and
  // the components of sums); a factor of a product shares the product's.
  std::vector<int> parent;         // per PDF node: its user (-1 for the top)
  std::vector<int> canon;          // per PDF node: node whose Y sum it uses
  std::vector<int> ysum;           // per canonical node: index of Y_c (or -1)
  std::vector<Slot> slots;
  int n_sums = 0;                  // including sum 0 (= NLL)
  bool has_numconv = false, has_mlp = false, has_poisson = false;
  std::vector<double> aux;         // FP64 device inputs (Gauss-Legendre rules, ...)
  std::vector<int> aux_off;        // per node: offset into aux (or -1)
  std::vector<int> mlp_nodes;      // MLP leaves (need bound weights)
};

int lower(const std::vector<Node>& g, int top, int precision, Lowered& out);
// unfused = false: the fused kernels (values, NLL, NLL+gradient); true: the
// unfused per-node batch mode (one kernel per PDF node, then the NLL)
std::string generate_source(const Lowered& L, int block_size, int ept, int pfd, int tg, int prio,
                            bool unfused = false);
// unfused mode: slot of each PDF node's value array (-1: not a reachable PDF node)
std::vector<int> unfused_slots(const Lowered& L);
// the Hessian kernel (rf_k_hess) of a program: whether every leaf has second
// derivatives (else why not), its number of event sums, its source
bool hess_supported(const Lowered& L, std::string* why);
int hess_nsums(const Lowered& L);
std::string generate_hess_source(const Lowered& L, int block_size);

// code-object cache + compiler driver
struct Module {
  hipModule_t mod = nullptr;
  hipFunction_t k_values = nullptr, k_nll = nullptr, k_grad = nullptr;
};
int build_code_object(const std::string& src, std::string& path_out);
int load_module(const std::string& path, bool f32, Module& m);  // f32: FP32 form entry names
uint64_t fnv1a(const std::string& s);
std::string cache_dir();

// Synchronous results in mapped host memory: before a launch the host fills
// the n result words with RF_SENTINEL, a signalling-NaN pattern that no kernel
// result has (FP64 arithmetic produces only quiet NaNs); the kernel's last
// workgroup writes each word with a system-scope store; the host polls until
// no word holds the sentinel (every aligned 8-byte word arrives whole).  After
// 20 ms it synchronises the stream instead (long calls, errors).
constexpr uint64_t RF_SENTINEL = 0x7FF4D1CE5EED0001ull;
void arm_result(double* h, int n);
int wait_result(const double* h, int n, void* stream, int64_t* slow);
// before a launch on `stream`: wait for the previous launch's stream if it was
// another one (kernels of one program share their ticket words)
int order_launch(void*& last, bool& launched, void* stream);

// host-side domain checks of a parameter point
int check_theta(const Lowered& L, const double* theta);
void eval_paramlike(const Lowered& L, const double* theta, std::vector<double>& pv);

// surrogate normalisation kernel (rf_mlp.hip)
int mlp_renorm_launch(const void* w, const double* q5, const double* box12, const double* grid, int K, double* out,
                      void* stream);
// workgroups of the normalisation kernel for a K-point rule (256 points each);
// its partial sums take 6 doubles per workgroup
inline int mlp_renorm_blocks(int K) { return (K + 255) / 256; }

// column checks of rf_bind_columns with RF_VALIDATE (rf_validate.hip): the
// number of events outside [lo[c], hi[c]] (or not finite, or, for the
// columns in int_mask, not an integer) in columns c < n_range, plus the
// number of non-finite values in columns n_range .. n_cols - 1 (event
// weights); synchronises the stream
int validate_columns(const void* const* cols, int n_cols, int n_range, const double* lo, const double* hi,
                     unsigned int_mask, int64_t n, bool f32, void* stream, int64_t* n_bad);

// one NLL+gradient evaluation of a bound program (as rf_nll_grad_async) with
// the cross-workgroup partials (part_stride >= the workgroup count per sum),
// the ticket words (RF_TICKET_WORDS, zero) and the result block supplied by
// the caller instead of the program's workspace; allocates nothing
int enqueue_grad_on(rf_program* p, const double* theta, double* part, int32_t part_stride, unsigned* ticket,
                    double* out, void* stream);

// parameters of a binned model: 1 + J (mu, alpha_1..alpha_J)
int binned_n_params(const rf_binned* b);

// Gauss-Legendre rule (host)
void gauss_legendre(int K, double lo, double hi, double* x, double* w);

// What the BFGS minimiser (rf_fit.cpp) minimises: P parameters within
// [lo, hi], one NLL+gradient evaluation (RF_OK, RF_E_NONFINITE and
// RF_E_DOMAIN steer the line search; other codes end the fit), and
// optionally the exact Hessian at a point (else central differences of the
// gradient give the uncertainties).
struct Objective {
  int P = 0;
  std::vector<double> lo, hi;
  std::function<int(const double* x, double* f, double* g)> eval;
  std::function<int(const double* x, double* H)> hess;
};
int bfgs_fit(const Objective& obj, const double* theta0, const double* hinv0, double edm_tol, int32_t max_iter,
             double* theta_out, double* sigma_out, double* cov_out, double* info_out);

}  // namespace rf

struct rf_graph {
  std::vector<rf::Node> nodes;
  int n_obs = 0, n_params = 0;
};

struct rf_program {
  rf::Lowered L;
  std::string source;
  std::string co_path;
  rf::Module m;
  bool loaded = false;
  int block = 256;  // threads per workgroup (compile-time constant of the kernel)
  int ept = 4;      // events per lane and step of the event loop (compile-time)
  int pfd = 3;      // groups in flight per lane (load ring depth, compile-time)
  int tg = 16;      // ticket groups of the end-of-kernel hand-off (compile-time)
  int prio = 1;     // wavefront issue-priority policy of the event loop (compile-time)
  int resident = 4; // workgroups of the gradient kernel one CU holds at once (occupancy query)
  int64_t n_sync = 0, n_slow = 0;  // synchronous calls; those whose wait fell back to a stream sync
  // stream of the previous launch: a launch on another stream first waits for
  // it (the previous kernel's last workgroup resets the ticket words after
  // writing the result a synchronous call returns on)
  void* last_stream = nullptr;
  bool launched = false;
  int blocks_override = 0;
  uint32_t flags = 0;  // RF_COMPILE_* / RF_VALIDATE given to rf_compile
  // binding
  const void* cols[RF_MAX_COLS] = {};
  void* owned[RF_MAX_COLS + 1] = {};         // contiguous copies made by rf_bind_columns_strided
  size_t owned_bytes[RF_MAX_COLS + 1] = {};
  int64_t n = -1;
  int nblk = 0, nblk_max = 0;
  double* d_part = nullptr;
  unsigned* d_ticket = nullptr;
  double* d_out = nullptr;
  double* h_out = nullptr;   // pinned, mapped: the kernel writes the result here too
  double* d_hout = nullptr;  // device address of h_out
  double* d_aux = nullptr;   // auxiliary FP64 block (surrogate normalisation, ...)
  const void* d_weights = nullptr;
  int device = -1;
  // unfused per-node batch mode (rf_nll_unfused): built and allocated on first use
  struct Unfused {
    hipModule_t mod = nullptr;
    std::vector<hipFunction_t> nodes;  // kernels of the PDF nodes, inputs before users
    hipFunction_t k_nll = nullptr, k_sum = nullptr;
    void* vals = nullptr;  // node value arrays
    size_t vals_bytes = 0;
    double* part = nullptr;  // [3][part_n]: partial sums, bad-event counts, sums of weights
    int part_n = 0;
    double* out = nullptr;  // [NLL, bad events]
  } unf;
  // Hessian kernel (rf_nll_grad_hess): built and allocated on first use
  struct Hess {
    hipModule_t mod = nullptr;
    hipFunction_t k = nullptr;
    double* part = nullptr;    // [sums + 1][part_n]
    int part_n = 0;
    unsigned* ticket = nullptr;
    double* out = nullptr;     // [nll, grad[P], n_bad, hess[P * P]]
    double* h_out = nullptr;   // mapped host copy
    double* d_hout = nullptr;
  } hes;
};
