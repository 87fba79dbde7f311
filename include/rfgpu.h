/*
 * rfgpu.h -- C ABI of the MI355X batched-likelihood library.
 *
 * What it computes (Hageboeck & Moneta, "Making RooFit Ready for Run 3",
 * ACAT 2019):
 *   - A likelihood model is a computation graph of observables, parameters,
 *     functions and PDFs; every node evaluates to a real number and a PDF's
 *     value is the probability density of an event (Section 1, Fig. 1).
 *   - The likelihood needs the probability of every event; evaluating all
 *     events of a node in one call ("batch") replaces per-event recursion
 *     (Section 4, 4.1).  Here the whole compiled graph is evaluated for all
 *     events in ONE fused GPU kernel with intermediates in registers.
 *   - Parameter-only branches (normalisation integrals) are computed once per
 *     parameter point (Section 4) -- in FP64, in the kernel's prologue.
 *   - NLL(theta) = -sum_i log p(x_i | theta), each PDF normalised over the
 *     observables' ranges (a box); the sum is a deterministic compensated
 *     reduction (plain FP64 within a wavefront, double-double TwoSum across
 *     wavefronts and workgroups, fixed order).  The gradient dNLL/dtheta comes
 *     from a hand-written adjoint in the same kernel.
 *
 * Conventions for every function:
 *   - Return value: RF_OK (0) or a negative RF_E_* code; rf_last_error()
 *     then holds a message (thread-local, valid until the next call on the
 *     same thread).
 *   - Pointers named dev_* are device pointers (e.g. torch tensor data); they
 *     are BORROWED: the caller keeps them alive while they are bound.  Every
 *     other pointer is host memory owned by the caller.  theta is copied on
 *     each call.
 *   - stream is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it; the functions that return host values synchronise it.
 *   - A program is not re-entrant: do not call it from two threads at once.
 *     Distinct programs are independent.
 */
#ifndef RFGPU_H
#define RFGPU_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
  RF_OK = 0,
  RF_E_INVALID = -1,   /* bad argument, graph error (arity, unknown op, ...) */
  RF_E_DOMAIN = -2,    /* theta outside declared bounds or mathematically invalid */
  RF_E_NONFINITE = -3, /* some p_i <= 0 or not finite: nll = +inf, n_bad set, grad NaN */
  RF_E_DEVICE = -4,    /* HIP runtime or kernel-compiler failure */
  RF_E_OOM = -5,       /* device allocation failed */
  RF_E_STATE = -6      /* e.g. evaluation before columns are bound */
};

/* ---- precision forms ----------------------------------------------------- */
enum {
  RF_FP64 = 0,      /* plain FP64: FP64 columns and arithmetic */
  RF_FP32_COMP = 1  /* FP32 per-event arithmetic and FP32 columns; FP64 prologue
                       (normalisations), FP64 per-thread accumulation, FP64
                       re-evaluation of events with p_i < 1e-30 in FP32,
                       compensated FP64 cross-block reduction */
};

/* ---- compile flags ------------------------------------------------------- */
enum {
  RF_COMPILE_NO_LOAD = 1u << 0, /* generate + build the code object only (no GPU
                                   needed); the program can then only be queried */
  RF_VALIDATE = 1u << 1,        /* rf_bind_columns checks that every event lies in
                                   its observables' ranges, that the observables of
                                   Poisson leaves hold integers and that every event
                                   weight is finite (one device pass), RF_E_INVALID
                                   otherwise */
  RF_COMPILE_WEIGHTED = 1u << 2 /* weighted events: one more column after the
                                   observables holds per-event weights w_i (program
                                   dtype, any finite real); the NLL is
                                   -sum_i w_i log p_i and the gradient its derivative
                                   (uncertainties from its Hessian carry no
                                   sum-of-squared-weights correction); values p_i are
                                   unchanged.  At most 7 observables. */
};

/* ---- graph ops ----------------------------------------------------------- */
/* Inputs are node ids.  A PDF leaf's input 0 is an observable; its shape
 * inputs are parameter-like nodes (PARAM, CONST or FN_*).  Each leaf is
 * normalised over its observable's range. */
enum {
  RF_OP_GAUSS = 1,          /* (x, mu, sigma): exp(-(x-mu)^2/(2 sigma^2))            */
  RF_OP_CHEB = 2,           /* (x, c1..cn), n<=8: 1 + sum c_k T_k(x'), x' in [-1,1]  */
  RF_OP_EXP = 3,            /* (x, k); attrs[0] = 0: exp(-x/k) (k = tau > 0),
                                         attrs[0] = 1: exp(k x) (k = rate)          */
  RF_OP_DECAY_GAUSS = 4,    /* (t, tau, sigma, bias): single-sided exp(-t/tau) decay
                               convolved with a Gaussian resolution (analytic erfc) */
  RF_OP_ARGUS = 5,          /* (m, m0 [CONST], c <= 0): m sqrt(U) exp(c U), U = 1-(m/m0)^2 */
  RF_OP_BW = 6,             /* (x, M, Gamma): 1/((x-M)^2 + Gamma^2/4)                */
  RF_OP_NUMCONV_BW_CB = 7,  /* (x, M, Gamma, sigma, alpha, n); attrs (ylo, yhi, K):
                               sum_k w_k CB(y_k) BW(x - y_k) over a K-point
                               Gauss-Legendre rule on [ylo, yhi], K <= 1024       */
  RF_OP_MLP = 8,            /* (x, q1..q5); attrs: 6 (lo, hi) input boxes, K:
                               exp(s(u)) with s a 6-64-64-64-1 tanh MLP (BF16
                               weights bound with rf_bind_weights), u = affine maps
                               onto [-1,1] of (x - q1, q1..q5) with the boxes
                               (the first box is that of x - q1), normalised by a
                               K-point Gauss-Legendre sum over x's range; FP32 only */
  RF_OP_POISSON = 9,        /* (n, lambda > 0): lambda^n e^-lambda / n!, an unbinned
                               Poisson PDF; the observable holds integers and its
                               range [lo, hi] has integer ends, 0 <= lo < hi,
                               hi - lo < 2048 (normalised over lo..hi) */
  RF_OP_ADD_PDF = 20,       /* (pdf_1..pdf_n, f_1..f_{n-1}): sum_j f_j pdf_j +
                               (1 - sum f) pdf_n, each pdf normalised            */
  RF_OP_PROD_PDF = 21,      /* (pdf_1..pdf_n) over disjoint observables           */
  RF_OP_EXTENDED = 22,      /* (pdf, nu param-like > 0), only as the compiled top of
                               a program: the extended likelihood.  Event
                               values are pdf's; the NLL gains nu - N log nu (N the
                               number of bound events; in a weighted program the
                               sum of the weights), i.e. it is, up to the
                               constant log N!, -sum_i log(nu p_i) + nu.  Yields of
                               a sum: fractions nu_j / nu_tot (RF_OP_FN_RATIO) and
                               nu = nu_tot (RF_OP_FN_LINEAR of the yields). */
  RF_OP_FN_LINEAR = 40,     /* (a_1..a_n param-like); attrs (c0, c1..cn): c0 + sum c_j a_j */
  RF_OP_FN_PRODUCT = 41,    /* (a_1..a_n param-like): prod a_j                     */
  RF_OP_FN_RATIO = 42       /* (a, b param-like): a / b (b != 0)                     */
};

typedef struct rf_graph rf_graph;
typedef struct rf_program rf_program;
typedef struct rf_binned rf_binned;

const char* rf_last_error(void);
/* library version string; also names the device code-object cache layout */
const char* rf_version(void);

/* ---- graph construction (host only) -------------------------------------- */
/* A model is a graph of observables, parameters, functions and PDFs linked
 * into a computation graph whose every node evaluates to a real number
 * (Section 1, Fig. 1).  The graph is owned by the caller until
 * rf_graph_free; rf_compile copies what it needs. */
int rf_graph_new(rf_graph** out);
void rf_graph_free(rf_graph* g);
/* column index = declaration order of observables; [lo, hi] is the range
 * every PDF on this observable is normalised over (lo < hi, finite). */
int rf_graph_observable(rf_graph* g, const char* name, double lo, double hi, int32_t* id);
/* theta index = declaration order of parameters; [lo, hi] are the bounds
 * checked on every evaluation (lo <= theta <= hi). */
int rf_graph_parameter(rf_graph* g, const char* name, double lo, double hi, int32_t* id);
int rf_graph_constant(rf_graph* g, double value, int32_t* id);
/* A function or PDF node (the PDFs of Section 4.1: Gaussian, Poisson,
 * exponential, sums of PDFs; the others are the benchmark models'); inputs
 * must be ids of earlier nodes (so the graph is acyclic by construction);
 * RF_E_INVALID for an unknown op, a wrong arity or attribute count. */
int rf_graph_node(rf_graph* g, int32_t op, const int32_t* inputs, int32_t n_inputs,
                  const double* attrs, int32_t n_attrs, int32_t* id);

/* ---- compilation --------------------------------------------------------- */
/* The paper's two ideas for the hot path, on the GPU: parameter-only
 * branches (normalisation integrals) computed once per parameter point
 * (Section 4), and every event of the model evaluated in one batch call
 * (Section 4.1), here fused across nodes.
 * Validates the subgraph under top, lowers it to a flat node program,
 * generates one fused HIP kernel source for it (three entry points: values,
 * NLL, NLL+gradient) specialised to the precision form, builds a gfx950 code
 * object (content-addressed cache; built with the ROCm compiler on a miss) and
 * loads it.  The graph may be freed afterwards.
 * A PDF node may feed several sums or products (the paper's model is a graph,
 * Section 1): the lowering then copies it, with the PDF nodes below it, once
 * per use, so that the program is a tree (the adjoint's path constants are
 * single products); parameters, observables and parameter functions stay
 * shared.  rf_bind_weights takes the graph's id of an MLP leaf either way. */
int rf_compile(const rf_graph* g, int32_t top, int32_t precision, uint32_t flags,
               rf_program** out);
void rf_program_free(rf_program* p);
/* n_columns: observables, plus one for the weights of a RF_COMPILE_WEIGHTED
 * program; n_sums: number of FP64 event sums the gradient kernel accumulates */
int rf_program_info(const rf_program* p, int32_t* n_params, int32_t* n_columns,
                    int32_t* n_sums);
/* generated HIP source (NUL-terminated, owned by the program) */
const char* rf_program_source(const rf_program* p);
/* Counters of the synchronous calls (rf_nll, rf_nll_grad) of a program: how
 * many were made and how many waited longer than 20 ms for the result word
 * and fell back to a stream synchronisation.  Either pointer may be NULL. */
int rf_program_stats(const rf_program* p, int64_t* sync_calls, int64_t* slow_waits);

/* ---- binding ------------------------------------------------------------- */
/* The data as one contiguous array per observable (the structure-of-arrays
 * layout the batch interface reads, Section 4.1).
 * dev_cols[j]: contiguous column of observable j (n_events values, unit
 * stride), float64 for RF_FP64 programs, float32 for RF_FP32_COMP (the
 * kernels read 16-byte vectors of consecutive events; rf_bind_columns_strided
 * takes strided or other-dtype columns); for a RF_COMPILE_WEIGHTED
 * program dev_cols[n_observables] holds the event weights.  Allocates the
 * program's workspace (block partials, result block) on the current device;
 * with RF_VALIDATE, also checks the columns (synchronising the stream). */
int rf_bind_columns(rf_program* p, const void* const* dev_cols, int32_t n_cols,
                    int64_t n_events, void* stream);

/* Column element types for rf_bind_columns_strided. */
enum {
  RF_COL_F32 = 0, /* float */
  RF_COL_F64 = 1  /* double */
};
/* rf_bind_columns for columns given with a stride or in the other
 * floating-point type (one array per observable, Section 4.1, in any of the
 * two types and any positive element stride).
 * dev_cols[j]: device pointer to the first value of column j; strides[j]:
 * distance between consecutive events in elements (>= 1); dtypes[j]:
 * RF_COL_F32 or RF_COL_F64; the caller guarantees that
 * dev_cols[j] + (n_events - 1) * strides[j] lies in its allocation.
 * A column already in the program's type with unit stride is bound in place,
 * as rf_bind_columns binds it.  Any other is copied on the device into a
 * contiguous array in the program's type that the program owns (converted by
 * round-to-nearest; reused by later calls, freed with the program): the
 * binding is a snapshot of such a column, and the source may be freed once
 * the call returns (the call synchronises the stream after the copies).
 * Errors: RF_E_INVALID for a wrong column count, a NULL pointer, an unknown
 * dtype or a stride below 1, RF_E_STATE for a program compiled without
 * loading or loaded on another device, RF_E_DEVICE / RF_E_OOM from the copies;
 * then as rf_bind_columns. */
int rf_bind_columns_strided(rf_program* p, const void* const* dev_cols, const int64_t* strides,
                            const int32_t* dtypes, int32_t n_cols, int64_t n_events, void* stream);
/* MLP leaf weights: 8833 bf16 values (layout W1[64][6] b1[64] W2[64][64]
 * b2[64] W3[64][64] b3[64] W4[64] b4[1], row = output unit). */
int rf_bind_weights(rf_program* p, int32_t node, const void* dev_bf16, void* stream);
/* launch shape override (0 = automatic) */
int rf_set_launch(rf_program* p, int32_t blocks, int32_t threads);

/* ---- evaluation ---------------------------------------------------------- */
/* The probabilities of all events in a single call (Section 4.1); the NLL is
 * -sum_i log p_i over them (Section 4: the likelihood needs the probability of
 * every event).  RF_E_DOMAIN for theta outside its bounds or invalid for a
 * leaf, RF_E_STATE before binding, RF_E_NONFINITE (nll = +inf, grad NaN,
 * n_bad set) when some p_i <= 0 or is not finite.
 * per-event normalised p_i into dev_out (n_events, bound dtype); async */
int rf_eval_values(rf_program* p, const double* theta, void* dev_out, void* stream);
/* NLL only; synchronous.  n_bad may be NULL. */
int rf_nll(rf_program* p, const double* theta, double* nll, int64_t* n_bad, void* stream);
/* NLL and gradient (n_params); synchronous. */
int rf_nll_grad(rf_program* p, const double* theta, double* nll, double* grad,
                int64_t* n_bad, void* stream);
/* The unfused batch mode of the paper (Section 4.1: one call per node computes
 * that node's values for all events into an array), kept as an ablation of the
 * fused kernel: one kernel per PDF node writes the node's value of every event
 * into its own array in device memory (inputs before users), then the NLL of
 * the top node's array is summed in a fixed order (weighted and extended
 * programs included).  NLL only; programs without MLP leaves (RF_E_INVALID
 * otherwise: the surrogate evaluates whole wavefronts on MFMA).  The
 * first call builds its code object; the node arrays (PDF nodes x n_events
 * values of the program dtype) are allocated on first use and kept with the
 * program.  Synchronous; n_bad may be NULL. */
int rf_nll_unfused(rf_program* p, const double* theta, double* nll, int64_t* n_bad, void* stream);
/* builds the unfused mode's code object into the cache without loading it (no
 * GPU needed; also valid for a RF_COMPILE_NO_LOAD program) */
int rf_unfused_build(const rf_program* p);
/* enqueue one NLL+gradient evaluation without synchronising; the result
 * block [nll, grad[n_params], n_bad] stays in device memory at
 * rf_program_result(p) until the next evaluation of this program. */
int rf_nll_grad_async(rf_program* p, const double* theta, void* stream);
const double* rf_program_result(const rf_program* p);

/* For callers that cannot allocate device memory (code under stream capture
 * into a HIP graph, tight serving loops, harnesses that forbid allocation):
 * the NLL+gradient evaluation of rf_nll_grad_async without the program's
 * workspace.  The kernel's cross-workgroup scratch (ticket words and
 * per-workgroup partial sums, (n_sums + 1) x workgroups doubles) lives in a
 * fixed 256 KiB device array of the library, one per device, kept until the
 * process ends; the result block [nll, grad[n_params], n_bad, sums[n_sums]]
 * (n_params + 2 + n_sums doubles, see rf_program_info) is written to the
 * caller's device buffer dev_result.  Asynchronous on the stream; calls no
 * allocating routine.  The program must be bound (rf_bind_columns, and
 * rf_bind_weights for MLP leaves).  RF_E_INVALID if the partials do not fit
 * the array (lower the workgroup count with rf_set_launch).  Every call on a
 * device shares its array: calls that overlap on one device race, so
 * serialise them (one stream, or events). */
int rf_nll_grad_noalloc(rf_program* p, const double* theta, double* dev_result, void* stream);

/* The NLL, its gradient and its Hessian hess[n_params * n_params] (row-major)
 * at theta in one fused pass: the curvature from which a fit's uncertainties
 * come (the paper's fits, Section 3 and Fig. 5; its parameter-only caching,
 * Section 4, here for second derivatives of the normalisations too).
 * Per-event arithmetic in FP64 whatever the program's precision form; the
 * kernel accumulates log p, its gradient and its Hessian in the leaf and
 * fraction inputs and contracts them with the parameter functions' first and
 * second derivatives.  Programs whose leaves all have second derivatives
 * (Gaussian, Chebyshev, exponential, decay (x) resolution, ARGUS,
 * Breit-Wigner) and at most 16 parameters; RF_E_INVALID otherwise.  The first
 * call builds and loads its own code object and allocates its workspace
 * (kept with the program).  Synchronous; n_bad may be NULL; events with
 * p <= 0 give RF_E_NONFINITE, nll = +inf, grad and hess NaN. */
int rf_nll_grad_hess(rf_program* p, const double* theta, double* nll, double* grad, double* hess,
                     int64_t* n_bad, void* stream);
/* builds the Hessian kernel's code object into the cache without loading it
 * (no GPU needed; also valid for a RF_COMPILE_NO_LOAD program) */
int rf_hess_build(const rf_program* p);

/* ---- fit ------------------------------------------------------------------ */
/* The fits whose run time the paper's batch computation speeds up (Section 3
 * and Fig. 5).
 * Quasi-Newton (BFGS) minimisation of NLL with backtracking line search that
 * backs off infinite NLL and out-of-bounds points; converged when
 * EDM = g^T H^-1 g / 2 < edm_tol.  sigma_out: sqrt(diag(H^-1)) with H the
 * Hessian of rf_nll_grad_hess at the minimum, or central differences of the
 * analytic gradient for programs it does not take (may be NULL).
 * info_out[4] = {n_iterations, n_evaluations, edm, converged(0/1)}. */
int rf_fit_bfgs(rf_program* p, const double* theta0, double edm_tol, int32_t max_iter,
                double* theta_out, double* sigma_out, double* info_out, void* stream);
/* rf_fit_bfgs with two optional matrices (row-major P x P, host memory, may be
 * NULL): hinv0, the initial inverse Hessian (symmetrised; its diagonal must be
 * positive and finite, else RF_E_INVALID), in place of the one rf_fit_bfgs
 * builds from P forward differences of the gradient -- e.g. the covariance of
 * a fit of a cheaper model of the same data, which lets the exact fit start
 * with that fit's curvature; cov_out, the covariance at the minimum (the
 * inverse of the Hessian the uncertainties come from; NaN when that Hessian
 * is not positive definite).  rf_fit_bfgs(...) is rf_fit_bfgs_ex with both
 * NULL. */
int rf_fit_bfgs_ex(rf_program* p, const double* theta0, const double* hinv0, double edm_tol,
                   int32_t max_iter, double* theta_out, double* sigma_out, double* cov_out,
                   double* info_out, void* stream);

/* ---- binned template likelihood (HistFactory-like, Section 3) -------------- */
/* C channels, S samples (sample 0 scaled by the signal strength mu), B bins,
 * J nuisance parameters.  Host FP64 inputs: T[C][S][B] nominal yields,
 * Tp/Tm[C][S][J][B] the +-1 sigma yields, nobs[C][B] observed counts.
 * log(T+-/T) is taken once here (FP64) and stored as FP32 on the device.
 * theta = (mu, alpha_1..alpha_J):
 *   nu_csb = mu^[s=0] T_csb exp(sum_j |alpha_j| log(T^{sgn alpha_j}_csbj / T_csb)),
 *   NLL = sum_cb (nu_cb - n_cb log nu_cb) + sum_j alpha_j^2 / 2,
 * nu_cb = sum_s nu_csb; the constant sum log(n!) is left out. */
int rf_binned_new(int32_t C, int32_t S, int32_t B, int32_t J, const double* T,
                  const double* Tp, const double* Tm, const double* nobs, void* stream,
                  rf_binned** out);
void rf_binned_free(rf_binned* b);
int rf_binned_nll_grad(rf_binned* b, const double* theta, double* nll, double* grad,
                       void* stream);
int rf_binned_nll_grad_async(rf_binned* b, const double* theta, void* stream);
const double* rf_binned_result(const rf_binned* b);

/* ---- combined likelihoods and constraints (Section 3) ------------------------ */
/* A combined measurement: independent likelihoods that share parameters (the
 * paper's combined measurements of a parameter such as a signal strength,
 * Section 3), times Gaussian constraint factors on parameters.  With
 * global parameters theta[0..n_params-1]:
 *   NLL(theta) = sum_t NLL_t(theta[map_t[0]], .., theta[map_t[P_t - 1]])
 *              + sum_c (theta[k_c] - mean_c)^2 / (2 width_c^2),
 * each term t a compiled program (rf_compile, columns bound) or a binned model
 * (rf_binned_new), each NLL_t as its own rf_nll_grad / rf_binned_nll_grad
 * gives it; the gradient is the terms' gradients added through the maps plus
 * (theta[k_c] - mean_c) / width_c^2.  Terms may share parameters in any way;
 * a global parameter used by no term and no constraint has gradient 0.
 *
 * rf_sum_new: n_params in 1..256 global parameters; lo/hi (host, n_params
 * values each, or NULL for unbounded) are bounds the fit keeps to, narrowed
 * by every term's own bounds through its map (and mu >= 0 of a binned term).
 * Host only; device memory is taken at the first evaluation.
 * rf_sum_add_program / rf_sum_add_binned: map (host, the term's n_params
 * values, resp. 1 + J for (mu, alpha_1..alpha_J)) gives each of the term's
 * parameters its global index; RF_E_INVALID for an index outside
 * [0, n_params), a term already in this sum (its device result block is
 * reused by every evaluation), or more than 16 terms.  The sum refers to the
 * term and does not own it: the term must outlive the sum's use.
 * rf_sum_add_constraint: a Gaussian factor on theta[k] (width > 0, mean
 * finite); at most 64.
 * rf_sum_nll_grad: synchronous on `stream` (host result): each term's
 * evaluation is enqueued on the stream, then one combining kernel adds the
 * NLLs in term order, gathers each global parameter's gradient entries in
 * term order and adds the constraints, all in FP64 (results repeat bit for
 * bit).  Status as rf_nll_grad: RF_E_DOMAIN when a term's parameters are out
 * of its bounds (nothing is launched), RF_E_NONFINITE with nll = +inf and
 * grad NaN when a term has events with p <= 0 or a non-finite NLL; n_bad (may
 * be NULL) is the terms' total of such events.  Terms must not be evaluated
 * elsewhere while a sum's evaluation is in flight.
 * rf_sum_fit_bfgs: rf_fit_bfgs_ex's minimiser on the combined NLL (initial
 * inverse Hessian from forward differences, uncertainties from central
 * differences of the gradient); same outputs. */
typedef struct rf_sum rf_sum;
int rf_sum_new(int32_t n_params, const double* lo, const double* hi, rf_sum** out);
void rf_sum_free(rf_sum* s);
int rf_sum_add_program(rf_sum* s, rf_program* p, const int32_t* map);
int rf_sum_add_binned(rf_sum* s, rf_binned* b, const int32_t* map);
int rf_sum_add_constraint(rf_sum* s, int32_t k, double mean, double width);
int rf_sum_nll_grad(rf_sum* s, const double* theta, double* nll, double* grad, int64_t* n_bad,
                    void* stream);
int rf_sum_fit_bfgs(rf_sum* s, const double* theta0, double edm_tol, int32_t max_iter,
                    double* theta_out, double* sigma_out, double* cov_out, double* info_out,
                    void* stream);

/* ---- MLP kernels used to train the surrogate ------------------------------- */
/* Not in the paper: the learned surrogate of the numerically convolved signal
 * of the benchmark workload (its expensive PDF), trained by these kernels on
 * the exact convolution's own values. */
/* 6-64-64-64-1 tanh network, BF16 weights (layout as rf_bind_weights), FP32
 * inputs in [-1,1] (n x 6 row-major), FP32 accumulation.
 * rf_mlp_forward: out[n]; act (n x 192 FP32, may be NULL) keeps the hidden
 * activations for rf_mlp_backward. */
int rf_mlp_forward(const void* dev_w_bf16, const float* dev_in, int64_t n, float* dev_out,
                   float* dev_act, void* stream);
/* dout[n] cotangents -> dw[8833] FP32 (overwritten with the sum over rows),
 * din (n x 6, may be NULL) input gradients.  The per-workgroup partial
 * gradients live in a library-owned workspace per (device, stream), grown on
 * demand and kept until the process ends, which rf_mlp_backward and
 * rf_mlp_train_step calls on that stream share in stream order; calls on
 * different streams use different workspaces. */
int rf_mlp_backward(const void* dev_w_bf16, const float* dev_in, const float* dev_act,
                    const float* dev_dout, int64_t n, float* dev_dw, float* dev_din,
                    void* stream);
/* one Adam step on FP32 master weights w32 (n values) with moments m, v;
 * writes the BF16 copy (round to nearest even) used by the kernels. */
int rf_adam_step(float* dev_w32, void* dev_w_bf16, float* dev_m, float* dev_v,
                 const float* dev_g, int64_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, void* stream);

/* dout[i] = scale * (out[i] - target[i])  (gradient of a mean-squared error) */
int rf_mse_grad(const float* dev_out, const float* dev_target, int64_t n, float scale, float* dev_dout,
                void* stream);
/* One optimiser step of the surrogate's training, as rf_mlp_forward +
 * rf_mse_grad (scale 2/batch) + rf_mlp_backward + rf_adam_step on a batch of
 * rows, in two kernel launches.  Batch row r is row dev_idx[r] of dev_in
 * (n_rows x 6) and dev_target (n_rows; dev_idx NULL: rows 0..batch-1, and
 * n_rows >= batch).  An index outside [0, n_rows) is the caller's error: the
 * kernel clamps it into the arrays (no read leaves them); with
 * flags & RF_VALIDATE the indices are first checked on the host (the stream is
 * synchronised) and RF_E_INVALID returned if any is out of range.  The loss is
 * the mean of (s - target)^2 over the batch.  dev_w_bf16 (read by the step,
 * then refreshed), dev_w32, dev_m, dev_v are updated in place; dev_dw (8833
 * FP32, may be NULL) receives the summed gradient.  Asynchronous on the
 * stream; uses rf_mlp_backward's workspace of that stream. */
int rf_mlp_train_step(void* dev_w_bf16, float* dev_w32, float* dev_m, float* dev_v, const float* dev_in,
                      const float* dev_target, const int64_t* dev_idx, int64_t batch, int64_t n_rows,
                      uint32_t flags, float lr, float beta1, float beta2, float eps, int32_t step, float* dev_dw,
                      void* stream);
/* Exact log p_sig of the Breit-Wigner (x) Crystal Ball signal at per-sample
 * parameters: dev_xq[n][6] = (x, M, Gamma, sigma, alpha, n) FP64; the same
 * K-point Gauss-Legendre rule on [ylo, yhi] and normalisation over [lo, hi]
 * as RF_OP_NUMCONV_BW_CB; dev_out[n] FP64.  The surrogate's training targets. */
int rf_bwcb_logpdf(const double* dev_xq, int64_t n, int32_t K, double ylo, double yhi, double lo, double hi,
                   double* dev_out, void* stream);

/* The surrogate's training targets: log p_sig - log b at the rows of dev_xq
 * (as rf_bwcb_logpdf), b the surrogate leaf's analytic base evaluated exactly
 * as the leaf evaluates it (RF_OP_MLP: its FP64 parameter-only constants and
 * its FP32 value), so the network learns the residual the leaf adds to it;
 * dev_out[n] FP32. */
int rf_mlp_targets(const double* dev_xq, int64_t n, int32_t K, double ylo, double yhi, double lo, double hi,
                   float* dev_out, void* stream);

/* ---- measurement ------------------------------------------------------------ */
/* Microbenchmark of the ceilings the likelihood kernels are measured against,
 * on the current device: kind 0 FP32 FMA, 1 FP64 FMA, 2 FP32 exp2 (lane
 * operations/s); 3 the 1-D kernel's mix of 14 FP32 FMA per transcendental,
 * 4 the convolution's 12 FMA per reciprocal (lane-slots/s, a transcendental
 * counting 4); 5 FP64 exp, 6 FP64 log, 7 FP64 reciprocal with one Newton step
 * (lane calls/s); 8 streaming read of stream_bytes (0: 1 GiB) with 16-byte
 * loads (bytes/s); 9 the FP64 logarithm of the event loop (lane calls/s).
 * iters: loop iterations per lane (ignored for kind 8).
 * Synchronous; allocates and frees its own buffers. */
int rf_peak(int32_t kind, int32_t iters, int64_t stream_bytes, double* rate, double* seconds);
/* The library's own device math functions applied element by element to
 * dev_in[n] (FP64) into dev_out[n], for comparison with a host library:
 * fn 0 = the natural logarithm of the FP64 event loop (positive, finite,
 * normal arguments); fn 1 = the Gaussian's 2^t of the FP64 event loop
 * (t <= 0; 0 below 2^-1100).  Asynchronous on the stream. */
int rf_eval_math(int32_t fn, const double* dev_in, int64_t n, double* dev_out, void* stream);

/* ---- host utility ---------------------------------------------------------- */
/* (the fixed rule of the numerically convolved signal) */
/* K-point Gauss-Legendre nodes and weights on [lo, hi] (ascending) */
int rf_gauss_legendre(int32_t K, double lo, double hi, double* x, double* w);

#ifdef __cplusplus
}
#endif
#endif
