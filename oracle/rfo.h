/*
 * rfo.h -- the oracle: a plain, slow, scalar FP64 CPU evaluator of a
 * likelihood model graph (Hageboeck & Moneta, "Making RooFit Ready for
 * Run 3", ACAT 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  It shares no source,
 * header, table or helper with the GPU library; it is the judge of that
 * library's results, never a fallback for it.
 *
 * What it computes follows the paper's description of RooFit's scalar
 * evaluation (Section 4): load one event into the observable leaves,
 * evaluate the top PDF node, accumulate -log p, with parameter-only
 * branches (normalisation integrals) computed once per parameter point
 * (the node-value caching of Section 4).  Gradients are propagated in
 * forward mode through every node (value plus a dense d/dtheta vector).
 *
 * Conventions
 *   - Nodes are appended in dependency order; an input id must refer to an
 *     earlier node.  Parameter index = declaration order of PARAM nodes.
 *     Column index = declaration order of OBS nodes.
 *   - Every return code is 0 on success, negative on error; a static
 *     message is available from rfo_last_error().
 *   - The oracle is single threaded and not re-entrant per model.
 */
#ifndef RFO_H
#define RFO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* node kinds (the oracle's own numbering) */
enum {
  RFO_OBS = 1, RFO_PARAM = 2, RFO_CONST = 3,
  RFO_FN_LINEAR = 4,  /* attrs[0] + sum_j attrs[j+1]*in_j          */
  RFO_FN_PRODUCT = 5, /* prod_j in_j                                */
  RFO_FN_RATIO = 6,   /* in_0 / in_1                                */
  RFO_GAUSS = 10,     /* in: x, mu, sigma                           */
  RFO_CHEB = 11,      /* in: x, c1..cn  (T0 coefficient fixed to 1) */
  RFO_EXP = 12,       /* in: x, k ; attrs[0]=0: exp(-x/k), 1: exp(k*x) */
  RFO_DECAY_GAUSS = 13, /* in: t, tau, sigma, bias                  */
  RFO_ARGUS = 14,     /* in: m, m0 (constant), c                    */
  RFO_BW = 15,        /* in: x, M, Gamma                            */
  RFO_NUMCONV_BW_CB = 16, /* in: x, M, Gamma, sigma, alpha, n ;
                             attrs: ylo, yhi, K                      */
  RFO_MLP = 17,       /* in: x, q1..q5 ; attrs: 12 box bounds (lo,hi per
                         input; the first box is that of x - q1), K (grid
                         points on x's range)                        */
  RFO_POISSON = 18,   /* in: n, lambda: lambda^n e^-lambda / n! on the integers
                         of the observable's range [lo, hi] */
  RFO_ADD = 30,       /* in: pdf_1..pdf_n, f_1..f_{n-1}             */
  RFO_PROD = 31,      /* in: pdf_1..pdf_n (disjoint observables)    */
  RFO_EXTENDED = 32   /* in: pdf, nu; only as the top of an NLL: the
                         extended likelihood -sum_i w_i log p_i + nu - N log nu
                         with N = sum_i w_i (the event count unweighted);
                         values are pdf's */
};

const char* rfo_last_error(void);

typedef struct rfo_model rfo_model;
rfo_model* rfo_model_new(void);
void rfo_model_free(rfo_model* m);
/* returns the node id (>= 0) or a negative error */
int rfo_node(rfo_model* m, int kind, const int* in, int n_in,
             const double* attrs, int n_attrs);
int rfo_n_params(const rfo_model* m);
int rfo_n_obs(const rfo_model* m);
/* MLP weights for an RFO_MLP node: 8833 doubles, layout W1[64][6] b1[64]
   W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4[1] (row = output unit) */
int rfo_set_mlp_weights(rfo_model* m, int node, const double* w);

/* NLL (and optionally gradient) over n events; cols[j] = column of OBS j.
   nll: Neumaier-compensated sum of -log p_i.  n_bad counts events with
   p_i <= 0 or non-finite p_i (then nll = +inf). grad may be NULL. */
int rfo_nll(rfo_model* m, int top, const double* theta,
            const double* const* cols, int64_t n,
            double* nll, double* grad, int64_t* n_bad);
/* as rfo_nll, plus gabs[k] = sum_i |d(-log p_i)/d theta_k| (the scale of the
   gradient's cancellation; may be NULL) */
int rfo_nll_ex(rfo_model* m, int top, const double* theta,
               const double* const* cols, int64_t n,
               double* nll, double* grad, double* gabs, int64_t* n_bad);
/* as rfo_nll_ex for weighted events: -sum_i w_i log p_i and its gradient,
   gabs[k] = sum_i |w_i d(log p_i)/d theta_k|; w = NULL means every w_i = 1 */
int rfo_nll_w(rfo_model* m, int top, const double* theta,
              const double* const* cols, const double* w, int64_t n,
              double* nll, double* grad, double* gabs, int64_t* n_bad);
/* per-event normalised PDF values */
/* The NLL (weights w may be NULL), its gradient and its Hessian
 * hess[P][P] (row-major) at theta, by second-order forward mode through every
 * node; analytic leaves only (no convolution or MLP leaf), at most 16
 * parameters. */
int rfo_nll_hess(rfo_model* m, int top, const double* theta, const double* const* cols, const double* w,
                 int64_t n, double* nll, double* grad, double* hess, int64_t* n_bad);
int rfo_values(rfo_model* m, int top, const double* theta,
               const double* const* cols, int64_t n, double* out);
/* normalisation integral of a PDF leaf and its d/dtheta (n_params) */
int rfo_norm(rfo_model* m, int node, const double* theta,
             double* N, double* dN);

/* Gauss-Legendre rule of order K on [lo,hi] (Newton on P_K, long double) */
int rfo_gauss_legendre(int K, double lo, double hi, double* x, double* w);

/* 6 -> 64 -> 64 -> 64 -> 1 tanh MLP in FP64 (layout as above) */
int rfo_mlp_forward(const double* w, const double* in, int64_t n, double* out);
/* dout: dL/dout per row; dw += dL/dw (8833, accumulated), din (n x 6) may
   be NULL */
int rfo_mlp_backward(const double* w, const double* in, int64_t n,
                     const double* dout, double* dw, double* din);

/* Binned template likelihood (HistFactory-like, Section 3): C channels,
   S samples (sample 0 is scaled by mu), B bins, J nuisance parameters.
   T[c][s][b], Lp/Lm[c][s][j][b] = log(T+/T), log(T-/T), nobs[c][b].
   theta = (mu, alpha_1..alpha_J).  nll excludes sum lgamma(n+1). */
int rfo_binned_nll(int C, int S, int B, int J, const double* T,
                   const double* Lp, const double* Lm, const double* nobs,
                   const double* theta, double* nll, double* grad);

#ifdef __cplusplus
}
#endif
#endif
