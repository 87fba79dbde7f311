/*
 * rfo.c -- the oracle: scalar FP64 CPU evaluator of a likelihood model graph.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  Shares no code
 * with the GPU library.
 *
 * Reading of the paper (Section 4, "Batched likelihood computations"): a
 * likelihood is the probability of every event; RooFit loads one event into
 * the observable leaves and evaluates the top PDF, with branches that depend
 * only on parameters cached and computed once per parameter point.  This
 * file does exactly that, one event at a time, in FP64, and carries a dense
 * gradient vector through every node (forward mode).  NLL = -sum_i log p_i;
 * every sum uses Neumaier compensation.
 *
 * The PDFs are the textbook definitions of the shapes the paper names
 * (Gaussian, exponential, sum of PDFs and their normalisation, Section 4.1
 * and 4.2) plus the shapes of the benchmark workloads (Chebyshev polynomial,
 * decay (x) Gaussian resolution, ARGUS, Breit-Wigner, Breit-Wigner (x) Crystal
 * Ball by a fixed Gauss-Legendre rule, an MLP surrogate); each normalisation
 * is the integral over the observable's range [lo, hi].
 */
#include "rfo.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXN 64
#define MAXIN 16
#define MAXA 16
#define MAXP 64
#define NMLP 8833

static const char* g_err = "";
const char* rfo_last_error(void) { return g_err; }
#define FAIL(code, msg) do { g_err = (msg); return (code); } while (0)

/* ---- compensated (Neumaier) summation ---------------------------------- */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ---- model --------------------------------------------------------------- */
typedef struct {
  int kind, n_in, n_attrs;
  int in[MAXIN];
  double attrs[MAXA];
  int index;         /* PARAM: theta index; OBS: column index */
  double lo, hi;     /* OBS range */
  /* per-call caches for PDF leaves */
  double N, dN[MAXP];
  /* NUMCONV: y rule and per-call node table */
  int K;
  double *gy, *gw, *ck, *dck, *Ik;
  /* MLP: weights and x grid */
  double *mw, *mgx, *mgw;
} node;

struct rfo_model {
  int n, np, nobs;
  node nd[MAXN];
  /* per-call parameter-level values and gradients */
  double pv[MAXN];
  double pg[MAXN][MAXP];
};

rfo_model* rfo_model_new(void) {
  rfo_model* m = (rfo_model*)calloc(1, sizeof(rfo_model));
  return m;
}
void rfo_model_free(rfo_model* m) {
  if (!m) return;
  for (int i = 0; i < m->n; ++i) {
    node* d = &m->nd[i];
    free(d->gy); free(d->gw); free(d->ck); free(d->dck); free(d->Ik);
    free(d->mw); free(d->mgx); free(d->mgw);
  }
  free(m);
}
int rfo_n_params(const rfo_model* m) { return m->np; }
int rfo_n_obs(const rfo_model* m) { return m->nobs; }

static int is_pdf(int k) { return k >= RFO_GAUSS && k != RFO_EXTENDED; }
static int is_paramlike(int k) {
  return k == RFO_PARAM || k == RFO_CONST || k == RFO_FN_LINEAR || k == RFO_FN_PRODUCT || k == RFO_FN_RATIO;
}

/* ---- Gauss-Legendre nodes: Newton iteration on P_K in long double ------ */
int rfo_gauss_legendre(int K, double lo, double hi, double* x, double* w) {
  if (K < 1) FAIL(-1, "K < 1");
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < K; ++i) {
    long double z = cosl(pi * ((long double)i + 0.75L) / ((long double)K + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int j = 1; j < K; ++j) {
        long double p2 = ((2 * j + 1) * z * p1 - j * p0) / (j + 1);
        p0 = p1; p1 = p2;
      }
      /* p1 = P_K(z), p0 = P_{K-1}(z) */
      dp = K * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) {
        /* refresh derivative at the converged root */
        p0 = 1; p1 = z;
        for (int j = 1; j < K; ++j) {
          long double p2 = ((2 * j + 1) * z * p1 - j * p0) / (j + 1);
          p0 = p1; p1 = p2;
        }
        dp = K * (z * p1 - p0) / (z * z - 1);
        break;
      }
    }
    long double wi = 2.0L / ((1 - z * z) * dp * dp);
    /* ascending order */
    x[K - 1 - i] = (double)(0.5L * (hi - lo) * z + 0.5L * (hi + lo));
    w[K - 1 - i] = (double)(0.5L * (hi - lo) * wi);
  }
  return 0;
}

int rfo_node(rfo_model* m, int kind, const int* in, int n_in,
             const double* attrs, int n_attrs) {
  if (m->n >= MAXN) FAIL(-1, "too many nodes");
  if (n_in < 0 || n_in > MAXIN || n_attrs < 0 || n_attrs > MAXA) FAIL(-1, "arity");
  for (int j = 0; j < n_in; ++j)
    if (in[j] < 0 || in[j] >= m->n) FAIL(-1, "input id");
  node* d = &m->nd[m->n];
  memset(d, 0, sizeof(*d));
  d->kind = kind; d->n_in = n_in; d->n_attrs = n_attrs;
  for (int j = 0; j < n_in; ++j) d->in[j] = in[j];
  for (int j = 0; j < n_attrs; ++j) d->attrs[j] = attrs[j];
  switch (kind) {
    case RFO_OBS:
      if (n_attrs != 2) FAIL(-1, "OBS needs lo, hi");
      d->lo = attrs[0]; d->hi = attrs[1]; d->index = m->nobs++;
      break;
    case RFO_PARAM:
      if (m->np >= MAXP) FAIL(-1, "too many parameters");
      d->index = m->np++;
      break;
    case RFO_CONST:
      if (n_attrs != 1) FAIL(-1, "CONST needs a value");
      break;
    case RFO_FN_LINEAR:
      if (n_attrs != n_in + 1) FAIL(-1, "LINEAR attrs");
      break;
    case RFO_FN_PRODUCT:
      break;
    case RFO_FN_RATIO:
    case RFO_EXTENDED:
      if (n_in != 2) FAIL(-1, "RATIO and EXTENDED take two inputs");
      break;
    case RFO_NUMCONV_BW_CB: {
      if (n_in != 6 || n_attrs != 3) FAIL(-1, "NUMCONV arity");
      int K = (int)attrs[2];
      d->K = K;
      d->gy = malloc(sizeof(double) * K); d->gw = malloc(sizeof(double) * K);
      d->ck = malloc(sizeof(double) * K); d->dck = malloc(sizeof(double) * 3 * K);
      d->Ik = malloc(sizeof(double) * K);
      rfo_gauss_legendre(K, attrs[0], attrs[1], d->gy, d->gw);
      break;
    }
    case RFO_MLP: {
      if (n_in != 6 || n_attrs != 13) FAIL(-1, "MLP arity");
      int K = (int)attrs[12];
      d->K = K;
      d->mgx = malloc(sizeof(double) * K); d->mgw = malloc(sizeof(double) * K);
      const node* ob = &m->nd[in[0]];
      rfo_gauss_legendre(K, ob->lo, ob->hi, d->mgx, d->mgw);
      break;
    }
    default: break;
  }
  if (is_pdf(kind) && kind != RFO_ADD && kind != RFO_PROD) {
    if (n_in < 1 || m->nd[in[0]].kind != RFO_OBS) FAIL(-1, "leaf input 0 must be an observable");
  }
  return m->n++;
}

int rfo_set_mlp_weights(rfo_model* m, int id, const double* w) {
  if (id < 0 || id >= m->n || m->nd[id].kind != RFO_MLP) FAIL(-1, "not an MLP node");
  node* d = &m->nd[id];
  if (!d->mw) d->mw = malloc(sizeof(double) * NMLP);
  memcpy(d->mw, w, sizeof(double) * NMLP);
  return 0;
}

/* ---- MLP (6-64-64-64-1, tanh) -------------------------------------------- */
enum { OW1 = 0, OB1 = 384, OW2 = 448, OB2 = 4544, OW3 = 4608, OB3 = 8704, OW4 = 8768, OB4 = 8832 };

typedef struct { double h1[64], h2[64], h3[64], s; } mlp_act;

static void mlp_fwd1(const double* w, const double* u, mlp_act* a) {
  for (int o = 0; o < 64; ++o) {
    double z = w[OB1 + o];
    for (int i = 0; i < 6; ++i) z += w[OW1 + o * 6 + i] * u[i];
    a->h1[o] = tanh(z);
  }
  for (int o = 0; o < 64; ++o) {
    double z = w[OB2 + o];
    for (int i = 0; i < 64; ++i) z += w[OW2 + o * 64 + i] * a->h1[i];
    a->h2[o] = tanh(z);
  }
  for (int o = 0; o < 64; ++o) {
    double z = w[OB3 + o];
    for (int i = 0; i < 64; ++i) z += w[OW3 + o * 64 + i] * a->h2[i];
    a->h3[o] = tanh(z);
  }
  double s = w[OB4];
  for (int i = 0; i < 64; ++i) s += w[OW4 + i] * a->h3[i];
  a->s = s;
}

/* backprop of a scalar cotangent g through one row: accumulates weight
   gradients into dw (if non-NULL) and writes d/du into du (if non-NULL) */
static void mlp_bwd1(const double* w, const double* u, const mlp_act* a, double g,
                     double* dw, double* du) {
  double d3[64], d2[64], d1[64];
  for (int o = 0; o < 64; ++o) d3[o] = g * w[OW4 + o] * (1 - a->h3[o] * a->h3[o]);
  for (int i = 0; i < 64; ++i) {
    double s = 0;
    for (int o = 0; o < 64; ++o) s += w[OW3 + o * 64 + i] * d3[o];
    d2[i] = s * (1 - a->h2[i] * a->h2[i]);
  }
  for (int i = 0; i < 64; ++i) {
    double s = 0;
    for (int o = 0; o < 64; ++o) s += w[OW2 + o * 64 + i] * d2[o];
    d1[i] = s * (1 - a->h1[i] * a->h1[i]);
  }
  if (du) {
    for (int i = 0; i < 6; ++i) {
      double s = 0;
      for (int o = 0; o < 64; ++o) s += w[OW1 + o * 6 + i] * d1[o];
      du[i] = s;
    }
  }
  if (dw) {
    dw[OB4] += g;
    for (int i = 0; i < 64; ++i) dw[OW4 + i] += g * a->h3[i];
    for (int o = 0; o < 64; ++o) {
      dw[OB3 + o] += d3[o];
      for (int i = 0; i < 64; ++i) dw[OW3 + o * 64 + i] += d3[o] * a->h2[i];
      dw[OB2 + o] += d2[o];
      for (int i = 0; i < 64; ++i) dw[OW2 + o * 64 + i] += d2[o] * a->h1[i];
      dw[OB1 + o] += d1[o];
      for (int i = 0; i < 6; ++i) dw[OW1 + o * 6 + i] += d1[o] * u[i];
    }
  }
}

int rfo_mlp_forward(const double* w, const double* in, int64_t n, double* out) {
  mlp_act a;
  for (int64_t r = 0; r < n; ++r) { mlp_fwd1(w, in + 6 * r, &a); out[r] = a.s; }
  return 0;
}

int rfo_mlp_backward(const double* w, const double* in, int64_t n,
                     const double* dout, double* dw, double* din) {
  mlp_act a;
  for (int64_t r = 0; r < n; ++r) {
    mlp_fwd1(w, in + 6 * r, &a);
    mlp_bwd1(w, in + 6 * r, &a, dout[r], dw, din ? din + 6 * r : NULL);
  }
  return 0;
}

/* ---- analytic base of the surrogate ----------------------------------------
   The surrogate's log density is s = MLP(u) + log b, with the analytic base
   b(d = x - M; Gamma, sigma, alpha, n) a pseudo-Voigt (Thompson, Cox &
   Hastings, J. Appl. Cryst. 20 (1987) 79: a Lorentzian and a Gaussian of
   common full width f, mixed with weight eta; f_G = 2 sigma sqrt(2 ln 2),
   f_L = Gamma) whose Gaussian part carries the Crystal Ball tail below
   z = -alpha, z in units of that component's width f / (2 sqrt(2 ln 2)).
   Evaluated here with forward-mode dual numbers (value and the derivatives
   with respect to (d, Gamma, sigma, alpha, n)), straight from the
   definition. */
static const double SQRT2PI_ = 2.50662827463100050242;
typedef struct { double v, g[5]; } dual;
static dual dl_c(double v) { dual r = {v, {0, 0, 0, 0, 0}}; return r; }
static dual dl_var(double v, int i) { dual r = dl_c(v); r.g[i] = 1.0; return r; }
static dual dl_add(dual a, dual b) { for (int i = 0; i < 5; ++i) a.g[i] += b.g[i]; a.v += b.v; return a; }
static dual dl_sub(dual a, dual b) { for (int i = 0; i < 5; ++i) a.g[i] -= b.g[i]; a.v -= b.v; return a; }
static dual dl_mul(dual a, dual b) {
  dual r; r.v = a.v * b.v;
  for (int i = 0; i < 5; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
  return r;
}
static dual dl_div(dual a, dual b) {
  dual r; r.v = a.v / b.v;
  for (int i = 0; i < 5; ++i) r.g[i] = (a.g[i] * b.v - a.v * b.g[i]) / (b.v * b.v);
  return r;
}
static dual dl_scale(dual a, double c) { a.v *= c; for (int i = 0; i < 5; ++i) a.g[i] *= c; return a; }
static dual dl_exp(dual a) { dual r; r.v = exp(a.v); for (int i = 0; i < 5; ++i) r.g[i] = r.v * a.g[i]; return r; }
static dual dl_log(dual a) { dual r; r.v = log(a.v); for (int i = 0; i < 5; ++i) r.g[i] = a.g[i] / a.v; return r; }
static dual dl_powi(dual a, int k) { dual r = dl_c(1.0); for (int i = 0; i < k; ++i) r = dl_mul(r, a); return r; }

/* log b and its derivatives with respect to (d, Gamma, sigma, alpha, n) */
static dual mlp_base_log(double dx, double G, double sg, double al, double n) {
  const double c0 = 2.0 * sqrt(2.0 * log(2.0));
  const double PI = 3.14159265358979323846;
  dual d = dl_var(dx, 0), fl = dl_var(G, 1), s = dl_var(sg, 2), a = dl_var(al, 3), nn = dl_var(n, 4);
  dual fg = dl_scale(s, c0);
  dual P = dl_powi(fg, 5);
  P = dl_add(P, dl_scale(dl_mul(dl_powi(fg, 4), fl), 2.69269));
  P = dl_add(P, dl_scale(dl_mul(dl_powi(fg, 3), dl_powi(fl, 2)), 2.42843));
  P = dl_add(P, dl_scale(dl_mul(dl_powi(fg, 2), dl_powi(fl, 3)), 4.47163));
  P = dl_add(P, dl_scale(dl_mul(fg, dl_powi(fl, 4)), 0.07842));
  P = dl_add(P, dl_powi(fl, 5));
  dual f = dl_exp(dl_scale(dl_log(P), 0.2));
  dual r = dl_div(fl, f);
  dual eta = dl_add(dl_sub(dl_scale(r, 1.36603), dl_scale(dl_powi(r, 2), 0.47719)), dl_scale(dl_powi(r, 3), 0.11116));
  dual h = dl_scale(f, 0.5);
  dual L = dl_div(dl_scale(h, 1.0 / PI), dl_add(dl_mul(d, d), dl_mul(h, h)));
  dual se = dl_scale(f, 1.0 / c0);
  dual z = dl_div(d, se);
  dual C;
  if (z.v > -al) {
    C = dl_exp(dl_scale(dl_mul(z, z), -0.5));
  } else {
    /* A (B - z)^-n, A = (n/alpha)^n exp(-alpha^2/2), B = n/alpha - alpha */
    dual logA = dl_sub(dl_mul(nn, dl_log(dl_div(nn, a))), dl_scale(dl_mul(a, a), 0.5));
    dual B = dl_sub(dl_div(nn, a), a);
    C = dl_exp(dl_sub(logA, dl_mul(nn, dl_log(dl_sub(B, z)))));
  }
  dual Gn = dl_div(C, dl_scale(se, SQRT2PI_));
  dual pv = dl_add(dl_mul(eta, L), dl_mul(dl_sub(dl_c(1.0), eta), Gn));
  return dl_log(pv);
}

/* MLP surrogate.  Inputs: u0 = affine map of (x - q1) onto [-1, 1] (the
   position relative to the first shape parameter, the Breit-Wigner mass),
   u_j = affine map of q_j (j = 1..5), each with its (lo, hi) box.  Returns
   s = MLP(u) + log b and d s / d(raw input j), raw = (x, q1..q5). */
static double mlp_leaf(const node* d, const double* raw, double* ds /*6*/) {
  double u[6], du[6], sc[6];
  for (int j = 0; j < 6; ++j) {
    double lo = d->attrs[2 * j], hi = d->attrs[2 * j + 1];
    double r = j == 0 ? raw[0] - raw[1] : raw[j];
    sc[j] = 2.0 / (hi - lo);
    u[j] = (r - lo) * sc[j] - 1.0;
  }
  mlp_act a;
  mlp_fwd1(d->mw, u, &a);
  const dual lb = mlp_base_log(raw[0] - raw[1], raw[2], raw[3], raw[4], raw[5]);
  if (ds) {
    mlp_bwd1(d->mw, u, &a, 1.0, NULL, du);
    for (int j = 0; j < 6; ++j) ds[j] = du[j] * sc[j];
    ds[1] -= du[0] * sc[0];
    ds[0] += lb.g[0];
    ds[1] -= lb.g[0];
    for (int j = 1; j < 5; ++j) ds[j + 1] += lb.g[j];
  }
  return a.s + lb.v;
}

/* ---- shapes ---------------------------------------------------------------- */
static const double SQRT2 = 1.41421356237309504880;
static const double SQRTPI = 1.77245385090551602730;
static const double SQRT2PI = 2.50662827463100050242;

/* Crystal Ball (mean 0, low-side power-law tail) and d/d(sigma, alpha, n) */
static double cb_val(double y, double s, double al, double n, double* d) {
  double z = y / s;
  if (z > -al) {
    double v = exp(-0.5 * z * z);
    if (d) { d[0] = v * z * z / s; d[1] = 0; d[2] = 0; }
    return v;
  }
  double A = pow(n / al, n) * exp(-0.5 * al * al);
  double B = n / al - al;
  double r = B - z;
  double v = A * pow(r, -n);
  if (d) {
    d[0] = v * (-n * (z / s) / r);
    d[1] = v * (-n / al - al + n * (n / (al * al) + 1.0) / r);
    d[2] = v * (log(n / al) + 1.0 - log(r) - n / (al * r));
  }
  return v;
}

/* decay (x) Gaussian resolution: F(t) and dF/d(tau, s, b) */
static double decay_F(double t, double tau, double s, double b, double* d) {
  double u = t - b;
  double E = exp(s * s / (2 * tau * tau) - u / tau);
  double w = (s * s / tau - u) / (SQRT2 * s);
  double F = 0.5 * E * erfc(w);
  if (d) {
    double G = exp(-u * u / (2 * s * s));
    d[0] = F * (u / (tau * tau) - s * s / (tau * tau * tau)) + s * G / (SQRT2PI * tau * tau);
    d[1] = F * s / (tau * tau) - G * (1.0 / tau + u / (s * s)) / SQRT2PI;
    d[2] = F / tau - G / (SQRT2PI * s);
  }
  return F;
}
/* antiderivative A(t) = tau*(Phi(u/s) - F(t)) and dA/d(tau, s, b) */
static double decay_A(double t, double tau, double s, double b, double* d) {
  double dF[3];
  double u = t - b;
  double F = decay_F(t, tau, s, b, dF);
  double Phi = 0.5 * erfc(-u / (SQRT2 * s));
  double G = exp(-u * u / (2 * s * s));
  if (d) {
    d[0] = Phi - F - tau * dF[0];
    d[1] = tau * (-u * G / (SQRT2PI * s * s) - dF[1]);
    d[2] = tau * (-G / (SQRT2PI * s) - dF[2]);
  }
  return tau * (Phi - F);
}

/* ARGUS helper integrals for c = -k <= 0:
   J(U)  = int_0^U v^(1/2) e^{-k v} dv ,  J3(U) = int_0^U v^(3/2) e^{-k v} dv */
static void argus_J(double U, double k, double* J, double* J3) {
  if (U <= 0) { *J = 0; *J3 = 0; return; }
  if (k * U < 1e-3) {
    /* power series in (k U); the closed form cancels badly here */
    double sJ = 0, sJ3 = 0, term = 1;
    for (int nn = 0; nn < 30; ++nn) {
      sJ += term * pow(U, nn + 1.5) / (nn + 1.5);
      sJ3 += term * pow(U, nn + 2.5) / (nn + 2.5);
      term *= -k / (nn + 1);
    }
    *J = sJ; *J3 = sJ3; return;
  }
  double sq = sqrt(k * U);
  *J = SQRTPI / (2 * k * sqrt(k)) * erf(sq) - sqrt(U) * exp(-k * U) / k;
  *J3 = 1.5 / k * (*J) - U * sqrt(U) * exp(-k * U) / k;
}

/* unnormalised value u(x) of a leaf and du/d(input j), j = 1..n_in-1 stored at
   du[j-1] (input 0 is the observable).  v[] holds the input values. */
static double leaf_value(const node* d, double x, const double* v, double* du) {
  switch (d->kind) {
    case RFO_GAUSS: {
      double mu = v[1], s = v[2], z = (x - mu) / s;
      double g = exp(-0.5 * z * z);
      du[0] = g * z / s; du[1] = g * z * z / s;
      return g;
    }
    case RFO_CHEB: {
      /* x' in [-1, 1]; T_0 = 1, T_1 = x', T_{k+1} = 2 x' T_k - T_{k-1} */
      double lo = d->lo, hi = d->hi;
      double xp = (2 * x - lo - hi) / (hi - lo);
      double tkm = 1, tk = xp, h = 1;
      for (int j = 1; j < d->n_in; ++j) {
        h += v[j] * tk; du[j - 1] = tk;
        double tn = 2 * xp * tk - tkm; tkm = tk; tk = tn;
      }
      return h;
    }
    case RFO_EXP: {
      double k = v[1];
      if ((int)d->attrs[0] == 0) { double e = exp(-x / k); du[0] = e * x / (k * k); return e; }
      double e = exp(k * x); du[0] = e * x; return e;
    }
    case RFO_DECAY_GAUSS: {
      double dF[3];
      double F = decay_F(x, v[1], v[2], v[3], dF);
      du[0] = dF[0]; du[1] = dF[1]; du[2] = dF[2];
      return F;
    }
    case RFO_ARGUS: {
      double m0 = v[1], c = v[2];
      if (x >= m0) { du[0] = 0; du[1] = 0; return 0.0; }
      double U = (m0 - x) * (m0 + x) / (m0 * m0);
      double a = x * sqrt(U) * exp(c * U);
      du[0] = 0; /* m0 is a constant (checked in the normalisation) */
      du[1] = a * U;
      return a;
    }
    case RFO_BW: {
      double M = v[1], G = v[2], q = x - M;
      double b = 1.0 / (q * q + 0.25 * G * G);
      du[0] = 2 * q * b * b; du[1] = -0.5 * G * b * b;
      return b;
    }
    case RFO_POISSON: { /* the probability mass lambda^n e^-lambda / n! */
      double lam = v[1];
      double u = exp(x * log(lam) - lam - lgamma(x + 1.0));
      du[0] = u * (x / lam - 1.0);
      return u;
    }
    case RFO_NUMCONV_BW_CB: {
      double M = v[1], G = v[2];
      nsum S = {0, 0}, dM = {0, 0}, dG = {0, 0}, ds = {0, 0}, da = {0, 0}, dn = {0, 0};
      for (int k = 0; k < d->K; ++k) {
        double q = x - d->gy[k] - M;
        double b = 1.0 / (q * q + 0.25 * G * G);
        nadd(&S, d->ck[k] * b);
        nadd(&dM, d->ck[k] * 2 * q * b * b);
        nadd(&dG, -d->ck[k] * 0.5 * G * b * b);
        nadd(&ds, d->dck[3 * k + 0] * b);
        nadd(&da, d->dck[3 * k + 1] * b);
        nadd(&dn, d->dck[3 * k + 2] * b);
      }
      du[0] = nval(&dM); du[1] = nval(&dG); du[2] = nval(&ds); du[3] = nval(&da); du[4] = nval(&dn);
      return nval(&S);
    }
    case RFO_MLP: {
      double raw[6], ds[6];
      raw[0] = x;
      for (int j = 1; j < 6; ++j) raw[j] = v[j];
      double s = mlp_leaf(d, raw, ds);
      double e = exp(s);
      for (int j = 1; j < 6; ++j) du[j - 1] = e * ds[j];
      return e;
    }
  }
  return NAN;
}

/* normalisation N over the observable range and dN/d(input j) (j >= 1) */
static int leaf_norm(node* d, const double* v, double* dN) {
  double lo = d->lo, hi = d->hi;
  switch (d->kind) {
    case RFO_GAUSS: {
      double mu = v[1], s = v[2];
      if (!(s > 0)) FAIL(-2, "gauss: sigma <= 0");
      double za = (lo - mu) / (SQRT2 * s), zb = (hi - mu) / (SQRT2 * s);
      double diff;
      if (za >= 0) diff = erfc(za) - erfc(zb);
      else if (zb <= 0) diff = erfc(-zb) - erfc(-za);
      else diff = erf(zb) - erf(za);
      double N = s * (SQRT2PI * 0.5) * diff;
      double ea = exp(-za * za), eb = exp(-zb * zb);
      dN[0] = ea - eb;
      dN[1] = (N - (hi - mu) * eb + (lo - mu) * ea) / s;
      d->N = N; return 0;
    }
    case RFO_CHEB: {
      double N = 1;
      for (int j = 1; j < d->n_in; ++j) {
        int k = j;
        if (k % 2 == 0) { N += v[j] / (1.0 - k * k); dN[j - 1] = (hi - lo) / (1.0 - k * k); }
        else dN[j - 1] = 0;
      }
      d->N = (hi - lo) * N; return 0;
    }
    case RFO_EXP: {
      double k = v[1];
      if ((int)d->attrs[0] == 0) {
        if (!(k > 0)) FAIL(-2, "exp: tau <= 0");
        double ea = exp(-lo / k), eb = exp(-hi / k);
        d->N = -k * ea * expm1(-(hi - lo) / k);
        dN[0] = (1 + lo / k) * ea - (1 + hi / k) * eb;
        return 0;
      }
      if (fabs(k) < 1e-12) {
        d->N = hi - lo; dN[0] = 0.5 * (hi * hi - lo * lo); return 0;
      }
      double ea = exp(k * lo), eb = exp(k * hi);
      d->N = ea * expm1(k * (hi - lo)) / k;
      dN[0] = (hi * eb - lo * ea) / k - d->N / k;
      return 0;
    }
    case RFO_DECAY_GAUSS: {
      double tau = v[1], s = v[2], b = v[3];
      if (!(tau > 0) || !(s > 0)) FAIL(-2, "decay: tau or sigma <= 0");
      double dA[3], dB[3];
      double Ah = decay_A(hi, tau, s, b, dA);
      double Al = decay_A(lo, tau, s, b, dB);
      d->N = Ah - Al;
      for (int j = 0; j < 3; ++j) dN[j] = dA[j] - dB[j];
      return 0;
    }
    case RFO_ARGUS: {
      double m0 = v[1], c = v[2];
      if (!(m0 > 0)) FAIL(-2, "argus: m0 <= 0");
      if (c > 0) FAIL(-2, "argus: c > 0");
      double k = -c;
      double top = hi < m0 ? hi : m0;
      if (lo >= top) FAIL(-2, "argus: empty support");
      double Ul = (m0 - lo) * (m0 + lo) / (m0 * m0);
      double Ut = (m0 - top) * (m0 + top) / (m0 * m0);
      double Jl, J3l, Jt, J3t;
      argus_J(Ul, k, &Jl, &J3l);
      argus_J(Ut, k, &Jt, &J3t);
      d->N = 0.5 * m0 * m0 * (Jl - Jt);
      dN[0] = 0;
      dN[1] = 0.5 * m0 * m0 * (J3l - J3t);
      return 0;
    }
    case RFO_POISSON: { /* sum of the mass over the integers lo..hi */
      double lam = v[1];
      if (!(lam > 0)) FAIL(-2, "poisson: lambda <= 0");
      nsum N = {0, 0}, D = {0, 0};
      for (double k = ceil(lo); k <= hi; k += 1.0) {
        double u = exp(k * log(lam) - lam - lgamma(k + 1.0));
        nadd(&N, u);
        nadd(&D, u * (k / lam - 1.0));
      }
      dN[0] = nval(&D);
      d->N = nval(&N); return 0;
    }
    case RFO_BW: {
      double M = v[1], G = v[2];
      if (!(G > 0)) FAIL(-2, "bw: Gamma <= 0");
      double qh = 2 * (hi - M) / G, ql = 2 * (lo - M) / G;
      double N = 2.0 / G * (atan(qh) - atan(ql));
      double bl = 1.0 / ((lo - M) * (lo - M) + 0.25 * G * G);
      double bh = 1.0 / ((hi - M) * (hi - M) + 0.25 * G * G);
      dN[0] = bl - bh;
      dN[1] = -N / G - 2.0 / (G * G) * (qh / (1 + qh * qh) - ql / (1 + ql * ql));
      d->N = N; return 0;
    }
    case RFO_NUMCONV_BW_CB: {
      double M = v[1], G = v[2], s = v[3], al = v[4], n = v[5];
      if (!(G > 0) || !(s > 0) || !(al > 0) || !(n >= 1)) FAIL(-2, "numconv: domain");
      nsum N = {0, 0}, dM = {0, 0}, dG = {0, 0}, ds = {0, 0}, da = {0, 0}, dn = {0, 0};
      for (int k = 0; k < d->K; ++k) {
        double dc[3];
        double c = d->gw[k] * cb_val(d->gy[k], s, al, n, dc);
        d->ck[k] = c;
        for (int j = 0; j < 3; ++j) d->dck[3 * k + j] = d->gw[k] * dc[j];
        double a0 = lo - d->gy[k], a1 = hi - d->gy[k];
        double qh = 2 * (a1 - M) / G, ql = 2 * (a0 - M) / G;
        double I = 2.0 / G * (atan(qh) - atan(ql));
        double bl = 1.0 / ((a0 - M) * (a0 - M) + 0.25 * G * G);
        double bh = 1.0 / ((a1 - M) * (a1 - M) + 0.25 * G * G);
        double dIM = bl - bh;
        double dIG = -I / G - 2.0 / (G * G) * (qh / (1 + qh * qh) - ql / (1 + ql * ql));
        d->Ik[k] = I;
        nadd(&N, c * I); nadd(&dM, c * dIM); nadd(&dG, c * dIG);
        nadd(&ds, d->dck[3 * k] * I); nadd(&da, d->dck[3 * k + 1] * I); nadd(&dn, d->dck[3 * k + 2] * I);
      }
      d->N = nval(&N);
      dN[0] = nval(&dM); dN[1] = nval(&dG); dN[2] = nval(&ds); dN[3] = nval(&da); dN[4] = nval(&dn);
      return 0;
    }
    case RFO_MLP: {
      if (!d->mw) FAIL(-3, "mlp: weights not set");
      nsum N = {0, 0}, dq[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
      for (int g = 0; g < d->K; ++g) {
        double raw[6], ds[6];
        raw[0] = d->mgx[g];
        for (int j = 1; j < 6; ++j) raw[j] = v[j];
        double e = exp(mlp_leaf(d, raw, ds));
        nadd(&N, d->mgw[g] * e);
        for (int j = 1; j < 6; ++j) nadd(&dq[j - 1], d->mgw[g] * e * ds[j]);
      }
      d->N = nval(&N);
      for (int j = 0; j < 5; ++j) dN[j] = nval(&dq[j]);
      return 0;
    }
  }
  FAIL(-1, "not a leaf");
}

/* ---- per-call preparation --------------------------------------------------- */
static void mark(const rfo_model* m, int id, char* reach) {
  if (reach[id]) return;
  reach[id] = 1;
  for (int j = 0; j < m->nd[id].n_in; ++j) mark(m, m->nd[id].in[j], reach);
}

static int prepare(rfo_model* m, int top, const double* theta, char* reach) {
  int P = m->np;
  if (top < 0 || top >= m->n || !is_pdf(m->nd[top].kind)) FAIL(-1, "top is not a PDF");
  memset(reach, 0, MAXN);
  mark(m, top, reach);
  for (int id = 0; id < m->n; ++id) {
    node* d = &m->nd[id];
    double* g = m->pg[id];
    memset(g, 0, sizeof(double) * MAXP);
    switch (d->kind) {
      case RFO_PARAM: m->pv[id] = theta[d->index]; g[d->index] = 1; break;
      case RFO_CONST: m->pv[id] = d->attrs[0]; break;
      case RFO_FN_LINEAR: {
        double s = d->attrs[0];
        for (int j = 0; j < d->n_in; ++j) {
          s += d->attrs[j + 1] * m->pv[d->in[j]];
          for (int k = 0; k < P; ++k) g[k] += d->attrs[j + 1] * m->pg[d->in[j]][k];
        }
        m->pv[id] = s; break;
      }
      case RFO_FN_PRODUCT: {
        double s = 1;
        for (int j = 0; j < d->n_in; ++j) s *= m->pv[d->in[j]];
        for (int j = 0; j < d->n_in; ++j) {
          double o = 1;
          for (int i = 0; i < d->n_in; ++i) if (i != j) o *= m->pv[d->in[i]];
          for (int k = 0; k < P; ++k) g[k] += o * m->pg[d->in[j]][k];
        }
        m->pv[id] = s; break;
      }
      case RFO_FN_RATIO: {  /* d(a/b) = da/b - a db/b^2 */
        const double a = m->pv[d->in[0]], b = m->pv[d->in[1]];
        m->pv[id] = a / b;
        for (int k = 0; k < P; ++k) g[k] = m->pg[d->in[0]][k] / b - a * m->pg[d->in[1]][k] / (b * b);
        break;
      }
      default: break;
    }
  }
  for (int id = 0; id < m->n; ++id) {
    node* d = &m->nd[id];
    if (!reach[id] || !is_pdf(d->kind) || d->kind == RFO_ADD || d->kind == RFO_PROD) continue;
    const node* ob = &m->nd[d->in[0]];
    d->lo = ob->lo; d->hi = ob->hi;
    if (d->kind == RFO_ARGUS && m->nd[d->in[1]].kind != RFO_CONST) FAIL(-1, "argus: m0 must be a constant");
    double v[MAXIN], dNin[MAXIN];
    for (int j = 1; j < d->n_in; ++j) {
      if (!is_paramlike(m->nd[d->in[j]].kind)) FAIL(-1, "leaf shape input must be parameter-like");
      v[j] = m->pv[d->in[j]];
    }
    int rc = leaf_norm(d, v, dNin);
    if (rc) return rc;
    for (int k = 0; k < P; ++k) {
      double s = 0;
      for (int j = 1; j < d->n_in; ++j) s += dNin[j - 1] * m->pg[d->in[j]][k];
      d->dN[k] = s;
    }
  }
  return 0;
}

/* evaluate all reachable PDF nodes for one event; val[id], grd[id][P] */
static void eval_event(rfo_model* m, const double* xs, char* reach, double* val,
                       double (*grd)[MAXP], int want_grad) {
  int P = m->np;
  for (int id = 0; id < m->n; ++id) {
    node* d = &m->nd[id];
    if (!reach[id] || !is_pdf(d->kind)) continue;
    double* g = grd[id];
    if (d->kind == RFO_ADD) {
      int nc = (d->n_in + 1) / 2;
      double fsum = 0, v = 0;
      for (int j = 0; j < nc - 1; ++j) fsum += m->pv[d->in[nc + j]];
      for (int j = 0; j < nc; ++j) {
        double cj = j < nc - 1 ? m->pv[d->in[nc + j]] : 1.0 - fsum;
        v += cj * val[d->in[j]];
      }
      val[id] = v;
      if (want_grad) {
        for (int k = 0; k < P; ++k) {
          double s = 0;
          for (int j = 0; j < nc; ++j) {
            double cj = j < nc - 1 ? m->pv[d->in[nc + j]] : 1.0 - fsum;
            s += cj * grd[d->in[j]][k];
          }
          for (int j = 0; j < nc - 1; ++j)
            s += m->pg[d->in[nc + j]][k] * (val[d->in[j]] - val[d->in[nc - 1]]);
          g[k] = s;
        }
      }
    } else if (d->kind == RFO_PROD) {
      double v = 1;
      for (int j = 0; j < d->n_in; ++j) v *= val[d->in[j]];
      val[id] = v;
      if (want_grad) {
        for (int k = 0; k < P; ++k) {
          double s = 0;
          for (int j = 0; j < d->n_in; ++j) {
            double o = 1;
            for (int i = 0; i < d->n_in; ++i) if (i != j) o *= val[d->in[i]];
            s += o * grd[d->in[j]][k];
          }
          g[k] = s;
        }
      }
    } else {
      double v[MAXIN], du[MAXIN];
      for (int j = 1; j < d->n_in; ++j) v[j] = m->pv[d->in[j]];
      double x = xs[m->nd[d->in[0]].index];
      double u = leaf_value(d, x, v, du);
      val[id] = u / d->N;
      if (want_grad) {
        for (int k = 0; k < P; ++k) {
          double dudk = 0;
          for (int j = 1; j < d->n_in; ++j) dudk += du[j - 1] * m->pg[d->in[j]][k];
          g[k] = dudk / d->N - u * d->dN[k] / (d->N * d->N);
        }
      }
    }
  }
}

int rfo_nll(rfo_model* m, int top, const double* theta,
            const double* const* cols, int64_t n,
            double* nll, double* grad, int64_t* n_bad) {
  return rfo_nll_ex(m, top, theta, cols, n, nll, grad, NULL, n_bad);
}

int rfo_nll_ex(rfo_model* m, int top, const double* theta,
               const double* const* cols, int64_t n,
               double* nll, double* grad, double* gabs, int64_t* n_bad) {
  return rfo_nll_w(m, top, theta, cols, NULL, n, nll, grad, gabs, n_bad);
}

/* Weighted events: NLL = -sum_i w_i log p_i, straight from its definition
 * (w = NULL: every weight 1, the same arithmetic as unweighted since a
 * product with 1 is exact). */
int rfo_nll_w(rfo_model* m, int top, const double* theta,
              const double* const* cols, const double* w, int64_t n,
              double* nll, double* grad, double* gabs, int64_t* n_bad) {
  char reach[MAXN];
  int ext = -1; /* extended likelihood: node of nu */
  if (top >= 0 && top < m->n && m->nd[top].kind == RFO_EXTENDED) {
    ext = m->nd[top].in[1];
    top = m->nd[top].in[0];
  }
  int rc = prepare(m, top, theta, reach);
  if (rc) return rc;
  int P = m->np, no = m->nobs;
  double* val = malloc(sizeof(double) * MAXN);
  double (*grd)[MAXP] = malloc(sizeof(double) * MAXN * MAXP);
  nsum L = {0, 0};
  nsum G[MAXP], A[MAXP];
  memset(G, 0, sizeof(G));
  memset(A, 0, sizeof(A));
  int64_t bad = 0;
  double xs[MAXN];
  for (int64_t i = 0; i < n; ++i) {
    for (int j = 0; j < no; ++j) xs[j] = cols[j][i];
    eval_event(m, xs, reach, val, grd, grad != NULL || gabs != NULL);
    double p = val[top];
    if (!(p > 0) || !isfinite(p)) { ++bad; continue; }
    const double wi = w ? w[i] : 1.0;
    nadd(&L, -wi * log(p));
    if (grad)
      for (int k = 0; k < P; ++k) nadd(&G[k], -wi * (grd[top][k] / p));
    if (gabs)
      for (int k = 0; k < P; ++k) nadd(&A[k], fabs(wi * (grd[top][k] / p)));
  }
  if (ext >= 0) {
    /* + nu - N log nu, N = sum of the weights (the event count unweighted) */
    nsum Nw = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&Nw, w ? w[i] : 1.0);
    const double nu = m->pv[ext], N = nval(&Nw);
    if (!(nu > 0)) { free(val); free(grd); FAIL(-2, "extended: nu must be > 0"); }
    nadd(&L, nu - N * log(nu));
    for (int k = 0; k < P; ++k) {
      const double t = (1.0 - N / nu) * m->pg[ext][k];
      nadd(&G[k], t);
      nadd(&A[k], fabs(t));
    }
  }
  *nll = bad ? INFINITY : nval(&L);
  if (grad) for (int k = 0; k < P; ++k) grad[k] = nval(&G[k]);
  if (gabs) for (int k = 0; k < P; ++k) gabs[k] = nval(&A[k]);
  if (n_bad) *n_bad = bad;
  free(val); free(grd);
  return 0;
}

int rfo_values(rfo_model* m, int top, const double* theta,
               const double* const* cols, int64_t n, double* out) {
  char reach[MAXN];
  if (top >= 0 && top < m->n && m->nd[top].kind == RFO_EXTENDED) top = m->nd[top].in[0];
  int rc = prepare(m, top, theta, reach);
  if (rc) return rc;
  double* val = malloc(sizeof(double) * MAXN);
  double xs[MAXN];
  for (int64_t i = 0; i < n; ++i) {
    for (int j = 0; j < m->nobs; ++j) xs[j] = cols[j][i];
    eval_event(m, xs, reach, val, NULL, 0);
    out[i] = val[top];
  }
  free(val);
  return 0;
}

int rfo_norm(rfo_model* m, int id, const double* theta, double* N, double* dN) {
  char reach[MAXN];
  if (id < 0 || id >= m->n || !is_pdf(m->nd[id].kind) || m->nd[id].kind >= RFO_ADD)
    FAIL(-1, "not a leaf PDF");
  int rc = prepare(m, id, theta, reach);
  if (rc) return rc;
  *N = m->nd[id].N;
  if (dN) for (int k = 0; k < m->np; ++k) dN[k] = m->nd[id].dN[k];
  return 0;
}

/* ---- binned template likelihood ------------------------------------------ */
int rfo_binned_nll(int C, int S, int B, int J, const double* T,
                   const double* Lp, const double* Lm, const double* nobs,
                   const double* theta, double* nll, double* grad) {
  double mu = theta[0];
  const double* al = theta + 1;
  nsum L = {0, 0};
  nsum* G = calloc((size_t)(J + 1), sizeof(nsum));
  double* nu_s = malloc(sizeof(double) * S);
  double t0 = 0; /* d nu_{c,0,b} / d mu */
  for (int c = 0; c < C; ++c) {
    for (int b = 0; b < B; ++b) {
      double nu = 0;
      for (int s = 0; s < S; ++s) {
        double e = 0;
        for (int j = 0; j < J; ++j) {
          size_t o = (((size_t)c * S + s) * J + j) * B + b;
          e += al[j] >= 0 ? al[j] * Lp[o] : -al[j] * Lm[o];
        }
        double t = T[((size_t)c * S + s) * B + b] * exp(e);
        if (s == 0) { t0 = t; t *= mu; }
        nu_s[s] = t; nu += t;
      }
      double n = nobs[(size_t)c * B + b];
      nadd(&L, nu - n * log(nu));
      double r = 1.0 - n / nu; /* d/dnu of (nu - n log nu) */
      if (grad) {
        nadd(&G[0], r * t0);
        for (int j = 0; j < J; ++j) {
          double s2 = 0;
          for (int s = 0; s < S; ++s) {
            size_t o = (((size_t)c * S + s) * J + j) * B + b;
            s2 += nu_s[s] * (al[j] >= 0 ? Lp[o] : -Lm[o]);
          }
          nadd(&G[j + 1], r * s2);
        }
      }
    }
  }
  for (int j = 0; j < J; ++j) {
    nadd(&L, 0.5 * al[j] * al[j]);
    if (grad) nadd(&G[j + 1], al[j]);
  }
  *nll = nval(&L);
  if (grad) for (int j = 0; j <= J; ++j) grad[j] = nval(&G[j]);
  free(G); free(nu_s);
  return 0;
}

/* ===== second derivatives: the Hessian of the NLL ==========================
 * The paper's fits need uncertainties, which come from the curvature of the
 * NLL at its minimum.  This section carries, per event and node, the value,
 * the dense gradient and the dense Hessian in theta (forward mode, second
 * order), from the second derivatives of every analytic leaf and of its
 * normalisation written out below, and of the parameter functions.  The
 * convolution and MLP leaves have no second derivatives here.
 * H(NLL) = -sum_i w_i [ p_i'' / p_i - p_i' p_i'^T / p_i^2 ], plus, for an
 * extended likelihood, (N / nu^2) nu' nu'^T + (1 - N / nu) nu''. */
#define MAXPH 16 /* parameters of a model whose Hessian the oracle forms */
#define MAXS 8   /* shape inputs of a leaf */

typedef double hmat[MAXPH][MAXPH];

/* decay (x) resolution: F and its first and second derivatives in
   (tau, s, b); with u = t - b and phi = exp(-u^2 / (2 s^2)) / sqrt(2 pi) */
static double decay_F2(double t, double tau, double s, double b, double* d, double (*h)[MAXS]) {
  const double u = t - b;
  double d1[3];
  const double F = decay_F(t, tau, s, b, d1);
  const double phi = exp(-u * u / (2 * s * s)) / SQRT2PI;
  const double Ft = d1[0], Fs = d1[1], Fb = d1[2];
  const double at = u / (tau * tau) - s * s / (tau * tau * tau); /* d(log F)/dtau without the phi term */
  d[0] = Ft; d[1] = Fs; d[2] = Fb;
  h[0][0] = Ft * at + F * (-2 * u / (tau * tau * tau) + 3 * s * s / (tau * tau * tau * tau)) - 2 * s * phi / (tau * tau * tau);
  h[0][1] = Fs * at - 2 * s * F / (tau * tau * tau) + phi / (tau * tau) + phi * u * u / (s * s * tau * tau);
  h[0][2] = Fb * at - F / (tau * tau) + phi * u / (s * tau * tau);
  h[1][1] = Fs * s / (tau * tau) + F / (tau * tau) - phi * u * u / (s * s * s) * (1 / tau + u / (s * s)) + 2 * phi * u / (s * s * s);
  h[1][2] = Fb * s / (tau * tau) - phi * u / (s * s) * (1 / tau + u / (s * s)) + phi / (s * s);
  h[2][2] = Fb / tau - phi * u / (s * s * s);
  h[1][0] = h[0][1]; h[2][0] = h[0][2]; h[2][1] = h[1][2];
  return F;
}
/* A(t) = tau (Phi(u/s) - F(t)) with first and second derivatives */
static double decay_A2(double t, double tau, double s, double b, double* d, double (*h)[MAXS]) {
  const double u = t - b;
  double dF[3], hF[MAXS][MAXS];
  const double F = decay_F2(t, tau, s, b, dF, hF);
  const double Phi = 0.5 * erfc(-u / (SQRT2 * s));
  const double phi = exp(-u * u / (2 * s * s)) / SQRT2PI;
  d[0] = Phi - F - tau * dF[0];
  d[1] = tau * (-u * phi / (s * s) - dF[1]);
  d[2] = tau * (-phi / s - dF[2]);
  h[0][0] = -2 * dF[0] - tau * hF[0][0];
  h[0][1] = -u * phi / (s * s) - dF[1] - tau * hF[0][1];
  h[0][2] = -phi / s - dF[2] - tau * hF[0][2];
  h[1][1] = tau * (-u * u * u * phi / (s * s * s * s * s) + 2 * u * phi / (s * s * s) - hF[1][1]);
  h[1][2] = tau * (phi / (s * s) - u * u * phi / (s * s * s * s) - hF[1][2]);
  h[2][2] = tau * (-u * phi / (s * s * s) - hF[2][2]);
  h[1][0] = h[0][1]; h[2][0] = h[0][2]; h[2][1] = h[1][2];
  return tau * (Phi - F);
}

/* J5(U) = int_0^U v^(5/2) e^{-k v} dv (the ARGUS normalisation's second
   derivative in c); power series up to kU = 2, else by parts from J3 */
static double argus_J5(double U, double k) {
  if (U <= 0) return 0;
  if (k * U < 2.0) {
    double s = 0, term = 1;
    for (int nn = 0; nn < 60; ++nn) {
      s += term * pow(U, nn + 3.5) / (nn + 3.5);
      term *= -k / (nn + 1);
    }
    return s;
  }
  double J, J3;
  argus_J(U, k, &J, &J3);
  return 2.5 / k * J3 - U * U * sqrt(U) * exp(-k * U) / k;
}

/* u, du/d(input j) and d2u/d(input j)d(input k), inputs j = 1..n_in-1 at j-1 */
static int leaf_value2(const node* d, double x, const double* v, double* du, double (*h)[MAXS]) {
  for (int j = 0; j < MAXS; ++j) for (int k = 0; k < MAXS; ++k) h[j][k] = 0;
  switch (d->kind) {
    case RFO_GAUSS: {
      const double mu = v[1], s = v[2], z = (x - mu) / s, g = exp(-0.5 * z * z);
      du[0] = g * z / s; du[1] = g * z * z / s;
      h[0][0] = g * (z * z - 1) / (s * s);
      h[0][1] = h[1][0] = g * (z * z * z - 2 * z) / (s * s);
      h[1][1] = g * (z * z * z * z - 3 * z * z) / (s * s);
      return 0;
    }
    case RFO_CHEB: case RFO_ARGUS: case RFO_BW: case RFO_POISSON: case RFO_EXP: case RFO_DECAY_GAUSS: break;
    default: FAIL(-1, "no second derivatives for this leaf");
  }
  switch (d->kind) {
    case RFO_CHEB: leaf_value(d, x, v, du); return 0; /* linear in its coefficients */
    case RFO_EXP: {
      const double k = v[1];
      if ((int)d->attrs[0] == 0) {
        const double e = exp(-x / k);
        du[0] = e * x / (k * k);
        h[0][0] = e * (x * x / (k * k * k * k) - 2 * x / (k * k * k));
      } else {
        const double e = exp(k * x);
        du[0] = e * x; h[0][0] = e * x * x;
      }
      return 0;
    }
    case RFO_DECAY_GAUSS: decay_F2(x, v[1], v[2], v[3], du, h); return 0;
    case RFO_ARGUS: {
      const double m0 = v[1], c = v[2];
      du[0] = 0; du[1] = 0;
      if (x >= m0) return 0;
      const double U = (m0 - x) * (m0 + x) / (m0 * m0);
      const double a = x * sqrt(U) * exp(c * U);
      du[1] = a * U; h[1][1] = a * U * U;
      return 0;
    }
    case RFO_BW: {
      const double M = v[1], G = v[2], q = x - M, b = 1.0 / (q * q + 0.25 * G * G);
      du[0] = 2 * q * b * b; du[1] = -0.5 * G * b * b;
      h[0][0] = -2 * b * b + 8 * q * q * b * b * b;
      h[0][1] = h[1][0] = -2 * q * G * b * b * b;
      h[1][1] = -0.5 * b * b + 0.5 * G * G * b * b * b;
      return 0;
    }
    case RFO_POISSON: {
      const double lam = v[1], u = exp(x * log(lam) - lam - lgamma(x + 1.0)), r = x / lam - 1.0;
      du[0] = u * r; h[0][0] = u * (r * r - x / (lam * lam));
      return 0;
    }
  }
  FAIL(-1, "no second derivatives for this leaf");
}

/* second derivatives of the normalisation N over the observable's range in
   the leaf's inputs (d->N and the first derivatives come from leaf_norm) */
static int leaf_norm2(const node* d, const double* v, double (*h)[MAXS]) {
  const double lo = d->lo, hi = d->hi;
  for (int j = 0; j < MAXS; ++j) for (int k = 0; k < MAXS; ++k) h[j][k] = 0;
  switch (d->kind) {
    case RFO_GAUSS: {
      const double mu = v[1], s = v[2];
      const double ea = exp(-0.5 * (lo - mu) * (lo - mu) / (s * s)), eb = exp(-0.5 * (hi - mu) * (hi - mu) / (s * s));
      const double a = lo - mu, b = hi - mu;
      h[0][0] = (a * ea - b * eb) / (s * s);
      h[0][1] = h[1][0] = (a * a * ea - b * b * eb) / (s * s * s);
      h[1][1] = (a * a * a * ea - b * b * b * eb) / (s * s * s * s);
      return 0;
    }
    case RFO_CHEB: return 0;
    case RFO_EXP: {
      const double k = v[1];
      if ((int)d->attrs[0] == 0) {
        h[0][0] = (lo * lo * exp(-lo / k) - hi * hi * exp(-hi / k)) / (k * k * k);
        return 0;
      }
      if (fabs(k) < 1e-12) { h[0][0] = (hi * hi * hi - lo * lo * lo) / 3.0; return 0; }
      /* int x^2 e^{k x} dx = e^{k x} (x^2 / k - 2 x / k^2 + 2 / k^3) */
      const double Fh = exp(k * hi) * (hi * hi / k - 2 * hi / (k * k) + 2 / (k * k * k));
      const double Fl = exp(k * lo) * (lo * lo / k - 2 * lo / (k * k) + 2 / (k * k * k));
      h[0][0] = Fh - Fl;
      return 0;
    }
    case RFO_DECAY_GAUSS: {
      double dA[3], dB[3], hA[MAXS][MAXS], hB[MAXS][MAXS];
      decay_A2(hi, v[1], v[2], v[3], dA, hA);
      decay_A2(lo, v[1], v[2], v[3], dB, hB);
      for (int j = 0; j < 3; ++j) for (int k = 0; k < 3; ++k) h[j][k] = hA[j][k] - hB[j][k];
      return 0;
    }
    case RFO_ARGUS: {
      const double m0 = v[1], k = -v[2], top = hi < m0 ? hi : m0;
      const double Ul = (m0 - lo) * (m0 + lo) / (m0 * m0), Ut = (m0 - top) * (m0 + top) / (m0 * m0);
      h[1][1] = 0.5 * m0 * m0 * (argus_J5(Ul, k) - argus_J5(Ut, k));
      return 0;
    }
    case RFO_BW: {
      const double M = v[1], G = v[2];
      const double bl = 1.0 / ((lo - M) * (lo - M) + 0.25 * G * G);
      const double bh = 1.0 / ((hi - M) * (hi - M) + 0.25 * G * G);
      const double qh = 2 * (hi - M) / G, ql = 2 * (lo - M) / G;
      const double N = 2.0 / G * (atan(qh) - atan(ql));
      const double ph = qh / (1 + qh * qh), pl = ql / (1 + ql * ql);
      const double dph = (1 - qh * qh) / ((1 + qh * qh) * (1 + qh * qh)), dpl = (1 - ql * ql) / ((1 + ql * ql) * (1 + ql * ql));
      const double NG = -N / G - 2.0 / (G * G) * (ph - pl);
      h[0][0] = 2 * (lo - M) * bl * bl - 2 * (hi - M) * bh * bh;
      h[0][1] = h[1][0] = -0.5 * G * (bl * bl - bh * bh);
      h[1][1] = -NG / G + N / (G * G) + 4.0 / (G * G * G) * (ph - pl) + 2.0 / (G * G * G) * (qh * dph - ql * dpl);
      return 0;
    }
    case RFO_POISSON: {
      const double lam = v[1];
      nsum S = {0, 0};
      for (double k = ceil(lo); k <= hi; k += 1.0) {
        const double u = exp(k * log(lam) - lam - lgamma(k + 1.0)), r = k / lam - 1.0;
        nadd(&S, u * (r * r - k / (lam * lam)));
      }
      h[0][0] = nval(&S);
      return 0;
    }
  }
  FAIL(-1, "no second derivatives for this leaf");
}

/* second derivatives in theta of the parameter-like nodes */
static void param_hess(const rfo_model* m, hmat* ph) {
  const int P = m->np;
  for (int id = 0; id < m->n; ++id) {
    const node* d = &m->nd[id];
    double (*H)[MAXPH] = ph[id];
    for (int a = 0; a < MAXPH; ++a) for (int b = 0; b < MAXPH; ++b) H[a][b] = 0;
    switch (d->kind) {
      case RFO_FN_LINEAR:
        for (int j = 0; j < d->n_in; ++j)
          for (int a = 0; a < P; ++a) for (int b = 0; b < P; ++b) H[a][b] += d->attrs[j + 1] * ph[d->in[j]][a][b];
        break;
      case RFO_FN_PRODUCT:
        for (int j = 0; j < d->n_in; ++j) {
          double o = 1;
          for (int i = 0; i < d->n_in; ++i) if (i != j) o *= m->pv[d->in[i]];
          for (int a = 0; a < P; ++a) for (int b = 0; b < P; ++b) H[a][b] += o * ph[d->in[j]][a][b];
          for (int k = 0; k < d->n_in; ++k) {
            if (k == j) continue;
            double o2 = 1;
            for (int i = 0; i < d->n_in; ++i) if (i != j && i != k) o2 *= m->pv[d->in[i]];
            for (int a = 0; a < P; ++a)
              for (int b = 0; b < P; ++b) H[a][b] += o2 * m->pg[d->in[j]][a] * m->pg[d->in[k]][b];
          }
        }
        break;
      case RFO_FN_RATIO: { /* a/b */
        const double A = m->pv[d->in[0]], B = m->pv[d->in[1]];
        const double* ga = m->pg[d->in[0]]; const double* gb = m->pg[d->in[1]];
        for (int a = 0; a < P; ++a)
          for (int b = 0; b < P; ++b)
            H[a][b] = ph[d->in[0]][a][b] / B - (ga[a] * gb[b] + gb[a] * ga[b]) / (B * B) - A * ph[d->in[1]][a][b] / (B * B) +
                      2 * A * gb[a] * gb[b] / (B * B * B);
        break;
      }
      default: break;
    }
  }
}

int rfo_nll_hess(rfo_model* m, int top, const double* theta, const double* const* cols, const double* w,
                 int64_t n, double* nll, double* grad, double* hess, int64_t* n_bad) {
  char reach[MAXN];
  int ext = -1;
  if (top >= 0 && top < m->n && m->nd[top].kind == RFO_EXTENDED) {
    ext = m->nd[top].in[1];
    top = m->nd[top].in[0];
  }
  const int P = m->np, no = m->nobs;
  if (P > MAXPH) FAIL(-1, "the oracle's Hessian takes at most 16 parameters");
  int rc = prepare(m, top, theta, reach);
  if (rc) return rc;
  hmat* ph = calloc(MAXN, sizeof(hmat));
  hmat* lN2 = calloc(MAXN, sizeof(hmat)); /* per leaf: d2N/dtheta2 */
  double* val = malloc(sizeof(double) * MAXN);
  double (*grd)[MAXPH] = malloc(sizeof(double) * MAXN * MAXPH);
  hmat* hss = malloc(sizeof(hmat) * MAXN);
  nsum* HS = calloc(MAXPH * MAXPH, sizeof(nsum));
  nsum L = {0, 0}, G[MAXPH];
  memset(G, 0, sizeof(G));
  param_hess(m, ph);
  /* theta-space second derivatives of every leaf's normalisation */
  for (int id = 0; id < m->n && rc == 0; ++id) {
    node* d = &m->nd[id];
    if (!reach[id] || !is_pdf(d->kind) || d->kind == RFO_ADD || d->kind == RFO_PROD) continue;
    double v[MAXIN], h[MAXS][MAXS], dN[MAXIN];
    for (int j = 1; j < d->n_in; ++j) v[j] = m->pv[d->in[j]];
    leaf_norm(d, v, dN);
    rc = leaf_norm2(d, v, h);
    for (int a = 0; a < P && rc == 0; ++a)
      for (int b = 0; b < P; ++b) {
        double s = 0;
        for (int j = 1; j < d->n_in; ++j) {
          s += dN[j - 1] * ph[d->in[j]][a][b];
          for (int k = 1; k < d->n_in; ++k) s += h[j - 1][k - 1] * m->pg[d->in[j]][a] * m->pg[d->in[k]][b];
        }
        lN2[id][a][b] = s;
      }
  }
  int64_t bad = 0;
  double xs[MAXN];
  for (int64_t i = 0; i < n && rc == 0; ++i) {
    for (int j = 0; j < no; ++j) xs[j] = cols[j][i];
    for (int id = 0; id < m->n && rc == 0; ++id) {
      node* d = &m->nd[id];
      if (!reach[id] || !is_pdf(d->kind)) continue;
      double* g = grd[id];
      double (*H)[MAXPH] = hss[id];
      if (d->kind == RFO_ADD) {
        const int nc = (d->n_in + 1) / 2;
        double fs = 0, c[MAXIN];
        for (int j = 0; j < nc - 1; ++j) { c[j] = m->pv[d->in[nc + j]]; fs += c[j]; }
        c[nc - 1] = 1.0 - fs;
        /* d c_j: the fraction's own derivatives; the last one is minus their sum */
        double dc[MAXIN][MAXPH];
        hmat* hc = malloc(sizeof(hmat) * MAXIN);
        for (int a = 0; a < P; ++a) {
          double t = 0;
          for (int j = 0; j < nc - 1; ++j) { dc[j][a] = m->pg[d->in[nc + j]][a]; t += dc[j][a]; }
          dc[nc - 1][a] = -t;
        }
        for (int a = 0; a < P; ++a)
          for (int b = 0; b < P; ++b) {
            double t = 0;
            for (int j = 0; j < nc - 1; ++j) { hc[j][a][b] = ph[d->in[nc + j]][a][b]; t += hc[j][a][b]; }
            hc[nc - 1][a][b] = -t;
          }
        double vv = 0;
        for (int j = 0; j < nc; ++j) vv += c[j] * val[d->in[j]];
        val[id] = vv;
        for (int a = 0; a < P; ++a) {
          double t = 0;
          for (int j = 0; j < nc; ++j) t += c[j] * grd[d->in[j]][a] + dc[j][a] * val[d->in[j]];
          g[a] = t;
        }
        for (int a = 0; a < P; ++a)
          for (int b = 0; b < P; ++b) {
            double t = 0;
            for (int j = 0; j < nc; ++j) {
              const int cj = d->in[j];
              t += c[j] * hss[cj][a][b] + dc[j][a] * grd[cj][b] + dc[j][b] * grd[cj][a] + hc[j][a][b] * val[cj];
            }
            H[a][b] = t;
          }
        free(hc);
      } else if (d->kind == RFO_PROD) {
        /* fold the factors one at a time: (f g)'' = f'' g + f' g'^T + g' f'^T + f g'' */
        const int c0 = d->in[0];
        double vv = val[c0], gg[MAXPH];
        hmat hh;
        for (int a = 0; a < P; ++a) gg[a] = grd[c0][a];
        memcpy(hh, hss[c0], sizeof(hmat));
        for (int j = 1; j < d->n_in; ++j) {
          const int cj = d->in[j];
          hmat nh;
          for (int a = 0; a < P; ++a)
            for (int b = 0; b < P; ++b)
              nh[a][b] = hh[a][b] * val[cj] + gg[a] * grd[cj][b] + grd[cj][a] * gg[b] + vv * hss[cj][a][b];
          for (int a = 0; a < P; ++a) gg[a] = gg[a] * val[cj] + vv * grd[cj][a];
          vv *= val[cj];
          memcpy(hh, nh, sizeof(hmat));
        }
        val[id] = vv;
        for (int a = 0; a < P; ++a) g[a] = gg[a];
        memcpy(H, hh, sizeof(hmat));
      } else {
        double v[MAXIN], du[MAXIN], h2[MAXS][MAXS];
        for (int j = 1; j < d->n_in; ++j) v[j] = m->pv[d->in[j]];
        const double x = xs[m->nd[d->in[0]].index];
        const double u = leaf_value(d, x, v, du);
        rc = leaf_value2(d, x, v, du, h2);
        if (rc) break;
        /* U' and U'' in theta, through the parameter-like inputs */
        double Ug[MAXPH];
        hmat Uh;
        for (int a = 0; a < P; ++a) {
          double t = 0;
          for (int j = 1; j < d->n_in; ++j) t += du[j - 1] * m->pg[d->in[j]][a];
          Ug[a] = t;
        }
        for (int a = 0; a < P; ++a)
          for (int b = 0; b < P; ++b) {
            double t = 0;
            for (int j = 1; j < d->n_in; ++j) {
              t += du[j - 1] * ph[d->in[j]][a][b];
              for (int k = 1; k < d->n_in; ++k) t += h2[j - 1][k - 1] * m->pg[d->in[j]][a] * m->pg[d->in[k]][b];
            }
            Uh[a][b] = t;
          }
        /* v = U / N */
        const double N = d->N;
        val[id] = u / N;
        for (int a = 0; a < P; ++a) g[a] = Ug[a] / N - u * d->dN[a] / (N * N);
        for (int a = 0; a < P; ++a)
          for (int b = 0; b < P; ++b)
            H[a][b] = Uh[a][b] / N - (Ug[a] * d->dN[b] + d->dN[a] * Ug[b]) / (N * N) - u * lN2[id][a][b] / (N * N) +
                      2 * u * d->dN[a] * d->dN[b] / (N * N * N);
      }
    }
    if (rc) break;
    const double p = val[top];
    if (!(p > 0) || !isfinite(p)) { ++bad; continue; }
    const double wi = w ? w[i] : 1.0;
    nadd(&L, -wi * log(p));
    for (int a = 0; a < P; ++a) nadd(&G[a], -wi * grd[top][a] / p);
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b)
        nadd(&HS[a * MAXPH + b], -wi * (hss[top][a][b] / p - grd[top][a] * grd[top][b] / (p * p)));
  }
  if (rc == 0 && ext >= 0) {
    nsum Nw = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&Nw, w ? w[i] : 1.0);
    const double nu = m->pv[ext], N = nval(&Nw);
    if (!(nu > 0)) rc = -2, g_err = "extended: nu must be > 0";
    else {
      nadd(&L, nu - N * log(nu));
      for (int a = 0; a < P; ++a) nadd(&G[a], (1.0 - N / nu) * m->pg[ext][a]);
      for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b)
          nadd(&HS[a * MAXPH + b], N / (nu * nu) * m->pg[ext][a] * m->pg[ext][b] + (1.0 - N / nu) * ph[ext][a][b]);
    }
  }
  if (rc == 0) {
    *nll = bad ? INFINITY : nval(&L);
    if (grad) for (int a = 0; a < P; ++a) grad[a] = nval(&G[a]);
    if (hess)
      for (int a = 0; a < P; ++a) for (int b = 0; b < P; ++b) hess[a * P + b] = nval(&HS[a * MAXPH + b]);
    if (n_bad) *n_bad = bad;
  }
  free(ph); free(lN2); free(val); free(grd); free(hss); free(HS);
  return rc;
}
