// rf_fit.cpp -- host-side minimiser driving the GPU likelihood.
//
// Fits call the likelihood repeatedly (Section 3 and Fig. 5: the speed-ups
// are measured on fit run time).  The minimiser is a plain BFGS
// quasi-Newton iteration in FP64 on the host: each iteration is one
// NLL+gradient evaluation on the GPU plus a few backtracking steps.
//   - start: inverse Hessian = diag(1 / H_kk), H_kk from a one-sided
//     difference of the analytic gradient (scale-aware for parameters whose
//     natural scales differ by orders of magnitude);
//   - line search on the directional derivative (curvature condition, secant
//     bracketing); a trial point outside the declared bounds, with NLL = +inf
//     (events with p <= 0) or a clear rise of NLL counts as an overshoot;
//   - convergence: EDM = g^T H^-1 g / 2 < edm_tol;
//   - uncertainties: sigma_k = sqrt((H^-1)_kk) with H the Hessian kernel's
//     at the minimum (rf_nll_grad_hess), or, for programs with leaves that
//     have no second derivatives, central differences of the analytic
//     gradient.
// Gauss-Legendre nodes for the quadrature leaves are computed here as well.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "rf_internal.h"

namespace rf {

// Newton iteration on P_K from Tricomi's asymptotic initial guess, FP64,
// with the derivative from the three-term recurrence.
void gauss_legendre(int K, double lo, double hi, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  const int half = (K + 1) / 2;
  for (int i = 1; i <= half; ++i) {
    const double th = pi * (4.0 * i - 1.0) / (4.0 * K + 2.0);
    double z = (1.0 - (K - 1.0) / (8.0 * K * (double)K * K)) * std::cos(th);
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= K; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      dp = K * (z * p1 - p2) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * std::fabs(z) + 1e-300) {
        if (it > 0) break;
      }
    }
    // final derivative at the converged node
    double p1 = 1.0, p2 = 0.0;
    for (int j = 1; j <= K; ++j) {
      const double p3 = p2;
      p2 = p1;
      p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
    }
    dp = K * (z * p1 - p2) / (z * z - 1.0);
    const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    const double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo);
    // z is positive and decreasing in i: node K-i (ascending) is +z, node i-1 is -z
    x[K - i] = c + h * z;
    x[i - 1] = c - h * z;
    w[K - i] = h * wt;
    w[i - 1] = h * wt;
  }
  if (K % 2 == 1) x[K / 2] = 0.5 * (hi + lo);
}

}  // namespace rf

using namespace rf;

namespace {

struct Eval {
  const Objective& obj;
  int n_eval = 0;
  // returns RF_OK (finite), RF_E_NONFINITE, RF_E_DOMAIN, or another error
  int operator()(const double* x, double* f, double* g) {
    ++n_eval;
    return obj.eval(x, f, g);
  }
};

bool invert_spd(std::vector<double>& A, int n) {
  // Gauss-Jordan with partial pivoting (n <= 64)
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(I[c * n + k], I[piv * n + k]);
      }
    const double d = A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] /= d;
      I[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        I[r * n + k] -= f * I[c * n + k];
      }
    }
  }
  A = I;
  return true;
}

}  // namespace

namespace rf {

int bfgs_fit(const Objective& obj, const double* theta0, const double* hinv0, double edm_tol, int32_t max_iter,
             double* theta_out, double* sigma_out, double* cov_out, double* info_out) {
  if (!theta0 || !theta_out) return fail(RF_E_INVALID, "NULL argument");
  const int P = obj.P;
  if (P == 0) return fail(RF_E_INVALID, "no parameters to fit");
  if (!(edm_tol > 0)) return fail(RF_E_INVALID, "edm_tol must be > 0");
  // the caller's initial inverse Hessian: finite, with a positive diagonal
  // (a covariance matrix); checked before anything runs
  for (int i = 0; i < P && hinv0; ++i) {
    if (!(hinv0[i * P + i] > 0)) return fail(RF_E_INVALID, "hinv0 must have a positive diagonal");
    for (int j = 0; j < P; ++j)
      if (!std::isfinite(hinv0[i * P + j])) return fail(RF_E_INVALID, "hinv0 is not finite");
  }
  Eval ev{obj};
  std::vector<double> x(theta0, theta0 + P), g(P), xn(P), gn(P), H(P * P, 0.0), d(P), s(P), y(P), Hy(P);
  double f;
  int rc = ev(x.data(), &f, g.data());
  if (rc) return rc;
  const std::vector<double>& lo = obj.lo;
  const std::vector<double>& hi = obj.hi;
  if (hinv0)
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) H[i * P + j] = 0.5 * (hinv0[i * P + j] + hinv0[j * P + i]);
  // initial inverse Hessian from forward differences of the gradient
  for (int k = 0; k < P && !hinv0; ++k) {
    const double span = std::isfinite(hi[k] - lo[k]) ? hi[k] - lo[k] : 1.0;
    double h = 1e-5 * span;
    if (x[k] + h > hi[k]) h = -h;
    xn = x;
    xn[k] += h;
    double fk;
    double hkk = 0.0;
    if (ev(xn.data(), &fk, gn.data()) == RF_OK) hkk = (gn[k] - g[k]) / h;
    H[k * P + k] = hkk > 0 ? 1.0 / hkk : span * span * 1e-4;
  }
  int it = 0;
  double edm = 0.0;
  bool conv = false;
  auto calc_edm = [&]() {
    double e = 0.0;
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) e += g[i] * H[i * P + j] * g[j];
    return 0.5 * e;
  };
  edm = calc_edm();
  for (it = 0; it < max_iter && !(conv = edm < edm_tol); ++it) {
    double slope = 0.0;
    for (int i = 0; i < P; ++i) {
      double v = 0.0;
      for (int j = 0; j < P; ++j) v -= H[i * P + j] * g[j];
      d[i] = v;
      slope += g[i] * v;
    }
    if (!(slope < 0)) {  // lost positive definiteness: restart from the diagonal
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j)
          if (i != j) H[i * P + j] = 0.0;
      continue;
    }
    // Line search on phi'(a) = g(x + a d) . d, which the adjoint gives to
    // ~1e-7 of its scale even in FP32, while FP32 NLL values carry rounding
    // noise far above the decrease near a minimum.  Accept when the
    // directional derivative has dropped to half its start (curvature
    // condition); bracket and interpolate (secant) otherwise.  Points outside
    // the bounds, with p <= 0 events or with a clear rise of NLL count as
    // overshoot.
    double alpha = 1.0, fn = 0.0, lo_a = 0.0, hi_a = -1.0, s_lo = slope;
    bool ok = false;
    for (int ls = 0; ls < 40; ++ls) {
      bool inside = true;
      for (int i = 0; i < P; ++i) {
        xn[i] = x[i] + alpha * d[i];
        if (xn[i] < lo[i] || xn[i] > hi[i]) inside = false;
      }
      bool over = !inside;
      double sn = 0.0;
      if (inside) {
        rc = ev(xn.data(), &fn, gn.data());
        if (rc && rc != RF_E_NONFINITE && rc != RF_E_DOMAIN) return rc;
        if (rc) over = true;
        else {
          for (int i = 0; i < P; ++i) sn += gn[i] * d[i];
          const double rise_tol = 1e-6 * std::fabs(f) + 1e-9;
          if (fn > f + 0.5 * alpha * std::fabs(slope) + rise_tol) over = true;
        }
      }
      if (!over && std::fabs(sn) <= 0.5 * std::fabs(slope)) { ok = true; break; }
      if (!over && sn < 0) {  // still descending: move the lower end up
        lo_a = alpha;
        s_lo = sn;
        alpha = hi_a < 0 ? 2.0 * alpha : 0.5 * (lo_a + hi_a);
        if (hi_a < 0 && alpha > 64.0) break;
        continue;
      }
      hi_a = alpha;  // overshoot
      if (!over && sn > 0) {
        double a2 = lo_a - s_lo * (hi_a - lo_a) / (sn - s_lo);  // secant zero of phi'
        const double w = hi_a - lo_a;
        if (!(a2 > lo_a + 0.1 * w)) a2 = lo_a + 0.1 * w;
        if (!(a2 < hi_a - 0.1 * w)) a2 = hi_a - 0.1 * w;
        alpha = a2;
      } else {
        alpha = 0.5 * (lo_a + hi_a);
      }
      if (hi_a - lo_a < 1e-12) break;
    }
    if (!ok) break;
    double ys = 0.0;
    for (int i = 0; i < P; ++i) {
      s[i] = xn[i] - x[i];
      y[i] = gn[i] - g[i];
      ys += y[i] * s[i];
    }
    if (ys > 1e-300) {
      // H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T
      const double rho = 1.0 / ys;
      double yHy = 0.0;
      for (int i = 0; i < P; ++i) {
        double v = 0.0;
        for (int j = 0; j < P; ++j) v += H[i * P + j] * y[j];
        Hy[i] = v;
        yHy += y[i] * v;
      }
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j)
          H[i * P + j] += -rho * (Hy[i] * s[j] + s[i] * Hy[j]) + (rho * rho * yHy + rho) * s[i] * s[j];
    }
    x = xn;
    g = gn;
    f = fn;
    edm = calc_edm();
  }
  conv = edm < edm_tol;
  for (int i = 0; i < P; ++i) theta_out[i] = x[i];
  if (sigma_out || cov_out) {
    // the exact Hessian where the objective has one, else central
    // differences of the analytic gradient
    std::vector<double> Hf(P * P), gp(P), gm(P);
    bool good = true;
    const bool exact = (bool)obj.hess;
    if (exact) good = obj.hess(x.data(), Hf.data()) == RF_OK;
    for (int k = 0; k < P && good && !exact; ++k) {
      // a tenth of the estimated sigma: large enough that FP32 gradient noise is
      // negligible, small enough for the quadratic region
      double h = 0.1 * std::sqrt(std::fabs(H[k * P + k]));
      if (x[k] + h > hi[k] || x[k] - h < lo[k]) h = 0.5 * std::min(hi[k] - x[k], x[k] - lo[k]);
      if (!(h > 0)) h = 1e-8;
      xn = x;
      xn[k] = x[k] + h;
      double ft;
      good &= ev(xn.data(), &ft, gp.data()) == RF_OK;
      xn[k] = x[k] - h;
      good &= ev(xn.data(), &ft, gm.data()) == RF_OK;
      for (int i = 0; i < P; ++i) Hf[i * P + k] = (gp[i] - gm[i]) / (2 * h);
    }
    for (int i = 0; i < P; ++i)
      for (int j = i + 1; j < P; ++j) Hf[i * P + j] = Hf[j * P + i] = 0.5 * (Hf[i * P + j] + Hf[j * P + i]);
    if (!(good && invert_spd(Hf, P))) Hf.assign((size_t)P * P, NAN);
    if (sigma_out)
      for (int k = 0; k < P; ++k) sigma_out[k] = Hf[k * P + k] > 0 ? std::sqrt(Hf[k * P + k]) : NAN;
    if (cov_out)
      for (int k = 0; k < P * P; ++k) cov_out[k] = Hf[k];
  }
  if (info_out) {
    info_out[0] = it;
    info_out[1] = ev.n_eval;
    info_out[2] = edm;
    info_out[3] = conv ? 1.0 : 0.0;
  }
  return RF_OK;
}

}  // namespace rf

extern "C" int rf_fit_bfgs(rf_program* p, const double* theta0, double edm_tol, int32_t max_iter,
                           double* theta_out, double* sigma_out, double* info_out, void* stream) {
  return rf_fit_bfgs_ex(p, theta0, nullptr, edm_tol, max_iter, theta_out, sigma_out, nullptr, info_out, stream);
}

extern "C" int rf_fit_bfgs_ex(rf_program* p, const double* theta0, const double* hinv0, double edm_tol,
                              int32_t max_iter, double* theta_out, double* sigma_out, double* cov_out,
                              double* info_out, void* stream) {
  if (!p) return fail(RF_E_INVALID, "NULL argument");
  Objective obj;
  obj.P = p->L.n_params;
  obj.lo = p->L.plo;
  obj.hi = p->L.phi;
  obj.eval = [p, stream](const double* x, double* f, double* g) {
    int64_t bad = 0;
    return rf_nll_grad(p, x, f, g, &bad, stream);
  };
  // the Hessian kernel where every leaf has second derivatives
  if (hess_supported(p->L, nullptr))
    obj.hess = [p, stream](const double* x, double* H) {
      double fh;
      std::vector<double> gh(p->L.n_params);
      return rf_nll_grad_hess(p, x, &fh, gh.data(), H, nullptr, stream);
    };
  return bfgs_fit(obj, theta0, hinv0, edm_tol, max_iter, theta_out, sigma_out, cov_out, info_out);
}
