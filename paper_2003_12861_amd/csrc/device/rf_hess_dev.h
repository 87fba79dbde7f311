// rf_hess_dev.h -- second derivatives of the analytic leaves, for the
// Hessian kernel (FP64).  Requires rf_dev.h.
//
// Uncertainties of fitted parameters come from the curvature of the NLL at
// its minimum.  For every analytic leaf this header gives
//   * <op>_u2(x, in, lo, hi, du, d2): the unnormalised shape u(x) with
//     du[j] = du/d(input j) and d2[j*k + l] = d2u/d(input j)d(input l), j, l
//     over the k shape inputs (in[] holds their values);
//   * <op>_n2(in, lo, hi, d2): the second derivatives of the normalisation N
//     over the range [lo, hi] in the same inputs (N and dN come from the
//     leaf's prologue in rf_dev.h).
// The Hessian kernel combines them per event into d2 log p / d(slot)^2 and
// contracts with the parameter functions' derivatives at the end.
#pragma once

// ---------------------------------------------------------------- Gaussian
// u = exp(-z^2/2), z = (x - mu)/s:
//   d2u/dmu2 = u (z^2 - 1)/s^2, d2u/dmu ds = u (z^3 - 2z)/s^2,
//   d2u/ds2 = u (z^4 - 3z^2)/s^2.
RF_DEV double gauss_u2(double x, const double* in, double lo, double hi, double* du, double* d2) {
  (void)lo; (void)hi;
  const double s = in[1], is = 1.0 / s, z = (x - in[0]) * is, z2 = z * z;
  const double u = ::exp(-0.5 * z2);
  const double ui2 = u * is * is;
  du[0] = u * z * is;
  du[1] = u * z2 * is;
  d2[0] = ui2 * (z2 - 1.0);
  d2[1] = d2[2] = ui2 * z * (z2 - 2.0);
  d2[3] = ui2 * z2 * (z2 - 3.0);
  return u;
}
// N = s sqrt(pi/2) [erf(zb) - erf(za)]; with e_y = exp(-(y - mu)^2/(2 s^2)) and
// a = lo - mu, b = hi - mu: d2N/dmu2 = (a e_a - b e_b)/s^2,
// d2N/dmu ds = (a^2 e_a - b^2 e_b)/s^3, d2N/ds2 = (a^3 e_a - b^3 e_b)/s^4.
RF_DEV void gauss_n2(const double* in, double lo, double hi, double* d2) {
  const double s = in[1], a = lo - in[0], b = hi - in[0];
  const double ea = ::exp(-0.5 * a * a / (s * s)), eb = ::exp(-0.5 * b * b / (s * s));
  const double ta = a * ea, tb = b * eb, is2 = 1.0 / (s * s);
  d2[0] = (ta - tb) * is2;
  d2[1] = d2[2] = (a * ta - b * tb) * is2 / s;
  d2[3] = (a * a * ta - b * b * tb) * is2 * is2;
}

// --------------------------------------------------------------- Chebyshev
// linear in its coefficients: no second derivatives of u or N
template <int NC> RF_DEV double cheb_u2(double x, const double* in, double lo, double hi, double* du, double* d2) {
  const double y = (2.0 * x - lo - hi) / (hi - lo);
  double tkm = 1.0, tk = y, u = 1.0;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    u += in[j] * tk;
    du[j] = tk;
    const double tn = 2.0 * y * tk - tkm;
    tkm = tk;
    tk = tn;
  }
#pragma unroll
  for (int j = 0; j < NC * NC; ++j) d2[j] = 0.0;
  return u;
}
template <int NC> RF_DEV void cheb_n2(const double* in, double lo, double hi, double* d2) {
  (void)in; (void)lo; (void)hi;
#pragma unroll
  for (int j = 0; j < NC * NC; ++j) d2[j] = 0.0;
}

// ------------------------------------------------------------- exponential
// form 0: u = exp(-x/tau), du = u x/tau^2, d2u = u (x^2/tau^4 - 2x/tau^3);
//         d2N/dtau2 = (lo^2 e^{-lo/tau} - hi^2 e^{-hi/tau}) / tau^3.
// form 1: u = exp(lam (x - xc)) (xc the range midpoint, as in the fused
//         kernel), du = (x - xc) u, d2u = (x - xc)^2 u;
//         d2N/dlam2 = int (y - xc)^2 exp(lam (y - xc)) dy over the range.
template <int FORM> RF_DEV double exp_u2(double x, const double* in, double lo, double hi, double* du, double* d2) {
  if (FORM == 0) {
    const double it = 1.0 / in[0], e = ::exp(-x * it), q = x * it * it;
    du[0] = e * q;
    d2[0] = e * (q * q - 2.0 * q * it);
    return e;
  }
  const double s = x - 0.5 * (lo + hi), e = ::exp(in[0] * s);
  du[0] = s * e;
  d2[0] = s * s * e;
  return e;
}
template <int FORM> RF_DEV void exp_n2(const double* in, double lo, double hi, double* d2) {
  if (FORM == 0) {
    const double t = in[0];
    d2[0] = (lo * lo * ::exp(-lo / t) - hi * hi * ::exp(-hi / t)) / (t * t * t);
    return;
  }
  const double lam = in[0], a = lo - 0.5 * (lo + hi), b = hi - 0.5 * (lo + hi);
  const double r = ::fabs(lam) * (::fabs(a) > ::fabs(b) ? ::fabs(a) : ::fabs(b));
  if (r < 1.0) {
    // sum_n lam^n / n! (b^{n+3} - a^{n+3}) / (n + 3): every term is small
    double s = 0.0, c = 1.0, pa = a * a * a, pb = b * b * b;
    for (int n = 0; n < 40; ++n) {
      s += c * (pb - pa) / (n + 3);
      c *= lam / (n + 1);
      pa *= a;
      pb *= b;
    }
    d2[0] = s;
    return;
  }
  auto F = [&](double y) { return ::exp(lam * y) * (y * y / lam - 2.0 * y / (lam * lam) + 2.0 / (lam * lam * lam)); };
  d2[0] = F(b) - F(a);
}

// ------------------------------------------- decay (x) Gaussian resolution
// F(t; tau, s, b) and its first derivatives come from decay_F (rf_dev.h).
// With u = t - b, phi = exp(-u^2/(2 s^2))/sqrt(2 pi), c = u/tau^2 - s^2/tau^3
// (so that dF/dtau = F c + s phi/tau^2), and dF/d(tau, s, b) = (Ft, Fs, Fb):
//   Ftt = Ft c + F (3 s^2/tau^4 - 2u/tau^3) - 2 s phi/tau^3
//   Fts = Fs c - 2 s F/tau^3 + phi (1 + u^2/s^2)/tau^2
//   Ftb = Fb c - F/tau^2 + phi u/(s tau^2)
//   Fss = Fs s/tau^2 + F/tau^2 - phi (u^2/s^3)(1/tau + u/s^2) + 2 phi u/s^3
//   Fsb = Fb s/tau^2 - phi (u/s^2)(1/tau + u/s^2) + phi/s^2
//   Fbb = Fb/tau - phi u/s^3
RF_DEV double decay_F2(double u, double tau, double s, double* dF, double* h) {
  const double F = decay_F(u, tau, s, dF);
  const double phi = ::exp(-u * u / (2.0 * s * s)) * RF_INV_SQRT2PI;
  const double it = 1.0 / tau, is = 1.0 / s, it2 = it * it;
  const double c = u * it2 - s * s * it2 * it;
  const double Ft = dF[0], Fs = dF[1], Fb = dF[2];
  const double g = it + u * is * is;
  h[0] = Ft * c + F * (3.0 * s * s * it2 * it2 - 2.0 * u * it2 * it) - 2.0 * s * phi * it2 * it;
  h[1] = Fs * c - 2.0 * s * F * it2 * it + phi * (1.0 + u * u * is * is) * it2;
  h[2] = Fb * c - F * it2 + phi * u * is * it2;
  h[4] = Fs * s * it2 + F * it2 - phi * u * u * is * is * is * g + 2.0 * phi * u * is * is * is;
  h[5] = Fb * s * it2 - phi * u * is * is * g + phi * is * is;
  h[8] = Fb * it - phi * u * is * is * is;
  h[3] = h[1];
  h[6] = h[2];
  h[7] = h[5];
  return F;
}
RF_DEV double decay_u2(double x, const double* in, double lo, double hi, double* du, double* d2) {
  (void)lo; (void)hi;
  return decay_F2(x - in[2], in[0], in[1], du, d2);
}
// A(t) = tau [Phi(u/s) - F]: second derivatives at one end of the range
//   Att = -2 Ft - tau Ftt,  Ats = -u phi/s^2 - Fs - tau Fts,
//   Atb = -phi/s - Fb - tau Ftb,  Ass = tau (2u phi/s^3 - u^3 phi/s^5 - Fss),
//   Asb = tau (phi/s^2 - u^2 phi/s^4 - Fsb),  Abb = -tau (u phi/s^3 + Fbb)
RF_DEV void decay_A2(double t, const double* in, double* h) {
  const double tau = in[0], s = in[1], u = t - in[2];
  double dF[3], hF[9];
  decay_F2(u, tau, s, dF, hF);
  const double phi = ::exp(-u * u / (2.0 * s * s)) * RF_INV_SQRT2PI;
  const double is = 1.0 / s, is2 = is * is;
  h[0] = -2.0 * dF[0] - tau * hF[0];
  h[1] = -u * phi * is2 - dF[1] - tau * hF[1];
  h[2] = -phi * is - dF[2] - tau * hF[2];
  h[4] = tau * (2.0 * u * phi * is2 * is - u * u * u * phi * is2 * is2 * is - hF[4]);
  h[5] = tau * (phi * is2 - u * u * phi * is2 * is2 - hF[5]);
  h[8] = -tau * (u * phi * is2 * is + hF[8]);
  h[3] = h[1];
  h[6] = h[2];
  h[7] = h[5];
}
RF_DEV void decay_n2(const double* in, double lo, double hi, double* d2) {
  double hh[9], hl[9];
  decay_A2(hi, in, hh);
  decay_A2(lo, in, hl);
#pragma unroll
  for (int j = 0; j < 9; ++j) d2[j] = hh[j] - hl[j];
}

// ------------------------------------------------------------------ ARGUS
// inputs (m0 constant, c): u = m sqrt(U) e^{cU}, d2u/dc2 = U^2 u;
// d2N/dc2 = m0^2/2 [J5(U(lo)) - J5(U(top))], J5(U) = int_0^U v^{5/2} e^{-kv} dv,
// k = -c: its power series where kU < 2, else by parts from J3.
RF_DEV double argus_J5(double U, double k) {
  if (U <= 0) return 0.0;
  if (k * U < 2.0) {
    double s = 0.0, term = 1.0, p = U * U * U * ::sqrt(U);
    for (int n = 0; n < 60; ++n) {
      s += term * p / (n + 3.5);
      term *= -k * U / (n + 1);
    }
    return s;
  }
  double J, J3;
  argus_J(U, k, &J, &J3);
  return 2.5 / k * J3 - U * U * ::sqrt(U) * ::exp(-k * U) / k;
}
RF_DEV double argus_u2(double x, const double* in, double lo, double hi, double* du, double* d2) {
  (void)lo; (void)hi;
  const double m0 = in[0], c = in[1];
  du[0] = 0.0; du[1] = 0.0;
  d2[0] = d2[1] = d2[2] = d2[3] = 0.0;
  if (x >= m0) return 0.0;
  const double U = (m0 - x) * (m0 + x) / (m0 * m0);
  const double u = x * ::sqrt(U) * ::exp(c * U);
  du[1] = U * u;
  d2[3] = U * U * u;
  return u;
}
RF_DEV void argus_n2(const double* in, double lo, double hi, double* d2) {
  const double m0 = in[0], k = -in[1], top = hi < m0 ? hi : m0;
  const double Ul = (m0 - lo) * (m0 + lo) / (m0 * m0), Ut = (m0 - top) * (m0 + top) / (m0 * m0);
  d2[0] = d2[1] = d2[2] = 0.0;
  d2[3] = 0.5 * m0 * m0 * (argus_J5(Ul, k) - argus_J5(Ut, k));
}

// ----------------------------------------------------------- Breit-Wigner
// u = 1/(q^2 + G^2/4), q = x - M:
//   d2u/dM2 = 8 q^2 u^3 - 2 u^2, d2u/dM dG = -2 q G u^3, d2u/dG2 = (G^2 u - 1) u^2 / 2.
RF_DEV double bw_u2(double x, const double* in, double lo, double hi, double* du, double* d2) {
  (void)lo; (void)hi;
  const double G = in[1], q = x - in[0];
  const double u = 1.0 / (q * q + 0.25 * G * G), u2 = u * u, u3 = u2 * u;
  du[0] = 2.0 * q * u2;
  du[1] = -0.5 * G * u2;
  d2[0] = 8.0 * q * q * u3 - 2.0 * u2;
  d2[1] = d2[2] = -2.0 * q * G * u3;
  d2[3] = 0.5 * (G * G * u - 1.0) * u2;
  return u;
}
// N = (2/G)[atan(qh) - atan(ql)], q_y = 2 (y - M)/G, with u_y = u at x = y:
//   d2N/dM2 = 2 (lo - M) u_lo^2 - 2 (hi - M) u_hi^2,
//   d2N/dM dG = -(G/2)(u_lo^2 - u_hi^2),
//   d2N/dG2 = -N_G/G + N/G^2 + 4 [f(qh) - f(ql)]/G^3 + 2 [qh f'(qh) - ql f'(ql)]/G^3,
// f(q) = q/(1 + q^2), N_G = dN/dG = -N/G - 2 [f(qh) - f(ql)]/G^2.
RF_DEV void bw_n2(const double* in, double lo, double hi, double* d2) {
  const double M = in[0], G = in[1];
  const double ul = 1.0 / ((lo - M) * (lo - M) + 0.25 * G * G), uh = 1.0 / ((hi - M) * (hi - M) + 0.25 * G * G);
  const double qh = 2.0 * (hi - M) / G, ql = 2.0 * (lo - M) / G;
  const double N = 2.0 / G * (::atan(qh) - ::atan(ql));
  const double fh = qh / (1.0 + qh * qh), fl = ql / (1.0 + ql * ql);
  const double dfh = (1.0 - qh * qh) / ((1.0 + qh * qh) * (1.0 + qh * qh));
  const double dfl = (1.0 - ql * ql) / ((1.0 + ql * ql) * (1.0 + ql * ql));
  const double iG = 1.0 / G, NG = -N * iG - 2.0 * iG * iG * (fh - fl);
  d2[0] = 2.0 * (lo - M) * ul * ul - 2.0 * (hi - M) * uh * uh;
  d2[1] = d2[2] = -0.5 * G * (ul * ul - uh * uh);
  d2[3] = -NG * iG + N * iG * iG + iG * iG * iG * (4.0 * (fh - fl) + 2.0 * (qh * dfh - ql * dfl));
}
