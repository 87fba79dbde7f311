"""Pins of the oracle against values fixed by mathematics, not by itself.

Every normalisation is checked against adaptive quadrature and, where one
exists, against an independent library distribution (scipy.stats); every
analytic gradient against Richardson-extrapolated central differences;
special cases against the textbook function they reduce to.  These tests run
on the CPU only.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

from oracle import rfo
from paper_2003_12861_amd import synth, workloads


def quad(f, a, b, points=None):
    v, err = integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=500, points=points)
    return v


def single_leaf(kind, lo, hi, n_params, consts=(), attrs=()):
    """Model with one leaf: inputs = x, then params p0..p{n-1}, then constants."""
    m = rfo.Model()
    x = m.node("obs", [], [lo, hi])
    ins = [x] + [m.node("param") for _ in range(n_params)]
    ins += [m.node("const", [], [c]) for c in consts]
    if kind == "argus":  # inputs: m, m0 (const), c (param)
        ins = [x, ins[2], ins[1]]
    top = m.node(kind, ins, attrs)
    return m, top


def richardson_grad(f, theta, h=1e-4):
    theta = np.asarray(theta, float)
    g = np.empty_like(theta)
    for k in range(theta.size):
        def d(hh):
            tp, tm = theta.copy(), theta.copy()
            tp[k] += hh
            tm[k] -= hh
            return (f(tp) - f(tm)) / (2 * hh)
        g[k] = (4 * d(h / 2) - d(h)) / 3
    return g


# ---------------------------------------------------------------- Gaussian
@pytest.mark.parametrize("mu,sig,lo,hi", [(0.0, 1.0, -10, 10), (5.28, 0.003, 5.2, 5.29),
                                          (0.3, 2.0, -1.0, 4.0), (3.0, 0.5, -10, 0.5)])
def test_gauss_norm(mu, sig, lo, hi):
    m, top = single_leaf("gauss", lo, hi, 2)
    N, dN = m.norm(top, [mu, sig])
    ref = sig * math.sqrt(2 * math.pi) * (stats.norm.cdf(hi, mu, sig) - stats.norm.cdf(lo, mu, sig))
    if lo > mu:
        ref = sig * math.sqrt(2 * math.pi) * (stats.norm.sf(lo, mu, sig) - stats.norm.sf(hi, mu, sig))
    assert N == pytest.approx(ref, rel=1e-13)
    u = lambda x: math.exp(-0.5 * ((x - mu) / sig) ** 2)
    pts = [mu] if lo < mu < hi else None
    assert N == pytest.approx(quad(u, lo, hi, pts), rel=1e-11)
    dmu = quad(lambda x: u(x) * (x - mu) / sig**2, lo, hi, pts)
    dsg = quad(lambda x: u(x) * (x - mu) ** 2 / sig**3, lo, hi, pts)
    assert dN[0] == pytest.approx(dmu, rel=1e-9, abs=1e-14 * abs(N))
    assert dN[1] == pytest.approx(dsg, rel=1e-9)


def test_gauss_wide_range_limit():
    m, top = single_leaf("gauss", -60, 60, 2)
    N, _ = m.norm(top, [0.7, 1.3])
    assert N == pytest.approx(1.3 * math.sqrt(2 * math.pi), rel=1e-15)


def test_gauss_values_truncnorm():
    lo, hi, mu, sig = -2.0, 3.0, 0.4, 0.8
    m, top = single_leaf("gauss", lo, hi, 2)
    x = np.linspace(lo, hi, 37)
    v = m.values(top, [mu, sig], [x])
    ref = stats.truncnorm.pdf(x, (lo - mu) / sig, (hi - mu) / sig, loc=mu, scale=sig)
    np.testing.assert_allclose(v, ref, rtol=1e-12)


# ------------------------------------------------------------- Chebyshev
@pytest.mark.parametrize("coef", [(0.2, -0.1), (0.0, 0.0), (0.3, 0.1, -0.2, 0.05)])
def test_cheb(coef):
    lo, hi = -10.0, 7.0
    m, top = single_leaf("cheb", lo, hi, len(coef))
    N, dN = m.norm(top, list(coef))
    shape = lambda x: np.polynomial.chebyshev.chebval((2 * x - lo - hi) / (hi - lo), [1.0, *coef])
    assert N == pytest.approx(quad(shape, lo, hi), rel=1e-13)
    if not any(coef):
        assert N == pytest.approx(hi - lo, rel=1e-15)
    for k in range(len(coef)):
        Tk = lambda x, k=k: np.polynomial.chebyshev.chebval((2 * x - lo - hi) / (hi - lo), [0] * (k + 1) + [1])
        assert dN[k] == pytest.approx(quad(Tk, lo, hi), abs=1e-12)
    x = np.linspace(lo, hi, 11)
    np.testing.assert_allclose(m.values(top, list(coef), [x]), shape(x) / N, rtol=1e-13)


# ----------------------------------------------------------- exponential
def test_exp_tau_form():
    lo, hi, tau = 0.0, 10.0, 0.4
    m, top = single_leaf("exp", lo, hi, 1, attrs=[0.0])
    N, dN = m.norm(top, [tau])
    assert N == pytest.approx(quad(lambda t: math.exp(-t / tau), lo, hi), rel=1e-13)
    assert N == pytest.approx(tau * (1 - math.exp(-hi / tau)), rel=1e-15)
    assert dN[0] == pytest.approx(quad(lambda t: math.exp(-t / tau) * t / tau**2, lo, hi), rel=1e-11)
    x = np.linspace(lo, hi, 9)
    ref = stats.truncexpon.pdf(x, (hi - lo) / tau, loc=lo, scale=tau)
    np.testing.assert_allclose(m.values(top, [tau], [x]), ref, rtol=1e-12)


@pytest.mark.parametrize("lam", [-0.02, 0.03, 0.0, 1e-14])
def test_exp_rate_form(lam):
    lo, hi = 60.0, 120.0
    m, top = single_leaf("exp", lo, hi, 1, attrs=[1.0])
    N, dN = m.norm(top, [lam])
    assert N == pytest.approx(quad(lambda x: math.exp(lam * x), lo, hi), rel=1e-12)
    assert dN[0] == pytest.approx(quad(lambda x: x * math.exp(lam * x), lo, hi), rel=1e-9)


# ------------------------------------------------ decay (x) Gaussian resolution
def decay_ref(t, tau, s, b):
    """tau * exponentially-modified-Gaussian density (scipy.stats.exponnorm)."""
    return tau * stats.exponnorm.pdf(t, tau / s, loc=b, scale=s)


@pytest.mark.parametrize("tau,s,b", [(1.5, 0.05, 0.0), (1.2, 0.3, 0.1), (0.8, 0.02, -0.01)])
def test_decay_gauss(tau, s, b):
    lo, hi = 0.0, 10.0
    m, top = single_leaf("decay_gauss", lo, hi, 3)
    N, dN = m.norm(top, [tau, s, b])
    ref = tau * (stats.exponnorm.cdf(hi, tau / s, loc=b, scale=s) - stats.exponnorm.cdf(lo, tau / s, loc=b, scale=s))
    assert N == pytest.approx(ref, rel=1e-11)
    assert N == pytest.approx(quad(lambda t: decay_ref(t, tau, s, b), lo, hi, [b, b + s]), rel=1e-10)
    x = np.linspace(lo, hi, 23)
    np.testing.assert_allclose(m.values(top, [tau, s, b], [x]), decay_ref(x, tau, s, b) / N, rtol=1e-10)
    # normalisation derivatives vs differences of the library CDF
    def Nof(th):
        t2, s2, b2 = th
        return t2 * (stats.exponnorm.cdf(hi, t2 / s2, loc=b2, scale=s2) - stats.exponnorm.cdf(lo, t2 / s2, loc=b2, scale=s2))
    np.testing.assert_allclose(dN, richardson_grad(Nof, [tau, s, b], 1e-4), rtol=1e-6, atol=1e-9)


def test_decay_total_is_tau():
    m, top = single_leaf("decay_gauss", -20.0, 80.0, 3)
    N, _ = m.norm(top, [1.5, 0.3, 0.2])
    assert N == pytest.approx(1.5, rel=1e-12)


def test_decay_small_resolution_is_exponential():
    lo, hi, tau = 0.0, 10.0, 1.5
    m, top = single_leaf("decay_gauss", lo, hi, 3)
    x = np.linspace(0.5, 9.5, 10)
    v = m.values(top, [tau, 1e-7, 0.0], [x])
    ref = stats.truncexpon.pdf(x, (hi - lo) / tau, loc=lo, scale=tau)
    np.testing.assert_allclose(v, ref, rtol=1e-6)


# ------------------------------------------------------------------ ARGUS
def argus_series_J(U, k, terms=60):
    return sum((-k) ** n * U ** (n + 1.5) / (math.factorial(n) * (n + 1.5)) for n in range(terms))


@pytest.mark.parametrize("c,lo,hi", [(-20.0, 5.2, 5.29), (-2.0, 4.0, 5.29), (-60.0, 5.0, 5.25), (0.0, 5.0, 5.29)])
def test_argus(c, lo, hi):
    m0 = 5.29
    m, top = single_leaf("argus", lo, hi, 1, consts=[m0])
    N, dN = m.norm(top, [c])
    shape = lambda x: x * math.sqrt(max(0.0, 1 - (x / m0) ** 2)) * math.exp(c * (1 - (x / m0) ** 2)) if x < m0 else 0.0
    assert N == pytest.approx(quad(shape, lo, min(hi, m0)), rel=1e-11)
    # closed form of the paper-independent series in U = 1 - (m/m0)^2
    Ul, Uh = 1 - (lo / m0) ** 2, 1 - (min(hi, m0) / m0) ** 2
    assert N == pytest.approx(0.5 * m0 * m0 * (argus_series_J(Ul, -c) - argus_series_J(Uh, -c)), rel=1e-12)
    dshape = lambda x: shape(x) * (1 - (x / m0) ** 2)
    assert dN[0] == pytest.approx(quad(dshape, lo, min(hi, m0)), rel=1e-9)
    if c < 0:
        chi = math.sqrt(-2 * c)
        x = np.linspace(lo, min(hi, m0) - 1e-6, 15)
        rv = stats.argus(chi, scale=m0)
        ref = rv.pdf(x) / (rv.cdf(min(hi, m0)) - rv.cdf(lo))
        np.testing.assert_allclose(m.values(top, [c], [x]), ref, rtol=1e-9)


# ------------------------------------------------- Breit-Wigner, Crystal Ball
def test_breit_wigner():
    lo, hi, M, G = 60.0, 120.0, 91.19, 2.5
    m, top = single_leaf("bw", lo, hi, 2)
    N, dN = m.norm(top, [M, G])
    ref = math.pi / (G / 2) * (stats.cauchy.cdf(hi, M, G / 2) - stats.cauchy.cdf(lo, M, G / 2))
    assert N == pytest.approx(ref, rel=1e-13)
    x = np.linspace(lo, hi, 31)
    v = m.values(top, [M, G], [x])
    np.testing.assert_allclose(v, stats.cauchy.pdf(x, M, G / 2) / (ref * G / 2 / math.pi), rtol=1e-12)
    Nof = lambda th: math.pi / (th[1] / 2) * (stats.cauchy.cdf(hi, th[0], th[1] / 2) - stats.cauchy.cdf(lo, th[0], th[1] / 2))
    np.testing.assert_allclose(dN, richardson_grad(Nof, [M, G], 1e-3), rtol=1e-8)


def numconv_model(K=1024, window=(-30.0, 30.0), lo=60.0, hi=120.0):
    m = rfo.Model()
    x = m.node("obs", [], [lo, hi])
    ps = [m.node("param") for _ in range(5)]
    top = m.node("numconv_bw_cb", [x] + ps, [window[0], window[1], float(K)])
    return m, top


def cb_shape(y, s, a, n):
    """Crystal Ball shape from scipy.stats.crystalball, scaled to 1 at y = 0."""
    return stats.crystalball.pdf(y / s, a, n) / stats.crystalball.pdf(0.0, a, n)


@pytest.mark.parametrize("theta", [(91.19, 2.5, 1.5, 1.5, 3.0), (90.0, 3.0, 0.7, 0.8, 1.5), (92.0, 2.0, 2.5, 2.5, 8.0)])
def test_numconv_normalised_and_close_to_exact(theta):
    M, G, s, a, n = theta
    lo, hi = 60.0, 120.0
    m, top = numconv_model()
    N, _ = m.norm(top, list(theta))
    # the rule's normalisation is the exact x-integral of its own sum
    xs = np.linspace(lo, hi, 4001)
    p = m.values(top, list(theta), [xs])
    total = integrate.simpson(p, x=xs)
    assert total == pytest.approx(1.0, rel=2e-6)
    # distance from the adaptive convolution integral (rule error, small)
    def conv(x):
        f = lambda y: cb_shape(y, s, a, n) / ((x - y - M) ** 2 + G * G / 4)
        return quad(f, -30.0, 30.0, points=[-a * s, 0.0, x - M])
    for x in (80.0, 89.0, 91.0, 93.5, 110.0):
        exact = conv(x)
        ours = m.values(top, list(theta), [np.array([x])])[0] * N
        assert ours == pytest.approx(exact, rel=3e-4 if s < 1 else 2e-5)


def test_crystal_ball_continuity_via_numconv_tables():
    # C1 continuity of the shape at the junction z = -alpha, checked on the
    # library reference the oracle is compared against below
    s, a, n = 1.3, 1.1, 2.5
    z0 = -a * s
    e = 1e-7
    left, right = cb_shape(z0 - e, s, a, n), cb_shape(z0 + e, s, a, n)
    assert left == pytest.approx(right, rel=1e-6)


def test_numconv_value_vs_direct_rule():
    """S(x) = sum_k w_k CB(y_k) BW(x - y_k) written out with numpy's Gauss-Legendre
    nodes and scipy's Crystal Ball: agrees with the oracle to rounding."""
    theta = [91.19, 2.5, 1.5, 1.5, 3.0]
    M, G, s, a, n = theta
    m, top = numconv_model(K=256)
    N, _ = m.norm(top, theta)
    t, w = np.polynomial.legendre.leggauss(256)
    y, w = 30.0 * t, 30.0 * w
    c = w * cb_shape(y, s, a, n)
    xs = np.array([70.0, 91.0, 95.5])
    S = np.array([(c / ((x - y - M) ** 2 + G * G / 4)).sum() for x in xs])
    np.testing.assert_allclose(m.values(top, theta, [xs]) * N, S, rtol=1e-12)


# ------------------------------------------------------------ Gauss-Legendre
def test_gauss_legendre_nodes():
    x, w = rfo.gauss_legendre(64, -1.0, 1.0)
    xr, wr = np.polynomial.legendre.leggauss(64)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, rtol=1e-11)  # numpy weights carry ~1e-12 error
    x, w = rfo.gauss_legendre(1024, -1.0, 1.0)
    assert np.all(np.diff(x) > 0)
    for j in (0, 1, 5, 50, 400, 1000):
        assert (w * x ** (2 * j)).sum() == pytest.approx(2.0 / (2 * j + 1), rel=1e-12)
    x, w = rfo.gauss_legendre(1024, -30.0, 30.0)
    assert (w * np.cos(x)).sum() == pytest.approx(2 * math.sin(30.0), rel=1e-12)


# ---------------------------------------------------------------------- MLP
def _torch_mlp(w, u):
    import torch
    W = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    U = torch.tensor(u, dtype=torch.float64, requires_grad=True)
    W1 = W[0:384].view(64, 6); b1 = W[384:448]
    W2 = W[448:4544].view(64, 64); b2 = W[4544:4608]
    W3 = W[4608:8704].view(64, 64); b3 = W[8704:8768]
    W4 = W[8768:8832].view(1, 64); b4 = W[8832:8833]
    h = torch.tanh(U @ W1.T + b1)
    h = torch.tanh(h @ W2.T + b2)
    h = torch.tanh(h @ W3.T + b3)
    s = (h @ W4.T + b4)[:, 0]
    return W, U, s


def test_mlp_forward_backward_vs_torch():
    rng = np.random.default_rng(0)
    w = rng.normal(0, 0.3, 8833)
    u = rng.uniform(-1, 1, (17, 6))
    dout = rng.normal(size=17)
    W, U, s = _torch_mlp(w, u)
    np.testing.assert_allclose(rfo.mlp_forward(w, u), s.detach().numpy(), rtol=1e-13, atol=1e-14)
    import torch
    (s * torch.tensor(dout)).sum().backward()
    dw, din = rfo.mlp_backward(w, u, dout)
    np.testing.assert_allclose(dw, W.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(din, U.grad.numpy(), rtol=1e-11, atol=1e-13)


def _base_value(d, G, sg, al, n):
    """The surrogate's analytic base, written out: pseudo-Voigt of Thompson, Cox
    & Hastings (1987) with the Crystal Ball tail in its Gaussian part."""
    c0 = 2 * math.sqrt(2 * math.log(2))
    fg, fl = c0 * sg, G
    f = (fg**5 + 2.69269 * fg**4 * fl + 2.42843 * fg**3 * fl**2 + 4.47163 * fg**2 * fl**3
         + 0.07842 * fg * fl**4 + fl**5) ** 0.2
    r = fl / f
    eta = 1.36603 * r - 0.47719 * r**2 + 0.11116 * r**3
    h = f / 2
    L = (h / math.pi) / (d * d + h * h)
    se = f / c0
    z = d / se
    if z > -al:
        C = math.exp(-0.5 * z * z)
    else:
        C = (n / al) ** n * math.exp(-0.5 * al * al) * (n / al - al - z) ** (-n)
    return eta * L + (1 - eta) * C / (se * math.sqrt(2 * math.pi))


def test_mlp_leaf_normalisation_vs_quadrature():
    """The leaf's K-point Gauss-Legendre normalisation against adaptive
    quadrature of exp(MLP) x base: the base's tail junction (continuous value
    and slope) limits the rule to ~1e-9 at K = 1024, and the error must shrink
    at K = 4096."""
    rng = np.random.default_rng(1)
    w = rng.normal(0, 0.2, 8833)
    th = [91.0, 2.4, 1.2, 1.3, 4.0]
    box = synth.BWCB_MLP_BOX
    def s_of_x(x):
        raw = np.array([[x - th[0]] + th])  # first input: position relative to M
        u = 2 * (raw - [b[0] for b in box]) / np.array([b[1] - b[0] for b in box]) - 1
        return math.exp(_torch_mlp(w, u)[2].item()) * _base_value(x - th[0], *th[1:])
    c0 = 2 * math.sqrt(2 * math.log(2))
    fg, fl = c0 * th[2], th[1]
    f = (fg**5 + 2.69269 * fg**4 * fl + 2.42843 * fg**3 * fl**2 + 4.47163 * fg**2 * fl**3
         + 0.07842 * fg * fl**4 + fl**5) ** 0.2
    junction = th[0] - th[3] * f / c0
    from scipy import integrate
    ref = integrate.quad(s_of_x, 60.0, 120.0, points=[th[0], junction], epsabs=0, epsrel=1e-13, limit=500)[0]
    errs = []
    for K in (1024, 4096):
        m, top, ids = rfo.from_spec(workloads.spec_bwcb(surrogate=True, K=K))
        m.set_mlp_weights(ids["sig"], w)
        N, _ = m.norm(ids["sig"], th + [-0.02, 0.8])
        errs.append(abs(N - ref) / ref)
    assert errs[0] < 3e-9 and errs[1] < 3e-10 and errs[1] < errs[0] / 5, errs


def test_mlp_base_is_pseudo_voigt_without_tail():
    """With a zero network and the tail moved out of reach (alpha = 30) the
    surrogate leaf is the Thompson-Cox-Hastings pseudo-Voigt, which
    approximates the exact Voigt profile (Lorentzian of width Gamma convolved
    with a Gaussian of width sigma) to about 1% of the peak height."""
    from scipy.special import voigt_profile
    spec = workloads.spec_bwcb(surrogate=True)
    m, top, ids = rfo.from_spec(spec)
    m.set_mlp_weights(ids["sig"], np.zeros(8833))
    for M, G, sg in ((91.19, 2.5, 1.5), (90.0, 1.6, 2.8), (92.5, 3.4, 0.6), (91.0, 0.5, 3.0), (91.0, 6.0, 0.5)):
        th = [M, G, sg, 30.0, 3.0, -0.02, 1.0]  # f = 1 isolates the signal
        x = np.linspace(M - 8, M + 8, 161)
        p = m.values(top, th, [x])
        v = voigt_profile(x - M, sg, G / 2)
        v /= quad(lambda t: voigt_profile(t - M, sg, G / 2), 60.0, 120.0, points=[M])
        assert np.abs(p - v).max() <= 0.012 * v.max(), (M, G, sg, np.abs(p - v).max() / v.max())


def _zero_net_leaf():
    """The oracle's surrogate leaf with a zero network: its values are the
    analytic base b(x - M; Gamma, sigma, alpha, n), normalised."""
    m, top, ids = rfo.from_spec(workloads.spec_bwcb(surrogate=True))
    m.set_mlp_weights(ids["sig"], np.zeros(8833))
    return m, top


def _base_ratio(m, top, th, x):
    """b(x - M) / b(0): the normalisation cancels (f = 1 isolates the signal)."""
    v = m.values(top, list(th[:5]) + [-0.02, 1.0], [np.concatenate([[th[0]], np.atleast_1d(x)])])
    return v[1:] / v[0]


def test_mlp_base_limits_are_gaussian_and_lorentzian():
    """The pseudo-Voigt base in its two limits, without the tail (alpha =
    30): at Gamma -> 0 it is the Gaussian of width sigma, at sigma -> 0 the
    Lorentzian of full width Gamma (the mixing weight becomes exactly 1: its
    polynomial's coefficients add up to 1)."""
    m, top = _zero_net_leaf()
    for M, sg in ((91.19, 1.5), (90.0, 0.6), (92.0, 2.9)):
        d = np.linspace(-4 * sg, 4 * sg, 33)
        r = _base_ratio(m, top, [M, 1e-12, sg, 30.0, 3.0], M + d)
        np.testing.assert_allclose(r, stats.norm.pdf(d, 0, sg) / stats.norm.pdf(0, 0, sg), rtol=1e-7, atol=1e-12)
    for M, G in ((91.19, 2.5), (89.5, 0.5), (92.5, 6.0)):
        d = np.linspace(-5 * G, 5 * G, 41)
        r = _base_ratio(m, top, [M, G, 1e-9, 30.0, 3.0], M + d)
        np.testing.assert_allclose(r, stats.cauchy.pdf(d, 0, G / 2) / stats.cauchy.pdf(0, 0, G / 2), rtol=1e-7)


def _half_max_crossing(d, r):
    """First d where the ratio r(d) (decreasing from 1) falls to 1/2, by
    linear interpolation between grid neighbours."""
    k = int(np.argmax(r < 0.5))
    return d[k - 1] + (0.5 - r[k - 1]) * (d[k] - d[k - 1]) / (r[k] - r[k - 1])


def test_mlp_base_width_is_the_voigt_fwhm():
    """The full width at half maximum of the base (half-maximum crossings of
    the oracle's own values on a grid of spacing 5e-4) against that of the
    exact Voigt profile (scipy.special.voigt_profile, Lorentzian half width
    Gamma/2, crossing by root-finding) over the surrogate's (Gamma, sigma)
    box and beyond.  The pseudo-Voigt's width approximates that FWHM:
    measured within 0.45% over Gamma in [0.5, 6], sigma in [0.5, 3], so the
    bar is 0.5%; a wrong width coefficient or component width moves it
    further (a 10x slip in the smallest coefficient moves it 2.5%)."""
    from scipy.optimize import brentq
    from scipy.special import voigt_profile
    m, top = _zero_net_leaf()
    M = 91.19
    worst = 0.0
    for G in (0.5, 2.5, 6.0):
        for sg in (0.5, 1.5, 3.0):
            th = [M, G, sg, 30.0, 3.0]
            d = np.arange(0.0, 12.0, 5e-4)
            hi = _half_max_crossing(d, _base_ratio(m, top, th, M + d))
            lo = _half_max_crossing(d, _base_ratio(m, top, th, M - d))
            pk = voigt_profile(0.0, sg, G / 2)
            fv = 2 * brentq(lambda t: voigt_profile(t, sg, G / 2) - pk / 2, 1e-6, 50.0, xtol=1e-12)
            assert abs(hi - lo) <= 1e-6 * fv  # symmetric without the tail
            worst = max(worst, abs((hi + lo) - fv) / fv)
    assert worst <= 5e-3, worst


@pytest.mark.parametrize("G,sg,al,n", [(2.5, 1.5, 1.5, 3.0), (1.6, 2.8, 0.5, 1.0), (3.4, 0.6, 2.9, 9.5),
                                       (2.0, 1.0, 1.0, 5.0)])
def test_mlp_base_is_c1_at_the_tail_junction(G, sg, al, n):
    """The Crystal Ball tail joins the base's Gaussian part with a continuous
    value and slope.  Scanned on grids without knowing where the junction
    is: for a function with continuous value and slope, the change of the
    difference quotient of log b between neighbours shrinks in proportion to
    the spacing (it is about the second derivative times the spacing); a
    jump in the slope would keep it constant, a jump in the value would make
    it grow."""
    m, top = _zero_net_leaf()
    M = 91.19
    th = [M, G, sg, al, n, -0.02, 1.0]
    span = 6.0 * sg + 1.0
    worst = []
    for step in (2e-3, 2e-4):
        x = M - span + step * np.arange(int(span / step))
        q = np.diff(np.log(m.values(top, th, [x]))) / step
        worst.append(np.abs(np.diff(q)).max())
    assert worst[1] <= 0.3 * worst[0], worst


# ------------------------------------------------------------ binned model
def _binned_small(seed=3, C=3, S=2, B=5, J=4):
    d = synth.make_binned(seed, C, S, B, J)
    Lp = np.log(d["Tp"] / d["T"][:, :, None, :])
    Lm = np.log(d["Tm"] / d["T"][:, :, None, :])
    return d, Lp, Lm


def test_binned_reduces_to_poisson():
    d, Lp, Lm = _binned_small()
    J = Lp.shape[2]
    nll, g = rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], [1.0] + [0.0] * J)
    nu = d["T"].sum(axis=1)
    ref = -(stats.poisson.logpmf(d["nobs"], nu).sum()) - special.gammaln(d["nobs"] + 1).sum()
    assert nll == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_binned_interpolation_hits_variations(sign):
    d, Lp, Lm = _binned_small()
    J = Lp.shape[2]
    j = 2
    th = [1.0] + [0.0] * J
    th[1 + j] = sign
    nll, _ = rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], th)
    Tv = (d["Tp"] if sign > 0 else d["Tm"])[:, :, j, :]
    nu = Tv.sum(axis=1)
    ref = -(stats.poisson.logpmf(d["nobs"], nu).sum()) - special.gammaln(d["nobs"] + 1).sum() + 0.5
    assert nll == pytest.approx(ref, rel=1e-12)


def test_binned_gradient_fd_and_single_bin_minimum():
    d, Lp, Lm = _binned_small()
    J = Lp.shape[2]
    rng = np.random.default_rng(4)
    al = rng.uniform(-1, 1, J)
    al[np.abs(al) < 0.05] = 0.3
    th = np.concatenate([[1.07], al])
    f = lambda t: rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], t, grad=False)[0]
    _, g = rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], th)
    np.testing.assert_allclose(g, richardson_grad(f, th, 1e-4), rtol=1e-7, atol=1e-7)
    # one bin, one sample scaled by mu: minimum of nu - n log nu at nu = n
    T = np.array([[[40.0]]]); L0 = np.zeros((1, 1, 0, 1)); n = np.array([[52.0]])
    _, g1 = rfo.binned_nll(T, L0, L0, n, [52.0 / 40.0])
    assert abs(g1[0]) < 1e-12


# ------------------------------------------------------- mixture and NLL
TH0 = [0.0, 1.0, 0.3, 0.2, -0.1]


def cfg0_pdf_ref(x, mu, sig, f, c1, c2, lo=-10.0, hi=10.0):
    g = stats.truncnorm.pdf(x, (lo - mu) / sig, (hi - mu) / sig, loc=mu, scale=sig)
    xp = (2 * x - lo - hi) / (hi - lo)
    h = np.polynomial.chebyshev.chebval(xp, [1.0, c1, c2])
    Nc = quad(lambda t: np.polynomial.chebyshev.chebval((2 * t - lo - hi) / (hi - lo), [1.0, c1, c2]), lo, hi)
    return f * g + (1 - f) * h / Nc


def test_cfg0_tiny_samples():
    m, top, _ = rfo.from_spec(workloads.spec_gauss_cheb())
    for xs in ([0.0], [-1.0, 0.5, 2.0], [-9.99, 9.99, 3.3, -0.25]):
        x = np.array(xs)
        nll, _, nb = m.nll(top, TH0, [x])
        assert nb == 0
        assert nll == pytest.approx(-np.log(cfg0_pdf_ref(x, *TH0)).sum(), rel=1e-13)


def test_mixture_fraction_limits():
    x = synth.sample_gauss_cheb(500, 11)
    m, top, _ = rfo.from_spec(workloads.spec_gauss_cheb())
    th1 = [0.2, 1.1, 1.0, 0.2, -0.1]
    nll1, _, _ = m.nll(top, th1, [x])
    g = stats.truncnorm.pdf(x, (-10 - 0.2) / 1.1, (10 - 0.2) / 1.1, loc=0.2, scale=1.1)
    assert nll1 == pytest.approx(-np.log(g).sum(), rel=1e-12)
    th0 = [0.2, 1.1, 0.0, 0.2, -0.1]
    nll0, _, _ = m.nll(top, th0, [x])
    assert nll0 == pytest.approx(-np.log(cfg0_pdf_ref(x, 0.2, 1.1, 0.0, 0.2, -0.1)).sum(), rel=1e-12)


def test_decay_argus_small_sample_vs_scipy():
    tr = synth.DECAY_TRUTH
    t, mm = synth.sample_decay_argus(50, 12)
    m, top, _ = rfo.from_spec(workloads.spec_decay_argus())
    th = list(tr.values())
    nll, _, nb = m.nll(top, th, [t, mm])
    assert nb == 0
    tau_s, st, bt, mu, sm, tb, c, f = th
    tlo, thi = synth.DECAY_T_RANGE
    mlo, mhi = synth.DECAY_M_RANGE
    ed = stats.exponnorm(tau_s / st, loc=bt, scale=st)
    pst = ed.pdf(t) / (ed.cdf(thi) - ed.cdf(tlo))
    psm = stats.truncnorm.pdf(mm, (mlo - mu) / sm, (mhi - mu) / sm, loc=mu, scale=sm)
    pbt = stats.truncexpon.pdf(t, (thi - tlo) / tb, loc=tlo, scale=tb)
    ra = stats.argus(math.sqrt(-2 * c), scale=synth.ARGUS_M0)
    pbm = ra.pdf(mm) / (ra.cdf(mhi) - ra.cdf(mlo))
    ref = -np.log(f * pst * psm + (1 - f) * pbt * pbm).sum()
    assert nll == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("which", ["gauss_cheb", "decay_argus", "bwcb", "mlp"])
def test_gradient_vs_richardson(which):
    rng = np.random.default_rng(5)
    if which == "gauss_cheb":
        spec, cols, th = workloads.spec_gauss_cheb(), [synth.sample_gauss_cheb(300, 2)], [0.05, 0.95, 0.33, 0.18, -0.12]
    elif which == "decay_argus":
        spec, cols, th = workloads.spec_decay_argus(), list(synth.sample_decay_argus(300, 3)), synth.jitter_decay(1)
    elif which == "bwcb":
        spec, cols, th = workloads.spec_bwcb(K=128), [synth.sample_bw_cb(60, 4)], [91.0, 2.6, 1.4, 1.6, 3.2, -0.021, 0.78]
    else:
        spec, cols, th = workloads.spec_bwcb(surrogate=True, K=64), [synth.sample_bw_cb(40, 4)], [91.0, 2.6, 1.4, 1.6, 3.2, -0.021, 0.78]
    m, top, ids = rfo.from_spec(spec)
    if which == "mlp":
        m.set_mlp_weights(ids["sig"], rng.normal(0, 0.2, 8833))
    nll, g, nb = m.nll(top, th, cols)
    assert nb == 0
    f = lambda t: m.nll(top, t, cols, grad=False)[0]
    h = np.maximum(1e-4 * np.abs(np.asarray(th, float)), 1e-5)
    if which == "decay_argus":
        h[3] = 2e-5  # the mass mean moves on the scale of its 0.003 width
    fd = np.array([richardson_grad(lambda tt: f(tt), th, hk)[k] for k, hk in enumerate(h)])
    scale = np.abs(fd).max()
    np.testing.assert_allclose(g, fd, rtol=2e-6, atol=2e-7 * scale)


def test_additivity_and_permutation():
    x = synth.sample_gauss_cheb(1000, 8)
    m, top, _ = rfo.from_spec(workloads.spec_gauss_cheb())
    a, ga, _ = m.nll(top, TH0, [x[:400]])
    b, gb, _ = m.nll(top, TH0, [x[400:]])
    ab, gab, _ = m.nll(top, TH0, [x])
    assert ab == pytest.approx(a + b, rel=1e-14)
    np.testing.assert_allclose(gab, ga + gb, rtol=1e-12, atol=1e-12)
    perm = np.random.default_rng(0).permutation(x.size)
    pp, _, _ = m.nll(top, TH0, [x[perm]])
    assert pp == pytest.approx(ab, rel=1e-14)


def test_bad_events_make_nll_infinite():
    m, top, _ = rfo.from_spec(workloads.spec_gauss_cheb())
    x = np.linspace(-10, 10, 101)
    nll, _, nb = m.nll(top, [0.0, 1.0, 0.0, 1.5, 0.0], [x])  # 1 + 1.5 x' < 0 for x' < -2/3
    assert math.isinf(nll) and nb == np.sum((x / 10.0) * 1.5 + 1 <= 0)


# ---- weighted events: NLL = -sum_i w_i log p_i -------------------------------
def _weighted_cases():
    g = workloads.spec_gauss_cheb()
    d = workloads.spec_decay_argus()
    x = synth.sample_gauss_cheb(300, 41)
    t, m = synth.sample_decay_argus(300, 42)
    return [(g, [x], [0.1, 1.2, 0.3, 0.15, -0.05]),
            (d, [t, m], workloads.truth_vector(synth.DECAY_TRUTH))]


@pytest.mark.parametrize("case", [0, 1])
def test_oracle_unit_weights_equal_unweighted(case):
    spec, cols, th = _weighted_cases()[case]
    om, top, _ = rfo.from_spec(spec)
    a = om.nll_ex(top, th, cols)
    b = om.nll_ex(top, th, cols, weights=np.ones(cols[0].size))
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and a[3] == b[3] == 0


@pytest.mark.parametrize("case", [0, 1])
def test_oracle_integer_weights_equal_repeated_events(case):
    """w_i in {0, 1, 2, 3} is the unweighted NLL of the sample with event i
    repeated w_i times (zero drops it): value, gradient and gradient scale."""
    spec, cols, th = _weighted_cases()[case]
    om, top, _ = rfo.from_spec(spec)
    w = np.random.default_rng(7).integers(0, 4, cols[0].size)
    rep = [np.repeat(c, w) for c in cols]
    a = om.nll_ex(top, th, cols, weights=w.astype(np.float64))
    b = om.nll_ex(top, th, rep)
    assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-12 * np.abs(b[2]).max())
    np.testing.assert_allclose(a[2], b[2], rtol=1e-13)


def test_oracle_weights_are_linear():
    spec, cols, th = _weighted_cases()[1]
    om, top, _ = rfo.from_spec(spec)
    rng = np.random.default_rng(8)
    w1, w2 = rng.uniform(-0.5, 2, cols[0].size), rng.uniform(0, 1, cols[0].size)
    a, b, c = (om.nll_ex(top, th, cols, weights=w) for w in (w1, w2, w1 + w2))
    assert abs(c[0] - (a[0] + b[0])) <= 1e-13 * (abs(a[0]) + abs(b[0]))
    np.testing.assert_allclose(c[1], a[1] + b[1], rtol=0, atol=1e-12 * (np.abs(a[2]) + np.abs(b[2])).max())


# ---- extended likelihood: -sum_i log(sum_k nu_k u_k(x_i)) + sum_k nu_k ------
def _leaf_values(kind, th, x):
    spec = [("obs", "x", [], [-10.0, 10.0]), ("param", "a", [], [-5, 5]), ("param", "b", [], [-5, 10]),
            (kind, "leaf", ["x", "a", "b"], [])]
    om, top, _ = rfo.from_spec(spec)
    return om.values(top, th, [x])


def test_oracle_extended_is_the_textbook_extended_likelihood():
    """Yields as fractions nu_s / nu plus the term nu - N log nu equal the
    textbook form built from the normalised components."""
    x = synth.sample_gauss_cheb(500, 51)
    mu, sg, ns, nb, c1, c2 = 0.2, 1.1, 180.0, 290.0, 0.15, -0.05
    om, top, _ = rfo.from_spec(workloads.spec_gauss_cheb_extended())
    nll, g, nbad = om.nll(top, [mu, sg, ns, nb, c1, c2], [x])
    ug, uc = _leaf_values("gauss", [mu, sg], x), _leaf_values("cheb", [c1, c2], x)
    ref = -np.sum(np.log(ns * ug + nb * uc)) + ns + nb
    assert nbad == 0 and abs(nll - ref) <= 1e-13 * abs(ref)


def test_oracle_extended_gradient_central_differences():
    x = synth.sample_gauss_cheb(400, 52)
    th = np.array([0.2, 1.1, 180.0, 290.0, 0.15, -0.05])
    om, top, _ = rfo.from_spec(workloads.spec_gauss_cheb_extended())
    _, g, ga, _ = om.nll_ex(top, th, [x])
    for k in range(th.size):
        h = 1e-6 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (om.nll(top, tp, [x], grad=False)[0] - om.nll(top, tm, [x], grad=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * ga[k], (k, fd, g[k])


def test_oracle_extended_single_component_yield_stationary_at_n():
    """One component: d NLL / d nu = 1 - N / nu, zero at nu = N."""
    x = synth.sample_gauss_cheb(250, 53)
    spec = [("obs", "x", [], [-10.0, 10.0]), ("param", "mu", [], [-5, 5]), ("param", "sigma", [], [0.05, 10]),
            ("param", "nu", [], [0, 1e9]), ("gauss", "sig", ["x", "mu", "sigma"], []),
            ("extended", "model", ["sig", "nu"], [])]
    om, top, _ = rfo.from_spec(spec)
    for nu in (100.0, 250.0, 400.0):
        _, g, _ = om.nll(top, [0.1, 1.5, nu], [x])
        assert abs(g[2] - (1.0 - 250.0 / nu)) <= 1e-14


# ---- unbinned Poisson PDF of an integer observable -------------------------
def _poisson_leaf(lo, hi):
    spec = [("obs", "n", [], [lo, hi]), ("param", "lam", [], [0.1, 100.0]), ("poisson", "p", ["n", "lam"], [])]
    om, top, _ = rfo.from_spec(spec)
    return om, top


@pytest.mark.parametrize("lo,hi,lam", [(0.0, 60.0, 7.3), (3.0, 15.0, 9.0), (20.0, 400.0, 55.5), (0.0, 1.0, 0.4)])
def test_poisson_leaf_vs_scipy_truncated(lo, hi, lam):
    """Values are scipy's Poisson mass renormalised over the integers lo..hi."""
    om, top = _poisson_leaf(lo, hi)
    n = np.arange(lo, hi + 1.0)
    v = om.values(top, [lam], [n])
    z = stats.poisson.cdf(hi, lam) - stats.poisson.cdf(lo - 1, lam)
    ref = stats.poisson.pmf(n, lam) / z
    assert np.max(np.abs(v / ref - 1.0)) <= 2e-12
    assert abs(v.sum() - 1.0) <= 1e-13


def test_poisson_mle_is_the_sample_mean():
    """With a range holding all the mass, d NLL / d lambda = N - sum n / lambda,
    which vanishes at the sample mean."""
    rng = np.random.default_rng(61)
    n = rng.poisson(10.0, 2000).astype(np.float64)
    om, top = _poisson_leaf(0.0, 300.0)
    for lam in (6.0, n.mean(), 14.5):
        _, g, _ = om.nll(top, [lam], [n])
        ref = n.size - n.sum() / lam
        assert abs(g[0] - ref) <= 1e-11 * n.sum() / lam
    nll_at = lambda lam: om.nll(top, [lam], [n], grad=False)[0]
    assert nll_at(n.mean()) < min(nll_at(n.mean() * 0.99), nll_at(n.mean() * 1.01))


def test_poisson_truncation_gradient_central_differences():
    """A range that cuts the mass on both sides makes d log N / d lambda
    matter; the analytic gradient must follow the finite differences."""
    rng = np.random.default_rng(62)
    n = np.clip(rng.poisson(9.0, 500), 4, 13).astype(np.float64)
    om, top = _poisson_leaf(4.0, 13.0)
    _, g, ga, _ = om.nll_ex(top, [8.7], [n])
    h = 1e-5
    fd = (om.nll(top, [8.7 + h], [n], grad=False)[0] - om.nll(top, [8.7 - h], [n], grad=False)[0]) / (2 * h)
    assert abs(fd - g[0]) <= 1e-7 * ga[0]
    assert abs(g[0] - (n.size - n.sum() / 8.7)) > 1.0  # the truncation term is not negligible here


def test_poisson_gauss_cheb_mixture_vs_scipy():
    """The 2-D count x mass mixture equals the mixture assembled from scipy's
    Poisson mass (renormalised over the count range) and the normalised
    Gauss and Chebyshev leaves."""
    k, x = synth.sample_poisson_gauss_cheb(600, 63)
    th = [11.0, 5.5, 0.1, 1.2, 0.15, -0.05, 0.35]
    om, top, _ = rfo.from_spec(workloads.spec_poisson_gauss_cheb())
    nll, g, ga, nbad = om.nll_ex(top, th, [k, x])
    z = lambda lam: stats.poisson.cdf(40, lam) - stats.poisson.cdf(-1, lam)
    ps = stats.poisson.pmf(k, th[0]) / z(th[0])
    pb = stats.poisson.pmf(k, th[1]) / z(th[1])
    ug, uc = _leaf_values("gauss", th[2:4], x), _leaf_values("cheb", th[4:6], x)
    ref = -np.sum(np.log(th[6] * ps * ug + (1 - th[6]) * pb * uc))
    assert nbad == 0 and abs(nll - ref) <= 1e-12 * abs(ref)
    th = np.array(th)
    for j in range(th.size):
        h = 1e-6 * max(1.0, abs(th[j]))
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (om.nll(top, tp, [k, x], grad=False)[0] - om.nll(top, tm, [k, x], grad=False)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * ga[j], (j, fd, g[j])


def test_oracle_weighted_extended_equals_repeated_events():
    """Integer weights in the extended likelihood: N becomes the sum of the
    weights, and the result equals the unweighted extended NLL of the sample
    with each event repeated w_i times."""
    x = synth.sample_gauss_cheb(300, 54)
    w = np.random.default_rng(55).integers(0, 4, x.size).astype(np.float64)
    th = [0.2, 1.1, 150.0, 320.0, 0.15, -0.05]
    om, top, _ = rfo.from_spec(workloads.spec_gauss_cheb_extended())
    a, ga, _, _ = om.nll_ex(top, th, [x], weights=w)
    b, gb, _, _ = om.nll_ex(top, th, [np.repeat(x, w.astype(int))])
    assert abs(a - b) <= 1e-12 * abs(b)
    np.testing.assert_allclose(ga, gb, rtol=1e-11, atol=1e-9)


# ------------------------------------------------------ second derivatives
def _hess_fd(om, otop, th, cols, weights=None, h=None):
    """Central differences of the oracle's analytic gradient, Richardson-
    extrapolated, one column per parameter."""
    th = np.asarray(th, float)
    P = th.size
    H = np.empty((P, P))
    for k in range(P):
        hk = (h[k] if h is not None else 1e-4 * max(1.0, abs(th[k])))

        def d(hh):
            tp, tm = th.copy(), th.copy()
            tp[k] += hh
            tm[k] -= hh
            return (om.nll_ex(otop, tp, cols, weights=weights)[1] - om.nll_ex(otop, tm, cols, weights=weights)[1]) / (2 * hh)
        H[:, k] = (4 * d(hk / 2) - d(hk)) / 3
    return H


def _hess_close(H, Href, tol):
    s = np.sqrt(np.abs(np.outer(np.diag(Href), np.diag(Href))))
    err = np.abs(H - Href) / s
    assert err.max() <= tol, (err.max(), np.unravel_index(np.argmax(err), err.shape), H, Href)


def _spec_product_fn():
    """Two Gaussians whose widths are tied by a product function s2 = k s1 and
    whose fraction is a ratio of yields (second derivatives of the parameter
    functions); theta = (mu1, s1, mu2, k, y1, y2)."""
    return [
        ("obs", "x", [], [-10.0, 10.0]),
        ("param", "mu1", [], [-5.0, 5.0]), ("param", "s1", [], [0.05, 5.0]),
        ("param", "mu2", [], [-5.0, 5.0]), ("param", "k", [], [0.1, 10.0]),
        ("param", "y1", [], [0.0, 1e9]), ("param", "y2", [], [0.0, 1e9]),
        ("product", "s2", ["s1", "k"], []),
        ("gauss", "g1", ["x", "mu1", "s1"], []), ("gauss", "g2", ["x", "mu2", "s2"], []),
        ("linear", "yt", ["y1", "y2"], [0.0, 1.0, 1.0]), ("ratio", "f", ["y1", "yt"], []),
        ("add", "model", ["g1", "g2", "f"], []),
    ]


HESS_CASES = {
    "gauss_cheb": (workloads.spec_gauss_cheb, lambda: [synth.sample_gauss_cheb(3000, 61)], [0.05, 0.97, 0.31, 0.21, -0.09]),
    "decay_argus": (workloads.spec_decay_argus, lambda: list(synth.sample_decay_argus(3000, 62)),
                    list(synth.jitter_decay(3)), [1.5e-3, 5e-5, 5e-5, 3e-6, 3e-6, 4e-4, 2e-2, 2e-4]),
    "poisson_mix": (workloads.spec_poisson_gauss_cheb, lambda: list(synth.sample_poisson_gauss_cheb(3000, 63)),
                    [11.5, 5.2, 0.03, 1.02, 0.19, -0.11, 0.31]),
    "two_gauss_ext": (workloads.spec_two_gauss_extended,
                      lambda: [np.concatenate([np.random.default_rng(64).normal(-2, 0.5, 1200),
                                               np.random.default_rng(65).normal(2, 0.5, 1800)]).clip(-9.9, 9.9)],
                      [-1.98, 0.51, 2.01, 0.49, 1190.0, 1815.0]),
    "product_ratio": (_spec_product_fn,
                      lambda: [np.concatenate([np.random.default_rng(66).normal(-2, 0.5, 1200),
                                               np.random.default_rng(67).normal(2, 1.0, 1800)]).clip(-9.9, 9.9)],
                      [-1.98, 0.51, 2.01, 1.9, 1190.0, 1815.0]),
    "bw_exp": (lambda: [("obs", "x", [], [60.0, 120.0]), ("param", "M", [], [85.0, 97.0]),
                        ("param", "G", [], [0.5, 6.0]), ("param", "lam", [], [-0.2, 0.2]), ("param", "f", [], [0.0, 1.0]),
                        ("bw", "s", ["x", "M", "G"], []), ("exp", "b", ["x", "lam"], [1.0]),
                        ("add", "model", ["s", "b", "f"], [])],
               lambda: [np.random.default_rng(68).uniform(60, 120, 3000)], [91.1, 2.6, -0.021, 0.7]),
    "argus_steep": (lambda: [("obs", "m", [], [5.2, 5.29]), ("param", "c", [], [-200.0, 0.0]),
                             ("const", "m0", [], [5.29]), ("argus", "a", ["m", "m0", "c"], [])],
                    lambda: [np.random.default_rng(73).uniform(5.2, 5.2899, 2000)], [-80.0]),
    "exp_tau": (lambda: [("obs", "t", [], [0.3, 7.0]), ("param", "tau", [], [0.1, 10.0]), ("exp", "e", ["t", "tau"], [0.0])],
                lambda: [np.random.default_rng(69).uniform(0.3, 7.0, 2000)], [1.3]),
}


@pytest.mark.parametrize("case", sorted(HESS_CASES))
@pytest.mark.parametrize("weighted", [False, True])
def test_oracle_hessian_vs_gradient_differences(case, weighted):
    """The oracle's analytic Hessian against Richardson-extrapolated central
    differences of its analytic gradient (which is pinned against differences
    of the NLL itself), relative to sqrt(H_jj H_kk); also symmetric, and its
    NLL and gradient are the ones rfo_nll_w gives."""
    make_spec, make_cols, th = HESS_CASES[case][:3]
    steps = HESS_CASES[case][3] if len(HESS_CASES[case]) > 3 else None
    om, otop, _ = rfo.from_spec(make_spec())
    cols = [synth._f32(c) for c in make_cols()]
    w = np.random.default_rng(70).uniform(0.5, 2.0, cols[0].size) if weighted else None
    nll, g, H, nb = om.nll_hess(otop, th, cols, weights=w)
    n2, g2, _, _ = om.nll_ex(otop, th, cols, weights=w)
    assert nb == 0 and nll == pytest.approx(n2, rel=1e-14) and np.allclose(g, g2, rtol=1e-12, atol=1e-9)
    assert np.array_equal(H, H.T) or np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    _hess_close(H, _hess_fd(om, otop, th, cols, weights=w, h=steps), 2e-7)


def test_oracle_hessian_closed_forms():
    """A lone Gaussian on a range wide enough that its normalisation is
    sigma sqrt(2 pi) to the last bit, and a lone exponential likewise tau:
    the NLL's Hessian in closed form."""
    rng = np.random.default_rng(71)
    x = synth._f32(rng.normal(0.3, 1.7, 5000))
    m, top = single_leaf("gauss", -1000.0, 1000.0, 2)
    mu, s = 0.25, 1.65
    _, _, H, _ = m.nll_hess(top, [mu, s], [x])
    d = x - mu
    n = x.size
    ref = np.array([[n / s**2, 2 * d.sum() / s**3], [2 * d.sum() / s**3, 3 * (d * d).sum() / s**4 - n / s**2]])
    np.testing.assert_allclose(H, ref, rtol=1e-12)
    t = synth._f32(rng.exponential(1.4, 5000))
    m, top = single_leaf("exp", 0.0, 1e4, 1, attrs=[0.0])
    tau = 1.35
    _, _, H, _ = m.nll_hess(top, [tau], [t])
    np.testing.assert_allclose(H[0, 0], 2 * t.sum() / tau**3 - t.size / tau**2, rtol=1e-12)


def test_oracle_hessian_fraction_entry_vs_scipy():
    """For f g + (1 - f) c the fraction-fraction entry is
    sum_i ((g_i - c_i) / p_i)^2, with the normalised Gaussian from
    scipy.stats.truncnorm and the normalised Chebyshev polynomial written
    out."""
    x = synth.sample_gauss_cheb(4000, 72)
    th = [0.05, 0.97, 0.31, 0.21, -0.09]
    om, otop, _ = rfo.from_spec(workloads.spec_gauss_cheb())
    _, _, H, _ = om.nll_hess(otop, th, [x])
    mu, s, f, c1, c2 = th
    gpdf = stats.truncnorm.pdf(x, (-10 - mu) / s, (10 - mu) / s, loc=mu, scale=s)
    xp = x / 10.0
    cpdf = (1 + c1 * xp + c2 * (2 * xp * xp - 1)) / (20.0 * (1 - c2 / 3))
    p = f * gpdf + (1 - f) * cpdf
    np.testing.assert_allclose(H[2, 2], np.sum(((gpdf - cpdf) / p) ** 2), rtol=1e-11)


def test_oracle_hessian_rejects_leaves_without_second_derivatives():
    om, otop, _ = rfo.from_spec(workloads.spec_bwcb(K=64))
    with pytest.raises(RuntimeError):
        om.nll_hess(otop, workloads.truth_vector(synth.BWCB_TRUTH), [synth.sample_bw_cb(10, 4)])
