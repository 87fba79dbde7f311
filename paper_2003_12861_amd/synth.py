"""Seeded synthetic inputs for the likelihood workloads.

This module only draws random numbers: it holds no likelihood, normalisation
or gradient arithmetic, and it is the one module that the GPU path and the
oracle both consume.  Every sampler is exact for the model it names and uses
``numpy.random.default_rng(seed)`` (PCG64), so a seed fixes every value.

Data precision: values are drawn in FP64, rounded once to FP32 (round to
nearest even), and only then checked against the observable range (and the
ARGUS endpoint); draws that fail are replaced.  The returned FP64 arrays hold
FP32-representable values, so the FP32 and FP64 paths and the oracle all see
bit-identical events.
"""
import math

import numpy as np


def _fill(n, seed, draw, rng=None):
    """Collect n accepted FP32-representable draws from draw(rng, m)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    parts, have = [], 0
    while have < n:
        m = max(1024, int(1.15 * (n - have)) + 64)
        got = draw(rng, m)
        parts.append(got)
        have += len(got if not isinstance(got, tuple) else got[0])
    if n == 0:
        return None
    if isinstance(parts[0], tuple):
        return tuple(np.concatenate([p[k] for p in parts])[:n] for k in range(len(parts[0])))
    return np.concatenate(parts)[:n]


def _mixture(n, seed, f, draw_sig, draw_bkg):
    """Exact sampler of f * sig + (1 - f) * bkg with both components normalised
    over the box: n_sig ~ Binomial(n, f), each component drawn truncated to the
    box (rejection inside the component), then a random permutation."""
    rng = np.random.default_rng(seed)
    ns = int(rng.binomial(n, f))
    a = _fill(ns, None, draw_sig, rng) if ns else None
    b = _fill(n - ns, None, draw_bkg, rng) if n - ns else None
    perm = rng.permutation(n)
    if isinstance(a if a is not None else b, tuple):
        k = len(a if a is not None else b)
        cols = [np.concatenate([c for c in (a[j] if a is not None else None, b[j] if b is not None else None)
                                if c is not None]) for j in range(k)]
        return tuple(c[perm] for c in cols)
    return np.concatenate([c for c in (a, b) if c is not None])[perm]


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _inside(a, lo, hi):
    return (a >= lo) & (a <= hi)


# --------------------------------------------------------------------------
# 1-D: fraction f of a Gaussian, 1-f of an order-2 Chebyshev polynomial
# --------------------------------------------------------------------------
GAUSS_CHEB_TRUTH = dict(mu=0.0, sigma=1.0, f=0.3, c1=0.2, c2=-0.1)
GAUSS_CHEB_RANGE = (-10.0, 10.0)


def sample_gauss_cheb(n, seed, mu=0.0, sigma=1.0, f=0.3, c1=0.2, c2=-0.1,
                      lo=-10.0, hi=10.0):
    """Mixture sampled exactly (component counts ~ Binomial(n, f)); Gaussian by
    rejection of N(mu, sigma) outside [lo, hi]; polynomial 1 + c1 T1 + c2 T2 by
    accept-reject against its maximum over [-1, 1] (mapped onto [lo, hi])."""
    # maximum of the polynomial on [-1,1]: at an end point or the vertex
    cand = [-1.0, 1.0]
    if c2 != 0.0:
        v = -c1 / (4.0 * c2)
        if -1.0 <= v <= 1.0:
            cand.append(v)
    hmax = max(1.0 + c1 * t + c2 * (2 * t * t - 1) for t in cand)

    def sig(rng, m):
        x = _f32(rng.normal(mu, sigma, m))
        return x[_inside(x, lo, hi)]

    def bkg(rng, m):
        t = rng.uniform(-1.0, 1.0, m)
        acc = rng.random(m) * hmax <= 1.0 + c1 * t + c2 * (2 * t * t - 1)
        x = _f32(0.5 * (hi - lo) * t + 0.5 * (hi + lo))
        return x[acc & _inside(x, lo, hi)]

    return _mixture(n, seed, f, sig, bkg)


# --------------------------------------------------------------------------
# 2-D with a count: per-event multiplicity n (Poisson) and a mass x;
# signal Poisson(n; lam_s) Gauss(x; mu, sigma), background Poisson(n; lam_b)
# times the order-2 Chebyshev polynomial, fraction f of signal
# --------------------------------------------------------------------------
POISSON_TRUTH = dict(lam_s=12.0, lam_b=5.0, mu=0.0, sigma=1.0, c1=0.2, c2=-0.1, f=0.3)
POISSON_N_RANGE = (0.0, 40.0)


def sample_poisson_gauss_cheb(n, seed, lam_s=12.0, lam_b=5.0, mu=0.0, sigma=1.0, c1=0.2, c2=-0.1, f=0.3,
                              nlo=0.0, nhi=40.0, lo=-10.0, hi=10.0):
    """Returns (counts, x): the component's count by numpy's Poisson draw,
    rejected outside [nlo, nhi]; x as in sample_gauss_cheb."""
    cand = [-1.0, 1.0]
    if c2 != 0.0:
        v = -c1 / (4.0 * c2)
        if -1.0 <= v <= 1.0:
            cand.append(v)
    hmax = max(1.0 + c1 * t + c2 * (2 * t * t - 1) for t in cand)

    def sig(rng, m):
        k = rng.poisson(lam_s, m).astype(np.float64)
        x = _f32(rng.normal(mu, sigma, m))
        ok = _inside(k, nlo, nhi) & _inside(x, lo, hi)
        return k[ok], x[ok]

    def bkg(rng, m):
        k = rng.poisson(lam_b, m).astype(np.float64)
        t = rng.uniform(-1.0, 1.0, m)
        acc = rng.random(m) * hmax <= 1.0 + c1 * t + c2 * (2 * t * t - 1)
        x = _f32(0.5 * (hi - lo) * t + 0.5 * (hi + lo))
        ok = acc & _inside(k, nlo, nhi) & _inside(x, lo, hi)
        return k[ok], x[ok]

    if n == 0:
        return np.zeros(0), np.zeros(0)
    return _mixture(n, seed, f, sig, bkg)


def jitter_gauss_cheb(k, truth=GAUSS_CHEB_TRUTH, base_seed=1000):
    """Parameter point k of the +-10% jitter: theta_j = truth_j + 0.1 s_j U(-1,1),
    s_j = |truth_j| (1 for a zero truth value), one uniform per parameter in the
    order (mu, sigma, f, c1, c2), seed base_seed + k."""
    rng = np.random.default_rng(base_seed + k)
    out = []
    for name in ("mu", "sigma", "f", "c1", "c2"):
        t = truth[name]
        s = abs(t) if t != 0 else 1.0
        out.append(t + 0.1 * s * rng.uniform(-1.0, 1.0))
    return np.array(out)


# --------------------------------------------------------------------------
# 2-D: decay (x) resolution times Gaussian mass, over exponential times ARGUS
# --------------------------------------------------------------------------
DECAY_TRUTH = dict(tau_s=1.5, sigma_t=0.05, bias_t=0.0, mu_m=5.28, sigma_m=0.003,
                   tau_b=0.4, c=-20.0, f=0.2)
DECAY_T_RANGE = (0.0, 10.0)
DECAY_M_RANGE = (5.2, 5.29)
ARGUS_M0 = 5.29


def sample_decay_argus(n, seed, tau_s=1.5, sigma_t=0.05, bias_t=0.0, mu_m=5.28,
                       sigma_m=0.003, tau_b=0.4, c=-20.0, f=0.2, m0=ARGUS_M0,
                       t_range=DECAY_T_RANGE, m_range=DECAY_M_RANGE):
    """Mixture sampled exactly (component counts ~ Binomial(n, f)).
    Signal: t = Exp(tau_s) + N(bias_t, sigma_t), m = N(mu_m, sigma_m).
    Background: t = Exp(tau_b); m = m0 sqrt(1 - U) with U ~ Gamma(3/2, 1/k),
    k = -c (the ARGUS law with power 1/2 in the variable U = 1 - (m/m0)^2).
    Draws outside the box, or with m >= m0 after FP32 rounding, are redrawn
    within their component."""
    tlo, thi = t_range
    mlo, mhi = m_range
    k = -c

    def sig(rng, mm):
        t = _f32(rng.exponential(tau_s, mm) + rng.normal(bias_t, sigma_t, mm))
        m = _f32(rng.normal(mu_m, sigma_m, mm))
        keep = _inside(t, tlo, thi) & _inside(m, mlo, mhi) & (m < m0)
        return t[keep], m[keep]

    def bkg(rng, mm):
        t = _f32(rng.exponential(tau_b, mm))
        U = rng.gamma(1.5, 1.0 / k, mm)
        m = _f32(m0 * np.sqrt(np.clip(1.0 - U, 0.0, None)))
        keep = _inside(t, tlo, thi) & _inside(m, mlo, mhi) & (m < m0) & (U < 1.0)
        return t[keep], m[keep]

    return _mixture(n, seed, f, sig, bkg)


def jitter_decay(k, truth=DECAY_TRUTH, base_seed=3000):
    """theta*(1 + 0.01 U(-1,1)) per scale-type parameter; the two location
    parameters move additively: the resolution bias by +-0.001 (its truth is
    0) and the mass mean by +-0.001 GeV (1% of 5.28 GeV would be 17 widths and
    leave the mass range).  Order as DECAY_TRUTH."""
    rng = np.random.default_rng(base_seed + k)
    out = []
    for name, t in truth.items():
        u = rng.uniform(-1.0, 1.0)
        out.append(t + 0.001 * u if name in ("bias_t", "mu_m") else t * (1.0 + 0.01 * u))
    return np.array(out)


# --------------------------------------------------------------------------
# Breit-Wigner (x) Crystal Ball signal over an exponential background
# --------------------------------------------------------------------------
BWCB_TRUTH = dict(M=91.19, Gamma=2.5, sigma=1.5, alpha=1.5, n=3.0, lam=-0.02, f=0.8)
BWCB_RANGE = (60.0, 120.0)
BWCB_WINDOW = (-30.0, 30.0)
# box of the surrogate's raw inputs (x, M, Gamma, sigma, alpha, n)
BWCB_BOX = ((60.0, 120.0), (89.19, 93.19), (1.5, 3.5), (0.5, 3.0), (0.5, 3.0), (1.0, 10.0))
# the network's first input is x - M, on the box of x - M implied by the above
BWCB_MLP_BOX = ((60.0 - 93.19, 120.0 - 89.19),) + BWCB_BOX[1:]


def _sample_cb(rng, m, sigma, alpha, n, ylo, yhi):
    """Crystal Ball (mean 0, low tail) restricted to [ylo, yhi]: accept-reject
    of a uniform proposal against the shape's maximum (1, at y = 0)."""
    out, have = [], 0
    while have < m:
        y = rng.uniform(ylo, yhi, 4 * m)
        z = y / sigma
        A = (n / alpha) ** n * math.exp(-0.5 * alpha * alpha)
        B = n / alpha - alpha
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            shape = np.where(z > -alpha, np.exp(-0.5 * z * z), A * np.power(np.maximum(B - z, 1e-300), -n))
        acc = rng.random(4 * m) <= shape
        out.append(y[acc])
        have += int(acc.sum())
    return np.concatenate(out)[:m]


def sample_bw_cb(n, seed, M=91.19, Gamma=2.5, sigma=1.5, alpha=1.5, nn=3.0, lam=-0.02,
                 f=0.8, x_range=BWCB_RANGE, window=BWCB_WINDOW):
    """Mixture sampled exactly (component counts ~ Binomial(n, f)).  Signal:
    x = M + (Gamma/2) tan(pi (u - 1/2)) + y with y ~ Crystal Ball on the window,
    redrawn until inside the range; background: exp(lam x) on the range by
    inverse CDF."""
    lo, hi = x_range

    def sig(rng, m):
        y = _sample_cb(rng, m, sigma, alpha, nn, window[0], window[1])
        x = _f32(M + 0.5 * Gamma * np.tan(np.pi * (rng.random(m) - 0.5)) + y)
        return x[_inside(x, lo, hi)]

    def bkg(rng, m):
        u = rng.random(m)
        if abs(lam) < 1e-12:
            xb = lo + (hi - lo) * u
        else:
            xb = lo + np.log1p(u * np.expm1(lam * (hi - lo))) / lam
        x = _f32(xb)
        return x[_inside(x, lo, hi)]

    return _mixture(n, seed, f, sig, bkg)


def _sample_cb_vec(rng, sigma, alpha, n, ylo, yhi):
    """Crystal Ball draws with per-row parameters (accept-reject, uniform proposal)."""
    m = sigma.size
    out = np.empty(m)
    todo = np.arange(m)
    while todo.size:
        y = rng.uniform(ylo, yhi, todo.size)
        s, a, nn = sigma[todo], alpha[todo], n[todo]
        z = y / s
        A = (nn / a) ** nn * np.exp(-0.5 * a * a)
        B = nn / a - a
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            shape = np.where(z > -a, np.exp(-0.5 * z * z), A * np.power(np.maximum(B - z, 1e-300), -nn))
        acc = rng.random(todo.size) <= shape
        out[todo[acc]] = y[acc]
        todo = todo[~acc]
    return out


def surrogate_design(n, seed=7, box=BWCB_BOX, frac_signal=0.5, window=BWCB_WINDOW, focus=None, frac_focus=0.0):
    """Training inputs of the surrogate: the five parameters from a scrambled
    Sobol sequence over the box; x drawn, for a fraction frac_signal of the
    rows, from the signal law at that row's parameters (Breit-Wigner plus
    Crystal Ball, redrawn until inside x's range) and uniformly otherwise, so
    that the training points follow where events fall.  With a focus box (a
    sub-box of the parameters, same layout as box), a fraction frac_focus of
    the rows takes its parameters from a second Sobol sequence over it, rows
    of the two sequences interleaved in a seeded order."""
    q = sobol_design(n, seed=seed, box=box)
    nf = int(round(frac_focus * n)) if focus is not None else 0
    if nf > 0:
        q[:nf, 1:] = sobol_design(nf, seed=seed + 101, box=focus)[:, 1:]
        q = q[np.random.default_rng(seed + 2).permutation(n)]
    rng = np.random.default_rng(seed + 1)
    lo, hi = box[0]
    xs = rng.uniform(lo, hi, n)
    sig = rng.random(n) < frac_signal
    idx = np.nonzero(sig)[0]
    todo = idx
    while todo.size:
        M, G, s, a, nn = (q[todo, j] for j in range(1, 6))
        y = _sample_cb_vec(rng, s, a, nn, window[0], window[1])
        x = M + 0.5 * G * np.tan(np.pi * (rng.random(todo.size) - 0.5)) + y
        ok = (x >= lo) & (x <= hi)
        xs[todo[ok]] = x[ok]
        todo = todo[~ok]
    q[:, 0] = xs
    return q


def sobol_design(n, seed=7, box=BWCB_BOX, skip=0):
    """Scrambled 6-D Sobol points (x, M, Gamma, sigma, alpha, n) in the box."""
    from scipy.stats import qmc
    eng = qmc.Sobol(d=6, scramble=True, seed=seed)
    if skip:
        eng.fast_forward(skip)
    u = eng.random(n)
    lo = np.array([b[0] for b in box])
    hi = np.array([b[1] for b in box])
    return lo + u * (hi - lo)


# --------------------------------------------------------------------------
# Binned templates: channels x samples x bins, +-1 sigma variations
# --------------------------------------------------------------------------
def make_binned(seed=5, C=200, S=4, B=100, J=60, delta_max=0.05):
    """lambda_cs ~ log-uniform[50, 5000]; T_csb ~ Poisson(lambda_cs) (>= 1);
    T+- = T (1 +- delta+-), delta+- ~ U(0, delta_max) per (c, s, j, b);
    observed n_cb ~ Poisson(sum_s T_csb) (signal strength 1, nuisances 0).
    Returns FP64 arrays T[C,S,B], Tp/Tm[C,S,J,B], nobs[C,B]."""
    rng = np.random.default_rng(seed)
    lam = np.exp(rng.uniform(np.log(50.0), np.log(5000.0), (C, S)))
    T = np.maximum(rng.poisson(lam[:, :, None], (C, S, B)), 1).astype(np.float64)
    dp = rng.uniform(0.0, delta_max, (C, S, J, B))
    dm = rng.uniform(0.0, delta_max, (C, S, J, B))
    Tp = T[:, :, None, :] * (1.0 + dp)
    Tm = T[:, :, None, :] * (1.0 - dm)
    nobs = rng.poisson(T.sum(axis=1)).astype(np.float64)
    return dict(T=T, Tp=Tp, Tm=Tm, nobs=nobs)
