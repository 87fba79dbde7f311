"""Declarative model graphs of the benchmark workloads.

A spec is a list of ``(kind, name, inputs, attrs)`` entries in dependency
order; the last entry is the top PDF.  ``Graph.from_spec`` turns a spec into a
compiled-ready graph.  OBS attrs are the range (lo, hi); PARAM attrs are the
declared bounds (lo, hi); CONST attrs are (value,).  Parameter order (the
layout of theta) is the order of the PARAM entries.
"""
from . import synth


def spec_gauss_cheb(lo=-10.0, hi=10.0):
    """f * Gauss(x; mu, sigma) + (1 - f) * Chebyshev2(x; c1, c2) on [lo, hi];
    theta = (mu, sigma, f, c1, c2)."""
    return [
        ("obs", "x", [], [lo, hi]),
        ("param", "mu", [], [-5.0, 5.0]),
        ("param", "sigma", [], [0.05, 10.0]),
        ("param", "f", [], [0.0, 1.0]),
        ("param", "c1", [], [-1.0, 1.0]),
        ("param", "c2", [], [-1.0, 1.0]),
        ("gauss", "sig", ["x", "mu", "sigma"], []),
        ("cheb", "bkg", ["x", "c1", "c2"], []),
        ("add", "model", ["sig", "bkg", "f"], []),
    ]


def spec_gauss_cheb_extended(lo=-10.0, hi=10.0):
    """The extended 1-D mixture with yields: nu_s Gauss(x; mu, sigma) +
    nu_b Chebyshev2(x; c1, c2), fraction nu_s / (nu_s + nu_b), extended term
    on nu = nu_s + nu_b; theta = (mu, sigma, nu_s, nu_b, c1, c2)."""
    return [
        ("obs", "x", [], [lo, hi]),
        ("param", "mu", [], [-5.0, 5.0]),
        ("param", "sigma", [], [0.05, 10.0]),
        ("param", "nu_s", [], [0.0, 1e12]),
        ("param", "nu_b", [], [0.0, 1e12]),
        ("param", "c1", [], [-1.0, 1.0]),
        ("param", "c2", [], [-1.0, 1.0]),
        ("gauss", "sig", ["x", "mu", "sigma"], []),
        ("cheb", "bkg", ["x", "c1", "c2"], []),
        ("linear", "nu", ["nu_s", "nu_b"], [0.0, 1.0, 1.0]),
        ("ratio", "f", ["nu_s", "nu"], []),
        ("add", "mix", ["sig", "bkg", "f"], []),
        ("extended", "model", ["mix", "nu"], []),
    ]


def spec_poisson_gauss_cheb(nlo=0.0, nhi=40.0, lo=-10.0, hi=10.0):
    """Multiplicity n and mass x: f * Poisson(n; lam_s) Gauss(x; mu, sigma) +
    (1 - f) * Poisson(n; lam_b) Chebyshev2(x; c1, c2), each Poisson normalised
    over the integers nlo..nhi; theta = (lam_s, lam_b, mu, sigma, c1, c2, f)."""
    return [
        ("obs", "n", [], [nlo, nhi]),
        ("obs", "x", [], [lo, hi]),
        ("param", "lam_s", [], [0.1, 40.0]),
        ("param", "lam_b", [], [0.1, 40.0]),
        ("param", "mu", [], [-5.0, 5.0]),
        ("param", "sigma", [], [0.05, 10.0]),
        ("param", "c1", [], [-1.0, 1.0]),
        ("param", "c2", [], [-1.0, 1.0]),
        ("param", "f", [], [0.0, 1.0]),
        ("poisson", "sig_n", ["n", "lam_s"], []),
        ("gauss", "sig_x", ["x", "mu", "sigma"], []),
        ("prod", "sig", ["sig_n", "sig_x"], []),
        ("poisson", "bkg_n", ["n", "lam_b"], []),
        ("cheb", "bkg_x", ["x", "c1", "c2"], []),
        ("prod", "bkg", ["bkg_n", "bkg_x"], []),
        ("add", "model", ["sig", "bkg", "f"], []),
    ]


def spec_poisson(lo, hi, lam_lo=0.1, lam_hi=2000.0):
    """One Poisson leaf of a count n on the integers lo..hi; theta = (lam,)."""
    return [("obs", "n", [], [lo, hi]), ("param", "lam", [], [lam_lo, lam_hi]), ("poisson", "p", ["n", "lam"], [])]


def spec_decay_argus():
    """Signal: [decay(tau_s) (x) Gauss resolution(sigma_t, bias_t)](t) * Gauss(m; mu_m, sigma_m);
    background: exp(-t/tau_b) * ARGUS(m; m0 = 5.29 constant, c); fraction f.
    theta = (tau_s, sigma_t, bias_t, mu_m, sigma_m, tau_b, c, f)."""
    tlo, thi = synth.DECAY_T_RANGE
    mlo, mhi = synth.DECAY_M_RANGE
    return [
        ("obs", "t", [], [tlo, thi]),
        ("obs", "m", [], [mlo, mhi]),
        ("param", "tau_s", [], [0.1, 10.0]),
        ("param", "sigma_t", [], [0.005, 1.0]),
        ("param", "bias_t", [], [-0.5, 0.5]),
        ("param", "mu_m", [], [5.2, 5.29]),
        ("param", "sigma_m", [], [0.0005, 0.05]),
        ("param", "tau_b", [], [0.05, 5.0]),
        ("param", "c", [], [-100.0, 0.0]),
        ("param", "f", [], [0.0, 1.0]),
        ("const", "m0", [], [synth.ARGUS_M0]),
        ("decay_gauss", "sig_t", ["t", "tau_s", "sigma_t", "bias_t"], []),
        ("gauss", "sig_m", ["m", "mu_m", "sigma_m"], []),
        ("prod", "sig", ["sig_t", "sig_m"], []),
        ("exp", "bkg_t", ["t", "tau_b"], [0.0]),
        ("argus", "bkg_m", ["m", "m0", "c"], []),
        ("prod", "bkg", ["bkg_t", "bkg_m"], []),
        ("add", "model", ["sig", "bkg", "f"], []),
    ]


def spec_bwcb(surrogate=False, K=1024):
    """Signal: Breit-Wigner(M, Gamma) (x) Crystal Ball(sigma, alpha, n) by a K-point
    Gauss-Legendre rule on the resolution window (or the MLP surrogate of its
    log density), background exp(lam x); fraction f of signal.
    theta = (M, Gamma, sigma, alpha, n, lam, f)."""
    lo, hi = synth.BWCB_RANGE
    spec = [
        ("obs", "x", [], [lo, hi]),
        ("param", "M", [], [85.0, 97.0]),
        ("param", "Gamma", [], [0.5, 6.0]),
        ("param", "sigma", [], [0.5, 3.0]),
        ("param", "alpha", [], [0.5, 3.0]),
        ("param", "n", [], [1.0, 10.0]),
        ("param", "lam", [], [-0.2, 0.2]),
        ("param", "f", [], [0.0, 1.0]),
    ]
    if surrogate:
        box = [v for b in synth.BWCB_MLP_BOX for v in b]
        spec.append(("mlp", "sig", ["x", "M", "Gamma", "sigma", "alpha", "n"], box + [float(K)]))
    else:
        spec.append(("numconv_bw_cb", "sig", ["x", "M", "Gamma", "sigma", "alpha", "n"],
                     [synth.BWCB_WINDOW[0], synth.BWCB_WINDOW[1], float(K)]))
    spec += [
        ("exp", "bkg", ["x", "lam"], [1.0]),
        ("add", "model", ["sig", "bkg", "f"], []),
    ]
    return spec


def spec_two_gauss_extended(lo=-10.0, hi=10.0):
    """nu1 Gauss(x; mu1, s1) + nu2 Gauss(x; mu2, s2), extended with
    nu = nu1 + nu2; theta = (mu1, s1, mu2, s2, nu1, nu2).  Between and beyond
    two narrow peaks the density falls far below FP32's tail threshold."""
    return [
        ("obs", "x", [], [lo, hi]),
        ("param", "mu1", [], [-5.0, 5.0]),
        ("param", "s1", [], [0.05, 5.0]),
        ("param", "mu2", [], [-5.0, 5.0]),
        ("param", "s2", [], [0.05, 5.0]),
        ("param", "nu1", [], [0.0, 1e12]),
        ("param", "nu2", [], [0.0, 1e12]),
        ("gauss", "g1", ["x", "mu1", "s1"], []),
        ("gauss", "g2", ["x", "mu2", "s2"], []),
        ("linear", "nu", ["nu1", "nu2"], [0.0, 1.0, 1.0]),
        ("ratio", "f", ["nu1", "nu"], []),
        ("add", "mix", ["g1", "g2", "f"], []),
        ("extended", "model", ["mix", "nu"], []),
    ]


def spec_decay_leaf():
    """One decay (x) Gaussian resolution leaf on t in [0, 10]; theta = (tau, s, b)."""
    tlo, thi = synth.DECAY_T_RANGE
    return [
        ("obs", "t", [], [tlo, thi]),
        ("param", "tau", [], [0.1, 10.0]),
        ("param", "s", [], [0.005, 1.0]),
        ("param", "b", [], [-0.5, 0.5]),
        ("decay_gauss", "d", ["t", "tau", "s", "b"], []),
    ]


def spec_gauss_sum(k=5, lo=-10.0, hi=10.0):
    """A sum of k Gaussians with their own means and widths and k - 1
    fractions; theta = (mu_1, s_1, ..., mu_k, s_k, f_1, ..., f_{k-1})."""
    spec = [("obs", "x", [], [lo, hi])]
    for j in range(k):
        spec += [("param", "mu%d" % j, [], [-8.0, 8.0]), ("param", "s%d" % j, [], [0.05, 5.0])]
    spec += [("param", "f%d" % j, [], [0.0, 1.0]) for j in range(k - 1)]
    spec += [("gauss", "g%d" % j, ["x", "mu%d" % j, "s%d" % j], []) for j in range(k)]
    spec.append(("add", "model", ["g%d" % j for j in range(k)] + ["f%d" % j for j in range(k - 1)], []))
    return spec


def truth_vector(truth):
    return [float(v) for v in truth.values()]


def spec_shared_sum(tree=False, lo=-10.0, hi=10.0):
    """One Gaussian peak G shared by two sums (a graph, not a tree):
    g (f1 G + (1 - f1) C) + (1 - g) (f2 G + (1 - f2) E) on [lo, hi], with
    G = Gauss(x; mu, sigma), C = Chebyshev2(x; c1, c2), E = exp(lam x);
    theta = (mu, sigma, f1, f2, g, c1, c2, lam).  tree=True gives the same
    model with the peak written twice."""
    return [
        ("obs", "x", [], [lo, hi]),
        ("param", "mu", [], [-5.0, 5.0]),
        ("param", "sigma", [], [0.05, 10.0]),
        ("param", "f1", [], [0.0, 1.0]),
        ("param", "f2", [], [0.0, 1.0]),
        ("param", "g", [], [0.0, 1.0]),
        ("param", "c1", [], [-1.0, 1.0]),
        ("param", "c2", [], [-1.0, 1.0]),
        ("param", "lam", [], [-1.0, 1.0]),
        ("gauss", "peak", ["x", "mu", "sigma"], []),
    ] + ([("gauss", "peak2", ["x", "mu", "sigma"], [])] if tree else []) + [
        ("cheb", "poly", ["x", "c1", "c2"], []),
        ("exp", "slope", ["x", "lam"], [1.0]),
        ("add", "m1", ["peak", "poly", "f1"], []),
        ("add", "m2", ["peak2" if tree else "peak", "slope", "f2"], []),
        ("add", "model", ["m1", "m2", "g"], []),
    ]


def spec_shared_prod(tree=False, lo=-10.0, hi=10.0):
    """One Gaussian in x shared by two products (a graph, not a tree):
    f Gx Gy + (1 - f) Gx Cy on [lo, hi]^2, with Gx = Gauss(x; mux, sx),
    Gy = Gauss(y; muy, sy), Cy = Chebyshev2(y; c1, c2);
    theta = (mux, sx, muy, sy, f, c1, c2).  tree=True gives the same model
    with Gx written twice."""
    return [
        ("obs", "x", [], [lo, hi]),
        ("obs", "y", [], [lo, hi]),
        ("param", "mux", [], [-5.0, 5.0]),
        ("param", "sx", [], [0.05, 10.0]),
        ("param", "muy", [], [-5.0, 5.0]),
        ("param", "sy", [], [0.05, 10.0]),
        ("param", "f", [], [0.0, 1.0]),
        ("param", "c1", [], [-1.0, 1.0]),
        ("param", "c2", [], [-1.0, 1.0]),
        ("gauss", "gx", ["x", "mux", "sx"], []),
    ] + ([("gauss", "gx2", ["x", "mux", "sx"], [])] if tree else []) + [
        ("gauss", "gy", ["y", "muy", "sy"], []),
        ("cheb", "cy", ["y", "c1", "c2"], []),
        ("prod", "s", ["gx", "gy"], []),
        ("prod", "b", ["gx2" if tree else "gx", "cy"], []),
        ("add", "model", ["s", "b", "f"], []),
    ]
