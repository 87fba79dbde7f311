"""Combined likelihoods (terms sharing parameters, Gaussian constraints): the
oracle's definition pinned on the CPU."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import rfo
from paper_2003_12861_amd import synth, workloads

TH = [0.1, 1.1, 0.3, 0.2, -0.1]


def _term(spec, cols):
    om, top, _ = rfo.from_spec(spec)

    def f(th):
        nll, g, ga, nb = om.nll_ex(top, th, cols)
        assert nb == 0
        return nll, np.asarray(g), np.asarray(ga)
    return f


def test_oracle_split_sample_equals_whole():
    """The likelihood of a sample is the product of the likelihoods of its
    parts: the same model on two halves, combined with identity maps, equals
    the model on the whole sample (sum over terms, gradient scatter)."""
    x = synth.sample_gauss_cheb(20001, 5)
    spec = workloads.spec_gauss_cheb()
    whole = _term(spec, [x])
    a, b = _term(spec, [x[:7000]]), _term(spec, [x[7000:]])
    ident = list(range(5))
    n, g, s = rfo.combined_nll([(a, ident), (b, ident)], [], TH)
    n0, g0, s0 = whole(np.array(TH))
    assert abs(n - n0) <= 1e-12 * abs(n0)
    assert np.all(np.abs(g - g0) <= 1e-12 * s0)
    np.testing.assert_allclose(s, s0, rtol=1e-12)


def test_oracle_reordered_parameters():
    """A model whose parameters are declared in another order, mapped back to
    the global order, gives the original model's NLL and gradient (the
    gather into the term and the scatter out of it use the same map)."""
    x = synth.sample_gauss_cheb(5003, 6)
    spec = workloads.spec_gauss_cheb()
    params = [e for e in spec if e[0] == "param"]
    names = [e[1] for e in params]
    order = ["c2", "f", "mu", "c1", "sigma"]
    perm_spec = [e for e in spec if e[0] == "obs"] + [params[names.index(nm)] for nm in order] + \
        [e for e in spec if e[0] not in ("obs", "param")]
    index_map = [names.index(nm) for nm in order]
    n, g, s = rfo.combined_nll([(_term(perm_spec, [x]), index_map)], [], TH)
    n0, g0, s0 = _term(spec, [x])(np.array(TH))
    assert abs(n - n0) <= 1e-13 * abs(n0)
    assert np.all(np.abs(g - g0) <= 1e-13 * s0)


def test_oracle_constraint_is_the_gaussian_factor():
    """A constraint adds -log of a normal density less its normalisation
    (scipy), and its gradient matches central differences; two factors on one
    parameter add."""
    cons = [(1, 0.7, 0.25), (0, -1.0, 2.0), (1, 1.2, 0.5)]
    for th in ([0.3, 0.9], [-2.0, 0.1], [5.0, -3.0]):
        n, g, s = rfo.combined_nll([], cons, th)
        ref = -sum(norm.logpdf(th[k], m, w) + math.log(w * math.sqrt(2 * math.pi)) for k, m, w in cons)
        assert abs(n - ref) <= 1e-12 * max(1.0, abs(ref))
        h = 1e-6
        for k in range(2):
            tp, tm = list(th), list(th)
            tp[k] += h
            tm[k] -= h
            fd = (rfo.combined_nll([], cons, tp)[0] - rfo.combined_nll([], cons, tm)[0]) / (2 * h)
            assert abs(g[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (th, k, g[k], fd)
        assert np.all(s >= np.abs(g))
