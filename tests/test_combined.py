"""Combined likelihoods (terms sharing parameters, Gaussian constraints): the
oracle's definition pinned on the CPU, and the host-side checks of the
rf_sum_* entry points (no kernel is launched here)."""
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


# ---- host-side checks of the entry points (programs compiled without loading)
api = pytest.importorskip("paper_2003_12861_amd.api")


def _prog():
    return api.Program(api.Graph.from_spec(workloads.spec_gauss_cheb()), precision=api.FP64, load=False)


def test_sum_host_checks():
    s = api.Sum(6)
    p, q = _prog(), _prog()
    with pytest.raises(api.RfError, match="one index per parameter"):
        s.add(p, [0, 1, 2])
    with pytest.raises(api.RfError, match="outside"):
        s.add(p, [0, 1, 2, 3, 6])
    s.add(p, [0, 1, 2, 3, 4])
    with pytest.raises(api.RfError, match="already in this sum"):
        s.add(p, [0, 1, 2, 3, 4])
    s.add(q, [5, 1, 2, 3, 4])  # a second program sharing four parameters
    for k, m, w in ((6, 0.0, 1.0), (0, float("nan"), 1.0), (0, 0.0, 0.0), (0, 0.0, -1.0), (0, 0.0, float("inf"))):
        with pytest.raises(api.RfError):
            s.constrain(k, m, w)
    s.constrain(0, 0.0, 1.0)
    # bounds are the terms' (mu in [-5, 5]), checked before anything runs
    th = np.array([0.1, 1.0, 0.3, 0.2, -0.1, 0.0])
    for bad in ((0, 5.5), (5, -6.0), (1, float("nan")), (2, float("inf"))):
        t = th.copy()
        t[bad[0]] = bad[1]
        with pytest.raises(api.RfError) as e:
            s.nll_grad(t, stream=0)
        assert e.value.code == -2, e.value
    # global bounds that exclude a term's range
    s2 = api.Sum(5, lo=[6.0, 0, 0, -1, -1], hi=[7.0, 10, 1, 1, 1])
    with pytest.raises(api.RfError, match="do not overlap"):
        s2.add(_prog(), [0, 1, 2, 3, 4])
    with pytest.raises(api.RfError):
        api.Sum(3, lo=[0.0, 1.0, 2.0], hi=[1.0, 0.5, 3.0])
    with pytest.raises(api.RfError):
        api.Sum(257)
    api.Sum(256)  # a combination may have up to 256 global parameters


def test_sum_term_limit():
    s = api.Sum(5)
    progs = [_prog() for _ in range(17)]
    for p in progs[:16]:
        s.add(p, [0, 1, 2, 3, 4])
    with pytest.raises(api.RfError, match="at most 16"):
        s.add(progs[16], [0, 1, 2, 3, 4])
