"""Combined likelihoods on the GPU (rf_sum_*): terms sharing parameters and
Gaussian constraints, against the oracle's definition of the combination
(oracle.rfo.combined_nll) and against the whole-sample program."""
import numpy as np
import pytest

from helpers import rel, scaled_grad_err, to_dev
from oracle import rfo
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")
from test_gpu_binned import _grad_scale, _logs  # noqa: E402

TOL = {api.FP64: 1e-9, api.FP32: 1e-6}
TH = np.array([0.1, 1.1, 0.3, 0.2, -0.1])


def _prog(spec, cols, prec):
    p = api.Program(api.Graph.from_spec(spec), precision=prec)
    p.bind(to_dev(cols, prec, api))
    return p


def _oracle_term(spec, cols):
    om, top, _ = rfo.from_spec(spec)

    def f(th):
        nll, g, ga, nb = om.nll_ex(top, th, cols)
        return nll, np.asarray(g), np.asarray(ga)
    return f


def _oracle_binned(d):
    Lp, Lm = _logs(d)

    def f(th):
        nll, g = rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], th)
        return nll, np.asarray(g), _grad_scale(d, Lp, Lm, th)
    return f


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_sum_split_equals_whole(prec):
    """The same model on two parts of a sample, combined with identity maps,
    against the oracle's combination and the program on the whole sample."""
    print("case sum split prec=%d" % prec, flush=True)
    x = synth.sample_gauss_cheb(30001, 7)
    spec = workloads.spec_gauss_cheb()
    whole = _prog(spec, [x], prec)
    a, b = _prog(spec, [x[:11000]], prec), _prog(spec, [x[11000:]], prec)
    s = api.Sum(5).add(a, range(5)).add(b, range(5))
    ident = list(range(5))
    terms = [(_oracle_term(spec, [x[:11000]]), ident), (_oracle_term(spec, [x[11000:]]), ident)]
    for th in (TH, synth.jitter_gauss_cheb(3)):
        nll, g, nb = s.nll_grad(th)
        assert nb == 0
        on, og, osc = rfo.combined_nll(terms, [], th)
        assert rel(nll, on) <= TOL[prec], (nll, on)
        assert scaled_grad_err(g, og, osc).max() <= TOL[prec]
        wn, wg, _ = whole.nll_grad(th)
        assert rel(nll, wn) <= TOL[prec]
        assert scaled_grad_err(g, wg, osc).max() <= TOL[prec]


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_sum_binned_and_unbinned_with_constraints(prec):
    """An unbinned mixture and a binned template model sharing one parameter
    (the binned model's signal strength is the mixture's fraction f), two
    Gaussian constraints (one on a parameter of each term); the binned
    model's FP32 terms set the 1e-6 bar."""
    print("case sum binned+unbinned prec=%d" % prec, flush=True)
    x = synth.sample_gauss_cheb(20001, 8)
    spec = workloads.spec_gauss_cheb()
    prog = _prog(spec, [x], prec)
    d = synth.make_binned(4, 3, 2, 10, 4)
    bn = api.Binned(d["T"], d["Tp"], d["Tm"], d["nobs"])
    bmap = [2, 5, 6, 7, 8]  # (mu_signal, alpha_1..alpha_4)
    cons = [(5, 0.1, 0.5), (0, 0.05, 0.2)]
    s = api.Sum(9).add(prog, range(5)).add(bn, bmap)
    for k, m, w in cons:
        s.constrain(k, m, w)
    terms = [(_oracle_term(spec, [x]), list(range(5))), (_oracle_binned(d), bmap)]
    rng = np.random.default_rng(5)
    for it in range(3):
        th = np.concatenate([TH, rng.uniform(-0.8, 0.8, 4)])
        th[2] = 0.3 + 0.05 * it
        nll, g, nb = s.nll_grad(th)
        assert nb == 0
        on, og, osc = rfo.combined_nll(terms, cons, th)
        assert rel(nll, on) <= 1e-6, (nll, on)
        assert scaled_grad_err(g, og, osc).max() <= 1e-6, scaled_grad_err(g, og, osc)
        # the shared parameter's gradient is the two terms' gradients added
        _, pg, _ = prog.nll_grad(th[:5])
        _, bg = bn.nll_grad(th[bmap])
        assert abs(g[2] - (pg[2] + bg[0])) <= 1e-12 * (abs(pg[2]) + abs(bg[0]))


def test_sum_constraints_only():
    print("case sum constraints only", flush=True)
    cons = [(0, 1.5, 0.3), (2, -0.5, 2.0), (0, 1.0, 1.0)]
    s = api.Sum(3)
    for c in cons:
        s.constrain(*c)
    th = np.array([1.2, 7.0, 0.25])
    nll, g, nb = s.nll_grad(th)
    on, og, _ = rfo.combined_nll([], cons, th)
    assert nb == 0 and abs(nll - on) <= 1e-15 * abs(on)
    np.testing.assert_allclose(g, og, rtol=1e-15, atol=0)
    assert g[1] == 0.0


def test_sum_repeat_and_streams():
    """Bit-identical results on repeat and on another stream."""
    print("case sum repeat", flush=True)
    x = synth.sample_gauss_cheb(50001, 9)
    spec = workloads.spec_gauss_cheb()
    a, b = _prog(spec, [x[:20000]], api.FP32), _prog(spec, [x[20000:]], api.FP64)
    s = api.Sum(6).add(a, [0, 1, 2, 3, 4]).add(b, [5, 1, 2, 3, 4]).constrain(5, 0.0, 0.1)
    th = np.array([0.1, 1.1, 0.3, 0.2, -0.1, -0.05])
    r0 = s.nll_grad(th)
    r1 = s.nll_grad(th)
    st = torch.cuda.Stream()
    r2 = s.nll_grad(th, stream=st)
    r3 = s.nll_grad(th)
    for r in (r1, r2, r3):
        assert r[0] == r0[0] and np.array_equal(r[1], r0[1])


def test_sum_fit_matches_whole_sample_fit():
    """Fitting the combination of two halves finds the whole-sample fit's
    minimum; its uncertainties (central differences of the gradient) match
    the whole-sample fit's (Hessian kernel)."""
    print("case sum fit", flush=True)
    x = synth.sample_gauss_cheb(40000, 10)
    spec = workloads.spec_gauss_cheb()
    whole = _prog(spec, [x], api.FP64)
    s = api.Sum(5).add(_prog(spec, [x[:25000]], api.FP64), range(5)).add(_prog(spec, [x[25000:]], api.FP64), range(5))
    start = [0.3, 0.8, 0.4, 0.1, 0.0]
    # tight convergence (EDM 1e-9: each fit within about 5e-5 sigma of the minimum)
    tw, sw, _, iw = whole.fit_ex(start, edm_tol=1e-9)
    ts, ss, _, info = s.fit(start, edm_tol=1e-9)
    assert info["converged"] and iw["converged"]
    assert np.all(np.abs(ts - tw) <= 1e-3 * sw), (ts, tw, sw)
    np.testing.assert_allclose(ss, sw, rtol=2e-3)


def test_sum_constrained_fit_against_scipy():
    """A fit with a tight constraint on sigma: the minimum of the combination
    as scipy's BFGS finds it on the oracle's combination."""
    from scipy.optimize import minimize
    print("case sum constrained fit", flush=True)
    x = synth.sample_gauss_cheb(8000, 11)
    spec = workloads.spec_gauss_cheb()
    cons = [(1, 0.9, 0.02)]
    s = api.Sum(5).add(_prog(spec, [x], api.FP64), range(5)).constrain(*cons[0])
    terms = [(_oracle_term(spec, [x]), list(range(5)))]
    start = np.array([0.2, 1.0, 0.35, 0.15, -0.05])
    th, sig, _, info = s.fit(start, edm_tol=1e-9)
    assert info["converged"]
    res = minimize(lambda t: rfo.combined_nll(terms, cons, t)[0], start, jac=lambda t: rfo.combined_nll(terms, cons, t)[1],
                   method="BFGS", options=dict(gtol=1e-8, maxiter=1000))
    assert np.all(np.abs(th - res.x) <= 2e-3 * sig), (th, res.x, sig)
    # the constraint pulls sigma to within a few widths of 0.9
    assert abs(th[1] - 0.9) < 0.1


def test_sum_nonfinite_term():
    """A term with events of p <= 0 makes the combination non-finite: nll =
    inf, grad NaN, n_bad the term's count."""
    print("case sum non-finite", flush=True)
    x = synth.sample_gauss_cheb(5000, 12)
    spec = workloads.spec_gauss_cheb()
    p = _prog(spec, [x], api.FP64)
    th = np.array([0.0, 1.0, 0.3, 1.0, -1.0])  # the polynomial is negative near x = -10
    pn, _, pb = p.nll_grad(th)
    assert pb > 0
    s = api.Sum(5).add(p, range(5))
    nll, g, nb = s.nll_grad(th)
    assert nll == np.inf and np.all(np.isnan(g)) and nb == pb


def test_sum_term_rebound_to_more_events():
    """A program re-bound to a larger sample gets a new result block; the
    combination follows it (against the oracle on the new sample)."""
    print("case sum rebind", flush=True)
    spec = workloads.spec_gauss_cheb()
    small, big = synth.sample_gauss_cheb(3000, 13), synth.sample_gauss_cheb(400001, 14)
    p = _prog(spec, [small], api.FP64)
    s = api.Sum(5).add(p, range(5))
    n0, _, _ = s.nll_grad(TH)
    assert rel(n0, rfo.combined_nll([(_oracle_term(spec, [small]), list(range(5)))], [], TH)[0]) <= 1e-9
    p.bind(to_dev([big], api.FP64, api))
    nll, g, nb = s.nll_grad(TH)
    on, og, osc = rfo.combined_nll([(_oracle_term(spec, [big]), list(range(5)))], [], TH)
    assert nb == 0 and rel(nll, on) <= 1e-9, (nll, on)
    assert scaled_grad_err(g, og, osc).max() <= 1e-9


def test_sum_full_size_combination():
    """At the combined benchmark's size and launch shape (the 1e7-event FP32
    mixture and the 200 x 4 x 100 binned model with 60 nuisances, 65 global
    parameters, the binned signal strength sharing the mixture's fraction, a
    constraint on the mean): the combination equals the terms' own results
    added plus the constraint, and each gradient entry the terms' entries
    mapped to it plus the constraint's, to rounding.  (Each term is checked
    against the oracle on its own at this size.)"""
    print("case sum full size", flush=True)
    spec = workloads.spec_gauss_cheb()
    p = _prog(spec, [synth.sample_gauss_cheb(10_000_000, 4)], api.FP32)
    d = synth.make_binned(5, 200, 4, 100, 60)
    bn = api.Binned(d["T"], d["Tp"], d["Tm"], d["nobs"])
    bmap = [2] + list(range(5, 65))
    w = 0.05
    s = api.Sum(65).add(p, range(5)).add(bn, bmap).constrain(0, 0.0, w)
    rng = np.random.default_rng(7)
    for it in range(2):
        th = np.concatenate([TH, rng.uniform(-0.5, 0.5, 60)])
        th[0] = 0.02 * (it + 1)
        nll, g, nb = s.nll_grad(th)
        pn, pg, pb = p.nll_grad(th[:5])
        bnl, bg = bn.nll_grad(th[bmap])
        assert nb == 0 and pb == 0
        cn, cg = 0.5 * (th[0] / w) ** 2, th[0] / w ** 2
        assert abs(nll - (pn + bnl + cn)) <= 1e-14 * (abs(pn) + abs(bnl) + cn), (nll, pn, bnl, cn)
        gref, sc = np.zeros(65), np.zeros(65)
        gref[:5] += pg
        sc[:5] += np.abs(pg)
        gref[bmap] += bg
        sc[bmap] += np.abs(bg)
        gref[0] += cg
        sc[0] += abs(cg)
        assert np.all(np.abs(g - gref) <= 1e-14 * sc + 1e-300), np.max(np.abs(g - gref) / (sc + 1e-300))


def test_sum_many_entries():
    """A larger sum: three binned models with 60 nuisances each, sharing the
    signal strength (181 global parameters, 183 gradient entries), against
    the oracle's combination; and one of them as a sum of its own."""
    print("case sum many entries", flush=True)
    ds = [synth.make_binned(20 + t, 3, 2, 10, 60) for t in range(3)]
    bns = [api.Binned(d["T"], d["Tp"], d["Tm"], d["nobs"]) for d in ds]
    maps = [[0] + list(range(1 + 60 * t, 61 + 60 * t)) for t in range(3)]
    s = api.Sum(181)
    for bn, m in zip(bns, maps):
        s.add(bn, m)
    s.constrain(0, 1.0, 0.2)
    rng = np.random.default_rng(11)
    th = np.concatenate([[1.05], rng.uniform(-0.5, 0.5, 180)])
    nll, g, nb = s.nll_grad(th)
    terms = [(_oracle_binned(d), m) for d, m in zip(ds, maps)]
    on, og, osc = rfo.combined_nll(terms, [(0, 1.0, 0.2)], th)
    assert nb == 0 and rel(nll, on) <= 1e-6, (nll, on)
    assert scaled_grad_err(g, og, osc).max() <= 1e-6
    one = api.Sum(61).add(bns[0], range(61))
    n1, g1, _ = one.nll_grad(th[maps[0]])
    o1, og1, osc1 = rfo.combined_nll([(_oracle_binned(ds[0]), list(range(61)))], [], th[maps[0]])
    assert rel(n1, o1) <= 1e-6 and scaled_grad_err(g1, og1, osc1).max() <= 1e-6
