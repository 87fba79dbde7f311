"""The Hessian kernel (rf_nll_grad_hess: NLL, gradient and Hessian in one
fused pass, per-event arithmetic in FP64 whatever the columns' dtype) against
the oracle's second-order forward mode, and the fit's uncertainties taken
from it.

Bars: NLL relative 1e-9 (FP64 per-event arithmetic in both precision forms),
gradient 1e-9 of the oracle's scale sum_i |d(-log p_i)/d theta|, Hessian
entries 1e-9 of sqrt(H_jj H_kk) (the scale on which uncertainties and
correlations depend), with a floor of 1e-13 of the largest entry for entries
whose diagonal cancels to nothing."""
import numpy as np
import pytest

from helpers import build_pair, oracle_hess_threads, rel, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")


def spec_product_ratio():
    """Two Gaussians with widths tied by a product function s2 = k s1 and a
    fraction that is a ratio of yields; theta = (mu1, s1, mu2, k, y1, y2)."""
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


def spec_bw_exp():
    return [("obs", "x", [], [60.0, 120.0]), ("param", "M", [], [85.0, 97.0]), ("param", "G", [], [0.5, 6.0]),
            ("param", "lam", [], [-0.2, 0.2]), ("param", "f", [], [0.0, 1.0]),
            ("bw", "s", ["x", "M", "G"], []), ("exp", "b", ["x", "lam"], [1.0]), ("add", "model", ["s", "b", "f"], [])]


def _two_peaks(n, seed, s2=0.5):
    rng = np.random.default_rng(seed)
    x = np.where(rng.random(n) < 0.4, rng.normal(-2.0, 0.5, n), rng.normal(2.0, s2, n))
    return synth._f32(np.clip(x, -9.9, 9.9))


CASES = {
    "gauss_cheb": (workloads.spec_gauss_cheb, lambda n: [synth.sample_gauss_cheb(n, 81)],
                   [0.05, 0.97, 0.31, 0.21, -0.09]),
    "decay_argus": (workloads.spec_decay_argus, lambda n: list(synth.sample_decay_argus(n, 82)),
                    list(synth.jitter_decay(5))),
    "two_gauss_ext": (workloads.spec_two_gauss_extended, lambda n: [_two_peaks(n, 83)],
                      lambda n: [-1.98, 0.51, 2.01, 0.49, 0.41 * n, 0.6 * n + 3.0]),
    "gauss_cheb_ext": (workloads.spec_gauss_cheb_extended, lambda n: [synth.sample_gauss_cheb(n, 84)],
                       lambda n: [0.02, 1.01, 0.29 * n + 1, 0.7 * n, 0.19, -0.11]),
    "product_ratio": (spec_product_ratio, lambda n: [_two_peaks(n, 85, s2=1.0)],
                      lambda n: [-1.98, 0.51, 2.01, 1.9, 0.4 * n, 0.6 * n]),
    "bw_exp": (spec_bw_exp, lambda n: [synth._f32(np.random.default_rng(86).uniform(60, 120, n))],
               [91.1, 2.6, -0.021, 0.7]),
    "gauss_sum": (lambda: workloads.spec_gauss_sum(5), lambda n: [_two_peaks(n, 87)],
                  [-3.0, 0.8, -1.0, 0.5, 0.0, 1.2, 1.5, 0.6, 3.0, 2.0, 0.2, 0.2, 0.2, 0.2]),
    "decay_leaf": (workloads.spec_decay_leaf, lambda n: [synth.sample_decay_argus(n, 88, bias_t=0.4, f=1.0)[0]],
                   [1.5, 0.05, 0.4]),
}


def _check(prog, om, otop, th, cols, w=None, label=""):
    nll, g, H, nb = prog.nll_grad_hess(th)
    onll, og, oH, onb = om.nll_hess(otop, th, cols, weights=w)
    _, _, oga, _ = om.nll_ex(otop, th, cols, weights=w)
    assert nb == onb == 0, label
    # the NLL bar relative to the magnitudes of its parts (an extended NLL's
    # event sum and yield term partly cancel)
    v = om.values(otop, th, cols)
    wa = np.abs(w) if w is not None else np.ones(v.size)
    scale = float(np.sum(wa * np.abs(np.log(v)))) + abs(onll)
    assert abs(nll - onll) <= 1e-9 * scale, (label, nll, onll)
    assert scaled_grad_err(g, og, oga).max() <= 1e-9, (label, g, og)
    # entries to 1e-9 of sqrt(H_jj H_kk); entries that cancel to nothing
    # (a diagonal near zero: one event and six parameters) to FP64 rounding
    # of the largest entry
    s = np.sqrt(np.abs(np.outer(np.diag(oH), np.diag(oH)))) + 1e-4 * np.abs(oH).max()
    err = np.abs(H - oH) / s
    assert err.max() <= 1e-9, (label, err.max(), np.unravel_index(np.argmax(err), err.shape), H, oH)
    assert np.array_equal(H, H.T) or np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    return nll, g, H


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("n", [1, 1000, 100_003])
def test_hessian_vs_oracle(case, prec, n):
    print("case hessian %s prec=%d n=%d" % (case, prec, n), flush=True)
    make_spec, make_cols, th = CASES[case]
    th = th(n) if callable(th) else th
    spec = make_spec()
    cols = make_cols(n)
    prog, (om, otop, _) = build_pair(spec, prec, api)
    prog.bind(to_dev(cols, prec, api))
    nll, g, H = _check(prog, om, otop, th, cols, label=case)
    # the same NLL and gradient as the fused kernel, to its own precision
    n2, g2, _ = prog.nll_grad(th)
    assert rel(n2, nll) <= (1e-12 if prec == api.FP64 else 1e-6)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("case", ["gauss_cheb", "two_gauss_ext", "gauss_cheb_ext"])
def test_hessian_weighted(case, prec):
    print("case hessian weighted %s prec=%d" % (case, prec), flush=True)
    n = 50_001
    make_spec, make_cols, th = CASES[case]
    cols = make_cols(n)
    w = synth._f32(np.random.default_rng(89).uniform(0.5, 2.0, n))
    th = th(int(np.sum(w))) if callable(th) else th
    prog, (om, otop, _) = build_pair(make_spec(), prec, api, weighted=True)
    prog.bind(to_dev(cols + [w], prec, api))
    _check(prog, om, otop, th, cols, w=w, label=case)


def test_hessian_full_size():
    """The 1e7-event 1-D model against the oracle over all events (threads)."""
    n = 10_000_000
    x = synth.sample_gauss_cheb(n, 2)
    spec = workloads.spec_gauss_cheb()
    th = [0.0, 1.0, 0.3, 0.2, -0.1]
    print("case hessian full size: oracle", flush=True)
    onll, og, oH, onb = oracle_hess_threads(spec, th, [x])
    for prec in (api.FP64, api.FP32):
        prog, _ = build_pair(spec, prec, api)
        prog.bind(to_dev([x], prec, api))
        nll, g, H, nb = prog.nll_grad_hess(th)
        assert nb == onb == 0
        assert rel(nll, onll) <= 1e-9
        s = np.sqrt(np.abs(np.outer(np.diag(oH), np.diag(oH))))
        assert (np.abs(H - oH) / s).max() <= 1e-9, (H, oH)


def test_hessian_unsupported_leaves_and_bad_events():
    prog, _ = build_pair(workloads.spec_bwcb(K=100), api.FP64, api)
    prog.bind(to_dev([synth.sample_bw_cb(100, 4)], api.FP64, api))
    with pytest.raises(api.RfError) as e:
        prog.nll_grad_hess(workloads.truth_vector(synth.BWCB_TRUTH))
    assert e.value.code == -1
    # an event with p <= 0: infinite NLL, NaN gradient and Hessian, the count
    x = np.linspace(-10, 10, 1001)
    th = [0.0, 1.0, 0.0, 1.5, 0.0]
    spec = [e if e[1] != "c1" else ("param", "c1", [], [-5.0, 5.0]) for e in workloads.spec_gauss_cheb()]
    prog, (om, otop, _) = build_pair(spec, api.FP64, api)
    prog.bind(to_dev([x], api.FP64, api))
    nll, g, H, nb = prog.nll_grad_hess(th)
    assert np.isinf(nll) and nb == om.nll(otop, th, [x])[2] > 0 and np.all(np.isnan(H))


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_fit_sigma_from_hessian(prec):
    """rf_fit_bfgs takes its uncertainties from the Hessian kernel: they equal
    the inverse of the oracle's Hessian at the fitted point, and those from
    central differences of the analytic gradient (the fallback for leaves
    without second derivatives) to 1e-3 relative."""
    n = 200_000
    t, m = synth.sample_decay_argus(n, 90)
    spec = workloads.spec_decay_argus()
    prog, (om, otop, _) = build_pair(spec, prec, api)
    prog.bind(to_dev([t, m], prec, api))
    th0 = list(synth.jitter_decay(7))
    th, sig, info = prog.fit(th0, edm_tol=1e-7, max_iter=500)
    assert info["converged"], info
    _, _, oH, _ = om.nll_hess(otop, th, [t, m])
    osig = np.sqrt(np.diag(np.linalg.inv(oH)))
    np.testing.assert_allclose(sig, osig, rtol=1e-6 if prec == api.FP64 else 1e-4)
    # central differences of the GPU gradient, a tenth of sigma apart
    P = len(th)
    Hf = np.empty((P, P))
    for k in range(P):
        h = 0.1 * sig[k]
        tp, tm = np.array(th), np.array(th)
        tp[k] += h
        tm[k] -= h
        Hf[:, k] = (prog.nll_grad(tp)[1] - prog.nll_grad(tm)[1]) / (2 * h)
    fsig = np.sqrt(np.diag(np.linalg.inv(0.5 * (Hf + Hf.T))))
    np.testing.assert_allclose(sig, fsig, rtol=1e-3)
