"""The extended likelihood (RF_OP_EXTENDED with yields through RF_OP_FN_RATIO)
on the GPU against the oracle, and the fit property of its minimum."""
import numpy as np
import pytest

from helpers import build_pair, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")

TOL = {api.FP64: (1e-9, 1e-9), api.FP32: (1e-6, 1e-6)}


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("n", [1, 100_003])
def test_extended_parity(prec, n):
    print("case extended n=%d prec=%d" % (n, prec), flush=True)
    x = synth.sample_gauss_cheb(n, 31)
    th = [0.2, 1.1, 0.3 * n + 0.5, 0.7 * n + 0.25, 0.15, -0.05]
    prog, (om, otop, _) = build_pair(workloads.spec_gauss_cheb_extended(), prec, api)
    prog.bind(to_dev([x], prec, api))
    nll, g, nb = prog.nll_grad(th)
    onll, og, oga, onb = om.nll_ex(otop, th, [x])
    assert nb == onb == 0
    tn, tg = TOL[prec]
    # the NLL bar relative to the magnitudes of its parts (they partly cancel)
    nu = th[2] + th[3]
    scale = float(np.sum(np.abs(np.log(om.values(otop, th, [x]))))) + nu + n * abs(np.log(nu))
    assert abs(nll - onll) <= tn * scale, (nll, onll)
    assert scaled_grad_err(g, og, oga).max() <= tg
    assert abs(prog.nll(th)[0] - onll) <= tn * scale  # the NLL-only kernel


def test_extended_fit_total_yield_is_the_event_count():
    """At the minimum of the extended NLL the fitted yields add up to N."""
    n = 200_000
    x = synth.sample_gauss_cheb(n, 32)
    prog, _ = build_pair(workloads.spec_gauss_cheb_extended(), api.FP64, api)
    prog.bind(to_dev([x], api.FP64, api))
    th, sig, info = prog.fit([0.1, 1.2, 0.25 * n, 0.8 * n, 0.1, 0.0], edm_tol=1e-9, max_iter=500)
    assert info["converged"], info
    assert abs(th[2] + th[3] - n) <= 1e-3 * np.sqrt(n), (th, n)
    # signal fraction near the sample's (0.3), yields' uncertainties ~ sqrt
    assert abs(th[2] / n - 0.3) < 5 * sig[2] / n


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("n", [1, 100_003])
def test_weighted_extended_parity(prec, n):
    """Weighted events in the extended likelihood: N of the term is the sum of
    the weights, formed on the GPU as one more event sum."""
    print("case weighted extended n=%d prec=%d" % (n, prec), flush=True)
    x = synth.sample_gauss_cheb(n, 33)
    w = np.random.default_rng(34).uniform(-0.5, 2.0, n).astype(np.float32).astype(np.float64)
    nw = float(np.sum(w))
    th = [0.2, 1.1, abs(0.3 * nw) + 0.5, abs(0.7 * nw) + 0.25, 0.15, -0.05]
    prog, (om, otop, _) = build_pair(workloads.spec_gauss_cheb_extended(), prec, api, weighted=True)
    prog.bind(to_dev([x, w], prec, api))
    nll, g, nb = prog.nll_grad(th)
    onll, og, oga, onb = om.nll_ex(otop, th, [x], weights=w)
    assert nb == onb == 0
    tn, tg = TOL[prec]
    nu = th[2] + th[3]
    v = om.values(otop, th, [x])
    scale = float(np.sum(np.abs(w * np.log(v)))) + nu + np.sum(np.abs(w)) * abs(np.log(nu))
    assert abs(nll - onll) <= tn * scale, (nll, onll)
    assert scaled_grad_err(g, og, oga).max() <= tg
    assert abs(prog.nll(th)[0] - onll) <= tn * scale  # the NLL-only entry point
    # unit weights reproduce the unweighted extended program
    prog.bind(to_dev([x, np.ones(n)], prec, api))
    ref, _ = build_pair(workloads.spec_gauss_cheb_extended(), prec, api)
    ref.bind(to_dev([x], prec, api))
    a, b = prog.nll_grad(th)[0], ref.nll_grad(th)[0]
    # FP64: the same arithmetic event by event.  FP32: the same per-event
    # arithmetic, but each program adds its events into FP32 partial sums per
    # round of its load ring (8 events with the weight column, 12 without), so
    # the two agree to the rounding of those partials
    bar = 1e-14 if prec == api.FP64 else 1e-9
    assert abs(a - b) <= bar * max(1.0, abs(b)), (a, b)
