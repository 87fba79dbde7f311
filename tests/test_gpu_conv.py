"""GPU parity of the Breit-Wigner (x) Crystal Ball model (1024-point rule) plus
exponential background against the oracle."""
import numpy as np
import pytest

from helpers import build_pair, oracle_nll_threads, rel, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")

TRUTH = workloads.truth_vector(synth.BWCB_TRUTH)
POINTS = [TRUTH, [91.0, 2.6, 1.2, 1.8, 4.0, -0.018, 0.75], [91.5, 2.3, 2.2, 1.0, 1.5, -0.025, 0.85]]


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("K", [1024, 100])
def test_conv_parity(prec, K):
    n = 20_000 if K == 1024 else 5_000
    x = synth.sample_bw_cb(n, 4)
    prog, (om, otop, oids) = build_pair(workloads.spec_bwcb(K=K), prec, api)
    prog.bind(to_dev([x], prec, api))
    tn, tg = (1e-9, 1e-9) if prec == api.FP64 else (1e-6, 1e-6)
    for th in POINTS:
        print("case conv prec=%d K=%d theta=%s" % (prec, K, th), flush=True)
        nll, g, nb = prog.nll_grad(th)
        onll, og, oga, onb = om.nll_ex(otop, th, [x])
        assert nb == onb == 0
        assert rel(nll, onll) <= tn, (nll, onll)
        err = scaled_grad_err(g, og, oga)
        assert err.max() <= tg, err


_FULL = {}


def _full_conv_oracle():
    """The oracle's NLL and gradient over all 1e7 events (host threads), once."""
    if not _FULL:
        n = 10_000_000
        x = synth.sample_bw_cb(n, 4)
        print("case conv full size: oracle over all events", flush=True)
        _FULL["x"] = x
        _FULL["ref"] = oracle_nll_threads(workloads.spec_bwcb(), TRUTH, [x])
    return _FULL["x"], _FULL["ref"]


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_conv_full_size(prec):
    """1e7 events in the benchmark's launch shape: the NLL and gradient against
    the oracle over all events, per-event values on a sample of events."""
    x, (onll, og, oga, onb) = _full_conv_oracle()
    n = x.size
    prog, (om, otop, _) = build_pair(workloads.spec_bwcb(), prec, api)
    prog.bind(to_dev([x], prec, api))
    th = TRUTH
    print("case conv full size prec=%d" % prec, flush=True)
    nll, g, nb = prog.nll_grad(th)
    assert nb == onb == 0
    tn, tg = (1e-9, 1e-9) if prec == api.FP64 else (1e-6, 1e-6)
    assert rel(nll, onll) <= tn, (nll, onll)
    err = scaled_grad_err(g, og, oga)
    assert err.max() <= tg, err
    v = prog.values(th).double().cpu().numpy()
    idx = np.random.default_rng(0).choice(n, 2000, replace=False)
    ref = om.values(otop, th, [x[idx]])
    np.testing.assert_allclose(v[idx], ref, rtol=1e-12 if prec == api.FP64 else 2e-6)


def test_conv_gradient_vs_central_differences():
    x = synth.sample_bw_cb(5_000, 9)
    prog, _ = build_pair(workloads.spec_bwcb(K=256), api.FP64, api)
    prog.bind(to_dev([x], api.FP64, api))
    th = np.array(POINTS[1])
    _, g, _ = prog.nll_grad(th)
    h = 1e-5
    fd = np.empty(th.size)
    for k in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (prog.nll(tp)[0] - prog.nll(tm)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=2e-5, atol=2e-3)
