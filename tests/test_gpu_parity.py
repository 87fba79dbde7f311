"""GPU parity of the fused likelihood kernels against the oracle.

Every test calls the C ABI (through the ctypes binding) and compares with the
FP64 CPU oracle on identical, FP32-representable events.  Bars:
  FP64 path: NLL relative error <= 1e-9, gradient error <= 1e-9 of
             sum_i |d(-log p_i)/d theta| (the cancellation-aware scale);
  FP32 path: NLL relative error <= 1e-6, gradient error <= 1e-6 of that scale.
"""
import math

import numpy as np
import pytest

from helpers import build_pair, rel, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2003_12861_amd.api")

TH0 = [0.0, 1.0, 0.3, 0.2, -0.1]
TOL = {0: (1e-9, 1e-9), 1: (1e-6, 1e-6)}


def _check(prog, oracle, cols_host, theta, prec, label=""):
    om, otop, _ = oracle
    nll, g, nb = prog.nll_grad(theta)
    onll, og, oga, onb = om.nll_ex(otop, theta, cols_host)
    assert nb == onb == 0, label
    tn, tg = TOL[prec]
    assert rel(nll, onll) <= tn, (label, nll, onll, rel(nll, onll))
    err = scaled_grad_err(g, og, oga)
    assert err.max() <= tg, (label, err, g, og)
    return nll, g


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 10000, (1 << 20) + 7])
def test_gauss_cheb_sizes(prec, n):
    print("case gauss_cheb prec=%d n=%d" % (prec, n), flush=True)
    x = synth.sample_gauss_cheb(n, 1)
    prog, orc = build_pair(workloads.spec_gauss_cheb(), prec, api)
    prog.bind(to_dev([x], prec, api))
    _check(prog, orc, [x], TH0, prec, "n=%d" % n)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("mu,sigma", [(0.37, 0.7), (-1.1, 1.3), (2.05, 0.45), (0.0, 1.0)])
def test_single_tail_events(prec, mu, sigma):
    """One event at a time, deep in the Gaussian's tails (|z| from 6 to 13):
    the mu and sigma gradients come from the Gaussian component alone, so
    they need the component's relative accuracy, not just the mixture's."""
    f, c1, c2 = 0.3, 0.2, -0.1
    th = [mu, sigma, f, c1, c2]
    prog, (om, otop, _) = build_pair(workloads.spec_gauss_cheb(), prec, api)
    tn, tg = TOL[prec]
    for z in (-13.0, -9.5, -6.0, 6.5, 8.75, 11.0):
        x = np.float32(mu + z * sigma)
        if not -10.0 <= x <= 10.0:
            continue
        print("case tail prec=%d mu=%g sigma=%g z=%g" % (prec, mu, sigma, z), flush=True)
        col = np.array([x], dtype=np.float64)
        prog.bind(to_dev([col], prec, api))
        nll, g, nb = prog.nll_grad(th)
        onll, og, oga, onb = om.nll_ex(otop, th, [col])
        assert nb == onb == 0
        assert rel(nll, onll) <= tn, (z, nll, onll)
        err = scaled_grad_err(g, og, oga)
        # mu, sigma: the Gaussian component's own accuracy
        assert err[:2].max() <= tg, (z, err, g, og)
        # f, c1, c2: within one event, each derivative is a difference of two
        # terms (component shape and normalisation, or the two components);
        # rounding of the FP32 arguments is relative to the terms, so the bar
        # is scaled by the event's cancellation factor (closed forms, FP64)
        xp = float(x) / 10.0
        T = (xp, 2.0 * xp * xp - 1.0)
        u = 1.0 + c1 * T[0] + c2 * T[1]
        sN = 1.0 + c2 / (1.0 - 4.0)
        dlogN = (0.0, 1.0 / ((1.0 - 4.0) * sN))
        kappa = [1.0, 1.0, 1.0]
        for kk in range(2):
            a_, b_ = T[kk] / u, dlogN[kk]
            kappa[1 + kk] = (abs(a_) + abs(b_)) / max(abs(a_ - b_), 1e-300)
        zz = (float(x) - mu) / sigma
        from scipy.special import erf
        Ng = sigma * math.sqrt(math.pi / 2) * (erf((10 - mu) / (math.sqrt(2) * sigma)) - erf((-10 - mu) / (math.sqrt(2) * sigma)))
        gs, gb = math.exp(-0.5 * zz * zz) / Ng, u / (20.0 * sN)
        kappa[0] = (gs + gb) / max(abs(gs - gb), 1e-300)
        assert np.all(err[2:] <= tg * np.array(kappa)), (z, err, kappa, g, og)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_empty_dataset(prec):
    prog, _ = build_pair(workloads.spec_gauss_cheb(), prec, api)
    prog.bind(to_dev([np.zeros(0)], prec, api))
    nll, g, nb = prog.nll_grad(TH0)
    assert nll == 0.0 and nb == 0 and np.all(g == 0.0)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_values_match_oracle(prec):
    x = synth.sample_gauss_cheb(5000, 3)
    prog, (om, otop, _) = build_pair(workloads.spec_gauss_cheb(), prec, api)
    prog.bind(to_dev([x], prec, api))
    v = prog.values(TH0).double().cpu().numpy()
    ref = om.values(otop, TH0, [x])
    np.testing.assert_allclose(v, ref, rtol=1e-12 if prec == api.FP64 else 2e-6)


def test_gauss_cheb_full_size_jitters():
    """1e7 events, the +-10% jitter points: FP32 and FP64 paths vs the oracle."""
    n = 10_000_000
    x = synth.sample_gauss_cheb(n, 2)
    spec = workloads.spec_gauss_cheb()
    p32, orc = build_pair(spec, api.FP32, api)
    p64, _ = build_pair(spec, api.FP64, api)
    p32.bind(to_dev([x], api.FP32, api))
    p64.bind(to_dev([x], api.FP64, api))
    worst32, worst64 = 0.0, 0.0
    for k in range(0, 100, 10):
        th = synth.jitter_gauss_cheb(k)
        print("case jitter k=%d" % k, flush=True)
        n32, _ = _check(p32, orc, [x], th, api.FP32, "fp32 k=%d" % k)
        n64, _ = _check(p64, orc, [x], th, api.FP64, "fp64 k=%d" % k)
    # the remaining jitter points: NLL only (the oracle's NLL is cheaper)
    om, otop, _ = orc
    for k in range(100):
        if k % 10 == 0:
            continue
        th = synth.jitter_gauss_cheb(k)
        onll = om.nll(otop, th, [x], grad=False)[0]
        worst32 = max(worst32, rel(p32.nll(th)[0], onll))
        worst64 = max(worst64, rel(p64.nll(th)[0], onll))
    print("worst NLL rel error fp32 %.3g fp64 %.3g" % (worst32, worst64))
    assert worst32 <= 1e-6 and worst64 <= 1e-9


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_decay_argus_parity(prec):
    n = 200_000
    t, m = synth.sample_decay_argus(n, 3)
    prog, orc = build_pair(workloads.spec_decay_argus(), prec, api)
    prog.bind(to_dev([t, m], prec, api))
    for k in range(4):
        th = workloads.truth_vector(synth.DECAY_TRUTH) if k == 0 else synth.jitter_decay(k)
        print("case decay prec=%d k=%d" % (prec, k), flush=True)
        _check(prog, orc, [t, m], th, prec, "k=%d" % k)


def test_decay_argus_full_size_sampled():
    """5e7 events in the benchmark's launch shape.  Per-event values on a
    sample against the oracle and the NLL against -sum log p of the values
    (both paths); the FP64 gradient against central differences of the FP64
    NLL and the FP32 gradient against the FP64 one.  Gradient bars are
    relative to the scale sum_i |d(-log p_i)/d theta|, estimated from the
    oracle on a random 20000-event subset times n / 20000 (the scale is a sum
    over events)."""
    n = 50_000_000
    t, m = synth.sample_decay_argus(n, 3)
    spec = workloads.spec_decay_argus()
    p64, (om, otop, _) = build_pair(spec, api.FP64, api)
    p32, _ = build_pair(spec, api.FP32, api)
    p64.bind(to_dev([t, m], api.FP64, api))
    p32.bind(to_dev([t, m], api.FP32, api))
    th = np.array(workloads.truth_vector(synth.DECAY_TRUTH))
    rng = np.random.default_rng(0)
    idx = rng.choice(n, 2000, replace=False)
    ref = om.values(otop, th, [t[idx], m[idx]])
    for prog, prec in ((p64, api.FP64), (p32, api.FP32)):
        print("case decay full size prec=%d" % prec, flush=True)
        v = prog.values(th).double().cpu().numpy()
        np.testing.assert_allclose(v[idx], ref, rtol=1e-12 if prec == api.FP64 else 2e-6)
        nll = prog.nll(th)[0]
        assert rel(nll, -np.log(v).sum()) <= TOL[prec][0]
    sub = rng.choice(n, 20_000, replace=False)
    _, _, oga, _ = om.nll_ex(otop, th, [t[sub], m[sub]])
    scale = np.asarray(oga) * (n / sub.size)
    nll64, g64, nb = p64.nll_grad(th)
    assert nb == 0
    # central differences, steps 1e-4 of each parameter's natural width
    h = np.array([1.5e-4, 5e-6, 5e-6, 3e-7, 3e-7, 4e-5, 2e-3, 2e-5])
    assert h.size == th.size
    fd = np.empty(th.size)
    for k in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[k] += h[k]
        tm[k] -= h[k]
        fd[k] = (p64.nll(tp)[0] - p64.nll(tm)[0]) / (2 * h[k])
    assert (np.abs(g64 - fd) / scale).max() <= 1e-7, (g64, fd, scale)
    nll32, g32, nb = p32.nll_grad(th)
    assert nb == 0
    assert rel(nll32, nll64) <= 1e-6
    assert (np.abs(g32 - g64) / scale).max() <= 1e-6, (g32, g64, scale)


def test_determinism_and_invariants():
    x = synth.sample_gauss_cheb(300_001, 5)
    for prec in (api.FP64, api.FP32):
        prog, _ = build_pair(workloads.spec_gauss_cheb(), prec, api)
        prog.bind(to_dev([x], prec, api))
        a = prog.nll_grad(TH0)
        b = prog.nll_grad(TH0)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])  # bitwise repeatable
        perm = np.random.default_rng(1).permutation(x.size)
        prog2, _ = build_pair(workloads.spec_gauss_cheb(), prec, api)
        prog2.bind(to_dev([x[perm]], prec, api))
        c = prog2.nll_grad(TH0)
        assert rel(c[0], a[0]) < (1e-12 if prec == api.FP64 else 1e-9)
        # additivity over a split of the events
        pa, _ = build_pair(workloads.spec_gauss_cheb(), prec, api)
        pa.bind(to_dev([x[:100_000]], prec, api))
        pb, _ = build_pair(workloads.spec_gauss_cheb(), prec, api)
        pb.bind(to_dev([x[100_000:]], prec, api))
        s = pa.nll_grad(TH0)[0] + pb.nll_grad(TH0)[0]
        assert rel(s, a[0]) < (1e-12 if prec == api.FP64 else 1e-9)


def test_bad_events_reported():
    x = np.linspace(-10, 10, 1001)
    th = [0.0, 1.0, 0.0, 1.5, 0.0]  # 1 + 1.5 x' <= 0 for x' <= -2/3
    spec = [e if e[1] != "c1" else ("param", "c1", [], [-5.0, 5.0]) for e in workloads.spec_gauss_cheb()]
    for prec in (api.FP64, api.FP32):
        prog, (om, otop, _) = build_pair(spec, prec, api)
        prog.bind(to_dev([x], prec, api))
        nll, g, nb = prog.nll_grad(th)
        onll, _, onb = om.nll(otop, th, [x])
        assert math.isinf(nll) and nb == onb > 0 and np.all(np.isnan(g))
        nll1, nb1 = prog.nll(th)
        assert math.isinf(nll1) and nb1 == onb


def test_domain_errors():
    prog, _ = build_pair(workloads.spec_gauss_cheb(), api.FP64, api)
    prog.bind(to_dev([np.zeros(10)], api.FP64, api))
    with pytest.raises(api.RfError) as e:
        prog.nll_grad([0.0, -1.0, 0.3, 0.2, -0.1])
    assert e.value.code == -2
    with pytest.raises(api.RfError) as e:
        prog.nll_grad([0.0, 1.0, 1.3, 0.2, -0.1])  # fraction outside its bounds
    assert e.value.code == -2


def test_gradient_vs_central_differences():
    """FP64 adjoint vs central differences (h = 1e-5) of the GPU NLL itself."""
    x = synth.sample_gauss_cheb(20_000, 6)
    prog, _ = build_pair(workloads.spec_gauss_cheb(), api.FP64, api)
    prog.bind(to_dev([x], api.FP64, api))
    th = np.array([0.05, 0.97, 0.31, 0.21, -0.09])
    _, g, _ = prog.nll_grad(th)
    h = 1e-5
    fd = np.empty(5)
    for k in range(5):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (prog.nll(tp)[0] - prog.nll(tm)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-4)
