"""The unbinned Poisson PDF (RF_OP_POISSON) on the GPU against the oracle:
the 2-D count x mass mixture, a range that truncates the mass on both sides,
and the widest range the leaf accepts."""
import numpy as np
import pytest

from helpers import build_pair, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")

TOL = {api.FP64: (1e-9, 1e-9), api.FP32: (1e-6, 1e-6)}
TH = [11.0, 5.5, 0.1, 1.2, 0.15, -0.05, 0.35]  # lam_s, lam_b, mu, sigma, c1, c2, f


def _check(prog, om, otop, th, cols, prec, n):
    prog.bind(to_dev(cols, prec, api))
    nll, g, nb = prog.nll_grad(th)
    onll, og, oga, onb = om.nll_ex(otop, th, cols)
    assert nb == onb == 0
    tn, tg = TOL[prec]
    assert abs(nll - onll) <= tn * max(1.0, abs(onll)), (nll, onll)
    assert scaled_grad_err(g, og, oga).max() <= tg, (g, og)
    assert abs(prog.nll(th)[0] - onll) <= tn * max(1.0, abs(onll))
    m = min(n, 20_000)
    v = prog.values(th).double().cpu().numpy()[:m]
    ref = om.values(otop, th, [c[:m] for c in cols])
    np.testing.assert_allclose(v, ref, rtol=1e-12 if prec == api.FP64 else 2e-6)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("n", [1, 100_003])
def test_poisson_gauss_cheb_parity(prec, n):
    print("case poisson_gauss_cheb n=%d prec=%d" % (n, prec), flush=True)
    k, x = synth.sample_poisson_gauss_cheb(n, 41)
    prog, (om, otop, _) = build_pair(workloads.spec_poisson_gauss_cheb(), prec, api)
    _check(prog, om, otop, TH, [k, x], prec, n)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("lo,hi,lam,n", [(4.0, 13.0, 8.7, 5000), (0.0, 2047.0, 1000.0, 50_000),
                                         (0.0, 1.0, 0.4, 777)])
def test_poisson_leaf_ranges(prec, lo, hi, lam, n):
    """Truncation on both sides (d log N / d lambda matters), the 2048-value
    table, and the two-value range."""
    print("case poisson_leaf [%g, %g] lam=%g n=%d prec=%d" % (lo, hi, lam, n, prec), flush=True)
    rng = np.random.default_rng(42)
    k = np.clip(rng.poisson(lam, n), lo, hi).astype(np.float64)
    prog, (om, otop, _) = build_pair(workloads.spec_poisson(lo, hi), prec, api)
    _check(prog, om, otop, [lam * 1.03], [k], prec, n)


def test_poisson_fit_recovers_the_sample_mean():
    """Untruncated in practice (range 0..200 around lambda = 10): the fitted
    lambda is the sample mean."""
    rng = np.random.default_rng(43)
    k = rng.poisson(10.0, 300_000).astype(np.float64)
    prog, _ = build_pair(workloads.spec_poisson(0.0, 200.0), api.FP64, api)
    prog.bind(to_dev([k], api.FP64, api))
    th, sig, info = prog.fit([7.0], edm_tol=1e-10, max_iter=200)
    assert info["converged"], info
    assert abs(th[0] - k.mean()) <= 1e-6 * k.mean(), (th[0], k.mean())
    assert abs(sig[0] - np.sqrt(k.mean() / k.size)) <= 1e-3 * sig[0]


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_validate_rejects_non_integer_counts(prec):
    """RF_VALIDATE: the observable of a Poisson leaf must hold integers; the
    continuous observable beside it need not."""
    k, x = synth.sample_poisson_gauss_cheb(1000, 44)
    prog, _ = build_pair(workloads.spec_poisson_gauss_cheb(), prec, api, validate=True)
    prog.bind(to_dev([k, x], prec, api))  # integer counts, continuous x: accepted
    assert prog.nll(TH)[1] == 0
    kb = k.copy()
    kb[[3, 500]] += 0.5
    with pytest.raises(api.RfError, match="integer"):
        prog.bind(to_dev([kb, x], prec, api))
