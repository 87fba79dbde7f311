"""Weighted events (NLL = -sum_i w_i log p_i, RF_COMPILE_WEIGHTED) and the
bind-time column check (RF_VALIDATE) on the GPU."""
import numpy as np
import pytest

from helpers import build_pair, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")

TOL = {api.FP64: (1e-9, 1e-9), api.FP32: (1e-6, 1e-6)}


def _case(model, n, seed):
    if model == "gauss_cheb":
        return workloads.spec_gauss_cheb(), [synth.sample_gauss_cheb(n, seed)], [0.1, 1.2, 0.3, 0.15, -0.05]
    t, m = synth.sample_decay_argus(n, seed)
    return workloads.spec_decay_argus(), [t, m], workloads.truth_vector(synth.DECAY_TRUTH)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("model,n", [("gauss_cheb", 1), ("gauss_cheb", 100_003), ("decay_argus", 50_001)])
def test_weighted_parity(prec, model, n):
    """Weights in [-0.5, 2] (FP32-representable; negative ones as in background
    subtraction) against the oracle's weighted NLL and gradient."""
    print("case weighted %s n=%d prec=%d" % (model, n, prec), flush=True)
    spec, cols, th = _case(model, n, 11)
    w = np.random.default_rng(n).uniform(-0.5, 2.0, n).astype(np.float32).astype(np.float64)
    prog, (om, otop, _) = build_pair(spec, prec, api, weighted=True)
    assert prog.n_columns == len(cols) + 1
    prog.bind(to_dev(cols + [w], prec, api))
    nll, g, nb = prog.nll_grad(th)
    onll, og, oga, onb = om.nll_ex(otop, th, cols, weights=w)
    assert nb == onb == 0
    tn, tg = TOL[prec]
    # the NLL bar relative to sum_i |w_i log p_i| (weights of both signs)
    scale = float(np.sum(np.abs(w * np.log(om.values(otop, th, cols)))))
    assert abs(nll - onll) <= tn * scale, (nll, onll, scale)
    assert scaled_grad_err(g, og, oga).max() <= tg
    assert abs(prog.nll(th)[0] - onll) <= tn * scale  # the NLL-only kernel


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_unit_weights_equal_unweighted(prec):
    """All weights 1: the weighted program gives the unweighted one's result
    bit for bit (a product with 1 is exact)."""
    spec, cols, th = _case("decay_argus", 30_001, 12)
    pw, _ = build_pair(spec, prec, api, weighted=True)
    pu, _ = build_pair(spec, prec, api)
    pw.bind(to_dev(cols + [np.ones(cols[0].size)], prec, api))
    pu.bind(to_dev(cols, prec, api))
    a, b = pw.nll_grad(th), pu.nll_grad(th)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    assert torch.equal(pw.values(th), pu.values(th))


def test_weighted_bind_needs_the_weight_column():
    spec, cols, th = _case("gauss_cheb", 100, 13)
    prog, _ = build_pair(spec, api.FP64, api, weighted=True)
    with pytest.raises(api.RfError):
        prog.bind(to_dev(cols, api.FP64, api))


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_validate_rejects_out_of_range_and_nonfinite(prec):
    spec, cols, th = _case("decay_argus", 10_000, 14)
    t, m = cols
    prog, _ = build_pair(spec, prec, api, validate=True, weighted=True)
    w = np.ones(t.size)
    prog.bind(to_dev([t, m, w], prec, api))  # in range: accepted
    assert np.isfinite(prog.nll(th)[0])
    for bad in ("t_high", "m_low", "t_nan", "w_inf"):
        t2, m2, w2 = t.copy(), m.copy(), w.copy()
        if bad == "t_high":
            t2[1234] = 10.5
        elif bad == "m_low":
            m2[9999] = 5.1
        elif bad == "t_nan":
            t2[0] = np.nan
        else:
            w2[5000] = np.inf
        with pytest.raises(api.RfError) as e:
            prog.bind(to_dev([t2, m2, w2], prec, api))
        assert e.value.code == -1, bad  # RF_E_INVALID
        # the program is left unbound
        with pytest.raises(api.RfError) as e2:
            prog.nll(th)
        assert e2.value.code == -6, bad  # RF_E_STATE
    prog.bind(to_dev([t, m, w], prec, api))
    assert np.isfinite(prog.nll(th)[0])
