"""The weighted-event, extended and count x mass workloads at their full size
(1e7 events), in the automatic launch configuration that the benchmark times,
against the oracle's NLL and gradient over all events."""
import numpy as np
import pytest

from helpers import build_pair, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")

N = 10_000_000
TOL = {api.FP64: 1e-9, api.FP32: 1e-6}


def _case(name):
    """(spec, observable columns, weights or None, theta)"""
    if name == "poisson_gauss_cheb":
        k, x = synth.sample_poisson_gauss_cheb(N, 5)
        th = np.asarray(workloads.truth_vector(synth.POISSON_TRUTH)) * 1.03
        return workloads.spec_poisson_gauss_cheb(), [k, x], None, th
    x = synth.sample_gauss_cheb(N, 2)
    t = synth.jitter_gauss_cheb(3)
    if name == "gauss_cheb_weighted":
        w = np.random.default_rng(21).uniform(0.5, 1.5, N).astype(np.float32).astype(np.float64)
        return workloads.spec_gauss_cheb(), [x], w, t
    th = np.array([t[0], t[1], t[2] * N, (1.0 - t[2]) * N, t[3], t[4]])
    return workloads.spec_gauss_cheb_extended(), [x], None, th


@pytest.mark.parametrize("name", ["gauss_cheb_weighted", "gauss_cheb_extended", "poisson_gauss_cheb"])
def test_full_size_vs_oracle(name):
    spec, cols, w, th = _case(name)
    om, otop, _ = build_pair(spec, api.FP64, api, weighted=w is not None)[1]
    onll, og, oga, onb = om.nll_ex(otop, th, cols, weights=w)
    assert onb == 0
    # NLL bar relative to the magnitudes of its parts (the extended term
    # partly cancels the event sum)
    lp = np.abs(np.log(om.values(otop, th, cols)))
    scale = float(np.sum(lp * (w if w is not None else 1.0)))
    if name == "gauss_cheb_extended":
        nu = th[2] + th[3]
        scale += nu + N * abs(np.log(nu))
    for prec in (api.FP32, api.FP64):
        print("case full size %s prec=%d" % (name, prec), flush=True)
        prog, _ = build_pair(spec, prec, api, weighted=w is not None)
        prog.bind(to_dev(cols + ([w] if w is not None else []), prec, api))
        nll, g, nb = prog.nll_grad(th)
        assert nb == 0
        assert abs(nll - onll) <= TOL[prec] * scale, (prec, nll, onll)
        assert scaled_grad_err(g, og, oga).max() <= TOL[prec], (prec, g, og)
        del prog
