"""The unfused per-node batch mode (rf_nll_unfused, an ablation of the fused
kernel): its NLL against the oracle and against the fused kernel's."""
import numpy as np
import pytest

from helpers import build_pair, rel, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")

TOL = {api.FP64: 1e-9, api.FP32: 1e-6}


def _case(model, n, seed):
    if model == "gauss_cheb":
        return workloads.spec_gauss_cheb(), [synth.sample_gauss_cheb(n, seed)], [0.1, 1.2, 0.3, 0.15, -0.05]
    t, m = synth.sample_decay_argus(n, seed)
    return workloads.spec_decay_argus(), [t, m], workloads.truth_vector(synth.DECAY_TRUTH)


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("model,n", [("gauss_cheb", 1), ("gauss_cheb", 100_003), ("decay_argus", 50_001)])
def test_unfused_nll(prec, model, n):
    print("case unfused %s n=%d prec=%d" % (model, n, prec), flush=True)
    spec, cols, th = _case(model, n, 21)
    prog, (om, otop, _) = build_pair(spec, prec, api)
    prog.bind(to_dev(cols, prec, api))
    nll, nb = prog.nll_unfused(th)
    onll = om.nll(otop, th, cols, grad=False)[0]
    assert nb == 0
    assert rel(nll, onll) <= TOL[prec], (nll, onll)
    # same per-node arithmetic as the fused kernel; the sums differ in order
    assert rel(nll, prog.nll(th)[0]) <= (1e-12 if prec == api.FP64 else 1e-6)
    assert prog.nll_unfused(th)[0] == nll  # repeatable


def test_unfused_empty_and_rejected_programs():
    spec, th = workloads.spec_gauss_cheb(), [0.1, 1.2, 0.3, 0.15, -0.05]
    cols = [np.zeros(0)]
    prog, _ = build_pair(spec, api.FP64, api)
    prog.bind(to_dev(cols, api.FP64, api))
    assert prog.nll_unfused(th)[0] == 0.0
    pw, _ = build_pair(spec, api.FP64, api, weighted=True)
    pw.bind(to_dev(cols + [np.zeros(0)], api.FP64, api))
    with pytest.raises(api.RfError):
        pw.nll_unfused(th)
    pc, _ = build_pair(workloads.spec_bwcb(K=100), api.FP64, api)
    pc.bind(to_dev([synth.sample_bw_cb(10, 3)], api.FP64, api))
    with pytest.raises(api.RfError):
        pc.nll_unfused(workloads.truth_vector(synth.BWCB_TRUTH))
