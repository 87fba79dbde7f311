"""The quasi-Newton fit loop on the GPU likelihood (2-D decay x mass model)."""
import numpy as np
import pytest

from helpers import build_pair, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")


def test_decay_fit_converges_and_recovers_truth():
    n = 1_000_000
    t, m = synth.sample_decay_argus(n, 21)
    truth = np.array(workloads.truth_vector(synth.DECAY_TRUTH))
    start = synth.jitter_decay(5)
    res = {}
    for prec in (api.FP64, api.FP32):
        prog, _ = build_pair(workloads.spec_decay_argus(), prec, api)
        prog.bind(to_dev([t, m], prec, api))
        th, sig, info = prog.fit(start, edm_tol=1e-6, max_iter=500)
        print("prec", prec, info, th, sig, flush=True)
        assert np.all(np.isfinite(sig)) and np.all(sig > 0)
        assert np.all(np.abs(th - truth) < 5 * sig), (th - truth) / sig
        res[prec] = (th, sig, info)
    assert res[api.FP64][2]["converged"]
    # the FP32 path lands on the FP64 minimum to a small fraction of sigma
    d = (res[api.FP32][0] - res[api.FP64][0]) / res[api.FP64][1]
    assert np.all(np.abs(d) < 0.05), d


def test_gauss_cheb_fit_uncertainty_is_hessian_based():
    x = synth.sample_gauss_cheb(200_000, 31)
    prog, _ = build_pair(workloads.spec_gauss_cheb(), api.FP64, api)
    prog.bind(to_dev([x], api.FP64, api))
    th, sig, info = prog.fit([0.1, 1.1, 0.25, 0.15, -0.05])
    assert info["converged"]
    # at the minimum the analytic gradient vanishes
    _, g, _ = prog.nll_grad(th)
    assert np.all(np.abs(g * sig) < 1e-2)
