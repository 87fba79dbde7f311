"""Graphs with a PDF node shared by two sums or two products, on the GPU:
the program compiled from the shared graph against the oracle's evaluation
of the same graph (which computes the shared node once per event), and
against the program compiled from the tree with the node written twice."""
import numpy as np
import pytest

from helpers import rel, scaled_grad_err, to_dev
from oracle import rfo
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")

TOL = {api.FP64: 1e-9, api.FP32: 1e-6}
CASES = {
    "sum": (workloads.spec_shared_sum, [0.2, 1.1, 0.4, 0.3, 0.6, 0.2, -0.1, -0.05]),
    "prod": (workloads.spec_shared_prod, [0.1, 1.2, -0.3, 0.9, 0.35, 0.2, -0.1]),
}


def _cols(which, n):
    if which == "sum":
        return [synth.sample_gauss_cheb(n, 41)]
    return [synth.sample_gauss_cheb(n, 42), synth.sample_gauss_cheb(n, 43, mu=-0.3, sigma=0.9)]


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
@pytest.mark.parametrize("which", ["sum", "prod"])
def test_shared_graph_parity(which, prec):
    print("case shared %s prec=%d" % (which, prec), flush=True)
    spec, th = CASES[which]
    for n in (1, 100003):
        cols = _cols(which, n)
        p = api.Program(api.Graph.from_spec(spec()), precision=prec)
        p.bind(to_dev(cols, prec, api))
        nll, g, nb = p.nll_grad(th)
        om, top, _ = rfo.from_spec(spec())
        on, og, oga, onb = om.nll_ex(top, th, cols)
        assert nb == 0 and onb == 0
        assert rel(nll, on) <= TOL[prec], (n, nll, on)
        assert scaled_grad_err(g, og, oga).max() <= TOL[prec], (n, scaled_grad_err(g, og, oga))
        # the program of the tree form (the node written twice)
        t = api.Program(api.Graph.from_spec(spec(tree=True)), precision=prec)
        t.bind(to_dev(cols, prec, api))
        tn, tg, _ = t.nll_grad(th)
        assert rel(nll, tn) <= TOL[prec] and scaled_grad_err(g, tg, oga).max() <= TOL[prec]
