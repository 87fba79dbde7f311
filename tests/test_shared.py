"""PDF nodes shared by several sums or products (a graph rather than a
tree), on the host: the oracle evaluates a shared node once per event and
uses it in every parent (forward mode); pinned here against the same model
with the shared node written once per use, and against central differences.
The library compiles such graphs by expanding them into that tree."""
import numpy as np
import pytest

from oracle import rfo
from paper_2003_12861_amd import synth, workloads

TH_SUM = [0.2, 1.1, 0.4, 0.3, 0.6, 0.2, -0.1, -0.05]
TH_PROD = [0.1, 1.2, -0.3, 0.9, 0.35, 0.2, -0.1]


def _cols_sum():
    return [synth.sample_gauss_cheb(4001, 31)]


def _cols_prod():
    return [synth.sample_gauss_cheb(4001, 32), synth.sample_gauss_cheb(4001, 33, mu=-0.3, sigma=0.9)]


def _oracle(spec, th, cols):
    om, top, _ = rfo.from_spec(spec)
    nll, g, ga, nb = om.nll_ex(top, th, cols)
    assert nb == 0
    return nll, np.asarray(g), np.asarray(ga)


@pytest.mark.parametrize("which", ["sum", "prod"])
def test_oracle_shared_equals_tree(which):
    spec, th, cols = ((workloads.spec_shared_sum, TH_SUM, _cols_sum()) if which == "sum"
                      else (workloads.spec_shared_prod, TH_PROD, _cols_prod()))
    n, g, _ = _oracle(spec(), th, cols)
    n0, g0, s0 = _oracle(spec(tree=True), th, cols)
    assert abs(n - n0) <= 1e-13 * abs(n0)
    assert np.all(np.abs(g - g0) <= 1e-13 * s0)
    # and the gradient of the shared form against central differences of its NLL
    h = 1e-6
    for k in range(len(th)):
        tp, tm = list(th), list(th)
        tp[k] += h
        tm[k] -= h
        fd = (_oracle(spec(), tp, cols)[0] - _oracle(spec(), tm, cols)[0]) / (2 * h)
        assert abs(g[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (which, k, g[k], fd)


api = pytest.importorskip("paper_2003_12861_amd.api")


@pytest.mark.parametrize("which", ["sum", "prod"])
def test_shared_graph_compiles(which):
    """The library accepts the shared graph (it used to reject it), with the
    same parameters as the tree form, and evaluates the shared leaf in each
    of its copies."""
    spec = workloads.spec_shared_sum if which == "sum" else workloads.spec_shared_prod
    for prec in (api.FP64, api.FP32):
        p = api.Program(api.Graph.from_spec(spec()), precision=prec, load=False)
        t = api.Program(api.Graph.from_spec(spec(tree=True)), precision=prec, load=False)
        assert (p.n_params, p.n_columns, p.n_sums) == (t.n_params, t.n_columns, t.n_sums)
