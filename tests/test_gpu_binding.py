"""The binding's two call paths on the GPU: the CPython call module and the
plain ctypes call give bit-identical results for every accepted form of
theta, for a program in both precisions, a binned model and a combined
likelihood."""
import ctypes

import numpy as np
import pytest

from helpers import to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")

TH = [0.1, 1.1, 0.3, 0.2, -0.1]


def _forms(th):
    a = np.array(th, dtype=np.float64)
    wide = np.zeros(2 * len(th))
    wide[::2] = a
    return [a, list(th), tuple(th), wide[::2], [np.float64(v) for v in th]]


def _ctypes_nll_grad(fn, h, th, n, stream, with_bad=True):
    t = np.ascontiguousarray(th, dtype=np.float64)
    g = np.zeros(n)
    v, nb = ctypes.c_double(), ctypes.c_int64()
    dp = ctypes.POINTER(ctypes.c_double)
    if with_bad:
        rc = fn(h, t.ctypes.data_as(dp), ctypes.byref(v), g.ctypes.data_as(dp), ctypes.byref(nb), stream)
    else:
        rc = fn(h, t.ctypes.data_as(dp), ctypes.byref(v), g.ctypes.data_as(dp), stream)
    assert rc == 0, api.rf_last_error()
    return v.value, g


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_program_paths_agree(prec):
    print("case binding program prec=%d" % prec, flush=True)
    x = synth.sample_gauss_cheb(100003, 21)
    p = api.Program(api.Graph.from_spec(workloads.spec_gauss_cheb()), precision=prec)
    p.bind(to_dev([x], prec, api))
    st = torch.cuda.current_stream()
    ref_v, ref_g = _ctypes_nll_grad(api.rf_nll_grad, p.h, TH, 5, st.cuda_stream)
    for th in _forms(TH):
        for s in (st, st.cuda_stream, None):
            v, g, nb = p.nll_grad(th, stream=s)
            assert nb == 0 and v == ref_v and np.array_equal(g, ref_g), (type(th), s)


def test_binned_and_sum_paths_agree():
    print("case binding binned and sum", flush=True)
    d = synth.make_binned(4, 3, 2, 10, 4)
    bn = api.Binned(d["T"], d["Tp"], d["Tm"], d["nobs"])
    th = [1.1, 0.2, -0.3, 0.4, -0.1]
    st = torch.cuda.current_stream().cuda_stream
    ref_v, ref_g = _ctypes_nll_grad(api.rf_binned_nll_grad, bn.h, th, 5, st, with_bad=False)
    for t in _forms(th):
        v, g = bn.nll_grad(t, stream=st)
        assert v == ref_v and np.array_equal(g, ref_g), type(t)
    s = api.Sum(5).add(bn, range(5)).constrain(1, 0.0, 0.5)
    ref_v, ref_g = _ctypes_nll_grad(api.rf_sum_nll_grad, s.h, th, 5, st)
    for t in _forms(th):
        v, g, nb = s.nll_grad(t, stream=st)
        assert nb == 0 and v == ref_v and np.array_equal(g, ref_g), type(t)
