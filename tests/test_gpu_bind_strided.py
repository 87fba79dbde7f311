"""rf_bind_columns_strided on the GPU: columns with a stride or in the other
floating-point type give bit for bit the results of the same values bound
as contiguous arrays of the program's type; argument checks."""
import ctypes

import numpy as np
import pytest

from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")

TH = [0.1, 1.1, 0.3, 0.2, -0.1]


def _prog(prec, weighted=False):
    return api.Program(api.Graph.from_spec(workloads.spec_gauss_cheb()), precision=prec, weighted=weighted)


def _strided(values, stride, dtype):
    big = torch.zeros(len(values) * stride, dtype=dtype, device="cuda")
    big[::stride] = torch.tensor(values, dtype=dtype, device="cuda")
    return big[::stride]


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_strided_and_converted_columns(prec):
    print("case bind strided prec=%d" % prec, flush=True)
    pdt = torch.float64 if prec == api.FP64 else torch.float32
    odt = torch.float32 if prec == api.FP64 else torch.float64
    for n in (100003, 250001):  # the second call grows the program's copy
        x = synth.sample_gauss_cheb(n, 51 + n % 7)
        ref = _prog(prec).bind([torch.tensor(x, dtype=pdt, device="cuda")])
        r = ref.nll_grad(TH)
        for col in (_strided(x, 2, pdt), _strided(x, 3, odt), torch.tensor(x, dtype=odt, device="cuda")):
            # the same values in the program's type, contiguous
            same = _prog(prec).bind([col.to(pdt).contiguous()])
            want = same.nll_grad(TH)
            got = _prog(prec).bind([col]).nll_grad(TH)
            assert got[0] == want[0] and np.array_equal(got[1], want[1]), (n, col.dtype, col.stride())
            if col.dtype == pdt:
                assert got[0] == r[0] and np.array_equal(got[1], r[1])
        # one program re-bound from a strided column to a larger one
    p = _prog(prec)
    for n in (1000, 50001):
        x = synth.sample_gauss_cheb(n, 60)
        got = p.bind([_strided(x, 2, odt)]).nll_grad(TH)
        want = _prog(prec).bind([torch.tensor(x, dtype=odt, device="cuda").to(pdt)]).nll_grad(TH)
        assert got[0] == want[0] and np.array_equal(got[1], want[1]), n


def test_strided_weights():
    print("case bind strided weights", flush=True)
    n = 20001
    x = synth.sample_gauss_cheb(n, 61)
    w = np.random.default_rng(3).uniform(0.5, 1.5, n)
    for prec, pdt in ((api.FP64, torch.float64), (api.FP32, torch.float32)):
        want = _prog(prec, True).bind([torch.tensor(x, dtype=pdt, device="cuda"),
                                       torch.tensor(w, dtype=pdt, device="cuda")]).nll_grad(TH)
        got = _prog(prec, True).bind([torch.tensor(x, dtype=pdt, device="cuda"), _strided(w, 4, pdt)]).nll_grad(TH)
        assert got[0] == want[0] and np.array_equal(got[1], want[1])


def test_strided_argument_checks():
    print("case bind strided checks", flush=True)
    p = _prog(api.FP32)
    col = torch.zeros(100, dtype=torch.float32, device="cuda")
    arr = (ctypes.c_void_p * 1)(col.data_ptr())
    for stride, dt in ((0, 0), (-1, 0), (1, 2), (1, -1)):
        st = (ctypes.c_int64 * 1)(stride)
        d = (ctypes.c_int32 * 1)(dt)
        assert api.rf_bind_columns_strided(p.h, arr, st, d, 1, 100, 0) == -1, (stride, dt)
    st, d = (ctypes.c_int64 * 1)(1), (ctypes.c_int32 * 1)(0)
    assert api.rf_bind_columns_strided(p.h, arr, st, d, 2, 100, 0) == -1  # column count
    assert api.rf_bind_columns_strided(p.h, arr, None, d, 1, 100, 0) == -1
    assert api.rf_bind_columns_strided(p.h, arr, st, d, 1, 0, 0) == 0  # no events
    nl = api.Program(api.Graph.from_spec(workloads.spec_gauss_cheb()), precision=api.FP32, load=False)
    assert api.rf_bind_columns_strided(nl.h, arr, st, d, 1, 100, 0) == -6
