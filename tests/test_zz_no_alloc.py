"""rf_nll_grad_noalloc (the NLL+gradient evaluation that allocates nothing)
through the C ABI, against rf_nll_grad_async (the same kernel on the
program's own workspace) and the oracle: two calls in a row, the second on a
smaller input, in both precision forms; oversized partials are rejected."""
import ctypes

import numpy as np
import pytest

from helpers import build_pair, rel, scaled_grad_err, to_dev
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")

TOL = {0: (1e-9, 1e-9), 1: (1e-6, 1e-6)}
TH = [0.05, 0.97, 0.31, 0.21, -0.09]


def _abi():
    lib = ctypes.CDLL(api.LIB_PATH)
    f = lib.rf_nll_grad_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int32
    g = lib.rf_nll_grad_async
    g.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    g.restype = ctypes.c_int32
    r = lib.rf_program_result
    r.argtypes = [ctypes.c_void_p]
    r.restype = ctypes.c_void_p
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    return f, g, r, hip


@pytest.mark.parametrize("prec", [api.FP64, api.FP32])
def test_noalloc_matches_async_entry_point(prec):
    f_noalloc, f_async, f_result, hip = _abi()
    spec = workloads.spec_gauss_cheb()
    prog, (om, otop, _) = build_pair(spec, prec, api)
    nres = prog.n_params + 2 + prog.n_sums
    stream = torch.cuda.current_stream().cuda_stream
    th = np.array(TH, dtype=np.float64)
    thp = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for n in (1_000_003, 20_011):  # the second call on a smaller input
        print("case noalloc prec=%d n=%d" % (prec, n), flush=True)
        x = synth.sample_gauss_cheb(n, 50 + n % 7)
        prog.bind(to_dev([x], prec, api))
        out = torch.full((nres,), float("nan"), dtype=torch.float64, device="cuda")
        assert f_noalloc(prog.h, thp, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)) == 0
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        assert f_async(prog.h, thp, ctypes.c_void_p(stream)) == 0
        torch.cuda.synchronize()
        b = np.empty(nres)
        assert hip.hipMemcpy(b.ctypes.data, f_result(prog.h), 8 * nres, 2) == 0  # device to host
        # the same kernel in the same launch shape: bitwise the same result
        assert np.array_equal(a, b), (a, b)
        onll, og, oga, onb = om.nll_ex(otop, TH, [x])
        assert a[prog.n_params + 1] == onb == 0
        tn, tg = TOL[prec]
        assert rel(a[0], onll) <= tn
        assert scaled_grad_err(a[1:1 + prog.n_params], og, oga).max() <= tg


def test_noalloc_rejects_partials_beyond_its_scratch():
    """Five Gaussians: 17 rows of partials.  At the automatic launch shape they
    fit the 256 KiB array; at 2048 workgroups (278 KB) the call is refused
    before anything is enqueued, and the program still evaluates afterwards."""
    f_noalloc, _, _, _ = _abi()
    spec = workloads.spec_gauss_sum(5)
    prog, (om, otop, _) = build_pair(spec, api.FP32, api)
    x = synth.sample_gauss_cheb(300_000, 51)
    prog.bind(to_dev([x], api.FP32, api))
    th = [-3.0, 0.8, -1.0, 0.5, 0.0, 1.2, 1.5, 0.6, 3.0, 2.0, 0.2, 0.2, 0.2, 0.2]
    out = torch.zeros(prog.n_params + 2 + prog.n_sums, dtype=torch.float64, device="cuda")
    thp = np.array(th).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert f_noalloc(prog.h, thp, ctypes.c_void_p(out.data_ptr()), stream) == 0
    torch.cuda.synchronize()
    ref = prog.nll_grad(th)
    assert out[0].item() == ref[0]
    prog.set_launch(blocks=2048)
    rc = f_noalloc(prog.h, thp, ctypes.c_void_p(out.data_ptr()), stream)
    assert rc == -1 and b"scratch" in api.rf_last_error()
    prog.set_launch(blocks=0)
    assert f_noalloc(prog.h, thp, ctypes.c_void_p(out.data_ptr()), stream) == 0
    torch.cuda.synchronize()
    assert out[0].item() == ref[0]
    onll, og, oga, _ = om.nll_ex(otop, th, [x])
    assert rel(out[0].item(), onll) <= 1e-6
