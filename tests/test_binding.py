"""The Python binding's CPython call module (_rfcall), on the host: the
synchronous calls reach the library with the same arguments as the ctypes
path, and arguments it does not take directly go to the checked path.  No
kernel is launched (the programs are compiled without loading)."""
import numpy as np
import pytest

from paper_2003_12861_amd import workloads

api = pytest.importorskip("paper_2003_12861_amd.api")
from paper_2003_12861_amd import _rfcall  # noqa: E402


def _prog():
    return api.Program(api.Graph.from_spec(workloads.spec_gauss_cheb()), precision=api.FP32, load=False)


def test_call_reaches_the_library():
    """Every accepted form of theta reaches rf_nll_grad, which reports the
    unloaded program (RF_E_STATE) as the ctypes path does."""
    p = _prog()
    for th in (np.array([0.1, 1.1, 0.3, 0.2, -0.1]), [0.1, 1.1, 0.3, 0.2, -0.1], (0, 1, 0.3, 0.2, -0.1),
               np.array([0.1, 1.1, 0.3, 0.2, -0.1], dtype=np.float32),
               np.array([0.0, 9.0, 0.1, 0.2, 0.3, 1.1, 0.3, 0.2, -0.1, 0.0])[4:9],  # a view, offset
               np.array([0.1, 0.0, 1.1, 0.0, 0.3, 0.0, 0.2, 0.0, -0.1, 0.0])[::2]):  # strided
        r = _rfcall.nll_grad(p.h.value, th, p.n_params, 0)
        assert r is not None and r[0] == -6, (th, r)
        with pytest.raises(api.RfError) as e:
            p.nll_grad(th, stream=0)
        assert e.value.code == -6, e.value


def test_other_arguments_take_the_checked_path():
    p = _prog()
    h = p.h.value
    assert _rfcall.nll_grad(None, [0.0] * 5, 5, 0) is None
    for th in ([0.0] * 4, [0.0] * 6, np.zeros(4), ["a", 1, 2, 3, 4], 3.0, np.zeros((5, 2))):
        assert _rfcall.nll_grad(h, th, 5, 0) is None, th
    for th in ([0.0] * 4, np.zeros(6)):
        with pytest.raises(api.RfError) as e:
            p.nll_grad(th, stream=0)
        assert e.value.code == -1
    with pytest.raises(TypeError):
        _rfcall.nll_grad(h, [0.0] * 5, 5)
    with pytest.raises(TypeError):
        _rfcall.nll_grad("not a handle", [0.0] * 5, 5, 0)


def test_sum_call():
    """The combined likelihood's call: a point outside the bounds reaches the
    library (RF_E_DOMAIN before anything runs); a wrong length takes the
    checked path."""
    s = api.Sum(3, lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0])
    r = _rfcall.sum_nll_grad(s.h.value, [0.5, 2.0, 0.5], 3, 0)
    assert r is not None and r[0] == -2
    with pytest.raises(api.RfError) as e:
        s.nll_grad(np.array([0.5, 2.0, 0.5]), stream=0)
    assert e.value.code == -2
    assert _rfcall.sum_nll_grad(s.h.value, [0.5, 0.5], 3, 0) is None
    with pytest.raises(api.RfError) as e:
        s.nll_grad([0.5, 0.5], stream=0)
    assert e.value.code == -1
