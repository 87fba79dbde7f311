"""The library's own FP64 logarithm (the event loop's log p) against the
host's libm (numpy), over the arguments a likelihood meets: probabilities
from 1e-300 to 1e300, dense around 1 where log x is small and m - 1 matters."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")


def test_log64_vs_libm():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        np.exp(rng.uniform(-690.0, 690.0, 400_000)),
        rng.uniform(0.5, 2.0, 400_000),
        1.0 + rng.uniform(-1e-6, 1e-6, 100_000),
        np.nextafter(1.0, [0.0, 2.0]),
        [1.0, 2.0, 0.5, 0.7071067811865476, 0.7071067811865475, 1e-300, 1e300, 2.2250738585072014e-308],
    ])
    got = api.eval_math(0, torch.tensor(x, device="cuda")).cpu().numpy()
    ref = np.log(x)
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    # relative to the value, and absolute near 1 where log x -> 0
    assert np.all((rel <= 1e-15) | (np.abs(got - ref) <= 4.5e-16)), (rel.max(), x[np.argmax(rel)])
    assert got[-8] == 0.0  # log 1 = 0 exactly


def _ulp_err(got, ref):
    """error in units of the last place of the reference (subnormal results: of
    the smallest subnormal)"""
    ulp = np.spacing(np.abs(ref))
    return np.abs(got - ref) / np.maximum(ulp, 5e-324)


def test_exp2_neg_vs_libm():
    """2^t for t <= 0 of the FP64 event loop (the Gaussian's 2^(-q): rint
    reduction, Taylor series of e^r to r^13, ldexp) against the host's libm:
    within 2 units of the last place, subnormal results included."""
    rng = np.random.default_rng(2)
    t = np.concatenate([-rng.uniform(0.0, 1080.0, 300_000), -rng.uniform(0.0, 30.0, 300_000),
                        -np.arange(0, 1100) * 1.0, -np.arange(0, 2200) * 0.5, [0.0, -1e-300, -1074.0, -1075.0, -1076.0, -2000.0]])
    got = api.eval_math(1, torch.tensor(t, device="cuda")).cpu().numpy()
    ref = np.exp2(t)
    err = _ulp_err(got, ref)
    assert err.max() <= 2.0, (err.max(), t[np.argmax(err)])
    assert got[-1] == 0.0 and got[-6] == 1.0 and got[-5] == 1.0  # 2^-2000 = 0, 2^0 = 1, 2^-1e-300 = 1
    sp = api.eval_math(1, torch.tensor([-np.inf, np.nan], device="cuda")).cpu().numpy()
    assert sp[0] == 0.0 and np.isnan(sp[1])
