"""GPU tests of the learned surrogate: MFMA MLP kernels against the FP64 oracle
MLP evaluated with the same BF16-rounded weights, the training kernels, the
exact-target kernel, and the surrogate PDF leaf inside a compiled likelihood."""
import numpy as np
import pytest

from helpers import build_pair, oracle_nll_threads, rel, scaled_grad_err, to_dev
from oracle import rfo
from paper_2003_12861_amd import synth, workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2003_12861_amd.api")
torch = pytest.importorskip("torch")
from paper_2003_12861_amd import surrogate  # noqa: E402


# FP32 per-event values of the surrogate leaf: its exponentials take
# arguments up to ~25 in the tails (relative rounding 2^-24 times the
# argument) and the activations enter the MFMA products as two BF16 parts
# (relative 2^-17 per product); measured within 1.7e-6.  The NLL and the
# gradient meet the FP32 bar of 1e-6.
VALUES_RTOL = 3e-6


# weight and input gradients: each entry against its own scale, the sum
# over rows of the magnitudes of its terms (entries far smaller than the
# largest one are checked to their own accuracy).  The kernels' products take
# FP32 operands as BF16 parts (2^-17 relative per product) and the
# back-propagated cotangents are 64-term sums that can cancel: bar 4e-5 of the
# entry's scale (measured up to 1e-5 for a single row, 2e-7 over 1000 rows).
DW_TOL = 4e-5


def _dw_scale(w64, u, dout):
    """sum over rows r of |dout_r d s_r / d w| per weight (the oracle, row by row)"""
    sc = np.zeros(8833)
    for r in range(u.shape[0]):
        dw_r, _ = rfo.mlp_backward(w64, u[r:r + 1], np.abs(dout[r:r + 1]))
        sc += np.abs(dw_r)
    return sc


def _assert_dw(dw, dw_ref, scale):
    err = np.abs(dw - dw_ref)
    ratio = err / np.maximum(scale, 1e-300)
    print("weight gradient: max error / entry scale %.3g" % ratio.max(), flush=True)
    assert np.all(err <= DW_TOL * scale + 1e-30), (ratio.max(), int(np.argmax(ratio)))


def _weights(seed, scale=1.0):
    w32 = torch.tensor(surrogate.init_weights(seed) * scale, device="cuda")
    rng = np.random.default_rng(seed + 100)
    for off in (384, 4544, 8704):  # non-zero biases exercise the bias path
        w32[off:off + 64] = torch.tensor(rng.uniform(-0.2, 0.2, 64), dtype=torch.float32, device="cuda")
    w32[8832] = 0.3
    wbf = w32.to(torch.bfloat16)
    return wbf, wbf.float().double().cpu().numpy()


@pytest.mark.parametrize("n", [1, 64, 1037])
def test_mlp_forward_backward_vs_oracle(n):
    print("case mlp fwd/bwd n=%d" % n, flush=True)
    wbf, w64 = _weights(1)
    rng = np.random.default_rng(n)
    u = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
    dout = rng.normal(size=n).astype(np.float32)
    ud = torch.tensor(u, device="cuda")
    s = api.mlp_forward(wbf, ud).double().cpu().numpy()
    s_ref = rfo.mlp_forward(w64, u.astype(np.float64))
    np.testing.assert_allclose(s, s_ref, rtol=2e-6, atol=2e-6)
    din = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    dw, _ = api.mlp_backward(wbf, ud, torch.tensor(dout, device="cuda"), din=din)
    dw_ref, din_ref = rfo.mlp_backward(w64, u.astype(np.float64), dout.astype(np.float64))
    dw = dw.double().cpu().numpy()
    _assert_dw(dw, dw_ref, _dw_scale(w64, u.astype(np.float64), dout.astype(np.float64)))
    # input gradients: each row against its own largest component
    din = din.double().cpu().numpy()
    row = np.abs(din_ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(din - din_ref) <= DW_TOL * row), np.max(np.abs(din - din_ref) / row)


def test_mlp_activations_layout():
    n = 70
    wbf, w64 = _weights(2)
    u = torch.rand((n, 6), device="cuda") * 2 - 1
    act = torch.empty((n, 192), dtype=torch.float32, device="cuda")
    s1 = api.mlp_forward(wbf, u)
    s2 = api.mlp_forward(wbf, u, act=act)
    assert torch.equal(s1, s2)
    # layer 1 by hand from the stored inputs
    W1 = w64[:384].reshape(64, 6)
    b1 = w64[384:448]
    h1 = np.tanh(u.double().cpu().numpy() @ W1.T + b1)
    np.testing.assert_allclose(act[:, :64].double().cpu().numpy(), h1, atol=2e-6)


def test_adam_step_and_bf16_copy():
    n = 8833
    rng = np.random.default_rng(3)
    w = rng.normal(size=n).astype(np.float32)
    w32 = torch.tensor(w, device="cuda")
    wbf = w32.to(torch.bfloat16)
    m = torch.zeros_like(w32)
    v = torch.zeros_like(w32)
    mm, vv, ww = np.zeros(n), np.zeros(n), w.astype(np.float64)
    for step in (1, 2, 3):
        g = rng.normal(size=n).astype(np.float32)
        api.adam_step(w32, wbf, m, v, torch.tensor(g, device="cuda"), 1e-3, step)
        mm = 0.9 * mm + 0.1 * g
        vv = 0.999 * vv + 0.001 * g.astype(np.float64) ** 2
        ww = ww - 1e-3 * (mm / (1 - 0.9 ** step)) / (np.sqrt(vv / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(w32.double().cpu().numpy(), ww, rtol=1e-6, atol=1e-7)
    assert torch.equal(wbf, w32.to(torch.bfloat16))  # round to nearest even


@pytest.mark.parametrize("batch,gather", [(1, True), (200, True), (4096, True), (64, False)])
def test_train_step_vs_oracle(batch, gather):
    """The fused step (gathered rows, MSE cotangent from its own forward pass,
    Adam inside the gradient reduction) against the oracle's batch gradient,
    the separate kernels, and Adam written out on the host."""
    print("case train step batch=%d gather=%s" % (batch, gather), flush=True)
    n = 5000
    wbf, w64 = _weights(6)
    rng = np.random.default_rng(batch)
    u = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    idx = rng.integers(0, n, batch).astype(np.int64) if gather else np.arange(batch, dtype=np.int64)
    ud, yd = torch.tensor(u, device="cuda"), torch.tensor(y, device="cuda")
    idd = torch.tensor(idx, device="cuda") if gather else None
    if not gather:  # no index: the batch is all rows of the arrays passed
        ud, yd = ud[:batch], yd[:batch]
    w0 = wbf.float()
    w32, m, v = w0.clone(), torch.zeros_like(w0), torch.zeros_like(w0)
    wbf_s = wbf.clone()
    dw = torch.empty(8833, dtype=torch.float32, device="cuda")
    lr = 1e-3
    api.mlp_train_step(wbf_s, w32, m, v, ud, yd, idd, lr, 1, dw=dw)
    torch.cuda.synchronize()
    # oracle: gradient of mean (s - y)^2 over the batch rows
    ub, yb = u[idx].astype(np.float64), y[idx].astype(np.float64)
    s_ref = rfo.mlp_forward(w64, ub)
    dw_ref, _ = rfo.mlp_backward(w64, ub, 2.0 / batch * (s_ref - yb))
    g = dw.double().cpu().numpy()
    # the cotangent 2 (s - y)/B cannot be more accurate than the kernel's
    # forward value s (FP32 accumulation of BF16 parts, about 2e-6): that
    # bound enters each row's scale, which matters where s is close to y
    cot = 2.0 / batch * (np.abs(s_ref - yb) + 4e-6 * (1.0 + np.abs(s_ref)))
    _assert_dw(g, dw_ref, _dw_scale(w64, ub, cot))
    scale = np.abs(dw_ref).max()
    # the separate kernels on the gathered batch give the same gradient
    ubd = torch.tensor(u[idx], device="cuda")
    out = api.mlp_forward(wbf, ubd)
    dout = torch.empty_like(out)
    api.mse_grad(out, torch.tensor(y[idx], device="cuda"), 2.0 / batch, dout)
    g2, _ = api.mlp_backward(wbf, ubd, dout)
    np.testing.assert_allclose(g, g2.double().cpu().numpy(), rtol=0, atol=1e-6 * scale)
    # Adam (first step) on the fused gradient
    gm, gv = 0.1 * g, 0.001 * g * g
    ww = w0.double().cpu().numpy() - lr * (gm / 0.1) / (np.sqrt(gv / 0.001) + 1e-8)
    np.testing.assert_allclose(w32.double().cpu().numpy(), ww, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(m.double().cpu().numpy(), gm, rtol=1e-6, atol=1e-12)
    assert torch.equal(wbf_s, w32.to(torch.bfloat16))


def test_train_step_index_checks():
    """Batch indices outside the arrays: with validation the call is refused
    before any launch; without it the kernel clamps each index into the
    arrays, so the step equals the one on the clamped indices."""
    n = 300
    wbf, _ = _weights(8)
    rng = np.random.default_rng(9)
    u = torch.tensor(rng.uniform(-1, 1, (n, 6)).astype(np.float32), device="cuda")
    y = torch.tensor(rng.normal(size=n).astype(np.float32), device="cuda")
    idx = np.array([0, 5, n - 1, n, n + 7, -3, 42], dtype=np.int64)
    w0 = wbf.float()
    args = lambda: (wbf.clone(), w0.clone(), torch.zeros_like(w0), torch.zeros_like(w0))
    wb, w32, m, v = args()
    with pytest.raises(api.RfError) as e:
        api.mlp_train_step(wb, w32, m, v, u, y, torch.tensor(idx, device="cuda"), 1e-3, 1, validate=True)
    assert e.value.code == -1 and torch.equal(w32, w0)
    dw1 = torch.empty(8833, dtype=torch.float32, device="cuda")
    api.mlp_train_step(wb, w32, m, v, u, y, torch.tensor(idx, device="cuda"), 1e-3, 1, dw=dw1)
    wb2, w32b, m2, v2 = args()
    dw2 = torch.empty(8833, dtype=torch.float32, device="cuda")
    api.mlp_train_step(wb2, w32b, m2, v2, u, y, torch.tensor(np.clip(idx, 0, n - 1), device="cuda"), 1e-3, 1, dw=dw2)
    torch.cuda.synchronize()
    assert torch.equal(dw1, dw2) and torch.equal(w32, w32b)


def test_exact_targets_vs_oracle():
    raw = synth.sobol_design(200, seed=11)
    xq = torch.tensor(raw, dtype=torch.float64, device="cuda")
    y = api.bwcb_logpdf(xq, 1024, synth.BWCB_WINDOW, synth.BWCB_RANGE).cpu().numpy()
    m, top, ids = rfo.from_spec(workloads.spec_bwcb())
    ref = np.empty(raw.shape[0])
    for i, r in enumerate(raw):
        # p_sig(x) = S(x)/N: the mixture with f = 1 isolates the signal
        thf = list(r[1:]) + [-0.02, 1.0]
        ref[i] = np.log(m.values(top, thf, [np.array([r[0]])])[0])
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_training_targets_vs_oracle():
    """rf_mlp_targets: log p_sig - log b on the GPU against the oracle's exact
    signal and its surrogate leaf with a zero network (whose value times its
    normalisation is the base b).  FP32 output and an FP32 base: the bar is a
    few units of 2^-24 of the base's exponent arguments, 4e-6 absolute."""
    raw = synth.surrogate_design(300, seed=13)
    xq = torch.tensor(raw, dtype=torch.float64, device="cuda")
    y = api.mlp_targets(xq, 1024, synth.BWCB_WINDOW, synth.BWCB_RANGE).double().cpu().numpy()
    me, te, _ = rfo.from_spec(workloads.spec_bwcb())
    mz, tz, iz = rfo.from_spec(workloads.spec_bwcb(surrogate=True))
    mz.set_mlp_weights(iz["sig"], np.zeros(8833))
    ref = np.empty(raw.shape[0])
    for i, r in enumerate(raw):
        thf = list(r[1:]) + [-0.02, 1.0]  # f = 1 isolates the signal
        x = np.array([r[0]])
        lp = np.log(me.values(te, thf, [x])[0])
        Nb, _ = mz.norm(iz["sig"], thf)
        ref[i] = lp - np.log(mz.values(tz, thf, [x])[0] * Nb)
    np.testing.assert_allclose(y, ref, rtol=0, atol=4e-6)


@pytest.mark.parametrize("n", [1000, 20_001])
def test_surrogate_leaf_vs_oracle(n):
    print("case surrogate leaf n=%d" % n, flush=True)
    wbf, w64 = _weights(4, scale=0.7)
    x = synth.sample_bw_cb(n, 5)
    spec = workloads.spec_bwcb(surrogate=True)
    prog, (om, otop, oids) = build_pair(spec, api.FP32, api)
    prog.bind(to_dev([x], api.FP32, api))
    prog.bind_weights("sig", wbf)
    om.set_mlp_weights(oids["sig"], w64)
    for th in ([91.19, 2.5, 1.5, 1.5, 3.0, -0.02, 0.8], [90.5, 2.1, 2.2, 0.9, 6.0, -0.015, 0.7]):
        nll, g, nb = prog.nll_grad(th)
        onll, og, oga, onb = om.nll_ex(otop, th, [x])
        assert nb == onb == 0
        assert rel(nll, onll) <= 1e-6, (nll, onll)
        err = scaled_grad_err(g, og, oga)
        assert err.max() <= 1e-6, err
        v = prog.values(th).double().cpu().numpy()
        np.testing.assert_allclose(v, om.values(otop, th, [x]), rtol=VALUES_RTOL)


def test_surrogate_leaf_full_size():
    """1e7 events in the benchmark's launch shape: the NLL and gradient
    against the oracle over all events (host threads), per-event values on a
    sample of events."""
    n = 10_000_000
    wbf, w64 = _weights(4, scale=0.7)
    x = synth.sample_bw_cb(n, 4)
    spec = workloads.spec_bwcb(surrogate=True)
    prog, (om, otop, oids) = build_pair(spec, api.FP32, api)
    prog.bind(to_dev([x], api.FP32, api))
    prog.bind_weights("sig", wbf)
    om.set_mlp_weights(oids["sig"], w64)
    th = [91.19, 2.5, 1.5, 1.5, 3.0, -0.02, 0.8]
    print("case surrogate full size: oracle over all events", flush=True)
    onll, og, oga, onb = oracle_nll_threads(spec, th, [x], mlp_weights={"sig": w64})
    nll, g, nb = prog.nll_grad(th)
    assert nb == onb == 0
    assert rel(nll, onll) <= 1e-6, (nll, onll)
    err = scaled_grad_err(g, og, oga)
    assert err.max() <= 1e-6, err
    v = prog.values(th).double().cpu().numpy()
    rng = np.random.default_rng(0)
    idx = rng.choice(n, 2000, replace=False)
    np.testing.assert_allclose(v[idx], om.values(otop, th, [x[idx]]), rtol=VALUES_RTOL)


def test_training_reduces_error():
    res = surrogate.train_surrogate(n_train=131072, epochs=8, batch=4096, lr=3e-3, log=print)
    h = res["history"]
    assert h[-1]["holdout_rms"] < 0.5 * h[0]["holdout_rms"], h
