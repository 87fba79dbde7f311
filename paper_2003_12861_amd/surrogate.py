"""The learned part: an MLP surrogate of the numerically convolved signal PDF.

train_surrogate() trains a 6-64-64-64-1 tanh network s(x, M, Gamma, sigma,
alpha, n) ~ log p_sig on exact evaluations of the Breit-Wigner (x) Crystal
Ball convolution (the 1024-point rule of the exact leaf) at scrambled Sobol
points of the input box, using only the library's kernels:
    rf_bwcb_logpdf  (targets)  ->  rf_mlp_forward  ->  rf_mse_grad
    ->  rf_mlp_backward  ->  rf_adam_step
torch only holds the device buffers (and draws the per-epoch permutation).
The trained BF16 weights are served by the surrogate leaf (RF_OP_MLP) of a
compiled likelihood graph, normalised on a Gauss-Legendre grid over x.
"""
import math
import time

import numpy as np
import torch

from . import api, synth

BOX = synth.BWCB_BOX
N_W = 8833


def init_weights(seed=0):
    """Glorot-uniform weights, zero biases (FP32 master copy)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(N_W, dtype=np.float32)

    def glorot(off, fo, fi):
        a = math.sqrt(6.0 / (fi + fo))
        w[off:off + fo * fi] = rng.uniform(-a, a, fo * fi)

    glorot(0, 64, 6)
    glorot(448, 64, 64)
    glorot(4608, 64, 64)
    glorot(8768, 1, 64)
    return w


def normalise(raw, box=BOX):
    lo = np.array([b[0] for b in box])
    hi = np.array([b[1] for b in box])
    return 2.0 * (raw - lo) / (hi - lo) - 1.0


def to_bf16(w32):
    return w32.to(torch.bfloat16)


def make_training_set(n, seed=7, K=1024, device="cuda"):
    """Sobol (x, M, Gamma, sigma, alpha, n) in the box and exact log p_sig targets."""
    raw = synth.sobol_design(n, seed=seed)
    xq = torch.tensor(raw, dtype=torch.float64, device=device)
    y = api.bwcb_logpdf(xq, K, synth.BWCB_WINDOW, synth.BWCB_RANGE)
    u = torch.tensor(normalise(raw), dtype=torch.float32, device=device)
    return u, y.to(torch.float32), raw


def train_surrogate(n_train=2_000_000, epochs=60, batch=8192, lr=1e-3, lr_min=1e-5, seed=0, holdout=0.05,
                    K=1024, log=None, device="cuda"):
    """Returns dict(w32, w_bf16, history, holdout_rms, holdout_max)."""
    torch.cuda.set_device(0) if device == "cuda" else None
    u, y, _ = make_training_set(n_train, K=K, device=device)
    n_hold = int(holdout * n_train)
    u_tr, y_tr = u[n_hold:], y[n_hold:]
    u_ho, y_ho = u[:n_hold], y[:n_hold]
    n = u_tr.shape[0]
    w32 = torch.tensor(init_weights(seed), device=device)
    w32[8832] = float(y_tr.mean())  # output bias at the mean target
    wbf = to_bf16(w32)
    m = torch.zeros_like(w32)
    v = torch.zeros_like(w32)
    g = torch.empty_like(w32)
    out = torch.empty(batch, dtype=torch.float32, device=device)
    dout = torch.empty(batch, dtype=torch.float32, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    step = 0
    hist = []
    t0 = time.time()
    pred = api.mlp_forward(wbf, u_ho)
    hist.append(dict(epoch=-1, holdout_rms=float((pred - y_ho).double().pow(2).mean().sqrt()), seconds=0.0))
    for ep in range(epochs):
        perm = torch.randperm(n, device=device, generator=gen)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            ub = u_tr[idx].contiguous()
            yb = y_tr[idx].contiguous()
            api.mlp_forward(wbf, ub, out)
            api.mse_grad(out, yb, 2.0 / batch, dout)
            api.mlp_backward(wbf, ub, dout, g)
            step += 1
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / total))
            api.adam_step(w32, wbf, m, v, g, lr_t, step)
        pred = api.mlp_forward(wbf, u_ho)
        err = (pred - y_ho).double()
        rms = float(err.pow(2).mean().sqrt())
        hist.append(dict(epoch=ep, holdout_rms=rms, seconds=time.time() - t0))
        if log:
            log("epoch %d holdout rms %.3e (%.1fs)" % (ep, rms, time.time() - t0))
    pred = api.mlp_forward(wbf, u_ho)
    err = (pred - y_ho).double().abs()
    return dict(w32=w32, w_bf16=wbf, history=hist, holdout_rms=hist[-1]["holdout_rms"] if hist else None,
                holdout_max=float(err.max()), train_seconds=time.time() - t0)
