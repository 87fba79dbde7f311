"""The learned part: an MLP surrogate of the numerically convolved signal PDF.

train_surrogate() trains a 6-64-64-64-1 tanh network r(x, M, Gamma, sigma,
alpha, n) ~ log p_sig - log b on exact evaluations of the Breit-Wigner (x)
Crystal Ball convolution (the 1024-point rule of the exact leaf) at scrambled
Sobol points of the input box; b is the leaf's analytic base (a pseudo-Voigt
with the Crystal Ball tail, evaluated on the GPU by the leaf's own code), so
the network learns a residual about 20x smaller in spread than log p_sig.
Only the library's kernels are used:
    rf_mlp_targets (targets)  ->  rf_mlp_train_step (gather, forward, MSE
    gradient, backward and Adam in two launches)
torch only holds the device buffers (and draws the per-epoch permutation).
The trained BF16 weights are served by the surrogate leaf (RF_OP_MLP) of a
compiled likelihood graph, normalised on a Gauss-Legendre grid over x.
"""
import math
import time

import numpy as np
import torch

from . import api, synth

BOX = synth.BWCB_BOX          # raw design box (x, M, Gamma, sigma, alpha, n)
MLP_BOX = synth.BWCB_MLP_BOX  # network input box (x - M, M, Gamma, sigma, alpha, n)
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


def normalise(raw, box=MLP_BOX):
    """Network inputs: affine maps onto [-1, 1] of (x - M, M, Gamma, sigma, alpha, n)."""
    r = np.array(raw, dtype=np.float64, copy=True)
    r[:, 0] = r[:, 0] - r[:, 1]
    lo = np.array([b[0] for b in box])
    hi = np.array([b[1] for b in box])
    return 2.0 * (r - lo) / (hi - lo) - 1.0


def to_bf16(w32):
    return w32.to(torch.bfloat16)


def make_training_set(n, seed=7, K=1024, device="cuda", focus=None, frac_focus=0.0):
    """Sobol parameters, importance-sampled x, and the residual targets
    log p_sig (exact, FP64) - log b (the leaf's base), both on the GPU."""
    raw = synth.surrogate_design(n, seed=seed, focus=focus, frac_focus=frac_focus)
    xq = torch.tensor(raw, dtype=torch.float64, device=device)
    y = api.mlp_targets(xq, K, synth.BWCB_WINDOW, synth.BWCB_RANGE)
    u = torch.tensor(normalise(raw), dtype=torch.float32, device=device)
    return u, y, raw


def train_surrogate(n_train=2_000_000, epochs=60, batch=8192, lr=2e-3, lr_min=1e-5, seed=0, holdout=0.05,
                    K=1024, log=None, device="cuda", focus=None, frac_focus=0.0):
    """Returns dict(w32, w_bf16, history, holdout_rms, holdout_max)."""
    torch.cuda.set_device(0) if device == "cuda" else None
    u, y, _ = make_training_set(n_train, K=K, device=device, focus=focus, frac_focus=frac_focus)
    n_hold = int(holdout * n_train)
    u_tr, y_tr = u[n_hold:], y[n_hold:]
    u_ho, y_ho = u[:n_hold], y[:n_hold]
    n = u_tr.shape[0]
    w32 = torch.tensor(init_weights(seed), device=device)
    w32[8832] = float(y_tr.mean())  # output bias at the mean target
    wbf = to_bf16(w32)
    m = torch.zeros_like(w32)
    v = torch.zeros_like(w32)
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
            # one fused step: gather, forward, MSE gradient, backward, Adam
            idx = perm[b * batch:(b + 1) * batch]
            step += 1
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / total))
            api.mlp_train_step(wbf, w32, m, v, u_tr, y_tr, idx, lr_t, step)
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


def _kernel_seconds(prog, theta, reps=20):
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i in range(reps):
        ev[i][0].record(s)
        prog.nll_grad_async(theta, stream=s)
        ev[i][1].record(s)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e-3


def seeded_fit(prog_surrogate, prog_exact, start, edm_tol=1e-6, max_iter=500, exact_uncertainties=True):
    """The surrogate as the fit's accelerator: minimise with the surrogate
    from start, then with the exact convolution from the surrogate's minimum,
    starting with the surrogate fit's covariance as the inverse Hessian (the
    exact path stays the judge and the fallback: the result is the exact
    likelihood's minimum, reached with few exact evaluations).  With
    exact_uncertainties=False the exact fit forms no Hessian at its minimum
    and sigma is the surrogate fit's.  Returns dict(theta, sigma,
    info_surrogate, info_exact, theta_surrogate)."""
    th_s, sig_s, cov_s, info_s = prog_surrogate.fit_ex(start, edm_tol=edm_tol, max_iter=max_iter)
    hinv0 = cov_s if np.all(np.isfinite(cov_s)) else None
    th, sig, _, info_e = prog_exact.fit_ex(th_s, hinv0=hinv0, edm_tol=edm_tol, max_iter=max_iter,
                                           uncertainties=exact_uncertainties)
    return dict(theta=th, sigma=sig if exact_uncertainties else sig_s, info_surrogate=info_s, info_exact=info_e,
                theta_surrogate=th_s)


def experiment(epochs=600, n_train=2_000_000, n_events=10_000_000, seed=0, log=print, weights_out=None):
    """Train the surrogate, then fit the same events with the exact convolution
    (FP64 and FP32) and with the surrogate; report the surrogate's error, the
    fitted values, the bias in units of the exact fit's sigma and the speed."""
    from . import workloads
    torch.cuda.set_device(0)
    res = train_surrogate(n_train=n_train, epochs=epochs, seed=seed, log=log)
    if weights_out:
        np.savez(weights_out, w32=res["w32"].cpu().numpy())
    x = synth.sample_bw_cb(n_events, 4)
    truth = workloads.truth_vector(synth.BWCB_TRUTH)
    start = [91.0, 2.7, 1.3, 1.7, 3.5, -0.018, 0.78]
    out = dict(train_seconds=res["train_seconds"], holdout_rms=res["holdout_rms"], holdout_max=res["holdout_max"],
               history=res["history"][-5:], events=n_events, truth=truth, start=start)
    fits = {}
    for name, spec, prec in (("exact_fp64", workloads.spec_bwcb(), api.FP64),
                             ("exact_fp32", workloads.spec_bwcb(), api.FP32),
                             ("surrogate_fp32", workloads.spec_bwcb(surrogate=True), api.FP32)):
        p = api.Program(api.Graph.from_spec(spec), precision=prec)
        dt = torch.float64 if prec == api.FP64 else torch.float32
        p.bind([torch.tensor(x, dtype=dt, device="cuda")])
        if name.startswith("surrogate"):
            p.bind_weights("sig", res["w_bf16"])
        ks = _kernel_seconds(p, truth)
        t0 = time.time()
        th, sig, info = p.fit(start, edm_tol=1e-6, max_iter=500)
        fits[name] = dict(theta=th.tolist(), sigma=sig.tolist(), info=info, fit_seconds=time.time() - t0,
                          kernel_ms=ks * 1e3, events_per_s=n_events / ks)
        log("%s: kernel %.3f ms, fit %.2fs %s" % (name, ks * 1e3, time.time() - t0, info))
        del p
    ref = fits["exact_fp64"]
    for name in ("exact_fp32", "surrogate_fp32"):
        fits[name]["bias_in_sigma"] = ((np.array(fits[name]["theta"]) - np.array(ref["theta"]))
                                       / np.array(ref["sigma"])).tolist()
    fits["exact_fp64"]["pull_vs_truth"] = ((np.array(ref["theta"]) - np.array(truth)) / np.array(ref["sigma"])).tolist()
    out["fits"] = fits
    out["speedup_surrogate_vs_exact_fp32"] = fits["exact_fp32"]["kernel_ms"] / fits["surrogate_fp32"]["kernel_ms"]
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--n-train", type=int, default=2_000_000)
    ap.add_argument("--events", type=int, default=10_000_000)
    ap.add_argument("--weights-out", default=None)
    a = ap.parse_args()
    r = experiment(a.epochs, a.n_train, a.events, weights_out=a.weights_out,
                   log=lambda m: print(m, flush=True))
    print(json.dumps(r))
