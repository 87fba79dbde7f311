"""Benchmark: events/s for one NLL+gradient evaluation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete NLL+gradient evaluation of the model over all events
(FP64 prologue with the normalisations, every event through the fused
per-event program and its adjoint, the deterministic reduction and the
epilogue, result copied to the host and the stream synchronised) -- what a
minimiser waits for on every iteration.  Events are seeded synthetic data
already resident in HBM.  The headline value is the FP32+adjoint path; the
plain FP64 path is reported beside it, and both results are checked against
the oracle (FP32: NLL relative error <= 1e-6, FP64: <= 1e-9).

Prints ONE JSON line.  Extra fields: the fused kernel's roofline (average
kernel duration from HIP events on the launch stream) and the oracle's CPU
throughput on a bounded sample.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 3.93e13 lane-slots/s

WORKLOADS = {
    # name: (spec builder, sampler, truth, n events, per-event cost model)
    "gauss_cheb_1e7": dict(n=10_000_000, seed=2),
    "decay_argus_5e7": dict(n=50_000_000, seed=3),
}

# Algorithmic VALU slots per event of the fused NLL+gradient program (one
# slot = one full-rate lane operation; a transcendental -- exp, log, rcp,
# sqrt, erfc core -- counts 4, the quarter rate of the transcendental unit).
# Counted from the formulas (the design doc lists the breakdown).
SLOTS = {
    "gauss_cheb_1e7": {"fp32": 48 + 4 * 4, "fp64": 48 + 4 * 4},
    "decay_argus_5e7": {"fp32": 120 + 4 * 9, "fp64": 120 + 4 * 9},
}
BYTES_PER_EVENT = {"gauss_cheb_1e7": {"fp32": 4, "fp64": 8}, "decay_argus_5e7": {"fp32": 8, "fp64": 16}}


def make(workload):
    from paper_2003_12861_amd import synth, workloads
    w = WORKLOADS[workload]
    if workload.startswith("gauss_cheb"):
        spec = workloads.spec_gauss_cheb()
        cols = [synth.sample_gauss_cheb(w["n"], w["seed"])]
        theta = workloads.truth_vector(synth.GAUSS_CHEB_TRUTH)
        thetas = [synth.jitter_gauss_cheb(k) for k in range(100)]
    else:
        spec = workloads.spec_decay_argus()
        cols = list(synth.sample_decay_argus(w["n"], w["seed"]))
        theta = workloads.truth_vector(synth.DECAY_TRUTH)
        thetas = [synth.jitter_decay(k) for k in range(10)]
    return spec, cols, np.asarray(theta), thetas


def time_kernel(prog, thetas, reps, torch):
    """Average duration of the fused NLL+gradient kernel: HIP events recorded
    on the stream the kernel is launched on, one pair per launch."""
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i in range(reps):
        evs[i][0].record(stream)
        prog.nll_grad_async(thetas[i % len(thetas)], stream=stream)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3  # seconds


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="gauss_cheb_1e7", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 512 MiB device copy (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_12861_amd import api

    torch.cuda.set_device(0)
    spec, cols, theta, thetas = make(args.workload)
    n = cols[0].size
    progs = {}
    for key, prec, dt in (("fp32", api.FP32, torch.float32), ("fp64", api.FP64, torch.float64)):
        p = api.Program(api.Graph.from_spec(spec), precision=prec)
        p.bind([torch.tensor(c, dtype=dt, device="cuda") for c in cols])
        progs[key] = p

    if args.calib_copy:
        a = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    res = {}
    for key, p in progs.items():
        for i in range(args.warmup):
            p.nll_grad(thetas[i % len(thetas)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            nll, g, nb = p.nll_grad(thetas[i % len(thetas)])
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / args.steps
        kern_s = time_kernel(p, thetas, max(20, min(args.steps, 200)), torch)
        res[key] = dict(step_s=dt_s, kernel_s=kern_s)

    # validity of both paths against the oracle at the truth point
    check = {}
    cpu = None
    for key, p in progs.items():
        check[key] = p.nll_grad(theta)
    if not args.no_cpu_baseline:
        from oracle import rfo
        om, otop, _ = rfo.from_spec(spec)
        # bounded sample: repeat full-size oracle NLL+gradient evaluations for ~10-30 s
        t0 = time.perf_counter()
        reps = 0
        while True:
            onll, og, oga, _ = om.nll_ex(otop, theta, cols)
            reps += 1
            if time.perf_counter() - t0 > 10.0:
                break
        cpu_s = (time.perf_counter() - t0) / reps
        cpu = dict(value=n / cpu_s, unit="events/s", cores=1, kind="oracle",
                   sample="%d full NLL+gradient evaluations of %d events (single-threaded C, -O2)" % (reps, n),
                   host=platform.processor() or platform.machine(), nproc=os.cpu_count())
        for key, tol in (("fp32", 1e-6), ("fp64", 1e-9)):
            nll, g, _ = check[key]
            res[key]["nll_rel_err"] = abs(nll - onll) / abs(onll)
            res[key]["grad_scaled_err"] = float(np.max(np.abs(g - og) / oga))
            res[key]["valid"] = bool(res[key]["nll_rel_err"] <= tol)

    s32, s64 = SLOTS[args.workload], BYTES_PER_EVENT[args.workload]
    k32 = res["fp32"]["kernel_s"]
    achieved = n * s32["fp32"] / k32 / 1e12
    peak = VALU_LANE_OPS / 1e12
    line = {
        "metric": "events/s for NLL+gradient (FP32+adjoint vs FP64 plain) at <=1e-6 rel NLL error",
        "value": n / res["fp32"]["step_s"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["fp32"]["step_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "events": n, "precision": "fp32+adjoint, fp64 reductions",
                   "step": "one synchronous NLL+gradient evaluation"},
        "fp64_plain": {"value": n / res["fp64"]["step_s"], "unit": "events/s",
                       "ms_per_step": res["fp64"]["step_s"] * 1e3,
                       "kernel_ms": res["fp64"]["kernel_s"] * 1e3,
                       "kernel_events_per_s": n / res["fp64"]["kernel_s"],
                       "nll_rel_err": res["fp64"].get("nll_rel_err"),
                       "grad_scaled_err": res["fp64"].get("grad_scaled_err"),
                       "valid": res["fp64"].get("valid")},
        "fp32": {"kernel_ms": k32 * 1e3, "kernel_events_per_s": n / k32,
                 "nll_rel_err": res["fp32"].get("nll_rel_err"),
                 "grad_scaled_err": res["fp32"].get("grad_scaled_err"),
                 "valid": res["fp32"].get("valid")},
        "roofline": {"bound": "alu", "kernel": "rf_k_grad (fp32)", "achieved": achieved, "peak": peak,
                     "unit": "Tslot/s", "frac": achieved / peak, "traffic": None,
                     "slots_per_event": s32["fp32"], "bytes_per_event": s64["fp32"],
                     "hbm_GBps": n * s64["fp32"] / k32 / 1e9},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
