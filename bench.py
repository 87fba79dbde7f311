"""Benchmark: events/s for one NLL+gradient evaluation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete NLL+gradient evaluation of the model over all events:
the FP64 prologue with the normalisations, every event through the fused
per-event program and its adjoint, the deterministic reduction and the
epilogue, and the result in host memory -- what a minimiser waits for on
every iteration (synchronous call).  Events are seeded synthetic data already
resident in HBM.  The headline value is the FP32+adjoint path; the plain FP64
path is timed beside it, and both results are checked against the oracle
(FP32: NLL relative error <= 1e-6, FP64: <= 1e-9).

Prints ONE JSON line.  Extra fields:
  roofline      the fused kernel against the VALU issue rate: algorithmic
                lane-slots per event times events, over the kernel's average
                launch duration (HIP events on the launch stream around K
                back-to-back launches -- the duration a profiler reports per
                launch);
  cpu_baseline  the oracle's throughput on the host, on a bounded sample.
The Python garbage collector is paused inside the timed regions (a full
collection of this process takes tens of milliseconds).
"""
import argparse
import gc
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X unit counts: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz; one lane-slot is
# one full-rate (non-packed) VALU lane operation
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9  # 3.93e13
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "gauss_cheb_1e7": dict(n=10_000_000, seed=2),
    "decay_argus_5e7": dict(n=50_000_000, seed=3),
}

# Algorithmic VALU lane-slots per event of an NLL+gradient evaluation (a
# transcendental counts 4: the quarter-rate unit), and bytes read per event.
SLOTS = {
    "gauss_cheb_1e7": {"fp32": 48, "fp64": 90},
    "decay_argus_5e7": {"fp32": 165, "fp64": 400},
}
BYTES_PER_EVENT = {"gauss_cheb_1e7": {"fp32": 4, "fp64": 8}, "decay_argus_5e7": {"fp32": 8, "fp64": 16}}


def measured_traffic(workload, kernel, source):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on this exact kernel (same generated source); else None.  The summary
    holds lines 'traffic kernel=K workload=W source_sha1=H bytes_per_launch=B'."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha1(source.encode()).hexdigest()
    for line in open(path):
        if not line.startswith("traffic "):
            continue
        kv = dict(f.split("=", 1) for f in line.split()[1:] if "=" in f)
        if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("source_sha1") == sha:
            return float(kv["bytes_per_launch"])
    return None


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


def timed_steps(prog, thetas, steps, torch, stream):
    """K synchronous NLL+gradient evaluations; returns (seconds per step,
    median seconds of one step)."""
    per = np.zeros(steps)
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ti = time.perf_counter()
            prog.nll_grad(thetas[i % len(thetas)], stream=stream)
            per[i] = time.perf_counter() - ti
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / steps
    finally:
        gc.enable()
    return step_s, float(np.median(per))


def isolated_kernel(prog, thetas, reps, torch, stream):
    """Median duration of single launches (an event pair around each launch,
    the GPU idle before it): includes the dispatch of a launch from idle."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    gc.collect()
    gc.disable()
    try:
        for i in range(reps):
            evs[i][0].record(stream)
            prog.nll_grad_async(thetas[i % len(thetas)], stream=stream)
            evs[i][1].record(stream)
            torch.cuda.synchronize()
    finally:
        gc.enable()
    return float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e-3


def pipelined_kernel(prog, thetas, reps, torch, stream):
    """Average duration of back-to-back launches (no host round trip between
    them): the kernel's own time as a profiler reports it."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    try:
        a.record(stream)
        for i in range(reps):
            prog.nll_grad_async(thetas[i % len(thetas)], stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
    finally:
        gc.enable()
    return a.elapsed_time(b) * 1e-3 / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="gauss_cheb_1e7", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 path (profiling runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 512 MiB device copy (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_12861_amd import api

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    spec, cols, theta, thetas = make(args.workload)
    n = cols[0].size
    precs = (("fp32", api.FP32, torch.float32),) if args.fp32_only else (
        ("fp32", api.FP32, torch.float32), ("fp64", api.FP64, torch.float64))
    progs = {}
    for key, prec, dt in precs:
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
            p.nll_grad(thetas[i % len(thetas)], stream=stream)
        step_s, med_s = timed_steps(p, thetas, args.steps, torch, stream)
        kern_s = pipelined_kernel(p, thetas, max(20, min(args.steps, 200)), torch, stream)
        iso_s = isolated_kernel(p, thetas, 20, torch, stream)
        res[key] = dict(step_s=step_s, median_step_s=med_s, kernel_s=kern_s, isolated_s=iso_s)

    # validity of both paths against the oracle at the truth point
    cpu = None
    check = {key: p.nll_grad(theta) for key, p in progs.items()}
    if not args.no_cpu_baseline:
        from oracle import rfo
        om, otop, _ = rfo.from_spec(spec)
        # bounded sample: full-size oracle NLL+gradient evaluations for ~10 s
        t0 = time.perf_counter()
        reps = 0
        while True:
            onll, og, oga, _ = om.nll_ex(otop, theta, cols)
            reps += 1
            if time.perf_counter() - t0 > 10.0:
                break
        cpu_s = (time.perf_counter() - t0) / reps
        cpu = dict(value=n / cpu_s, unit="events/s", cores=1, kind="oracle",
                   sample="%d full NLL+gradient evaluations of the %d-event workload (single-threaded C, -O2)" % (reps, n),
                   host=platform.processor() or platform.machine(), nproc=os.cpu_count())
        for key, tol in (("fp32", 1e-6), ("fp64", 1e-9)):
            if key not in check:
                continue
            nll, g, _ = check[key]
            res[key]["nll_rel_err"] = abs(nll - onll) / abs(onll)
            res[key]["grad_scaled_err"] = float(np.max(np.abs(g - og) / oga))
            res[key]["valid"] = bool(res[key]["nll_rel_err"] <= tol)

    k32 = res["fp32"]["kernel_s"]
    slots = SLOTS[args.workload]["fp32"]
    achieved = n * slots / k32 / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
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
                   "step": "one synchronous NLL+gradient evaluation (result in host memory)"},
        "fp32": {"kernel_ms": k32 * 1e3, "isolated_kernel_ms": res["fp32"]["isolated_s"] * 1e3,
                 "median_step_ms": res["fp32"]["median_step_s"] * 1e3,
                 "kernel_events_per_s": n / k32,
                 "nll_rel_err": res["fp32"].get("nll_rel_err"),
                 "grad_scaled_err": res["fp32"].get("grad_scaled_err"),
                 "valid": res["fp32"].get("valid")},
        "roofline": {"bound": "alu", "kernel": "rf_k_grad_f32", "achieved": achieved, "peak": peak,
                     "unit": "Tslot/s", "frac": achieved / peak,
                     "traffic": measured_traffic(args.workload, "rf_k_grad_f32", progs["fp32"].source),
                     "source_sha1": hashlib.sha1(progs["fp32"].source.encode()).hexdigest(),
                     "slots_per_event": slots, "events_per_launch": n,
                     "bytes_per_event": BYTES_PER_EVENT[args.workload]["fp32"],
                     "hbm_GBps": n * BYTES_PER_EVENT[args.workload]["fp32"] / k32 / 1e9},
        "cpu_baseline": cpu,
    }
    if "fp64" in res:
        line["fp64_plain"] = {"value": n / res["fp64"]["step_s"], "unit": "events/s",
                              "ms_per_step": res["fp64"]["step_s"] * 1e3,
                              "median_step_ms": res["fp64"]["median_step_s"] * 1e3,
                              "kernel_ms": res["fp64"]["kernel_s"] * 1e3,
                              "isolated_kernel_ms": res["fp64"]["isolated_s"] * 1e3,
                              "kernel_events_per_s": n / res["fp64"]["kernel_s"],
                              "roofline_frac": n * SLOTS[args.workload]["fp64"] / res["fp64"]["kernel_s"] / VALU_SLOTS_PER_S,
                              "nll_rel_err": res["fp64"].get("nll_rel_err"),
                              "grad_scaled_err": res["fp64"].get("grad_scaled_err"),
                              "valid": res["fp64"].get("valid")}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
