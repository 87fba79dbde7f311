"""Benchmark: events/s for one NLL+gradient evaluation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete NLL+gradient evaluation of the model over all events:
the FP64 prologue with the normalisations, every event through the fused
per-event program and its adjoint, the deterministic reduction and the
epilogue, and the result in host memory -- what a minimiser waits for on
every iteration (synchronous call).  Events are seeded synthetic data already
resident in HBM.  The headline value is the FP32+adjoint path; the plain FP64
path is timed beside it where the model has one, and both results are checked
against the oracle (FP32: NLL relative error <= 1e-6, FP64: <= 1e-9).

Workloads (the default is the headline one):
  gauss_cheb_1e7        1-D Gaussian + Chebyshev mixture, 1e7 events
  gauss_cheb_weighted_1e7  the same with per-event weights (uniform in
                        [0.5, 1.5]): NLL = -sum_i w_i log p_i
  gauss_cheb_extended_1e7  the same mixture as an extended likelihood with
                        yields (nu_s, nu_b)
  decay_argus_5e7       2-D decay (x) resolution with mass peak, 5e7 events
  poisson_gauss_cheb_1e7  2-D count x mass: Poisson(n) Gauss(x) signal,
                        Poisson(n) Chebyshev(x) background, 1e7 events
  bwcb_exact_1e7        Breit-Wigner (x) Crystal Ball by the exact 1024-point
                        rule + exponential background, 1e7 events
  bwcb_surrogate_1e7    the same model with the MLP surrogate of the signal
                        (FP32; random-init weights: the cost does not depend
                        on their values), 1e7 events
  binned_200x4x100x60   binned templates: 200 channels x 4 samples x 100
                        bins, 60 nuisance parameters (a step is one
                        evaluation; the unit is evaluations/s)

--unfused-ablation (gauss_cheb_1e7 or decay_argus_5e7): instead, time the
NLL-only evaluation of the fused kernel against the paper's unfused per-node
batch mode (rf_nll_unfused: one kernel per PDF node writing its values to
device memory, then the NLL) in both precisions, and print one JSON line with
both step times, the ratio, and the unfused mode's device-memory traffic.

Prints ONE JSON line.  Extra fields:
  roofline      the dominant kernel against its bound: VALU issue rate
                (lane-slots), MFMA rate or HBM bandwidth; algorithmic work per
                launch over the kernel's average launch duration (HIP events
                on the launch stream around K back-to-back launches -- the
                duration a profiler reports per launch);
  cpu_baseline  the oracle's throughput on the host, on a bounded sample.
The Python garbage collector is paused inside the timed regions (a full
collection of this process takes tens of milliseconds).

The HSA runtime is asked to poll completion signals (HSA_ENABLE_INTERRUPT=0,
unless the environment sets it already): the timed region ends with
torch.cuda.synchronize(), which otherwise sleeps on an interrupt and wakes
tens of microseconds late.  Evaluations themselves do not depend on it (the
synchronous call polls its result in host memory).  The JSON line reports the
setting under "runtime".
"""
import argparse
import gc
import hashlib
import json
import os
import platform
import sys
import time

# before anything initialises the GPU runtime
os.environ.setdefault("HSA_ENABLE_INTERRUPT", "0")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X unit counts: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz; one lane-slot is
# one full-rate (non-packed) VALU lane operation
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9  # 3.93e13
HBM_PEAK_GBS = 8000.0
MFMA_BF16_TFLOPS = 2500.0  # dense

# VALU lane-slots per event of an NLL+gradient evaluation, and bytes read per
# event.  FP32: the algorithmic count (a transcendental counts 4: the
# quarter-rate unit).  FP64: the VALU instructions per event the hardware
# counters measured (SQ_INSTS_VALU x 64 / events), since the FP64 exp and log
# are instruction sequences whose length is the work.
SLOTS = {
    "gauss_cheb_1e7": {"fp32": 48, "fp64": 91},
    # weights: one more multiply on log p and one on 1/p
    "gauss_cheb_weighted_1e7": {"fp32": 50, "fp64": 93},
    # extended: the same per-event program (the yield term is parameter-only)
    "gauss_cheb_extended_1e7": {"fp32": 48, "fp64": 91},
    "decay_argus_5e7": {"fp32": 165, "fp64": 336},
    # the 1-D mixture's work, two Poisson leaves (an LDS table read each:
    # index, clamp, conversion) and the two products' adjoint terms
    "poisson_gauss_cheb_1e7": {"fp32": 68, "fp64": 120},
    "bwcb_exact_1e7": {"fp32": 16400, "fp64": 16400},
}
BYTES_PER_EVENT = {"gauss_cheb_1e7": {"fp32": 4, "fp64": 8}, "gauss_cheb_weighted_1e7": {"fp32": 8, "fp64": 16},
                   "gauss_cheb_extended_1e7": {"fp32": 4, "fp64": 8},
                   "decay_argus_5e7": {"fp32": 8, "fp64": 16},
                   "poisson_gauss_cheb_1e7": {"fp32": 8, "fp64": 16},
                   "bwcb_exact_1e7": {"fp32": 4, "fp64": 8}, "bwcb_surrogate_1e7": {"fp32": 4}}
# surrogate: network multiply-adds per event (forward and input gradient)
SURROGATE_MAC_PER_EVENT = 17300
WORKLOADS = ("gauss_cheb_1e7", "gauss_cheb_weighted_1e7", "gauss_cheb_extended_1e7", "decay_argus_5e7",
             "poisson_gauss_cheb_1e7", "bwcb_exact_1e7", "bwcb_surrogate_1e7",
             "binned_200x4x100x60")
WEIGHTED = ("gauss_cheb_weighted_1e7",)  # the last column holds the event weights


def emit(line):
    """Print the one JSON line, with the runtime setting it was measured under."""
    line["runtime"] = {"HSA_ENABLE_INTERRUPT": os.environ.get("HSA_ENABLE_INTERRUPT")}
    print(json.dumps(line))


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


def binned_source():
    """The binned kernel's sources (it is built into the library, not
    generated): the key under which its counter summary is valid."""
    d = os.path.join(ROOT, "paper_2003_12861_amd", "csrc")
    return "".join(open(os.path.join(d, f)).read() for f in ("rf_binned.hip", os.path.join("device", "rf_dev.h")))


def measured_ceiling(name):
    """A ceiling measured by bench.py --peaks on this device, from the
    committed summary's machine-read line 'ceiling name=N value=V unit=U'."""
    path = os.path.join(ROOT, "profiles", "peaks_mi355x.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("ceiling "):
            kv = dict(f.split("=", 1) for f in line.split()[1:] if "=" in f)
            if kv.get("name") == name:
                return float(kv["value"])
    return None


# the measured ceiling that bounds each workload's FP32 kernel: the issue rate
# of its instruction mix (lane-slots/s, a transcendental counting 4)
MIX = {"gauss_cheb_1e7": "fp32_mix_14fma_1trans", "gauss_cheb_weighted_1e7": "fp32_mix_14fma_1trans",
       "gauss_cheb_extended_1e7": "fp32_mix_14fma_1trans", "decay_argus_5e7": "fp32_mix_14fma_1trans",
       "poisson_gauss_cheb_1e7": "fp32_mix_14fma_1trans", "bwcb_exact_1e7": "fp32_mix_12fma_1rcp",
       "bwcb_surrogate_1e7": "fp32_mix_14fma_1trans"}
# surrogate leaf: VALU lane-slots per event (192 tanh, the BF16 splitting of
# the activations, the base): the binding bound, above the MFMA one
SURROGATE_SLOTS_PER_EVENT = 2700


def make(workload):
    """(spec, columns, truth theta, list of theta points, precisions, FP32 MLP weights or None)"""
    from paper_2003_12861_amd import synth, workloads
    if workload in ("gauss_cheb_1e7", "gauss_cheb_weighted_1e7"):
        cols = [synth.sample_gauss_cheb(10_000_000, 2)]
        if workload in WEIGHTED:
            w = np.random.default_rng(21).uniform(0.5, 1.5, cols[0].size)
            cols.append(w.astype(np.float32).astype(np.float64))  # exact in both precisions
        return (workloads.spec_gauss_cheb(), cols, np.asarray(workloads.truth_vector(synth.GAUSS_CHEB_TRUTH)),
                [synth.jitter_gauss_cheb(k) for k in range(100)], ("fp32", "fp64"), None)
    if workload == "gauss_cheb_extended_1e7":
        n = 10_000_000

        def ext(t):  # (mu, sigma, f, c1, c2) -> (mu, sigma, nu_s, nu_b, c1, c2), nu = n
            return np.array([t[0], t[1], t[2] * n, (1.0 - t[2]) * n, t[3], t[4]])
        return (workloads.spec_gauss_cheb_extended(), [synth.sample_gauss_cheb(n, 2)],
                ext(workloads.truth_vector(synth.GAUSS_CHEB_TRUTH)),
                [ext(synth.jitter_gauss_cheb(k)) for k in range(100)], ("fp32", "fp64"), None)
    if workload == "poisson_gauss_cheb_1e7":
        truth = np.asarray(workloads.truth_vector(synth.POISSON_TRUTH))
        rng = np.random.default_rng(12)
        thetas = [truth * (1.0 + 0.05 * rng.uniform(-1, 1, truth.size)) for _ in range(10)]
        return (workloads.spec_poisson_gauss_cheb(), list(synth.sample_poisson_gauss_cheb(10_000_000, 5)), truth,
                thetas, ("fp32", "fp64"), None)
    if workload == "decay_argus_5e7":
        return (workloads.spec_decay_argus(), list(synth.sample_decay_argus(50_000_000, 3)),
                np.asarray(workloads.truth_vector(synth.DECAY_TRUTH)),
                [synth.jitter_decay(k) for k in range(10)], ("fp32", "fp64"), None)
    truth = np.asarray(workloads.truth_vector(synth.BWCB_TRUTH))
    rng = np.random.default_rng(11)
    thetas = [truth * (1.0 + 0.002 * rng.uniform(-1, 1, truth.size)) for _ in range(10)]
    x = synth.sample_bw_cb(10_000_000, 4)
    if workload == "bwcb_exact_1e7":
        return workloads.spec_bwcb(), [x], truth, thetas, ("fp32", "fp64"), None
    from paper_2003_12861_amd import surrogate
    return workloads.spec_bwcb(surrogate=True), [x], truth, thetas, ("fp32",), surrogate.init_weights(0)


def timed_steps(call, thetas, steps, torch):
    """K synchronous evaluations; returns (seconds per step, median seconds of
    one step).  The collector is already paused (time_path pauses it before
    the warm-up, so that the warm-up steps run after its last collection)."""
    args = [thetas[i % len(thetas)] for i in range(steps)]
    stamps = []
    clock = time.perf_counter
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = clock()
        for th in args:
            call(th)
            stamps.append(clock())
        torch.cuda.synchronize()
        step_s = (clock() - t0) / steps
    finally:
        gc.enable()
    per = np.diff(np.array([t0] + stamps))  # each step from the end of the one before
    timed_steps.last = per
    return step_s, float(np.median(per))


def isolated_kernel(call_async, thetas, reps, torch, stream):
    """Median duration of single launches (an event pair around each launch,
    the GPU idle before it): includes the dispatch of a launch from idle."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    gc.collect()
    gc.disable()
    try:
        for i in range(reps):
            evs[i][0].record(stream)
            call_async(thetas[i % len(thetas)])
            evs[i][1].record(stream)
            torch.cuda.synchronize()
    finally:
        gc.enable()
    return float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e-3


def pipelined_kernel(call_async, thetas, reps, torch, stream):
    """Average duration of back-to-back launches (no host round trip between
    them): the kernel's own time as a profiler reports it."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    try:
        a.record(stream)
        for i in range(reps):
            call_async(thetas[i % len(thetas)])
        b.record(stream)
        torch.cuda.synchronize()
    finally:
        gc.enable()
    return a.elapsed_time(b) * 1e-3 / reps


def cold_kernel(call_async, thetas, reps, torch, stream):
    """Median duration of single launches whose inputs were evicted from the
    caches first: a 512 MiB fill (twice the 256 MB Infinity Cache) runs on the
    stream before each launch, outside the event pair."""
    flush = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    gc.collect()
    gc.disable()
    try:
        with torch.cuda.stream(stream):
            for i in range(reps):
                flush.fill_(float(i))
                evs[i][0].record(stream)
                call_async(thetas[i % len(thetas)])
                evs[i][1].record(stream)
        torch.cuda.synchronize()
    finally:
        gc.enable()
    del flush
    return float(np.median([a.elapsed_time(b) for a, b in evs])) * 1e-3


def time_path(call, call_async, thetas, args, torch, stream):
    """The kernel's own time first (10 launches after a cache eviction each,
    a lead-in, 200 back-to-back launches, then 20 isolated ones), then the W
    warm-up steps and the K timed synchronous steps.  On a freshly started
    process the GPU reaches its working clocks only after a few milliseconds
    of work: measured in that order, a 20-step run times the path at the
    speed it runs in a fit, with the inputs back in the caches."""
    cold_s = cold_kernel(call_async, thetas, 10, torch, stream)
    pipelined_kernel(call_async, thetas, 20, torch, stream)  # lead-in, not used
    kern_s = pipelined_kernel(call_async, thetas, 200, torch, stream)
    iso_s = isolated_kernel(call_async, thetas, 20, torch, stream)
    gc.collect()
    gc.disable()
    for i in range(args.warmup):
        call(thetas[i % len(thetas)])
    step_s, med_s = timed_steps(call, thetas, args.steps, torch)
    per = timed_steps.last
    return dict(step_s=step_s, median_step_s=med_s, kernel_s=kern_s, isolated_s=iso_s, cold_s=cold_s,
                step_us_min_max=[float(per.min()) * 1e6, float(per.max()) * 1e6])


def oracle_rate(fn, n_per_call, budget_s):
    """Units per second of fn() (n_per_call units each) over about budget_s seconds."""
    t0 = time.perf_counter()
    reps = 0
    while True:
        fn()
        reps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    return n_per_call / dt, reps


def run_binned(args, torch, stream):
    from paper_2003_12861_amd import api, synth
    C, S, B, J = 200, 4, 100, 60
    d = synth.make_binned(5, C, S, B, J)
    bn = api.Binned(d["T"], d["Tp"], d["Tm"], d["nobs"], stream=stream)
    rng = np.random.default_rng(3)
    thetas = [np.concatenate([[1.0 + 0.05 * rng.uniform(-1, 1)], rng.uniform(-0.5, 0.5, J)]) for _ in range(10)]
    r = time_path(lambda th: bn.nll_grad(th, stream=stream), lambda th: bn.nll_grad_async(th, stream=stream),
                  thetas, args, torch, stream)
    nll, _ = bn.nll_grad(thetas[0], stream=stream)
    cpu = None
    check = {}
    if not args.no_cpu_baseline:
        from oracle import rfo
        Lp = np.log(d["Tp"] / d["T"][:, :, None, :])
        Lm = np.log(d["Tm"] / d["T"][:, :, None, :])
        onll, _ = rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], thetas[0])
        rate, reps = oracle_rate(lambda: rfo.binned_nll(d["T"], Lp, Lm, d["nobs"], thetas[0]), 1, 5.0)
        cpu = dict(value=rate, unit="evaluations/s", cores=1, kind="oracle",
                   sample="%d full NLL+gradient evaluations (single-threaded C, -O2)" % reps,
                   host=platform.processor() or platform.machine(), nproc=os.cpu_count())
        check = dict(nll_rel_err=abs(nll - onll) / abs(onll), valid=bool(abs(nll - onll) <= 1e-6 * abs(onll)))
    # bytes per evaluation: T, one of the two variation tables per (j, cell), n
    nbytes = C * S * B * (1 + J) * 4 + C * B * 4
    k = r["kernel_s"]
    line = {
        "metric": "NLL+gradient evaluations/s of the binned template model",
        "value": 1.0 / r["step_s"], "unit": "evaluations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["step_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "channels": C, "samples": S, "bins": B, "nuisance": J,
                   "precision": "fp32 terms, fp64 exponent and sums",
                   "step": "one synchronous NLL+gradient evaluation (result in host memory)"},
        "binned": {"kernel_ms": k * 1e3, "isolated_kernel_ms": r["isolated_s"] * 1e3,
                   "cold_cache_kernel_ms": r["cold_s"] * 1e3,
                   "median_step_ms": r["median_step_s"] * 1e3, **check},
        "roofline": {"bound": "hbm", "kernel": "rf_binned_kernel<60>", "achieved": nbytes / k / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": nbytes / k / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, "rf_binned_kernel<60>", binned_source()),
                     "source_sha1": hashlib.sha1(binned_source().encode()).hexdigest(),
                     "bytes_per_launch": nbytes},
        "cpu_baseline": cpu,
    }
    sbw = measured_ceiling("stream_read_bytes")
    if sbw:
        line["roofline"]["measured_ceiling"] = {"stream_GBps": sbw / 1e9, "frac_hbm": nbytes / k / sbw}
    emit(line)


def run_peaks(api):
    """The ceilings, measured: median of three runs of each microbenchmark."""
    iters = {0: 20000, 1: 20000, 2: 5000, 3: 1500, 4: 1500, 5: 1000, 6: 1000, 7: 2000, 8: 1, 9: 1000}
    out = {}
    for kind, name in api.PEAK_KINDS.items():
        rates = [api.peak(kind, iters[kind], 1 << 31 if kind == 8 else 0)[0] for _ in range(3)]
        out[name] = float(np.median(rates))
    derived = {"valu_lane_slots_per_s": VALU_SLOTS_PER_S, "hbm_bytes_per_s": HBM_PEAK_GBS * 1e9}
    print(json.dumps({"metric": "measured ceilings", "unit": "per second", "measured": out, "derived": derived,
                      "ratios": {"fp32_fma/derived": out["fp32_fma"] / VALU_SLOTS_PER_S,
                                 "fp64_fma/derived": out["fp64_fma"] / VALU_SLOTS_PER_S,
                                 "mix_1d/derived": out["fp32_mix_14fma_1trans"] / VALU_SLOTS_PER_S,
                                 "mix_conv/derived": out["fp32_mix_12fma_1rcp"] / VALU_SLOTS_PER_S,
                                 "stream/8TB": out["stream_read_bytes"] / (HBM_PEAK_GBS * 1e9)}}))


def run_unfused_ablation(args, progs, cols, thetas, n, torch, stream):
    """Synchronous NLL-only steps: the fused kernel against the unfused
    per-node batch mode, same program, same events, same parameter points."""
    from paper_2003_12861_amd import api
    if args.workload not in ("gauss_cheb_1e7", "decay_argus_5e7"):
        raise SystemExit("--unfused-ablation takes gauss_cheb_1e7 or decay_argus_5e7")
    out = {}
    for key, p in progs.items():
        fused = lambda th, p=p: p.nll(th, stream=stream)
        unf = lambda th, p=p: p.nll_unfused(th, stream=stream)
        gc.collect()
        for f in (fused, unf):
            for i in range(args.warmup):
                f(thetas[i % len(thetas)])
        tf, _ = timed_steps(fused, thetas, args.steps, torch)
        tu, _ = timed_steps(unf, thetas, args.steps, torch)
        a, b = p.nll(thetas[0], stream=stream)[0], p.nll_unfused(thetas[0], stream=stream)[0]
        out[key] = {"fused_nll_ms": tf * 1e3, "unfused_nll_ms": tu * 1e3, "unfused_over_fused": tu / tf,
                    "nll_rel_diff": abs(a - b) / abs(b)}
    nodes = {"gauss_cheb_1e7": 3, "decay_argus_5e7": 7}[args.workload]
    # values moved per event by the unfused mode: each node reads its inputs
    # (a column or its input nodes' arrays) and writes its array, and the NLL
    # reads the top's array -- 1-D: 2 leaves x 2 + sum 3 + 1 = 8; 2-D:
    # 4 leaves x 2 + 2 products x 3 + sum 3 + 1 = 18 (the fused kernel: the
    # columns only)
    moved = {"gauss_cheb_1e7": 8, "decay_argus_5e7": 18}[args.workload]
    line = {
        "metric": "NLL evaluation time: fused kernel vs the paper's unfused per-node batch mode",
        "value": out["fp32"]["unfused_over_fused"], "unit": "unfused/fused step time (fp32)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": args.workload, "events": n, "pdf_nodes": nodes,
                   "step": "one synchronous NLL evaluation (no gradient)"},
        "unfused_bytes_per_event": {k: moved * (4 if k == "fp32" else 8) for k in out},
        "fused_bytes_per_event": {k: len(cols) * (4 if k == "fp32" else 8) for k in out},
        **out,
    }
    emit(line)


def run_hessian(args, progs, thetas, n, torch, stream):
    """Synchronous NLL + gradient + Hessian: the one-pass Hessian kernel
    (rf_nll_grad_hess, FP64 per event whatever the columns' dtype) against
    what it replaces in the fit, the Hessian from central differences of the
    analytic gradient (2P synchronous gradient evaluations, steps of a tenth
    of each parameter's uncertainty), and the uncertainties the two give."""
    if args.workload not in ("gauss_cheb_1e7", "gauss_cheb_extended_1e7", "decay_argus_5e7"):
        raise SystemExit("--hessian takes gauss_cheb_1e7, gauss_cheb_extended_1e7 or decay_argus_5e7")
    out = {}
    for key, p in progs.items():
        P = p.n_params
        hess = lambda th, p=p: p.nll_grad_hess(th, stream=stream)
        _, _, H0, _ = hess(thetas[0])
        sig0 = np.sqrt(np.diag(np.linalg.inv(H0)))
        h = 0.1 * sig0

        def fd(th, p=p):
            H = np.empty((P, P))
            for k in range(P):
                tp, tm = np.array(th, dtype=np.float64), np.array(th, dtype=np.float64)
                tp[k] += h[k]
                tm[k] -= h[k]
                H[:, k] = (p.nll_grad(tp, stream=stream)[1] - p.nll_grad(tm, stream=stream)[1]) / (2 * h[k])
            return 0.5 * (H + H.T)
        gc.collect()
        for f in (hess, fd):
            for i in range(args.warmup):
                f(thetas[i % len(thetas)])
        th_, _ = timed_steps(hess, thetas, args.steps, torch)
        tf_, _ = timed_steps(fd, thetas, max(1, args.steps // (2 * P)), torch)
        Hk, Hf = hess(thetas[0])[2], fd(thetas[0])
        sk, sf = np.sqrt(np.diag(np.linalg.inv(Hk))), np.sqrt(np.diag(np.linalg.inv(Hf)))
        out[key] = {"hessian_ms": th_ * 1e3, "fd_hessian_ms": tf_ * 1e3, "fd_over_hessian": tf_ / th_,
                    "gradient_evaluations_per_fd_hessian": 2 * P,
                    "sigma_rel_diff_max": float(np.max(np.abs(sk - sf) / sf))}
    first = "fp32" if "fp32" in out else "fp64"
    line = {
        "metric": "NLL, gradient and Hessian: one-pass Hessian kernel vs central differences of the gradient",
        "value": n / (out[first]["hessian_ms"] * 1e-3), "unit": "events/s (Hessian pass, %s columns)" % first,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": args.workload, "events": n, "parameters": progs[first].n_params,
                   "step": "one synchronous NLL + gradient + Hessian (FP64 per event)"},
        **out,
    }
    emit(line)


def run_combined(args, torch, stream):
    """A combined likelihood (rf_sum_*): the 1e7-event 1-D mixture (FP32+
    adjoint) and the 200 x 4 x 100 binned model with 60 nuisances, the
    binned signal strength sharing the mixture's fraction f, and a Gaussian
    constraint on the mixture's mean.  One synchronous combined evaluation
    against the two terms' own synchronous evaluations."""
    from paper_2003_12861_amd import api, synth
    spec, cols, theta, thetas, _, _ = make("gauss_cheb_1e7")
    p = api.Program(api.Graph.from_spec(spec), precision=api.FP32)
    p.bind([torch.tensor(c, dtype=torch.float32, device="cuda") for c in cols])
    d = synth.make_binned(5, 200, 4, 100, 60)
    bn = api.Binned(d["T"], d["Tp"], d["Tm"], d["nobs"], stream=stream)
    bmap = [2] + list(range(5, 65))
    s = api.Sum(65).add(p, range(5)).add(bn, bmap).constrain(0, 0.0, 0.05)
    rng = np.random.default_rng(7)
    ths = [np.concatenate([np.asarray(t), rng.uniform(-0.5, 0.5, 60)]) for t in thetas]
    calls = {"combined": lambda th: s.nll_grad(th, stream=stream),
             "mixture_alone": lambda th: p.nll_grad(th[:5], stream=stream),
             "binned_alone": lambda th: bn.nll_grad(th[bmap], stream=stream),
             "both_terms_enqueued": lambda th: (p.nll_grad_async(th[:5], stream=stream),
                                                bn.nll_grad(th[bmap], stream=stream))}
    out = {}
    gc.collect()
    for name, f in calls.items():
        for i in range(args.warmup):
            f(ths[i % len(ths)])
        step_s, med_s = timed_steps(f, ths, args.steps, torch)
        out[name] = {"ms_per_step": step_s * 1e3, "median_step_ms": med_s * 1e3}
    line = {
        "metric": "synchronous NLL+gradient of a combined likelihood (1-D mixture + binned model, shared parameter, constraint)",
        "value": 1.0 / (out["combined"]["ms_per_step"] * 1e-3), "unit": "evaluations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
        "config": {"terms": ["gauss_cheb_1e7 (fp32+adjoint)", "binned_200x4x100x60"], "global_parameters": 65,
                   "step": "one synchronous combined evaluation (terms' kernels and the combining kernel)"},
        **out,
    }
    emit(line)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="gauss_cheb_1e7", choices=WORKLOADS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 path (profiling runs)")
    ap.add_argument("--unfused-ablation", action="store_true",
                    help="fused vs unfused per-node NLL (gauss_cheb_1e7, decay_argus_5e7)")
    ap.add_argument("--hessian", action="store_true",
                    help="one-pass Hessian kernel vs central differences of the gradient (gauss_cheb_1e7, "
                         "gauss_cheb_extended_1e7, decay_argus_5e7)")
    ap.add_argument("--combined", action="store_true",
                    help="a combined likelihood: the 1-D mixture and the binned model with a shared parameter")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 512 MiB device copy (scale reference for HBM counters)")
    ap.add_argument("--peaks", action="store_true",
                    help="instead, measure the ceilings (issue rates of the kernels' instruction mixes, streaming "
                         "bandwidth) and print them as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_12861_amd import api

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.peaks:
        run_peaks(api)
        return
    if args.workload.startswith("binned"):
        run_binned(args, torch, stream)
        return
    if args.combined:
        run_combined(args, torch, stream)
        return
    spec, cols, theta, thetas, precs_avail, w32 = make(args.workload)
    n = cols[0].size
    precs = [p for p in precs_avail if not (args.fp32_only and p == "fp64")]
    pmap = {"fp32": (api.FP32, torch.float32), "fp64": (api.FP64, torch.float64)}
    wbf = torch.tensor(w32, device="cuda").to(torch.bfloat16) if w32 is not None else None

    weighted = args.workload in WEIGHTED

    def program(key, columns):
        prec, dt = pmap[key]
        p = api.Program(api.Graph.from_spec(spec), precision=prec, weighted=weighted)
        p.bind([torch.tensor(c, dtype=dt, device="cuda") for c in columns])
        if wbf is not None:
            p.bind_weights("sig", wbf)
        return p

    progs = {key: program(key, cols) for key in precs}

    if args.unfused_ablation:
        run_unfused_ablation(args, progs, cols, thetas, n, torch, stream)
        return
    if args.hessian:
        run_hessian(args, progs, thetas, n, torch, stream)
        return

    if args.calib_copy:
        a = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    res = {}
    for key, p in progs.items():
        res[key] = time_path(lambda th, p=p: p.nll_grad(th, stream=stream),
                             lambda th, p=p: p.nll_grad_async(th, stream=stream), thetas, args, torch, stream)

    # validity of each path against the oracle at the truth point
    cpu = None
    heavy = args.workload.startswith("bwcb")  # the convolution models: checked on a prefix
    if not args.no_cpu_baseline:
        from oracle import rfo
        om, otop, oids = rfo.from_spec(spec)
        if wbf is not None:
            om.set_mlp_weights(oids["sig"], wbf.float().double().cpu().numpy())
        # bounded sample: oracle evaluations for ~10 s (whole workload, or a
        # 20000-event prefix of the convolution models, scaled to events/s)
        sample = [c[:20000] for c in cols] if heavy else cols
        obs, wts = (sample[:-1], sample[-1]) if weighted else (sample, None)
        onll, og, oga, _ = om.nll_ex(otop, theta, obs, weights=wts)
        rate, reps = oracle_rate(lambda: om.nll_ex(otop, theta, obs, weights=wts), sample[0].size, 10.0)
        what = ("%d NLL+gradient evaluations of a %d-event prefix" % (reps, sample[0].size) if heavy
                else "%d full NLL+gradient evaluations of the %d-event workload" % (reps, n))
        cpu = dict(value=rate, unit="events/s", cores=1, kind="oracle",
                   sample=what + " (single-threaded C, -O2)",
                   host=platform.processor() or platform.machine(), nproc=os.cpu_count())
        tol = {"fp32": 1e-6, "fp64": 1e-9}
        for key, p in progs.items():
            q = program(key, sample) if heavy else p
            nll, g, _ = q.nll_grad(theta)
            res[key]["nll_rel_err"] = abs(nll - onll) / abs(onll)
            res[key]["grad_scaled_err"] = float(np.max(np.abs(g - og) / oga))
            res[key]["valid"] = bool(res[key]["nll_rel_err"] <= tol[key] and res[key]["grad_scaled_err"] <= tol[key])
            res[key]["checked_on"] = ("a %d-event prefix" % sample[0].size) if heavy else "all events"

    k32 = res["fp32"]["kernel_s"]
    if wbf is not None:
        # the roofline time is the largest of the bounds: VALU (the tanh and
        # operand splitting) over MFMA (the network's multiply-adds)
        achieved = n * SURROGATE_SLOTS_PER_EVENT / k32 / 1e12
        peak = VALU_SLOTS_PER_S / 1e12
        mfma = n * 2 * SURROGATE_MAC_PER_EVENT / k32 / 1e12
        roof = {"bound": "alu", "kernel": "rf_k_grad_f32 (MLP leaf) with its normalisation kernel",
                "achieved": achieved, "peak": peak, "unit": "Tslot/s", "frac": achieved / peak, "traffic": None,
                "slots_per_event": SURROGATE_SLOTS_PER_EVENT, "events_per_launch": n,
                "mfma": {"achieved_tflops": mfma, "peak_tflops": MFMA_BF16_TFLOPS, "frac": mfma / MFMA_BF16_TFLOPS,
                         "flop_per_event": 2 * SURROGATE_MAC_PER_EVENT}}
    else:
        slots = SLOTS[args.workload]["fp32"]
        achieved = n * slots / k32 / 1e12
        peak = VALU_SLOTS_PER_S / 1e12
        roof = {"bound": "alu", "kernel": "rf_k_grad_f32", "achieved": achieved, "peak": peak,
                "unit": "Tslot/s", "frac": achieved / peak,
                "traffic": measured_traffic(args.workload, "rf_k_grad_f32", progs["fp32"].source),
                "source_sha1": hashlib.sha1(progs["fp32"].source.encode()).hexdigest(),
                "slots_per_event": slots, "events_per_launch": n}
    roof["bytes_per_event"] = BYTES_PER_EVENT[args.workload]["fp32"]
    roof["hbm_GBps"] = n * BYTES_PER_EVENT[args.workload]["fp32"] / k32 / 1e9
    # against the ceilings measured on this device (profiles/peaks_mi355x.txt):
    # the issue rate of the kernel's instruction mix and the streaming read
    mix = measured_ceiling(MIX[args.workload])
    stream_bw = measured_ceiling("stream_read_bytes")
    if mix:
        roof["measured_ceiling"] = {"valu_mix": MIX[args.workload], "valu_Tslot_per_s": mix / 1e12,
                                    "frac_valu": roof["achieved"] / (mix / 1e12)}
        if stream_bw:
            roof["measured_ceiling"].update({"stream_GBps": stream_bw / 1e9,
                                             "frac_hbm": roof["hbm_GBps"] / (stream_bw / 1e9)})
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
        "data": "synthetic" + ("; random-init surrogate weights" if wbf is not None else ""),
        "config": {"workload": args.workload, "events": n, "precision": "fp32+adjoint, fp64 reductions",
                   "step": "one synchronous NLL+gradient evaluation (result in host memory)"},
        "fp32": {"kernel_ms": k32 * 1e3, "isolated_kernel_ms": res["fp32"]["isolated_s"] * 1e3,
                 "cold_cache_kernel_ms": res["fp32"]["cold_s"] * 1e3,
                 "median_step_ms": res["fp32"]["median_step_s"] * 1e3,
                 "step_us_min_max": res["fp32"]["step_us_min_max"],
                 "kernel_events_per_s": n / k32,
                 "nll_rel_err": res["fp32"].get("nll_rel_err"),
                 "grad_scaled_err": res["fp32"].get("grad_scaled_err"),
                 "valid": res["fp32"].get("valid"),
                 "checked_on": res["fp32"].get("checked_on")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "fp64" in res:
        slots64 = SLOTS.get(args.workload, {}).get("fp64")
        line["fp64_plain"] = {"value": n / res["fp64"]["step_s"], "unit": "events/s",
                              "ms_per_step": res["fp64"]["step_s"] * 1e3,
                              "median_step_ms": res["fp64"]["median_step_s"] * 1e3,
                              "kernel_ms": res["fp64"]["kernel_s"] * 1e3,
                              "isolated_kernel_ms": res["fp64"]["isolated_s"] * 1e3,
                              "cold_cache_kernel_ms": res["fp64"]["cold_s"] * 1e3,
                              "kernel_events_per_s": n / res["fp64"]["kernel_s"],
                              "roofline_frac": (n * slots64 / res["fp64"]["kernel_s"] / VALU_SLOTS_PER_S
                                                if slots64 else None),
                              "nll_rel_err": res["fp64"].get("nll_rel_err"),
                              "grad_scaled_err": res["fp64"].get("grad_scaled_err"),
                              "valid": res["fp64"].get("valid")}
    emit(line)


if __name__ == "__main__":
    main()
