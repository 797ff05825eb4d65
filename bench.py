"""Benchmark of the twofold exp/log hot path on one MI355X.

One step = the four binary64 twofold functions texp, texpm1, tlog, tlog1p,
each over its own 2^26-element split arrays x0, x1 -> z0, z1 (inputs resident
in HBM, seeded synthetic data of the paper's random-sample kind, 0.1% edge
arguments).  value = elements per second over the whole step (Gelem/s).

Printed as one JSON line on stdout; progress goes to stderr.  Extra fields:
per-function binary64 and binary32 rates from HIP events on the launch stream,
the roofline of the dominant kernel (algorithmic FP64 flops from the oracle's
counting build, tests/golden/opcounts.json, over the measured kernel time),
and the CPU oracle timed on the host cores on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 1 << 26
FUNCS = ("texp", "texpm1", "tlog", "tlog1p")
PEAK_FP64_TFLOPS = 78.6          # MI355X dense FP64 vector, FMA = 2 flops
PEAK_FP64_ISSUE_T = 39.3         # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz, one op per lane
PEAK_HBM_GBS = 8000.0
BYTES_PER_ELEM = {"f64": 32, "f32": 16}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1502_05216_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1502_05216_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_ms(fn, args, reps):
    """Average duration of one launch, HIP events on the launch stream."""
    import torch
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn(*args)
    e0.record(st)
    for _ in range(reps):
        fn(*args)
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def traffic_for(kernel, n_elem):
    """HBM bytes per launch measured by rocprofv3 counters for this kernel source,
    or None when the counters were taken on other kernel code."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    rec = t.get("kernels", {}).get(kernel)
    if not rec or rec.get("src_hash") != src_hash() or rec.get("n") != n_elem:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(inputs64, sample):
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    t = 0.0
    for fn in FUNCS:
        x0, x1 = inputs64[fn]
        a0 = np.ascontiguousarray(x0[:sample])
        a1 = np.ascontiguousarray(x1[:sample])
        t0 = time.perf_counter()
        getattr(oracle, fn)(a0, a1, threads=threads)
        t += time.perf_counter() - t0
    return {"value": 4 * sample / t / 1e9, "unit": "Gelem/s", "cores": threads, "kind": "oracle",
            "sample": "the first %d elements of each of the 4 binary64 benchmark arrays "
                      "(%d elements), scalar oracle, OpenMP static schedule" % (sample, 4 * sample),
            "seconds": t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f32", action="store_true", help="skip the binary32 rates")
    ap.add_argument("--cpu-sample", type=int, default=N)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the functions are "
              "elementwise; sharding is by contiguous element ranges, see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1502_05216_amd as tf
    from paper_1502_05216_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tf.lib()
    dev = torch.device("cuda:0")

    log("generating inputs (2^26 per function, binary64 and binary32)")
    host64 = {fn: workloads.twofold_inputs(fn, N, np.float64) for fn in FUNCS}
    dev64 = {fn: (torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
             for fn, (a, b) in host64.items()}
    out64 = {fn: (torch.empty_like(a), torch.empty_like(a)) for fn, (a, _) in dev64.items()}
    torch.cuda.synchronize()

    def step():
        for fn in FUNCS:
            getattr(tf, fn)(dev64[fn][0], dev64[fn][1], out=out64[fn])

    log("warmup %d steps" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = 4 * N * args.steps / dt / 1e9

    with open(os.path.join(ROOT, "tests", "golden", "opcounts.json")) as f:
        opc = json.load(f)

    per64 = {}
    for fn in FUNCS:
        ms = kernel_ms(lambda: getattr(tf, fn)(dev64[fn][0], dev64[fn][1], out=out64[fn]), (), 10)
        per64[fn] = {"ms": ms, "gelem_s": N / ms / 1e6,
                     "fp64_tflops": N * opc["f64"][fn]["flops"] / ms / 1e9,
                     "hbm_gbs": N * BYTES_PER_ELEM["f64"] / ms / 1e6}
        log("f64 %-7s %.3f ms  %.1f Gelem/s" % (fn, ms, per64[fn]["gelem_s"]))
    dom = max(FUNCS, key=lambda f: per64[f]["ms"])
    ach = per64[dom]["fp64_tflops"]
    traffic = traffic_for("f64_" + dom, N)
    roofline = {"bound": "alu", "kernel": "k_twofold<double,%s>" % dom, "achieved": ach,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                "traffic": traffic,
                "flops_per_elem": opc["f64"][dom]["flops"], "elems_per_launch": N,
                "issue_frac": N * opc["f64"][dom]["ops"] / (per64[dom]["ms"] * 1e-3)
                / (PEAK_FP64_ISSUE_T * 1e12),
                "hbm_frac": per64[dom]["hbm_gbs"] / PEAK_HBM_GBS}

    per32 = {}
    if not args.no_f32:
        del out64
        torch.cuda.empty_cache()
        for fn in FUNCS:
            a, b = workloads.twofold_inputs(fn, N, np.float32)
            x0 = torch.from_numpy(a).to(dev)
            x1 = torch.from_numpy(b).to(dev)
            o = (torch.empty_like(x0), torch.empty_like(x0))
            ms = kernel_ms(lambda: getattr(tf, fn)(x0, x1, out=o), (), 10)
            per32[fn] = {"ms": ms, "gelem_s": N / ms / 1e6,
                         "fp32_tflops": N * opc["f32"][fn]["flops"] / ms / 1e9,
                         "hbm_gbs": N * BYTES_PER_ELEM["f32"] / ms / 1e6}
            log("f32 %-7s %.3f ms  %.1f Gelem/s" % (fn, ms, per32[fn]["gelem_s"]))
            del x0, x1, o

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: oracle on %d elements per function" % args.cpu_sample)
        cpu = cpu_baseline(host64, args.cpu_sample)
        log("cpu baseline %.4f Gelem/s on %d threads (%.1f s)" % (cpu["value"], cpu["cores"],
                                                                cpu["seconds"]))

    rec = {
        "metric": "Gelem/s per twofold fn (double & float) + % FP64 peak; batched vs plain, 1 GPU",
        "value": value, "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "texp+texpm1+tlog+tlog1p binary64 twofolds, 2^26 elements each "
                               "(SoA x0,x1 -> z0,z1), 0.1% edge arguments",
                   "n_per_function": N, "functions": list(FUNCS)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_function_f64": per64,
        "per_function_f32": per32,
        "src_hash": src_hash(),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
