"""Benchmark of the twofold exp/log hot path on one MI355X.

One step = the four binary64 twofold functions texp, texpm1, tlog, tlog1p,
each over its own 2^26-element split arrays x0, x1 -> z0, z1 (inputs resident
in HBM, seeded synthetic data of the paper's random-sample kind, 0.1% edge
arguments).  value = elements per second over the whole step (Gelem/s).

Printed as one JSON line on stdout; progress goes to stderr.  Extra fields:
per-function binary64 and binary32 rates from HIP events on the launch stream;
the roofline of the dominant kernel (algorithmic FP64 flops from the oracle's
counting build, tests/golden/opcounts.json, over the measured kernel time);
the batched launch over 4096 ragged arrays of mixed function and format
against the per-array launches and the mix-weighted plain rate; the forward
and backward chain tlog1p(texpm1(texp(x))) at 2^24; the other entry points of
the paper's interface at 2^26; the twofold arithmetic (tadd, tsub, tmul, tdiv,
tsqrt, trenorm) at 2^26; texp on the small 65536-element workload, with the
oracle timed on it at one thread and all threads; and the CPU oracle timed on
the host cores over the step's arrays.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-f32]
                    [--no-batch] [--no-chain] [--no-interface] [--no-arith]
                    [--variant horner2x|k6|accexp]
"""
import argparse
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
# binary32: the published FP32 vector peak counts packed FP32 (two operations
# per lane per instruction): 256 x 4 x 16 x 2 x 2.4 GHz = 78.6 T lane-operations/s,
# 157.3 TFLOP/s with an FMA as 2.  The kernels are built without packed FP32,
# and plain FP32 arithmetic issues at the FP64 lane rate (a probe of long
# independent FMA, add and mul chains measures 38 T lane-operations/s at the
# clock under load), so 39.3 T is the ceiling of the code as built.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_ISSUE_T = 78.6
PEAK_FP32_NONPACKED_T = 39.3
PEAK_HBM_GBS = 8000.0
BYTES_PER_ELEM = {"f64": 32, "f32": 16}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash():
    from paper_1502_05216_amd._build import source_hash
    return source_hash()


def kernel_ms(fn, args, reps, warm=5, windows=2):
    """Duration of one launch: HIP events on the launch stream around `reps`
    back-to-back launches after `warm` untimed ones; the faster of `windows`
    such windows (the first can still see the clock ramp up)."""
    import torch
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(warm):
        fn(*args)
    best = float("inf")
    for _ in range(windows):
        e0.record(st)
        for _ in range(reps):
            fn(*args)
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


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


PAPER_MOPS_PER_CORE = {"texp": 11.86, "texpm1": 12.28, "tlog": 7.00, "tlog1p": 7.06}


def host_cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(inputs64, min_seconds, core_sample):
    """The oracle on the host: whole passes over the step's binary64 arrays on
    up to 16 threads until min_seconds have passed, plus a one-thread rate per
    function on the first core_sample elements (the paper's per-core figure)."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    t, passes = 0.0, 0
    while passes == 0 or t < min_seconds:
        for fn in FUNCS:
            x0, x1 = inputs64[fn]
            t0 = time.perf_counter()
            getattr(oracle, fn)(x0, x1, threads=threads)
            t += time.perf_counter() - t0
        passes += 1
        log("cpu baseline: pass %d, %.1f s" % (passes, t))
    n = inputs64[FUNCS[0]][0].size
    per_core = {}
    for fn in FUNCS:
        a0 = np.ascontiguousarray(inputs64[fn][0][:core_sample])
        a1 = np.ascontiguousarray(inputs64[fn][1][:core_sample])
        t0 = time.perf_counter()
        getattr(oracle, fn)(a0, a1, threads=1)
        per_core[fn] = {"mops": core_sample / (time.perf_counter() - t0) / 1e6,
                        "paper_mops": PAPER_MOPS_PER_CORE[fn]}
    # context: the comparison systems of the paper's performance table, one
    # thread, on the same arguments: libquadmath (expq ...) and the C library
    from oracle import qref
    context = {}
    for fn in FUNCS:
        x = np.ascontiguousarray(inputs64[fn][0][:1 << 16])
        xs = x[np.isfinite(x)]
        q = qref.context_mops(fn, xs, quad=True)
        c = qref.context_mops(fn, np.ascontiguousarray(inputs64[fn][0][:1 << 20]), quad=False)
        context[fn] = {"quadmath_mops": q, "libm_mops": c,
                       "twofold_over_quadmath": per_core[fn]["mops"] / q}
    return {"value": passes * 4 * n / t / 1e9, "unit": "Gelem/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d whole pass(es) over the step's 4 binary64 arrays of %d elements, "
                      "scalar oracle, OpenMP static schedule" % (passes, n),
            "seconds": t, "host_cpus": os.cpu_count(), "host_cpu_model": host_cpu_model(),
            "one_thread": {"sample": core_sample, "per_function": per_core},
            "context_one_thread": context}


def bench_small(tf, workloads, reps=200):
    """texp on the small binary64 workload (65536 twofolds, x0 ~ U[-700, 700],
    x1 = x0 u 2^-53, no edges): the launch-bound end of the range.  Two rates:
    the device time of one launch, from a HIP graph of `reps` launches replayed
    (no host work between launches), and the eager rate of `reps` back-to-back
    calls through the Python binding (host-bound at this size)."""
    import torch
    dev = torch.device("cuda:0")
    a, b = workloads.cfg1_inputs()
    x0 = torch.from_numpy(a).to(dev)
    x1 = torch.from_numpy(b).to(dev)
    o = (torch.empty_like(x0), torch.empty_like(x0))
    eager_ms = kernel_ms(lambda: tf.texp(x0, x1, out=o), (), reps, warm=20, windows=3)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            tf.texp(x0, x1, out=o)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            tf.texp(x0, x1, out=o)
    graph_ms = kernel_ms(g.replay, (), 1, warm=3, windows=5) / reps
    n = a.size
    return {"n": n, "us": graph_ms * 1e3, "gelem_s": n / graph_ms / 1e6,
            "timing": "device time per launch: a HIP graph of %d launches, replayed" % reps,
            "eager_us": eager_ms * 1e3, "eager_gelem_s": n / eager_ms / 1e6,
            "inputs": (a, b)}


def cpu_small(a, b, runs=5):
    """The oracle's texp on the small workload: median of `runs` passes on one
    thread and on up to 16 threads."""
    import oracle
    res = {}
    for label, th in (("one_thread", 1), ("all_threads", max(1, min(16, os.cpu_count() or 1)))):
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.texp(a, b, threads=th)
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[runs // 2]
        res[label] = {"threads": th, "us": t * 1e6, "mops": a.size / t / 1e6}
    return res


def bench_batch(tf, workloads, per64, per32, reps):
    """The batched ragged launch over 4096 arrays (function uniform over the
    four, binary64 with probability 3/4, lengths 2^U[0, 20]) against (i) one
    plain launch per array and (ii) the plain 2^26 rates weighted by the mix."""
    import torch
    from paper_1502_05216_amd.batch import BatchPlan
    dev = torch.device("cuda:0")
    descs = workloads.batch_descriptors()
    host = workloads.batch_inputs(descs)
    items = []
    for fn, dt, x0, x1 in host:
        a0 = torch.from_numpy(np.ascontiguousarray(x0)).to(dev)
        a1 = torch.from_numpy(np.ascontiguousarray(x1)).to(dev)
        items.append((fn, a0, a1, torch.empty_like(a0), torch.empty_like(a0)))
    del host
    total = sum(it[1].numel() for it in items)
    # autotuned tile parameters: every candidate configuration timed on this
    # batch (outside the timed region), then the fastest timed like the rest
    from paper_1502_05216_amd.batch import DEFAULT_CONFIG, autotune
    config, cand = autotune(items, reps=3)
    with BatchPlan(items, config=config) as plan:
        ms = kernel_ms(plan.launch, (), reps)

    def loop():
        for fn, a0, a1, z0, z1 in items:
            getattr(tf, fn)(a0, a1, out=(z0, z1))
    loop_ms = kernel_ms(loop, (), 2, warm=1, windows=1)
    mix_ms = None
    if per32:
        mix_ms = 0.0
        for fn, a0, _, _, _ in items:
            rate = (per64[fn]["windowed_gelem_s"] if a0.dtype == torch.float64
                    else per32[fn]["gelem_s"])
            mix_ms += a0.numel() / rate / 1e6
    del items
    torch.cuda.empty_cache()
    return {"arrays": len(descs), "elements": total, "config": list(config),
            "autotune": {"candidates": len(cand), "default_config": list(DEFAULT_CONFIG),
                         "default_config_ms": cand.get(tuple(DEFAULT_CONFIG))}, "ms": ms,
            "gelem_s": total / ms / 1e6, "per_array_launches_ms": loop_ms,
            "per_array_launches_gelem_s": total / loop_ms / 1e6,
            "mix_weighted_plain_gelem_s": None if mix_ms is None else total / mix_ms / 1e6,
            "vs_mix_weighted_plain": None if mix_ms is None else mix_ms / ms}


def bench_interface(tf, workloads, opc, reps, dtypes):
    """The other entry points of the paper's interface on 2^26 elements each
    (dotted argument: x0 -> z0, z1, 24 B per binary64 element; coupled
    argument: 32 B)."""
    import torch
    dev = torch.device("cuda:0")
    res = {}
    for key, dt in (("f64", np.float64), ("f32", np.float32)):
        if key not in dtypes:
            continue
        res[key] = {}
        for name in workloads.DOTTED + workloads.COUPLED:
            dotted = name in workloads.DOTTED
            a, b = workloads.twofold_inputs(name, N, dt, coupled=not dotted)
            x0 = torch.from_numpy(a).to(dev)
            x1 = None if dotted else torch.from_numpy(b).to(dev)
            out = (torch.empty_like(x0), torch.empty_like(x0))
            if dotted:
                ms = kernel_ms(lambda: getattr(tf, name)(x0, out=out), (), reps)
            else:
                ms = kernel_ms(lambda: getattr(tf, name)(x0, x1, out=out), (), reps)
            isz = 8 if key == "f64" else 4
            nbytes = (3 if dotted else 4) * isz
            c = opc[key][name]
            res[key][name] = {"ms": ms, "gelem_s": N / ms / 1e6,
                              "hbm_gbs": N * nbytes / ms / 1e6, "bytes_per_elem": nbytes,
                              "tflops": N * c["flops"] / ms / 1e9,
                              "issue_frac": N * c["ops"] / (ms * 1e-3) / (PEAK_FP64_ISSUE_T * 1e12),
                              "traffic": traffic_for("%s_%s" % (key, name), N)}
            log("%s %-8s %.3f ms  %.1f Gelem/s" % (key, name, ms, res[key][name]["gelem_s"]))
            del x0, x1, out
        torch.cuda.empty_cache()
    return res


def bench_arith(tf, reps, dtypes):
    """Twofold arithmetic (tadd, tsub, tmul, tdiv, tsqrt, trenorm) on 2^26
    elements: 48 B per binary64 element for the binary operations, 32 B for
    tsqrt and trenorm (of the pair x0, y0); all are bound by HBM."""
    import torch
    dev = torch.device("cuda:0")
    res = {}
    rng = np.random.default_rng(1502052161)
    for key, dt in (("f64", np.float64), ("f32", np.float32)):
        if key not in dtypes:
            continue
        eps = dt(2.0 ** (-53 if key == "f64" else -24))
        arrs = []
        for _ in range(2):
            a0 = (np.exp2(rng.uniform(-30, 30, N)) * np.where(rng.uniform(-1, 1, N) < 0, -1, 1)
                  ).astype(dt)
            arrs += [a0, ((a0 * rng.uniform(-1, 1, N).astype(dt)) * eps).astype(dt)]
        x0, x1, y0, y1 = [torch.from_numpy(a).to(dev) for a in arrs]
        ax0 = x0.abs()
        out = (torch.empty_like(x0), torch.empty_like(x0))
        res[key] = {}
        isz = 8 if key == "f64" else 4
        for op in ("tadd", "tsub", "tmul", "tdiv", "tsqrt", "trenorm"):
            if op == "tsqrt":
                ms = kernel_ms(lambda: tf.tsqrt(ax0, x1, out=out), (), reps)
                nbytes = 4 * isz
            elif op == "trenorm":
                ms = kernel_ms(lambda: tf.trenorm(x0, y0, out=out), (), reps)
                nbytes = 4 * isz
            else:
                ms = kernel_ms(lambda: getattr(tf, op)(x0, x1, y0, y1, out=out), (), reps)
                nbytes = 6 * isz
            res[key][op] = {"ms": ms, "gelem_s": N / ms / 1e6, "bytes_per_elem": nbytes,
                            "hbm_gbs": N * nbytes / ms / 1e6,
                            "hbm_frac": N * nbytes / ms / 1e6 / PEAK_HBM_GBS}
            log("%s %-6s %.3f ms  %.1f Gelem/s  %.0f GB/s" % (key, op, ms, res[key][op]["gelem_s"],
                                                             res[key][op]["hbm_gbs"]))
        del x0, x1, y0, y1, ax0, out
        torch.cuda.empty_cache()
    return res


def bench_chain(tf, workloads, reps):
    """Forward and backward of y = tlog1p(texpm1(texp(x))) on 2^24 binary64
    twofolds: three forward launches and one fused backward pass
    (tf_chain_bwd: reads g and the saved a, b once, writes gx); also timed
    with the three single-stage backward launches instead."""
    import torch
    dev = torch.device("cuda:0")
    n = 1 << 24
    arrs = [torch.from_numpy(a).to(dev) for a in workloads.chain_inputs(n)]
    x0, x1, g0, g1 = arrs
    buf = [torch.empty_like(x0) for _ in range(12)]

    def fwd():
        a = tf.texp(x0, x1, out=(buf[0], buf[1]))
        b = tf.texpm1(*a, out=(buf[2], buf[3]))
        tf.tlog1p(*b, out=(buf[4], buf[5]))
        return a, b

    def fwd_bwd():
        a, b = fwd()
        tf.chain_bwd(("texp", "texpm1", "tlog1p"), (a, b, b), g0, g1, out=(buf[10], buf[11]))

    def fwd_bwd_stagewise():
        a, b = fwd()
        c = tf.tlog1p_bwd(*b, g0, g1, out=(buf[6], buf[7]))
        d = tf.texpm1_bwd(*b, *c, out=(buf[8], buf[9]))
        tf.texp_bwd(*a, *d, out=(buf[10], buf[11]))
    ms = kernel_ms(fwd_bwd, (), reps)
    ms_stage = kernel_ms(fwd_bwd_stagewise, (), reps)
    # elements whose texpm1 stage overflows (x0 above ln ln DBL_MAX: y = inf
    # and a NaN gradient), counted apart as the chain's workload states
    fwd_bwd()
    overflow = int((~torch.isfinite(buf[4])).sum())
    nan_grad = int((~torch.isfinite(buf[10])).sum())
    del arrs, buf
    torch.cuda.empty_cache()
    return {"n": n, "ms": ms, "gelem_s": n / ms / 1e6,
            "overflow_elements": overflow, "nonfinite_gradients": nan_grad,
            "launches": 4, "hbm_bytes_per_elem": 3 * 32 + 64,
            "stagewise_backward": {"ms": ms_stage, "gelem_s": n / ms_stage / 1e6,
                                   "launches": 6, "hbm_bytes_per_elem": 3 * 32 + 3 * 48}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # After the host-side input generation the GPU has idled for seconds; its
    # clocks take about 10 steps (20 ms) of this load to settle, so the default
    # warmup covers that.
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f32", action="store_true", help="skip the binary32 rates")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched launch")
    ap.add_argument("--no-chain", action="store_true", help="skip the forward+backward chain")
    ap.add_argument("--no-interface", action="store_true",
                    help="skip the other entry points of the interface")
    ap.add_argument("--no-arith", action="store_true", help="skip the twofold arithmetic")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU oracle time (whole passes over the step)")
    ap.add_argument("--cpu-core-sample", type=int, default=1 << 21)
    ap.add_argument("--variant", default=None,
                    help="time the step with a flagged build variant of the library "
                         "(paper_1502_05216_amd/_build.py VARIANTS, e.g. k6)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the functions are "
              "elementwise; a multi-GPU run would give each GPU a contiguous element range)",
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

    stream = torch.cuda.current_stream()
    if args.variant:
        from paper_1502_05216_amd import _lib
        vlib = _lib.variant(args.variant)
        log("step timed with build variant %s: %s" % (args.variant, vlib.tf_version().decode()))

        def call(fn, a, b, out):
            return _lib.twofold_call(fn, a, b, out=out, lib=vlib)
    else:
        def call(fn, a, b, out):
            return getattr(tf, fn)(a, b, out=out)

    def step(marks=None):
        # marks: one HIP event before the first launch and one after each
        # launch, recorded on the stream the kernels run on
        if marks is not None:
            marks[0].record(stream)
        for k, fn in enumerate(FUNCS):
            call(fn, dev64[fn][0], dev64[fn][1], out64[fn])
            if marks is not None:
                marks[k + 1].record(stream)

    log("warmup %d steps" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    marks = [[torch.cuda.Event(enable_timing=True) for _ in range(len(FUNCS) + 1)]
             for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(marks[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = 4 * N * args.steps / dt / 1e9

    with open(os.path.join(ROOT, "tests", "golden", "opcounts.json")) as f:
        opc = json.load(f)

    # average launch duration of each kernel over the timed steps
    per64 = {}
    for j, fn in enumerate(FUNCS):
        ms = sum(m[j].elapsed_time(m[j + 1]) for m in marks) / args.steps
        per64[fn] = {"ms": ms, "gelem_s": N / ms / 1e6,
                     "fp64_tflops": N * opc["f64"][fn]["flops"] / ms / 1e9,
                     "hbm_gbs": N * BYTES_PER_ELEM["f64"] / ms / 1e6}
        # the same kernel timed like the binary32 and batched launches below
        w = kernel_ms(lambda: call(fn, dev64[fn][0], dev64[fn][1], out64[fn]), (), 10)
        per64[fn]["windowed_gelem_s"] = N / w / 1e6
        log("f64 %-7s %.3f ms  %.1f Gelem/s (windowed %.1f)" % (fn, ms, per64[fn]["gelem_s"],
                                                              per64[fn]["windowed_gelem_s"]))
    dom = max(FUNCS, key=lambda f: per64[f]["ms"])
    ach = per64[dom]["fp64_tflops"]
    traffic = None if args.variant else traffic_for("f64_" + dom, N)
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
            ms = kernel_ms(lambda: getattr(tf, fn)(x0, x1, out=o), (), 20, warm=10, windows=4)
            ops_s = N * opc["f32"][fn]["ops"] / (ms * 1e-3)
            per32[fn] = {"ms": ms, "gelem_s": N / ms / 1e6,
                         "fp32_tflops": N * opc["f32"][fn]["flops"] / ms / 1e9,
                         "frac": N * opc["f32"][fn]["flops"] / ms / 1e9 / PEAK_FP32_TFLOPS,
                         "issue_frac": ops_s / (PEAK_FP32_ISSUE_T * 1e12),
                         "nonpacked_issue_frac": ops_s / (PEAK_FP32_NONPACKED_T * 1e12),
                         "hbm_gbs": N * BYTES_PER_ELEM["f32"] / ms / 1e6,
                         "hbm_frac": N * BYTES_PER_ELEM["f32"] / ms / 1e6 / PEAK_HBM_GBS}
            log("f32 %-7s %.3f ms  %.1f Gelem/s" % (fn, ms, per32[fn]["gelem_s"]))
            del x0, x1, o

    log("small workload: texp, 65536 binary64 twofolds")
    small = bench_small(tf, workloads)
    small_in = small.pop("inputs")
    log("small texp %.2f us  %.1f Gelem/s (eager calls %.2f us)" % (small["us"], small["gelem_s"],
                                                                   small["eager_us"]))

    batch = None
    if not args.no_batch:
        log("batched launch: 4096 ragged arrays")
        batch = bench_batch(tf, workloads, per64, per32, 10)
        log("batched %.3f ms  %.1f Gelem/s  (per-array launches %.1f ms, vs mix-weighted plain %s)"
            % (batch["ms"], batch["gelem_s"], batch["per_array_launches_ms"],
               batch["vs_mix_weighted_plain"]))

    chain = None
    if not args.no_chain:
        log("forward+backward chain, 2^24")
        chain = bench_chain(tf, workloads, 10)
        log("chain %.3f ms  %.1f Gelem/s (single-stage backward launches %.3f ms); "
            "%d of %d elements overflow at texpm1" % (chain["ms"], chain["gelem_s"],
                                                      chain["stagewise_backward"]["ms"],
                                                      chain["overflow_elements"], chain["n"]))

    iface = None
    if not args.no_interface:
        log("other interface functions, 2^26 each")
        iface = bench_interface(tf, workloads, opc, 10, ("f64",) if args.no_f32 else ("f64", "f32"))

    arith = None
    if not args.no_arith:
        log("twofold arithmetic, 2^26 each")
        arith = bench_arith(tf, 10, ("f64",) if args.no_f32 else ("f64", "f32"))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: oracle, at least %.0f s" % args.cpu_seconds)
        cpu = cpu_baseline(host64, args.cpu_seconds, args.cpu_core_sample)
        log("cpu baseline %.4f Gelem/s on %d threads (%.1f s)" % (cpu["value"], cpu["cores"],
                                                                cpu["seconds"]))
        small["oracle"] = cpu_small(*small_in)
        for k in ("one_thread", "all_threads"):
            small["gpu_vs_oracle_" + k] = small["oracle"][k]["us"] / small["us"]
        log("small texp oracle: %.0f us on 1 thread, %.0f us on %d threads"
            % (small["oracle"]["one_thread"]["us"], small["oracle"]["all_threads"]["us"],
               small["oracle"]["all_threads"]["threads"]))

    rec = {
        "metric": "Gelem/s per twofold fn (double & float) + % FP64 peak; batched vs plain, 1 GPU",
        "value": value, "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "texp+texpm1+tlog+tlog1p binary64 twofolds, 2^26 elements each "
                               "(SoA x0,x1 -> z0,z1), 0.1% edge arguments",
                   "n_per_function": N, "functions": list(FUNCS)},
        "variant": args.variant,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_function_f64": per64,
        "per_function_f32": per32,
        "small_texp": small,
        "batched": batch,
        "fwd_bwd_chain": chain,
        "interface": iface,
        "arith": arith,
        "src_hash": src_hash(),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
