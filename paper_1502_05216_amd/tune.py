"""Autotuner of the launch configuration (elements per thread, workgroups per
compute unit) of every kernel, timed with HIP events on the device, and of
the batched launch (elements per thread, chunk size, workgroups per compute
unit) on the 4096-array ragged batch.

    python -m paper_1502_05216_amd.tune [--n 67108864] [--out PATH] [--batch]

For each function and format it times every candidate on seeded inputs of the
benchmark distribution (at a size well beyond the last-level cache, so that
HBM rather than cache bandwidth is measured), keeps the fastest, and writes a JSON cache keyed by
the device (name, compute units) and the library version.  `apply()` loads the
cache for the current device and sets the configuration in the library.  The
library's built-in defaults are the values this tuner found on MI355X.
"""
import argparse
import json
import os
import sys

import numpy as np

from . import _lib

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
EPTS = (1, 2, 4)
BPCS = (0, 2, 3, 4, 6, 8)
PDS = (1, 2)


def device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    return "%s|%d|%s" % (getattr(p, "gcnArchName", p.name), p.multi_processor_count,
                         _lib.lib().tf_version().decode())


def _time(fn, reps):
    import torch
    st = torch.cuda.current_stream()
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(n=1 << 26, reps=10, funcs=None, dtypes=("f64", "f32"), verbose=True, epts=EPTS,
         bpcs=BPCS):
    """Time all candidates; return {key: {"fn|dtype": [ept, bpc, pd, ms]}}."""
    import torch
    from . import workloads
    dev = torch.device("cuda:0")
    res = {}
    for dts in dtypes:
        dt = np.float64 if dts == "f64" else np.float32
        for fn in funcs or (_lib.TWOFOLD + _lib.ONEX):
            base = {"exp1x": "texp", "expm1_1x": "texpm1", "log1x": "tlog",
                    "log1p_1x": "tlog1p"}.get(fn, fn)
            a, b = workloads.twofold_inputs(base, n, dt)
            x0 = torch.from_numpy(a).to(dev)
            x1 = torch.from_numpy(b).to(dev)
            z0 = torch.empty_like(x0)
            z1 = torch.empty_like(x0)
            if fn in _lib.TWOFOLD:
                call = lambda: _lib.twofold_call(fn, x0, x1, out=(z0, z1))
            else:
                call = lambda: _lib.onex_call(fn, x0, out=z0)
            old = _lib.get_launch_config(fn, dts)
            best = None
            for ept in epts:
                for bpc in bpcs:
                    for pd in (PDS if fn in _lib.TWOFOLD else (1,)):
                        _lib.set_launch_config(fn, dts, ept, bpc, pd)
                        ms = _time(call, reps)
                        if verbose:
                            print("tune %-9s %s ept=%d bpc=%d pd=%d %.4f ms"
                                  % (fn, dts, ept, bpc, pd, ms), flush=True)
                        if best is None or ms < best[3]:
                            best = (ept, bpc, pd, ms)
            _lib.set_launch_config(fn, dts, *old)
            res["%s|%s" % (fn, dts)] = list(best)
            if verbose:
                print("best %-9s %s ept=%d bpc=%d pd=%d %.4f ms" % ((fn, dts) + best), flush=True)
            del x0, x1, z0, z1
    return {device_key(): res}


def save(result, path=CACHE):
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.update(result)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


_applied = False


def apply(path=CACHE):
    """Set the tuned configuration for the current device, if the cache has it."""
    global _applied
    if _applied:
        return True
    _applied = True
    if not os.path.exists(path):
        return False
    with open(path) as f:
        data = json.load(f)
    rec = data.get(device_key())
    if not rec:
        return False
    for key, (ept, bpc, pd, _) in rec.items():
        fn, dts = key.split("|")
        _lib.set_launch_config(fn, dts, int(ept), int(bpc), int(pd))
    return True


def tune_batch(verbose=True):
    """Tune the batched launch on the standard ragged batch (4096 arrays of
    mixed function and format); return {key|batch: [ept64, ept32, chunk_tiles,
    blocks_per_cu, ms]}."""
    import torch
    from . import batch, workloads
    dev = torch.device("cuda:0")
    items = []
    for fn, dt, x0, x1 in workloads.batch_inputs(workloads.batch_descriptors()):
        a0 = torch.from_numpy(np.ascontiguousarray(x0)).to(dev)
        a1 = torch.from_numpy(np.ascontiguousarray(x1)).to(dev)
        items.append((fn, a0, a1, torch.empty_like(a0), torch.empty_like(a0)))
    best, times = batch.autotune(items, verbose=verbose)
    if verbose:
        print("best batch %s %.4f ms" % (best, times[best]), flush=True)
    return {device_key() + "|batch": list(best) + [times[best]]}


def batch_config(path=CACHE):
    """The tuned batch configuration for the current device, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(device_key() + "|batch")
    return tuple(int(v) for v in rec[:4]) if rec else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 26)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--funcs", default="", help="comma-separated subset, e.g. texpm1,tlog")
    ap.add_argument("--dtypes", default="f64,f32")
    ap.add_argument("--bpcs", default=",".join(map(str, BPCS)))
    ap.add_argument("--epts", default=",".join(map(str, EPTS)))
    ap.add_argument("--batch", action="store_true", help="tune the batched launch only")
    args = ap.parse_args()
    if args.batch:
        r = tune_batch()
        save(r, args.out)
        print(json.dumps(r, indent=1))
        return 0
    r = tune(n=args.n, reps=args.reps, funcs=[f for f in args.funcs.split(",") if f] or None,
             dtypes=tuple(args.dtypes.split(",")), bpcs=tuple(int(b) for b in args.bpcs.split(",")),
             epts=tuple(int(e) for e in args.epts.split(",")))
    save(r, args.out)
    print(json.dumps(r, indent=1))


if __name__ == "__main__":
    sys.exit(main())
