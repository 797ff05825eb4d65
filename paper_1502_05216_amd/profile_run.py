"""Driver for rocprofv3 runs: a plain device copy of known size (the reference
for scaling HBM byte counters), then each selected twofold kernel `reps` times
on the benchmark's 2^26-element arrays.

    rocprofv3 --pmc FETCH_SIZE --kernel-trace -f csv -d OUT -- \\
        python3 -m paper_1502_05216_amd.profile_run --dtype f64 --reps 3

Prints one line per step so a long run shows progress.
"""
import argparse
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"))
    ap.add_argument("--n", type=int, default=1 << 26)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--fn", default="all")
    args = ap.parse_args()

    import torch
    import paper_1502_05216_amd as tf
    from paper_1502_05216_amd import workloads

    dev = torch.device("cuda:0")
    dt = np.float64 if args.dtype == "f64" else np.float32
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    src = torch.ones(args.n, dtype=tdt, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copy of %d x %d bytes done" % (args.n, src.element_size()), flush=True)
    del src, dst
    funcs = tf.TWOFOLD if args.fn == "all" else tuple(args.fn.split(","))
    for fn in funcs:
        a, b = workloads.twofold_inputs(fn, args.n, dt)
        x0 = torch.from_numpy(a).to(dev)
        x1 = torch.from_numpy(b).to(dev)
        z0 = torch.empty_like(x0)
        z1 = torch.empty_like(x0)
        for _ in range(args.reps):
            getattr(tf, fn)(x0, x1, out=(z0, z1))
        torch.cuda.synchronize()
        print("%s %s x%d done" % (fn, args.dtype, args.reps), flush=True)
        del x0, x1, z0, z1
    return 0


if __name__ == "__main__":
    sys.exit(main())
