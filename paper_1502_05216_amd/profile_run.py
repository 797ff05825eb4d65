"""Driver for rocprofv3 runs: a plain device copy of known size (the reference
for scaling HBM byte counters), then each selected twofold kernel `reps` times
on 2^26-element arrays, binary64 then binary32.

    cd /tmp && export TMPDIR=/tmp
    rocprofv3 --pmc FETCH_SIZE -f csv -d OUT -o run -- \\
        python3 -m paper_1502_05216_amd.profile_run --dtype f64,f32 --reps 2

Prints one line per step so a long run shows progress.
"""
import argparse
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="f64", help="f64, f32 or f64,f32")
    ap.add_argument("--n", type=int, default=1 << 26)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--fn", default="all",
                    help="comma-separated names; 'all' = the four twofold functions, "
                         "'iface' = the other 16 interface functions, 'arith' = the twofold "
                         "arithmetic, 'everything' = all of them")
    args = ap.parse_args()

    import torch
    import paper_1502_05216_amd as tf
    from paper_1502_05216_amd import workloads

    dev = torch.device("cuda:0")
    src = torch.ones(args.n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copy of %d x %d bytes done" % (args.n, src.element_size()), flush=True)
    del src, dst
    if args.fn == "all":
        funcs = tf.TWOFOLD
    elif args.fn == "iface":
        funcs = tf.DOTTED + tf.COUPLED
    elif args.fn == "arith":
        funcs = tf.ARITH + ("tsqrt", "trenorm")
    elif args.fn == "everything":
        funcs = tf.TWOFOLD + tf.DOTTED + tf.COUPLED + tf.ARITH + ("tsqrt", "trenorm")
    else:
        funcs = tuple(args.fn.split(","))
    for dname in args.dtype.split(","):
        dt = {"f64": np.float64, "f32": np.float32}[dname]
        for fn in funcs:
            arith = fn in tf.ARITH or fn in ("tsqrt", "trenorm")
            # the arithmetic takes texp's argument law (twofolds of many magnitudes)
            a, b = workloads.twofold_inputs("texp" if arith else fn, args.n, dt,
                                            coupled=fn in tf.COUPLED)
            x0 = torch.from_numpy(a).to(dev)
            x1 = torch.from_numpy(b).to(dev)
            z0 = torch.empty_like(x0)
            z1 = torch.empty_like(x0)
            if arith:                          # y = the same twofolds reversed
                y0, y1 = x0.flip(0), x1.flip(0)
                ax0 = x0.abs()
            for _ in range(args.reps):
                if fn in tf.DOTTED:
                    getattr(tf, fn)(x0, out=(z0, z1))
                elif fn in tf.ARITH:
                    getattr(tf, fn)(x0, x1, y0, y1, out=(z0, z1))
                elif fn == "tsqrt":
                    tf.tsqrt(ax0, x1, out=(z0, z1))
                elif fn == "trenorm":
                    tf.trenorm(x0, y0, out=(z0, z1))
                else:
                    getattr(tf, fn)(x0, x1, out=(z0, z1))
            torch.cuda.synchronize()
            print("%s %s x%d done" % (fn, dname, args.reps), flush=True)
            del x0, x1, z0, z1
            if arith:
                del y0, y1, ax0
    return 0


if __name__ == "__main__":
    sys.exit(main())
