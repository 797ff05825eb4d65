"""Writes tests/golden/opcounts.json: the floating-point operations per element
that the algorithm performs (the oracle's counting build), averaged over the
benchmark workloads -- the "algorithmic flops" of the roofline.

add counts + and -, mul counts *, fma counts fused multiply-adds (2 flops),
other counts rint/ldexp/frexp/divide.  Sample: the first 2^18 elements of the
2^26-element benchmark arrays of each function (binary64 and binary32): the
four twofold functions and the other entry points of the interface (coupled
arguments for the coupled-argument functions; x0 alone for the dotted ones).

Run:  python tests/golden/make_opcounts.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1502_05216_amd import workloads  # noqa: E402

SAMPLE = 1 << 18


def main():
    out = {"sample": "first 2^18 of workloads.twofold_inputs(fn, 2^26, dtype)", "f64": {},
           "f32": {}}
    for key, dt, sfx in (("f64", np.float64, ""), ("f32", np.float32, "f")):
        for fn in workloads.FUNCS + workloads.DOTTED + workloads.COUPLED:
            x0, x1 = workloads.twofold_inputs(fn, 1 << 26, dt, coupled=fn in workloads.COUPLED)
            if fn in workloads.DOTTED:
                c = oracle.op_count(fn + sfx, x0[:SAMPLE])
            else:
                c = oracle.op_count(fn + sfx, x0[:SAMPLE], x1[:SAMPLE])
            n = float(c["n"])
            rec = {k: c[k] / n for k in ("add", "mul", "fma", "other")}
            rec["ops"] = rec["add"] + rec["mul"] + rec["fma"]
            rec["flops"] = rec["add"] + rec["mul"] + 2 * rec["fma"]
            out[key][fn] = rec
            print(key, fn, rec)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "opcounts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
