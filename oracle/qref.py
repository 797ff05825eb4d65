"""Quad-precision etalon (oracle/qref.c, binary128 via libquadmath) for the
accuracy acceptance of the twofold functions on about a million arguments --
TEST INFRASTRUCTURE.

    rel, cls = qref.check("texp", x0, x1, z0, z1, l0=2**-95)
    parts, ex = qref.evaluate("tlog", x0, x1)   # f(x0 + x1) = parts[i].sum() 2^ex[i]

`cls` codes: 0 measured (rel holds |z0 + z1 - f| / |f|), 1 subnormal-range
result within l0*|f| + one subnormal ulp, 2 such a result outside it, 3 not
measured (non-finite or out-of-domain argument or result).  See qref.c.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qref.c")
LIB = os.path.join(HERE, "libqref.so")
FN = {"texp": 0, "texpm1": 1, "tlog": 2, "tlog1p": 3}
_lib = []


def build(verbose=False):
    """Compile qref.c into libqref.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lquadmath"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    _lib.clear()
    return LIB


def _load():
    if not _lib:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        P, S, I, D = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
        lib.qref_check.argtypes = [I, I, P, P, P, P, S, D, P, P, I]
        lib.qref_eval.argtypes = [I, P, P, P, P, S]
        lib.qref_quad.argtypes = [I, P, P, S]
        lib.qref_libm.argtypes = [I, P, P, S]
        _lib.append(lib)
    return _lib[0]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def check(fn, x0, x1, z0, z1, l0, threads=None):
    """Per-element relative error of the pairs (z0, z1) against fn(x0 + x1) in
    binary128; fn is the twofold function's name (texp texpm1 tlog tlog1p), the
    arrays all binary64 or all binary32.  Returns (rel float64[n], cls int8[n])."""
    arrs = [np.ascontiguousarray(a) for a in (x0, x1, z0, z1)]
    dt = arrs[0].dtype
    assert dt in (np.float64, np.float32) and all(a.dtype == dt for a in arrs)
    n = arrs[0].size
    rel = np.empty(n, np.float64)
    cls = np.empty(n, np.int8)
    threads = threads or max(1, min(os.cpu_count() or 1, 16))
    _load().qref_check(FN[fn], 0 if dt == np.float64 else 1, *[_p(a) for a in arrs], n,
                       float(l0), _p(rel), _p(cls), threads)
    return rel, cls


def evaluate(fn, x0, x1):
    """fn(x0 + x1) for binary64 arrays as (parts, ex): f = (parts[i, 0] +
    parts[i, 1] + parts[i, 2]) 2^ex[i], the quad significand in [1/2, 1) cut
    exactly into three doubles."""
    x0 = np.ascontiguousarray(x0, np.float64)
    x1 = np.ascontiguousarray(x1, np.float64)
    parts = np.empty((x0.size, 3), np.float64)
    ex = np.empty(x0.size, np.int32)
    _load().qref_eval(FN[fn], _p(x0), _p(x1), _p(parts), _p(ex), x0.size)
    return parts, ex


def context_mops(fn, x, quad=True):
    """Millions of calls per second of one libquadmath function (quad=True:
    expq, expm1q, logq, log1pq) or one C library function (exp, ...) of
    binary64 arguments, on one thread: the comparison systems the paper times
    its twofold functions against (section "Analysis > Performance")."""
    import time
    x = np.ascontiguousarray(x, np.float64)
    out = np.empty_like(x)
    f = _load().qref_quad if quad else _load().qref_libm
    f(FN[fn], _p(x), _p(out), min(x.size, 1024))          # warm
    t0 = time.perf_counter()
    f(FN[fn], _p(x), _p(out), x.size)
    return x.size / (time.perf_counter() - t0) / 1e6
