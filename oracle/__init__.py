"""Oracle for the twofold exp/log hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  It wraps the scalar CPU implementation in oracle/tfo.cpp (built
into oracle/libtfo.so) with numpy-array functions:

    z0, z1 = oracle.texp(x0, x1)        # and texpm1, tlog, tlog1p
    z0, z1 = oracle.texpf(x0, x1)       # binary32 variants
    z = oracle.exp1x(x)                 # the 1x main-part functions (+ f)
    z0, z1 = oracle.pexp0(x)            # dotted argument: pexp0 texp0 pexpm10
                                        # texpm10 plog0 tlog0 plog1p0 tlog1p0 (+ f)
    z0, z1 = oracle.pexp(x0, x1)        # coupled argument: texpp pexp texpm1p
                                        # pexpm1 tlogp plog tlog1pp plog1p (+ f)
    z0, z1 = oracle.tadd(x0, x1, y0, y1)   # twofold arithmetic: tadd tsub tmul
    z0, z1 = oracle.tsqrt(x0, x1)          # tdiv (+ f), tsqrt and trenorm (+ f)
    gx0, gx1 = oracle.texp_bwd(s0, s1, g0, g1)
    counts = oracle.op_count("texp", x0, x1)   # {add, mul, fma, other, n}

It shares no code with the GPU library (paper_1502_05216_amd).
"""
import ctypes
import os
import subprocess
import tempfile
import types

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtfo.so")
SRC = os.path.join(HERE, "tfo.cpp")

CXXFLAGS = ["-O2", "-mfma", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
            "-frounding-math", "-fopenmp", "-shared", "-fPIC"]

FUNCS_TW = ["texp", "texpm1", "tlog", "tlog1p"]
FUNCS_1X = ["exp1x", "expm1_1x", "log1x", "log1p_1x"]
# the other entry points of the paper's interface
FUNCS_D = ["pexp0", "texp0", "pexpm10", "texpm10", "plog0", "tlog0", "plog1p0", "tlog1p0"]
FUNCS_C = ["texpp", "pexp", "texpm1p", "pexpm1", "tlogp", "plog", "tlog1pp", "plog1p"]
# twofold arithmetic: binary operations on (x0, x1, y0, y1), and tsqrt(x0, x1)
FUNCS_ARITH = ["tadd", "tsub", "tmul", "tdiv"]


def build(verbose=False):
    """Compile oracle/tfo.cpp into oracle/libtfo.so and the quad etalon
    oracle/qref.c into oracle/libqref.so (always recompiles)."""
    cmd = ["g++"] + CXXFLAGS + [SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    _libs.pop(LIB, None)
    from . import qref              # the binary128 etalon of the accuracy tests
    qref.build(verbose)
    return LIB


def build_variant(src_text, out_path):
    """Compile a modified copy of the oracle source (tfo_tables.h from here)."""
    d = tempfile.mkdtemp(prefix="tfo_variant_")
    src = os.path.join(d, "tfo.cpp")
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["g++"] + CXXFLAGS + ["-I", HERE, src, "-o", out_path])
    return out_path


_libs = {}


def _load(path=None):
    path = path or LIB
    if path in _libs:
        return _libs[path]
    if path == LIB and not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(path)
    P, S, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    for base in FUNCS_TW:
        for sfx in ("", "f"):
            getattr(lib, "tfo_%s%s_n" % (base, sfx)).argtypes = [P, P, P, P, S, I]
            getattr(lib, "tfo_count_%s%s_n" % (base, sfx)).argtypes = [P, P, S, P]
            getattr(lib, "tfo_%s%s_bwd_n" % (base, sfx)).argtypes = [P, P, P, P, P, P, S, I]
            getattr(lib, "tfo_count_%s%s_bwd_n" % (base, sfx)).argtypes = [P, P, P, P, S, P]
    for base in FUNCS_1X:
        for sfx in ("", "f"):
            getattr(lib, "tfo_%s%s_n" % (base, sfx)).argtypes = [P, P, S, I]
    for base in FUNCS_C:
        for sfx in ("", "f"):
            getattr(lib, "tfo_%s%s_n" % (base, sfx)).argtypes = [P, P, P, P, S, I]
            getattr(lib, "tfo_count_%s%s_n" % (base, sfx)).argtypes = [P, P, S, P]
    for base in FUNCS_D:
        for sfx in ("", "f"):
            getattr(lib, "tfo_%s%s_n" % (base, sfx)).argtypes = [P, P, P, S, I]
            getattr(lib, "tfo_count_%s%s_n" % (base, sfx)).argtypes = [P, S, P]
    for base in FUNCS_ARITH:
        for sfx in ("", "f"):
            getattr(lib, "tfo_%s%s_n" % (base, sfx)).argtypes = [P, P, P, P, P, P, S, I]
            getattr(lib, "tfo_count_%s%s_n" % (base, sfx)).argtypes = [P, P, P, P, S, P]
    for sfx in ("", "f"):
        for u in ("tsqrt", "trenorm"):
            getattr(lib, "tfo_%s%s_n" % (u, sfx)).argtypes = [P, P, P, P, S, I]
            getattr(lib, "tfo_count_%s%s_n" % (u, sfx)).argtypes = [P, P, S, P]
    lib.tfo_eft_n.argtypes = [I, P, P, P, P, S]
    _libs[path] = lib
    return lib


def _arr(x, dt):
    return np.ascontiguousarray(np.asarray(x, dtype=dt))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads():
    return max(1, min(os.cpu_count() or 1, 16))


def _mk_tw(name, dt, path=None):
    def f(x0, x1, threads=1):
        lib = _load(path)
        x0 = _arr(x0, dt)
        x1 = _arr(x1, dt)
        assert x0.shape == x1.shape
        z0 = np.empty_like(x0)
        z1 = np.empty_like(x0)
        getattr(lib, "tfo_%s_n" % name)(_ptr(x0), _ptr(x1), _ptr(z0), _ptr(z1), x0.size,
                                        threads or 1)
        return z0, z1
    f.__name__ = name
    f.__doc__ = "oracle %s over %s twofold arrays -> (z0, z1)" % (name, np.dtype(dt).name)
    return f


def _mk_1x(name, dt, path=None):
    def f(x, threads=1):
        lib = _load(path)
        x = _arr(x, dt)
        z = np.empty_like(x)
        getattr(lib, "tfo_%s_n" % name)(_ptr(x), _ptr(z), x.size, threads or 1)
        return z
    f.__name__ = name
    return f


def _mk_d(name, dt, path=None):
    def f(x, threads=1):
        lib = _load(path)
        x = _arr(x, dt)
        z0 = np.empty_like(x)
        z1 = np.empty_like(x)
        getattr(lib, "tfo_%s_n" % name)(_ptr(x), _ptr(z0), _ptr(z1), x.size, threads or 1)
        return z0, z1
    f.__name__ = name
    f.__doc__ = "oracle %s over a %s array (dotted argument) -> (z0, z1)" % (name,
                                                                          np.dtype(dt).name)
    return f


def _mk_bwd(name, dt, path=None):
    def f(s0, s1, g0, g1, threads=1):
        lib = _load(path)
        s0, s1, g0, g1 = (_arr(a, dt) for a in (s0, s1, g0, g1))
        gx0 = np.empty_like(s0)
        gx1 = np.empty_like(s0)
        getattr(lib, "tfo_%s_n" % name)(_ptr(s0), _ptr(s1), _ptr(g0), _ptr(g1), _ptr(gx0),
                                        _ptr(gx1), s0.size, threads or 1)
        return gx0, gx1
    f.__name__ = name
    return f


def _bind(ns, path=None):
    for b in FUNCS_TW:
        ns[b] = _mk_tw(b, np.float64, path)
        ns[b + "f"] = _mk_tw(b + "f", np.float32, path)
        ns[b + "_bwd"] = _mk_bwd(b + "_bwd", np.float64, path)
        ns[b + "f_bwd"] = _mk_bwd(b + "f_bwd", np.float32, path)
    for b in FUNCS_1X:
        ns[b] = _mk_1x(b, np.float64, path)
        ns[b + "f"] = _mk_1x(b + "f", np.float32, path)
    for b in FUNCS_C:
        ns[b] = _mk_tw(b, np.float64, path)
        ns[b + "f"] = _mk_tw(b + "f", np.float32, path)
    for b in FUNCS_D:
        ns[b] = _mk_d(b, np.float64, path)
        ns[b + "f"] = _mk_d(b + "f", np.float32, path)
    for b in FUNCS_ARITH:      # same array shape as the backward: 4 in, 2 out
        ns[b] = _mk_bwd(b, np.float64, path)
        ns[b + "f"] = _mk_bwd(b + "f", np.float32, path)
    for u in ("tsqrt", "trenorm"):
        ns[u] = _mk_tw(u, np.float64, path)
        ns[u + "f"] = _mk_tw(u + "f", np.float32, path)


_bind(globals())


def variant(path):
    """The same array functions bound to another build of the oracle source."""
    ns = {}
    _bind(ns, path)
    return types.SimpleNamespace(**ns)


def eft(which, a, b):
    """which: 'two_sum' | 'fast_two_sum' | 'two_prod' -> (s, t) float64 arrays."""
    lib = _load()
    a = _arr(a, np.float64)
    b = _arr(b, np.float64)
    s = np.empty_like(a)
    t = np.empty_like(a)
    code = {"two_sum": 0, "fast_two_sum": 1, "two_prod": 2}[which]
    lib.tfo_eft_n(code, _ptr(a), _ptr(b), _ptr(s), _ptr(t), a.size)
    return s, t


def op_count(name, *arrays):
    """Floating-point operations the oracle performs for `name` over the given
    inputs: dict(add, mul, fma, other, n).  `name` is e.g. 'texp', 'tlogf',
    'texp_bwd' (backward takes s0, s1, g0, g1), 'plog0' (dotted argument: one
    array).  add counts + and -, other counts rint/ldexp/frexp and divisions."""
    lib = _load()
    base = name[:-4] if name.endswith("_bwd") else name
    dt = np.float32 if base.endswith("f") else np.float64
    arrs = [_arr(a, dt) for a in arrays]
    out = (ctypes.c_ulonglong * 4)()
    fn = getattr(lib, "tfo_count_%s_n" % name)
    fn(*[_ptr(a) for a in arrs], arrs[0].size, ctypes.cast(out, ctypes.c_void_p))
    return {"add": out[0], "mul": out[1], "fma": out[2], "other": out[3], "n": arrs[0].size}
