"""ctypes binding of libtwofold_hip.so (include/twofold_hip.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels.  Tensors must be contiguous CUDA (HIP) tensors of one dtype
(float64 -> tf_<fn>, float32 -> tf_<fn>f); calls are enqueued on
torch.cuda.current_stream().  There is no CPU fallback: without the built
library or a GPU the functions raise.
"""
import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libtwofold_hip.so")
HEADER = os.path.join(ROOT, "include", "twofold_hip.h")

TF_OK, TF_EINVAL, TF_ELAUNCH, TF_ENOMEM, TF_EUNSUPPORTED, TF_ENODEV, TF_ECAPACITY = range(7)

TWOFOLD = ("texp", "texpm1", "tlog", "tlog1p")
ONEX = ("exp1x", "expm1_1x", "log1x", "log1p_1x")
# the other entry points of the paper's interface
DOTTED = ("pexp0", "texp0", "pexpm10", "texpm10", "plog0", "tlog0", "plog1p0", "tlog1p0")
COUPLED = ("texpp", "pexp", "texpm1p", "pexpm1", "tlogp", "plog", "tlog1pp", "plog1p")
# twofold arithmetic: binary operations, and the square root
ARITH = ("tadd", "tsub", "tmul", "tdiv")

_lib = None


class TwofoldError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = _load().tf_status_string(status).decode() if _lib is not None else str(status)
        super().__init__("%s: %s (status %d)" % (what, msg, status))


_variants = {}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    _lib = _open(LIB_PATH)
    return _lib


def variant(name):
    """The ctypes handle of build variant `name` of the library (the same C ABI
    compiled with other defines; see _build.VARIANTS).  Pass it as `lib=` to
    twofold_call / dotted_call."""
    if name not in _variants:
        from . import _build
        _variants[name] = _open(_build.variant_path(name))
    return _variants[name]


def _open(path):
    if not os.path.exists(path):
        raise RuntimeError("%s is not built (run __graft_entry__.build())"
                           % os.path.basename(path))
    lib = ctypes.CDLL(path)
    P, S = ctypes.c_void_p, ctypes.c_size_t
    for f in TWOFOLD + COUPLED:
        for sfx in ("", "f"):
            fn = getattr(lib, "tf_" + f + sfx)
            fn.argtypes = [P, P, P, P, S, P]
            fn.restype = ctypes.c_int
    for f in DOTTED:
        for sfx in ("", "f"):
            fn = getattr(lib, "tf_" + f + sfx)
            fn.argtypes = [P, P, P, S, P]
            fn.restype = ctypes.c_int
    for f in ARITH:
        for sfx in ("", "f"):
            fn = getattr(lib, "tf_" + f + sfx)
            fn.argtypes = [P, P, P, P, P, P, S, P]
            fn.restype = ctypes.c_int
    for sfx in ("", "f"):
        for u in ("tsqrt", "trenorm"):
            fn = getattr(lib, "tf_" + u + sfx)
            fn.argtypes = [P, P, P, P, S, P]
            fn.restype = ctypes.c_int
    for f in ONEX:
        for sfx in ("", "f"):
            fn = getattr(lib, "tf_" + f + sfx)
            fn.argtypes = [P, P, S, P]
            fn.restype = ctypes.c_int
    for f in TWOFOLD:
        for sfx in ("", "f"):
            fn = getattr(lib, "tf_" + f + sfx + "_bwd")
            fn.argtypes = [P, P, P, P, P, P, S, P]
            fn.restype = ctypes.c_int
    for sfx in ("", "f"):
        fn = getattr(lib, "tf_chain_bwd" + sfx)
        fn.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(P),
                       ctypes.POINTER(P), P, P, P, P, S, P]
        fn.restype = ctypes.c_int
    lib.tf_set_launch_config.argtypes = [ctypes.c_int] * 5
    lib.tf_set_launch_config.restype = ctypes.c_int
    lib.tf_get_launch_config.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
    lib.tf_get_launch_config.restype = ctypes.c_int
    lib.tf_set_table_placement.argtypes = [ctypes.c_int]
    lib.tf_set_table_placement.restype = ctypes.c_int
    lib.tf_get_table_placement.argtypes = []
    lib.tf_get_table_placement.restype = ctypes.c_int
    lib.tf_status_string.argtypes = [ctypes.c_int]
    lib.tf_status_string.restype = ctypes.c_char_p
    lib.tf_version.restype = ctypes.c_char_p
    lib.tf_abi_version.restype = ctypes.c_int
    return lib


def lib():
    """The ctypes handle (loads the in-tree library)."""
    return _load()


def declared_functions():
    """Names of the functions include/twofold_hip.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tf_\w+)\s*\(", src)))


def _check(status, what):
    if status != TF_OK:
        raise TwofoldError(status, what)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_entries = {}
_raw_stream = None


def _current_raw_stream(dev):
    """torch's current stream on device `dev`, as the integer handle."""
    global _raw_stream
    if _raw_stream is None:
        import torch
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        _raw_stream = raw if raw is not None else (
            lambda d: torch.cuda.current_stream(d).cuda_stream)
    return _raw_stream(dev)


def _invoke(symbol, ref, args, lib=None):
    """Calls entry point `symbol` with `args` and torch's current stream of the
    device `ref` lives on, with that device current; raises on an error
    status.  The entry points and the stream handle are looked up once per
    call site's arguments, so a call costs a few microseconds of host time."""
    import torch
    lib = lib or _load()
    key = (id(lib), symbol)
    fn = _entries.get(key)
    if fn is None:
        fn = _entries[key] = getattr(lib, symbol)
    dev = ref.get_device()
    if dev == torch.cuda.current_device():
        _check(fn(*args, _current_raw_stream(dev)), symbol)
    else:
        with torch.cuda.device(dev):
            _check(fn(*args, _current_raw_stream(dev)), symbol)


def _suffix(t):
    import torch
    if t.dtype == torch.float64:
        return ""
    if t.dtype == torch.float32:
        return "f"
    raise TypeError("twofold arrays must be float64 or float32, got %s" % t.dtype)


def _validate(*ts):
    t0 = ts[0]
    for t in ts:
        if not t.is_cuda:
            raise ValueError("twofold arrays must be GPU tensors")
        if t.dtype != t0.dtype or t.shape != t0.shape or t.device != t0.device:
            raise ValueError("twofold arrays must share dtype, shape and device")
        if not t.is_contiguous():
            raise ValueError("twofold arrays must be contiguous")


def twofold_call(name, x0, x1, out=None, lib=None):
    """z0, z1 = name(x0 + x1) elementwise; name in TWOFOLD or COUPLED, or tsqrt
    or trenorm.  `lib`: a variant's handle (default: the library)."""
    import torch
    if name not in TWOFOLD + COUPLED + ("tsqrt", "trenorm"):
        raise ValueError(name)
    _validate(x0, x1)
    if out is None:
        z0 = torch.empty_like(x0)
        z1 = torch.empty_like(x0)
    else:
        z0, z1 = out
        _validate(x0, z0, z1)
    _invoke("tf_" + name + _suffix(x0), x0,
            (x0.data_ptr(), x1.data_ptr(), z0.data_ptr(), z1.data_ptr(), x0.numel()), lib)
    return z0, z1


def dotted_call(name, x0, out=None, lib=None):
    """z0, z1 = name(x0) elementwise for a dotted argument; name in DOTTED.
    `lib`: a variant's handle (default: the library)."""
    import torch
    if name not in DOTTED:
        raise ValueError(name)
    _validate(x0)
    if out is None:
        z0 = torch.empty_like(x0)
        z1 = torch.empty_like(x0)
    else:
        z0, z1 = out
        _validate(x0, z0, z1)
    _invoke("tf_" + name + _suffix(x0), x0,
            (x0.data_ptr(), z0.data_ptr(), z1.data_ptr(), x0.numel()), lib)
    return z0, z1


def arith_call(name, x0, x1, y0, y1, out=None):
    """z0, z1 = (x0 + x1) op (y0 + y1) elementwise; name in ARITH."""
    import torch
    if name not in ARITH:
        raise ValueError(name)
    _validate(x0, x1, y0, y1)
    if out is None:
        z0 = torch.empty_like(x0)
        z1 = torch.empty_like(x0)
    else:
        z0, z1 = out
        _validate(x0, z0, z1)
    _invoke("tf_" + name + _suffix(x0), x0,
            (x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr(), z0.data_ptr(),
             z1.data_ptr(), x0.numel()))
    return z0, z1


def onex_call(name, x, out=None):
    import torch
    if name not in ONEX:
        raise ValueError(name)
    _validate(x)
    z = torch.empty_like(x) if out is None else out
    _validate(x, z)
    _invoke("tf_" + name + _suffix(x), x, (x.data_ptr(), z.data_ptr(), x.numel()))
    return z


def backward_call(name, s0, s1, g0, g1, out=None):
    """Twofold gradient (gx0, gx1) of `name` at the saved forward value
    (s0, s1) for the twofold upstream gradient (g0, g1): texp g*z,
    texpm1 g*(z+1), tlog g/y, tlog1p g/(1+y)."""
    import torch
    if name not in TWOFOLD:
        raise ValueError(name)
    _validate(s0, s1, g0, g1)
    if out is None:
        gx0 = torch.empty_like(s0)
        gx1 = torch.empty_like(s0)
    else:
        gx0, gx1 = out
        _validate(s0, gx0, gx1)
    _invoke("tf_" + name + _suffix(s0) + "_bwd", s0,
            (s0.data_ptr(), s1.data_ptr(), g0.data_ptr(), g1.data_ptr(), gx0.data_ptr(),
             gx1.data_ptr(), s0.numel()))
    return gx0, gx1


CHAIN_MAX = 8          # TF_CHAIN_MAX


def chain_bwd_call(names, saved, g0, g1, out=None):
    """Twofold gradient (gx0, gx1) of y = names[-1](... names[0](x)) with
    respect to x, for the upstream gradient (g0, g1) of y, in one pass per
    CHAIN_MAX stages (tf_chain_bwd).  saved[j] = (s0, s1) is stage j's saved
    forward value as for backward_call; the result equals the chained
    backward_call results bit for bit."""
    import torch
    names = tuple(names)
    if not names or len(names) != len(saved):
        raise ValueError("one saved pair per stage, at least one stage")
    for nm in names:
        if nm not in TWOFOLD:
            raise ValueError(nm)
    _validate(g0, g1, *[t for pair in saved for t in pair])
    if out is None:
        gx0 = torch.empty_like(g0)
        gx1 = torch.empty_like(g0)
    else:
        gx0, gx1 = out
        _validate(g0, gx0, gx1)
    fn = getattr(_load(), "tf_chain_bwd" + _suffix(g0))
    cur = (g0, g1)
    hi = len(names)
    with torch.cuda.device(g0.device):
        while hi > 0:                  # the last CHAIN_MAX stages first
            lo = max(0, hi - CHAIN_MAX)
            k = hi - lo
            fns = (ctypes.c_int * k)(*[TWOFOLD.index(nm) for nm in names[lo:hi]])
            p0 = (ctypes.c_void_p * k)(*[saved[j][0].data_ptr() for j in range(lo, hi)])
            p1 = (ctypes.c_void_p * k)(*[saved[j][1].data_ptr() for j in range(lo, hi)])
            _check(fn(k, fns, p0, p1, cur[0].data_ptr(), cur[1].data_ptr(), gx0.data_ptr(),
                      gx1.data_ptr(), g0.numel(), _stream()), "tf_chain_bwd")
            cur = (gx0, gx1)
            hi = lo
    return gx0, gx1


FN_IDS = {name: i for i, name in enumerate(TWOFOLD + ONEX)}
DTYPE_IDS = {"f64": 0, "f32": 1}


def set_launch_config(fn, dtype, ept, blocks_per_cu, prefetch=1):
    """Launch configuration of one (function, dtype): elements per thread
    (1, 2, 4), workgroups per compute unit (0 = all that are resident) and
    tiles prefetched ahead (1, 2)."""
    _check(_load().tf_set_launch_config(FN_IDS[fn], DTYPE_IDS[dtype], ept, blocks_per_cu,
                                        prefetch), "tf_set_launch_config")


def get_launch_config(fn, dtype):
    e = ctypes.c_int()
    b = ctypes.c_int()
    p = ctypes.c_int()
    _check(_load().tf_get_launch_config(FN_IDS[fn], DTYPE_IDS[dtype], ctypes.byref(e),
                                        ctypes.byref(b), ctypes.byref(p)), "tf_get_launch_config")
    return e.value, b.value, p.value


TABLE_PLACEMENTS = {"auto": 0, "lds": 1, "global": 2}


def set_table_placement(mode):
    """Where the twofold-function kernels read their tables: "auto" (global
    memory for arrays of a few tiles per compute unit, an LDS copy otherwise),
    "lds" or "global".  Same results bit for bit."""
    _check(_load().tf_set_table_placement(TABLE_PLACEMENTS[mode]), "tf_set_table_placement")


def get_table_placement():
    v = _load().tf_get_table_placement()
    return {i: k for k, i in TABLE_PLACEMENTS.items()}[v]
