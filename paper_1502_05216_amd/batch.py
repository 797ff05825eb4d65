"""Batched ragged launch: many arrays, each with its own twofold function and
format, in one persistent hipGraph-captured launch (tf_batch_* in
include/twofold_hip.h).

    plan = BatchPlan([("texp", x0, x1, z0, z1), ("tlog1p", y0, y1, w0, w1), ...])
    plan.launch()          # enqueue on torch.cuda.current_stream()
    plan.close()

Arrays are contiguous GPU tensors (float64 or float32 per item); the plan
keeps references to them until it is closed.  Results equal the plain calls
bit for bit.
"""
import ctypes

from . import _lib

FUNC_IDS = {"texp": 0, "texpm1": 1, "tlog": 2, "tlog1p": 3}


class BatchDesc(ctypes.Structure):
    _fields_ = [("func", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_size_t),
                ("x0", ctypes.c_void_p), ("x1", ctypes.c_void_p), ("z0", ctypes.c_void_p),
                ("z1", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("ept64", ctypes.c_int32), ("ept32", ctypes.c_int32),
                ("chunk_tiles", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


DEFAULT_CONFIG = (2, 4, 32, 0)


def _bind(lib):
    if getattr(lib, "_tf_batch_bound", False):
        return lib
    P = ctypes.c_void_p
    lib.tf_batch_plan_create.argtypes = [ctypes.POINTER(BatchDesc), ctypes.c_size_t,
                                         ctypes.POINTER(BatchConfig), ctypes.POINTER(P)]
    lib.tf_batch_plan_create.restype = ctypes.c_int
    lib.tf_batch_launch.argtypes = [P, P]
    lib.tf_batch_launch.restype = ctypes.c_int
    lib.tf_batch_plan_destroy.argtypes = [P]
    lib.tf_batch_plan_destroy.restype = ctypes.c_int
    lib.tf_batch_plan_info.argtypes = [P, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]
    lib.tf_batch_plan_info.restype = ctypes.c_int
    lib._tf_batch_bound = True
    return lib


class BatchPlan:
    def __init__(self, items, config=None):
        """items: iterable of (func, x0, x1, z0, z1); config: (ept64, ept32,
        chunk_tiles, blocks_per_cu) or None for the library defaults."""
        import torch
        self._lib = _bind(_lib.lib())
        self._keep = []
        descs = []
        for func, x0, x1, z0, z1 in items:
            if func not in FUNC_IDS:
                raise ValueError(func)
            _lib._validate(x0, x1, z0, z1)
            dt = {torch.float64: 0, torch.float32: 1}.get(x0.dtype)
            if dt is None:
                raise TypeError("batch arrays must be float64 or float32")
            descs.append(BatchDesc(FUNC_IDS[func], dt, x0.numel(), x0.data_ptr(), x1.data_ptr(),
                                   z0.data_ptr(), z1.data_ptr()))
            self._keep += [x0, x1, z0, z1]
        arr = (BatchDesc * max(1, len(descs)))(*descs)
        cfg = BatchConfig(*(config or DEFAULT_CONFIG))
        handle = ctypes.c_void_p()
        _lib._check(self._lib.tf_batch_plan_create(arr, len(descs), ctypes.byref(cfg),
                                                   ctypes.byref(handle)), "tf_batch_plan_create")
        self._plan = handle
        self.config = tuple(config or DEFAULT_CONFIG)

    def info(self):
        c = ctypes.c_size_t()
        e = ctypes.c_size_t()
        _lib._check(self._lib.tf_batch_plan_info(self._plan, ctypes.byref(c), ctypes.byref(e)),
                    "tf_batch_plan_info")
        return {"chunks": c.value, "elements": e.value}

    def launch(self):
        if self._plan is None:
            raise RuntimeError("plan is closed")
        _lib._check(self._lib.tf_batch_launch(self._plan, _lib._stream()), "tf_batch_launch")

    def close(self):
        if self._plan is not None:
            _lib._check(self._lib.tf_batch_plan_destroy(self._plan), "tf_batch_plan_destroy")
            self._plan = None
            self._keep = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
