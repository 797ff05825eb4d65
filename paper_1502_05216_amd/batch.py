"""Batched ragged launch: many arrays, each with its own twofold function and
format, in one persistent hipGraph-captured launch (tf_batch_* in
include/twofold_hip.h).

    plan = BatchPlan([("texp", x0, x1, z0, z1), ("tlog1p", y0, y1, w0, w1), ...])
    plan.launch()          # enqueue on torch.cuda.current_stream()
    plan.close()

Arrays are contiguous GPU tensors (float64 or float32 per item); the plan
keeps references to them until it is closed.  Results equal the plain calls
bit for bit, under every configuration.

    best, times = autotune(items)           # time every candidate configuration
    plan = BatchPlan(items, config=best)    # or config="tuned": the tune cache

    run_noalloc(items)     # the same launch in one call that allocates nothing
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
# (elements per thread binary64, binary32) pairs the library instantiates
EPT_PAIRS = ((2, 4), (1, 2), (4, 4))
CHUNK_TILES = (8, 16, 32, 64)
BLOCKS_PER_CU = (0, 2)
CANDIDATES = tuple((e64, e32, ct, bpc) for e64, e32 in EPT_PAIRS for ct in CHUNK_TILES
                   for bpc in BLOCKS_PER_CU)


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
    lib.tf_batch_run_noalloc.argtypes = [ctypes.POINTER(BatchDesc), ctypes.c_size_t,
                                         ctypes.POINTER(BatchConfig), P]
    lib.tf_batch_run_noalloc.restype = ctypes.c_int
    lib._tf_batch_bound = True
    return lib


def _descs(items):
    import torch
    descs, keep = [], []
    for func, x0, x1, z0, z1 in items:
        if func not in FUNC_IDS:
            raise ValueError(func)
        _lib._validate(x0, x1, z0, z1)
        dt = {torch.float64: 0, torch.float32: 1}.get(x0.dtype)
        if dt is None:
            raise TypeError("batch arrays must be float64 or float32")
        descs.append(BatchDesc(FUNC_IDS[func], dt, x0.numel(), x0.data_ptr(), x1.data_ptr(),
                               z0.data_ptr(), z1.data_ptr()))
        keep += [x0, x1, z0, z1]
    return (BatchDesc * max(1, len(descs)))(*descs), len(descs), keep


MAX_ARRAYS_NOALLOC = 8192      # TF_BATCH_NOALLOC_MAX_ARRAYS
MAX_CHUNKS_NOALLOC = 65536     # TF_BATCH_NOALLOC_MAX_CHUNKS


def run_noalloc(items, config=None):
    """The batched launch of `items` in one call that allocates no device
    memory (tf_batch_run_noalloc): the library's static per-GPU scratch holds
    the descriptors, chunk list and work counter.  Enqueued on the current
    stream; results equal a BatchPlan's with the same config bit for bit.
    Calls that overlap on one GPU race on that scratch."""
    lib = _bind(_lib.lib())
    arr, count, _keep = _descs(items)
    cfg = BatchConfig(*(config or DEFAULT_CONFIG))
    _lib._check(lib.tf_batch_run_noalloc(arr, count, ctypes.byref(cfg), _lib._stream()),
                "tf_batch_run_noalloc")


class BatchPlan:
    def __init__(self, items, config=None):
        """items: iterable of (func, x0, x1, z0, z1); config: (ept64, ept32,
        chunk_tiles, blocks_per_cu) or None for the library defaults."""
        self._lib = _bind(_lib.lib())
        arr, count, self._keep = _descs(items)
        if config == "tuned":
            from . import tune
            config = tune.batch_config()
        cfg = BatchConfig(*(config or DEFAULT_CONFIG))
        handle = ctypes.c_void_p()
        _lib._check(self._lib.tf_batch_plan_create(arr, count, ctypes.byref(cfg),
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


def autotune(items, candidates=CANDIDATES, reps=5, verbose=False):
    """Time one plan of `items` per candidate configuration (ept64, ept32,
    chunk_tiles, blocks_per_cu) with HIP events on the current stream and
    return (best_config, {config: ms per launch}).  The outputs of `items` are
    overwritten (with the same values under every configuration)."""
    import torch
    items = list(items)
    times = {}
    stream = torch.cuda.current_stream()
    for cfg in candidates:
        cfg = tuple(cfg)
        with BatchPlan(items, config=cfg) as plan:
            plan.launch()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                plan.launch()
            e1.record(stream)
            e1.synchronize()
            times[cfg] = e0.elapsed_time(e1) / reps
        if verbose:
            print("batch config %s %.4f ms" % (cfg, times[cfg]), flush=True)
    best = min(times, key=times.get)
    return best, times
