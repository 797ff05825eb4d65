"""The device value type of include/twofold_device.hpp (the paper's C++
interface, section "Experimental code > C/C++ interface": twofold<T> with
value and error, one name for float and double, exp/expm1/log/log1p
overloads), through the check library tests/cxx/libtfcp_device.so, whose
kernels evaluate every function and operator of the header on
tfcp::twofold<T> values:

* without a GPU: the library loads and exports its entry point, and rejects
  an unknown operation without touching the GPU;
* on the GPU: for every function and operator, binary64 and binary32, the
  results equal the library's array entry points bit for bit on random
  arguments with 1% edge values (z0 and z1, signed zeros and NaN classes).
"""
import ctypes
import os
import sys

import numpy as np
import pytest

from paper_1502_05216_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "cxx", "libtfcp_device.so")

OPS = (["exp", "expm1", "log", "log1p"] + list(workloads.DOTTED) + list(workloads.COUPLED)
       + ["tadd", "tsub", "tmul", "tdiv", "tsqrt", "trenorm"])
STD = {"exp": "texp", "expm1": "texpm1", "log": "tlog", "log1p": "tlog1p"}


def _lib():
    if not os.path.exists(LIB):
        # built by __graft_entry__.build(); built here only on a host without one
        sys.path.insert(0, os.path.join(HERE, "cxx"))
        import build_check
        build_check.build_device()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.tfcp_dev_apply.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                   ctypes.c_size_t, P]
    lib.tfcp_dev_apply.restype = ctypes.c_int
    return lib


def test_device_check_library_loads():
    lib = _lib()
    assert lib.tfcp_dev_apply(99, 0, None, None, None, None, None, None, 5, None) == -1
    assert lib.tfcp_dev_apply(0, 7, None, None, None, None, None, None, 5, None) == -1
    assert lib.tfcp_dev_apply(0, 0, None, None, None, None, None, None, 0, None) == 0


def _inputs(name, dt, n):
    if name in STD:
        return workloads.twofold_inputs(STD[name], n, dt, seed=301, edges=0.01)
    if name in workloads.DOTTED:
        return workloads.twofold_inputs(name, n, dt, seed=302, edges=0.01)
    if name in workloads.COUPLED:
        return workloads.twofold_inputs(name, n, dt, seed=303, edges=0.01, coupled=True)
    return workloads.twofold_inputs("texp", n, dt, seed=304, edges=0.01)


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("op", range(len(OPS)), ids=OPS)
def test_device_type_equals_array_entry_points(op, dt):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as tf
    from parity_util import same_bits
    name = OPS[op]
    print("case device type", name, np.dtype(dt).name, flush=True)
    dev = torch.device("cuda:0")
    n = 50021
    a, b = _inputs(name, dt, n)
    x0 = torch.from_numpy(a).to(dev)
    x1 = torch.from_numpy(b).to(dev)
    y0, y1 = x0.flip(0).contiguous(), x1.flip(0).contiguous()
    if name == "tsqrt":
        x0 = x0.abs()
    if name == "trenorm":
        x1 = y0
    z0, z1 = torch.empty_like(x0), torch.empty_like(x0)
    dotted = name in workloads.DOTTED
    binary = name in ("tadd", "tsub", "tmul", "tdiv")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = _lib().tfcp_dev_apply(op, 0 if dt == np.float64 else 1, ptr(x0),
                               None if dotted else ptr(x1),
                               ptr(y0) if binary else None, ptr(y1) if binary else None,
                               ptr(z0), ptr(z1), n,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    if dotted:
        r0, r1 = getattr(tf, name)(x0)
    elif binary:
        r0, r1 = getattr(tf, name)(x0, x1, y0, y1)
    else:
        r0, r1 = getattr(tf, STD.get(name, name))(x0, x1)
    torch.cuda.synchronize()
    for what, g, r in (("z0", z0, r0), ("z1", z1, r1)):
        g, r = g.cpu().numpy(), r.cpu().numpy()
        ok = same_bits(g, r)
        assert ok.all(), "%s %s %s: %d of %d differ, e.g. %s vs %s" % (
            name, np.dtype(dt).name, what, (~ok).sum(), n, g[~ok][:3], r[~ok][:3])
