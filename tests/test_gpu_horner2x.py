"""GPU parity of the all-twofold Horner build (variant "horner2x",
TF_HORNER_1X_TAIL=0) against the oracle: z0 AND z1 bit for bit.

The default library evaluates the highest-degree Taylor steps of pexp0 and
pexpm10 in 1x arithmetic (the paper's cost discussion allows it), which moves
z1 in its last bits on a few elements per 10^5.  With those steps in twofold,
every kernel body (fast waves, general waves, texpm1's deferred lanes, the
ragged tail) runs the oracle's operation sequence, so z1 must be identical
everywhere: this is what shows that nothing else in the kernels departs from
the paper's sequence.  Cases: random arguments with 1% edges, the edge grid
crossed with special second parts, the other 16 entry points, and the full
2^26-element arrays of the benchmark in both formats, every element.
"""
import numpy as np
import pytest

import oracle
from paper_1502_05216_amd import workloads
from parity_util import same_bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FUNCS = ("texp", "texpm1", "tlog", "tlog1p")
DTS = (np.float64, np.float32)


@pytest.fixture(scope="module")
def vlib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_05216_amd import _lib
    lib = _lib.variant("horner2x")
    assert b"all-twofold Horner" in lib.tf_version()
    return lib


def sfx(dt):
    return "" if dt == np.float64 else "f"


def run(vlib, fn, x0, x1=None):
    from paper_1502_05216_amd import _lib
    d = torch.device("cuda:0")
    X0 = torch.from_numpy(x0).to(d)
    if x1 is None:
        g0, g1 = _lib.dotted_call(fn, X0, lib=vlib)
    else:
        g0, g1 = _lib.twofold_call(fn, X0, torch.from_numpy(x1).to(d), lib=vlib)
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy()


def assert_identical(g0, g1, o0, o1, what):
    for k, (g, o) in enumerate(((g0, o0), (g1, o1))):
        s = same_bits(g, o)
        if not s.all():
            i = np.flatnonzero(~s)[:5]
            raise AssertionError("%s: z%d differs at %d of %d elements, e.g. idx %s gpu %r "
                                 "oracle %r" % (what, k, (~s).sum(), s.size, i, g[i], o[i]))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_random_with_edges_bitwise(vlib, fn, dt):
    n = 200003
    print("case horner2x", fn, np.dtype(dt).name, n, flush=True)
    x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=101, edges=0.01)
    g0, g1 = run(vlib, fn, x0, x1)
    o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1, threads=8)
    assert_identical(g0, g1, o0, o1, "%s %s" % (fn, np.dtype(dt).name))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_edge_grid_bitwise(vlib, fn, dt):
    ev = workloads.edge_values(fn, dt)
    tiny = np.finfo(dt).smallest_subnormal
    x1s = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, tiny, -tiny, 1e-30, 0.25, -3.0], dt)
    x0 = np.repeat(ev, x1s.size)
    x1 = np.tile(x1s, ev.size)
    print("case horner2x edge grid", fn, np.dtype(dt).name, x0.size, flush=True)
    g0, g1 = run(vlib, fn, x0, x1)
    o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1)
    assert_identical(g0, g1, o0, o1, "%s %s edges" % (fn, np.dtype(dt).name))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_interface_bitwise(vlib, dt):
    from paper_1502_05216_amd import _lib
    n = 100003
    for fn in _lib.DOTTED + _lib.COUPLED:
        print("case horner2x", fn, np.dtype(dt).name, n, flush=True)
        x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=17, edges=0.01,
                                          coupled=fn in _lib.COUPLED)
        if fn in _lib.DOTTED:
            g0, g1 = run(vlib, fn, x0)
            o0, o1 = getattr(oracle, fn + sfx(dt))(x0)
        else:
            g0, g1 = run(vlib, fn, x0, x1)
            o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1)
        assert_identical(g0, g1, o0, o1, "%s %s" % (fn, np.dtype(dt).name))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_full_size_every_element_bitwise(vlib, dt):
    n = 1 << 26
    for fn in FUNCS:
        print("case horner2x full-size", fn, np.dtype(dt).name, n, flush=True)
        x0, x1 = workloads.twofold_inputs(fn, n, dt)
        g0, g1 = run(vlib, fn, x0, x1)
        torch.cuda.empty_cache()
        o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1, threads=16)
        assert_identical(g0, g1, o0, o1, "%s %s full size" % (fn, np.dtype(dt).name))
