"""GPU parity for every launch configuration the autotuner can pick.

Each (elements per thread, prefetch depth, workgroups per compute unit)
instantiation is its own kernel code path (vector width, register rotation,
the texpm1 queue capacity); all of them must match the oracle bit for bit on
z0 and within the parity bar on z1, on inputs that span many tiles, a ragged
tail, edge arguments, and a misaligned view (which forces one element per
thread).
"""
import numpy as np
import pytest

import oracle
from paper_1502_05216_amd import workloads
from parity_util import compare, same_bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FUNCS = ("texp", "texpm1", "tlog", "tlog1p")
ONEX = ("exp1x", "expm1_1x", "log1x", "log1p_1x")


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    from paper_1502_05216_amd import _lib
    m.lib()
    saved = {(f, d): _lib.get_launch_config(f, d) for f in FUNCS + ONEX for d in ("f64", "f32")}
    yield m
    for (f, d), c in saved.items():
        _lib.set_launch_config(f, d, *c)


@pytest.mark.parametrize("dts", ["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_all_launch_configs(tf, fn, dts):
    from paper_1502_05216_amd import _lib
    dt = np.float64 if dts == "f64" else np.float32
    sfx = "" if dts == "f64" else "f"
    n = 3 * 256 * 4 * 7 + 333
    x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=77, edges=0.02)
    o0, o1 = getattr(oracle, fn + sfx)(x0, x1)
    d = torch.device("cuda:0")
    a0 = torch.from_numpy(x0).to(d)
    a1 = torch.from_numpy(x1).to(d)
    for ept in (1, 2, 4):
        for pd in (1, 2):
            for bpc in (0, 1, 3):
                print("case", fn, dts, ept, pd, bpc, flush=True)
                _lib.set_launch_config(fn, dts, ept, bpc, pd)
                g0, g1 = getattr(tf, fn)(a0, a1)
                torch.cuda.synchronize()
                compare(g0.cpu().numpy(), g1.cpu().numpy(), o0, o1,
                        "%s %s ept=%d pd=%d bpc=%d" % (fn, dts, ept, pd, bpc))
    # misaligned view: element offset 1 breaks 16-byte alignment
    b0 = torch.from_numpy(np.concatenate([[dt(0.5)], x0])).to(d)[1:]
    b1 = torch.from_numpy(np.concatenate([[dt(0.0)], x1])).to(d)[1:]
    g0, g1 = getattr(tf, fn)(b0, b1)
    torch.cuda.synchronize()
    compare(g0.cpu().numpy(), g1.cpu().numpy(), o0, o1, "%s %s misaligned" % (fn, dts))


@pytest.mark.parametrize("dts", ["f64", "f32"])
@pytest.mark.parametrize("name", ONEX)
def test_onex_launch_configs(tf, name, dts):
    from paper_1502_05216_amd import _lib
    dt = np.float64 if dts == "f64" else np.float32
    sfx = "" if dts == "f64" else "f"
    base = {"exp1x": "texp", "expm1_1x": "texpm1", "log1x": "tlog", "log1p_1x": "tlog1p"}[name]
    x, _ = workloads.twofold_inputs(base, 2 * 256 * 4 * 5 + 77, dt, seed=78, edges=0.02)
    o = getattr(oracle, name + sfx)(x)
    a = torch.from_numpy(x).to(torch.device("cuda:0"))
    for ept in (1, 2, 4):
        for bpc in (0, 2):
            _lib.set_launch_config(name, dts, ept, bpc, 1)
            g = getattr(tf, name)(a)
            torch.cuda.synchronize()
            assert same_bits(g.cpu().numpy(), o).all(), (name, dts, ept, bpc)
