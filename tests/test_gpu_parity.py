"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs, element by element.

Sizes span many tiles (256 threads x 2 elements) and a ragged tail; the
edge cases are empty, single-element and sub-wave arrays, every edge argument
crossed with special second parts, and in-place calls.  The full-size case runs
the 2^26-element arrays in the launch configuration the benchmark times and
checks every element against the oracle.
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
DTS = (np.float64, np.float32)


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    m.lib()                       # fails loudly if the library is not built
    return m


def sfx(dt):
    return "" if dt == np.float64 else "f"


def gpu_call(tf, fn, x0, x1):
    d = torch.device("cuda:0")
    g0, g1 = getattr(tf, fn)(torch.from_numpy(x0).to(d), torch.from_numpy(x1).to(d))
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy()


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_parity_random_with_edges(tf, fn, dt):
    n = 200003
    print("case", fn, np.dtype(dt).name, n, flush=True)
    x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=101, edges=0.01)
    g0, g1 = gpu_call(tf, fn, x0, x1)
    o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1, threads=8)
    nd = compare(g0, g1, o0, o1, "%s %s" % (fn, np.dtype(dt).name))
    print("%s %s: z1 not bit-identical at %d of %d" % (fn, np.dtype(dt).name, nd, n))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_parity_edge_grid(tf, fn, dt):
    ev = workloads.edge_values(fn, dt)
    tiny = np.finfo(dt).smallest_subnormal
    x1s = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, tiny, -tiny, 1e-30, 0.25, -3.0], dt)
    x0 = np.repeat(ev, x1s.size)
    x1 = np.tile(x1s, ev.size)
    print("case edge grid", fn, np.dtype(dt).name, x0.size, flush=True)
    g0, g1 = gpu_call(tf, fn, x0, x1)
    o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1)
    compare(g0, g1, o0, o1, "%s %s edges" % (fn, np.dtype(dt).name))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("name", ONEX)
def test_parity_1x_functions(tf, name, dt):
    base = {"exp1x": "texp", "expm1_1x": "texpm1", "log1x": "tlog", "log1p_1x": "tlog1p"}[name]
    x, _ = workloads.twofold_inputs(base, 150001, dt, seed=7, edges=0.02)
    print("case 1x", name, np.dtype(dt).name, flush=True)
    d = torch.device("cuda:0")
    g = getattr(tf, name)(torch.from_numpy(x).to(d))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    o = getattr(oracle, name + sfx(dt))(x, threads=8)
    s = same_bits(g, o)
    assert s.all(), (name, (~s).sum(), x[~s][:5], g[~s][:5], o[~s][:5])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 511, 512, 513, 1537, 65536])
def test_sizes_and_ragged_tails(tf, n):
    for dt in DTS:
        for fn in FUNCS:
            x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=n, edges=0.0)
            g0, g1 = gpu_call(tf, fn, x0, x1)
            o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1)
            compare(g0, g1, o0, o1, "%s n=%d" % (fn, n))


def test_empty_arrays(tf):
    d = torch.device("cuda:0")
    for dt in (torch.float64, torch.float32):
        e = torch.empty(0, dtype=dt, device=d)
        z0, z1 = tf.texp(e, e)
        assert z0.numel() == 0 and z1.numel() == 0


def test_cfg1_texp_65536(tf):
    x0, x1 = workloads.cfg1_inputs()
    g0, g1 = gpu_call(tf, "texp", x0, x1)
    o0, o1 = oracle.texp(x0, x1, threads=8)
    compare(g0, g1, o0, o1, "cfg1 texp")


def test_in_place_and_determinism(tf):
    d = torch.device("cuda:0")
    for dt in DTS:
        for fn in FUNCS:
            x0, x1 = workloads.twofold_inputs(fn, 50001, dt, seed=3, edges=0.01)
            a0 = torch.from_numpy(x0).to(d)
            a1 = torch.from_numpy(x1).to(d)
            r0, r1 = getattr(tf, fn)(a0, a1)
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                q0, q1 = getattr(tf, fn)(a0, a1)
            s.synchronize()
            getattr(tf, fn)(a0, a1, out=(a0, a1))     # in place
            torch.cuda.synchronize()
            for u, v in ((r0, q0), (r1, q1), (r0, a0), (r1, a1)):
                assert same_bits(u.cpu().numpy(), v.cpu().numpy()).all(), fn


def test_rejects_bad_arguments(tf):
    d = torch.device("cuda:0")
    a = torch.zeros(10, dtype=torch.float64, device=d)
    with pytest.raises(ValueError):
        tf.texp(a, torch.zeros(11, dtype=torch.float64, device=d))
    with pytest.raises(ValueError):
        tf.texp(a, a.float())
    with pytest.raises(ValueError):
        tf.texp(a.cpu(), a.cpu())
    with pytest.raises(TypeError):
        tf.texp(a.half(), a.half())


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_full_size_every_element(tf, dt):
    """2^26 elements per function (the benchmark's arrays, edges included, in
    the launch configuration it times): every element against the oracle
    (z0 bit for bit, z1 within the bar), and z0 against the 1x kernel."""
    n = 1 << 26
    d = torch.device("cuda:0")
    onex = {"texp": "exp1x", "texpm1": "expm1_1x", "tlog": "log1x", "tlog1p": "log1p_1x"}
    it_ = torch.int64 if dt == np.float64 else torch.int32
    for fn in FUNCS:
        print("case full-size", fn, np.dtype(dt).name, n, flush=True)
        x0, x1 = workloads.twofold_inputs(fn, n, dt)
        X0 = torch.from_numpy(x0).to(d)
        g0, g1 = getattr(tf, fn)(X0, torch.from_numpy(x1).to(d))
        r0 = getattr(tf, onex[fn])(X0)
        same = (g0.view(it_) == r0.view(it_)) | (torch.isnan(g0) & torch.isnan(r0))
        assert bool(same.all()), "%s: z0 differs from %s at %d elements" % (
            fn, onex[fn], int((~same).sum()))
        del X0, r0, same
        s0 = g0.cpu().numpy()
        s1 = g1.cpu().numpy()
        del g0, g1
        torch.cuda.empty_cache()
        o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1, threads=16)
        nd = compare(s0, s1, o0, o1, "%s %s full size" % (fn, np.dtype(dt).name))
        print("%s %s: z1 not bit-identical at %d of %d" % (fn, np.dtype(dt).name, nd, n),
              flush=True)


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_log1p_tiny_arguments(tf, dt):
    """Arguments at and below the 1x log1p's tiny threshold (2^-60, binary32
    2^-30), subnormals and signed zeros, in whole arrays (so tlog1p's waves
    take the fast body): the 1x kernel, tlog1p and tlog1p0 against the oracle,
    main parts bit for bit."""
    rng = np.random.default_rng(23)
    fi = np.finfo(dt)
    n = 256 * 4 * 16
    lo = np.log2(float(fi.smallest_subnormal))
    x = (np.exp2(rng.uniform(lo, -20, n)) * np.where(rng.uniform(-1, 1, n) < 0, -1, 1)).astype(dt)
    x[:6] = np.array([0.0, -0.0, fi.smallest_subnormal, -fi.smallest_subnormal,
                      2.0 ** (-60 if dt == np.float64 else -30), -(2.0 ** (-60 if dt == np.float64 else -30))],
                     dtype=dt)
    x1 = (x * dt(fi.eps / 4)).astype(dt)
    print("case log1p tiny", np.dtype(dt).name, flush=True)
    d = torch.device("cuda:0")
    g = tf.log1p_1x(torch.from_numpy(x).to(d))
    torch.cuda.synchronize()
    o = getattr(oracle, "log1p_1x" + sfx(dt))(x)
    assert same_bits(g.cpu().numpy(), o).all()
    g0, g1 = gpu_call(tf, "tlog1p", x, x1)
    o0, o1 = getattr(oracle, "tlog1p" + sfx(dt))(x, x1)
    compare(g0, g1, o0, o1, "tlog1p tiny %s" % np.dtype(dt).name)
    h0, h1 = tf.tlog1p0(torch.from_numpy(x).to(d))
    torch.cuda.synchronize()
    p0, p1 = getattr(oracle, "tlog1p0" + sfx(dt))(x)
    compare(h0.cpu().numpy(), h1.cpu().numpy(), p0, p1, "tlog1p0 tiny %s" % np.dtype(dt).name)


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_table_placement_same_bits(tf, fn, dt):
    """The twofold kernels read their tables from an LDS copy or in place from
    global memory (automatically by size); both placements, forced, give the
    same bits at sizes from one element to several tiles per compute unit and
    at the size where the automatic choice switches, and meet the oracle."""
    from paper_1502_05216_amd import _lib
    per_cu = 8 if dt == np.float64 else 2
    ept = _lib.get_launch_config(fn, "f64" if dt == np.float64 else "f32")[0]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    switch = cus * per_cu * 256 * ept
    try:
        for n in (1, 700, 65536 + 3, switch, switch + 256 * ept, 3 * switch + 11):
            x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=n % 977, edges=0.01)
            print("case placement", fn, np.dtype(dt).name, n, flush=True)
            res = {}
            for mode in ("lds", "global"):
                _lib.set_table_placement(mode)
                res[mode] = gpu_call(tf, fn, x0, x1)
            for k in (0, 1):
                assert same_bits(res["lds"][k], res["global"][k]).all(), (fn, n, k)
            o0, o1 = getattr(oracle, fn + sfx(dt))(x0, x1, threads=8)
            compare(res["lds"][0], res["lds"][1], o0, o1, "%s n=%d placement" % (fn, n))
    finally:
        _lib.set_table_placement("auto")
