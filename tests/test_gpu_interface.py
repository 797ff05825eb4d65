"""GPU parity of the other entry points of the paper's interface: the HIP
library (through its C ABI) against the CPU oracle on the same seeded inputs.

Every function of a dotted argument (pexp0 texp0 pexpm10 texpm10 plog0 tlog0
plog1p0 tlog1p0) and of a coupled argument (texpp pexp texpm1p pexpm1 tlogp
plog tlog1pp plog1p), binary64 and binary32: random arguments of the
function's range with 1% edge arguments (for the coupled functions the edges
include non-finite second parts), ragged sizes from one element up, arrays
that are not 16-byte aligned, and a 2^24-element run checked on a sample.
Bar as for the four twofold functions: z0 bit for bit, z1 within 4 ulp.
"""
import numpy as np
import pytest

import oracle
from paper_1502_05216_amd import workloads
from parity_util import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DOTTED = list(workloads.DOTTED)
COUPLED = list(workloads.COUPLED)
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


def inputs(name, n, dt, seed, edges):
    return workloads.twofold_inputs(name, n, dt, seed=seed, edges=edges, coupled=name in COUPLED)


def on_gpu(tf, name, x0, x1, misalign=False):
    d = torch.device("cuda:0")
    if misalign:
        a = torch.from_numpy(np.concatenate([x0[:1], x0])).to(d)[1:]
        b = torch.from_numpy(np.concatenate([x1[:1], x1])).to(d)[1:]
    else:
        a = torch.from_numpy(np.ascontiguousarray(x0)).to(d)
        b = torch.from_numpy(np.ascontiguousarray(x1)).to(d)
    if name in DOTTED:
        g0, g1 = getattr(tf, name)(a)
    else:
        g0, g1 = getattr(tf, name)(a, b)
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy()


def on_oracle(name, dt, x0, x1):
    f = getattr(oracle, name + sfx(dt))
    return f(x0, threads=8) if name in DOTTED else f(x0, x1, threads=8)


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("name", DOTTED + COUPLED)
def test_parity_random_with_edges(tf, name, dt):
    n = 100003
    print("case", name, np.dtype(dt).name, n, flush=True)
    x0, x1 = inputs(name, n, dt, seed=201, edges=0.01)
    g0, g1 = on_gpu(tf, name, x0, x1)
    o0, o1 = on_oracle(name, dt, x0, x1)
    nd = compare(g0, g1, o0, o1, "%s %s" % (name, np.dtype(dt).name))
    print("%s %s: z1 not bit-identical at %d of %d" % (name, np.dtype(dt).name, nd, n))


@pytest.mark.parametrize("name", DOTTED + COUPLED)
def test_sizes_and_misaligned(tf, name):
    for dt in DTS:
        for n in (1, 2, 63, 64, 65, 511, 513, 4097):
            x0, x1 = inputs(name, n, dt, seed=203 + n, edges=0.05)
            g0, g1 = on_gpu(tf, name, x0, x1)
            o0, o1 = on_oracle(name, dt, x0, x1)
            compare(g0, g1, o0, o1, "%s %s n=%d" % (name, np.dtype(dt).name, n))
        x0, x1 = inputs(name, 20001, dt, seed=207, edges=0.01)
        g0, g1 = on_gpu(tf, name, x0, x1, misalign=True)
        o0, o1 = on_oracle(name, dt, x0, x1)
        compare(g0, g1, o0, o1, "%s %s misaligned" % (name, np.dtype(dt).name))


def test_empty(tf):
    d = torch.device("cuda:0")
    for name in DOTTED:
        z0, z1 = getattr(tf, name)(torch.empty(0, dtype=torch.float64, device=d))
        assert z0.numel() == 0 and z1.numel() == 0
    for name in COUPLED:
        e = torch.empty(0, dtype=torch.float32, device=d)
        z0, z1 = getattr(tf, name)(e, e)
        assert z0.numel() == 0


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_full_size_sampled(tf, dt):
    """2^24 elements per function, 20000 sampled indices against the oracle."""
    n = 1 << 24
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(n, 20000, replace=False))
    for name in DOTTED + COUPLED:
        print("case full", name, np.dtype(dt).name, flush=True)
        x0, x1 = inputs(name, n, dt, seed=211, edges=0.001)
        g0, g1 = on_gpu(tf, name, x0, x1)
        o0, o1 = on_oracle(name, dt, x0[idx], x1[idx])
        compare(g0[idx], g1[idx], o0, o1, "%s %s full-size sample" % (name, np.dtype(dt).name))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("name", DOTTED + COUPLED)
def test_fast_and_general_bodies_agree(tf, name, dt):
    """Ordinary arguments give the same bits on a fast wave and on a general
    one: the same inputs run as they are and with one NaN in every 64 elements
    (the argument of a dotted function, the second part of a coupled one),
    which sends every wave to the general body."""
    from parity_util import same_bits
    n = 256 * 4 * 24 + 45
    x0, x1 = inputs(name, n, dt, 95, 0.0)
    print("case", name, np.dtype(dt).name, flush=True)
    a0, a1 = on_gpu(tf, name, x0, x1)
    rng = np.random.default_rng(96)
    starts = np.arange(0, n, 64)
    idx = starts + rng.integers(0, 64, size=starts.size)
    idx = idx[idx < n]
    p0, p1 = x0.copy(), x1.copy()
    if name in DOTTED:
        p0[idx] = np.nan
    else:
        p1[idx] = np.nan
    b0, b1 = on_gpu(tf, name, p0, p1)
    keep = np.ones(n, bool)
    keep[idx] = False
    for part, a, b in (("z0", a0, b0), ("z1", a1, b1)):
        ok = same_bits(a[keep], b[keep])
        assert ok.all(), "%s %s: %s differs at %d elements" % (name, np.dtype(dt).name, part,
                                                               (~ok).sum())


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("name", ["tlog1pp", "plog1p"])
def test_log1p_coupled_with_loose_second_parts(tf, name, dt):
    """The coupled log1p functions on arguments that are not coupled but still
    take the fast body (|y1| up to 2^-30 |y0|, binary32 2^-26): on tlog1pp's
    fast waves the Newton seed then differs from the main part on every inner
    lane and is evaluated packed.  Fast against general body bit for bit (one
    NaN second part in every 64 elements), and against the oracle."""
    from parity_util import same_bits
    n = 256 * 4 * 16 + 45
    rng = np.random.default_rng(221)
    x0 = rng.uniform(-0.6, 1.2, n).astype(dt)
    x0[x0 <= -0.99] = dt(0.25)
    rel = 2.0 ** (-30 if dt == np.float64 else -26)
    x1 = (x0 * rng.uniform(-1, 1, n) * rel).astype(dt)
    print("case loose", name, np.dtype(dt).name, flush=True)
    a0, a1 = on_gpu(tf, name, x0, x1)
    o0, o1 = on_oracle(name, dt, x0, x1)
    compare(a0, a1, o0, o1, "%s %s loose second parts" % (name, np.dtype(dt).name))
    p1 = x1.copy()
    p1[::64] = np.nan
    b0, b1 = on_gpu(tf, name, x0, p1)
    keep = np.ones(n, bool)
    keep[::64] = False
    for part, a, b in (("z0", a0, b0), ("z1", a1, b1)):
        ok = same_bits(a[keep], b[keep])
        assert ok.all(), "%s %s: %s differs at %d elements" % (name, np.dtype(dt).name, part,
                                                               (~ok).sum())
