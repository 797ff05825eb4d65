"""GPU: the fast and general bodies of the twofold kernels give the same bits.

A wave whose lanes all hold ordinary arguments runs the straight-line fast body
(texpm1: the small path, with its |x0| > ln 2 lanes deferred to the wave's
queue and drained with pexp0 - 1 alone); any other wave runs the general body
with the edge handling.  For ordinary arguments the two must agree bit for bit.
The same ordinary inputs run twice: as they are, and with one NaN second part
in every 64 consecutive elements, which sends every wave (at any number of
elements per thread) to the general body.  All other elements must come out
identical.
"""
import numpy as np
import pytest

from paper_1502_05216_amd import workloads
from parity_util import same_bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FUNCS = ("texp", "texpm1", "tlog", "tlog1p")
DTS = (np.float64, np.float32)


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    from paper_1502_05216_amd import _lib
    m.lib()
    saved = {(f, d): _lib.get_launch_config(f, d) for f in FUNCS for d in ("f64", "f32")}
    yield m
    for (f, d), c in saved.items():
        _lib.set_launch_config(f, d, *c)
    _lib.set_table_placement("auto")


@pytest.fixture(autouse=True)
def auto_tables():
    """Every test leaves the table placement automatic."""
    yield
    from paper_1502_05216_amd import _lib
    if _lib._lib is not None:
        _lib.set_table_placement("auto")


def gpu_call(tf, fn, x0, x1):
    d = torch.device("cuda:0")
    g0, g1 = getattr(tf, fn)(torch.from_numpy(x0).to(d), torch.from_numpy(x1).to(d))
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy()


@pytest.mark.parametrize("tables", ["lds", "global"])
@pytest.mark.parametrize("ept", [0, 1, 4], ids=["default", "ept1", "ept4"])
@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", FUNCS)
def test_fast_and_general_bodies_agree(tf, fn, dt, ept, tables):
    from paper_1502_05216_amd import _lib
    dts = "f64" if dt == np.float64 else "f32"
    if ept:
        _, bpc, pd = _lib.get_launch_config(fn, dts)
        _lib.set_launch_config(fn, dts, ept, bpc, pd)
    _lib.set_table_placement(tables)
    n = 256 * 4 * 40 + 77
    x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=91, edges=0.0)
    # signed zero second parts: the fast renormalisation of the logs must give
    # two_sum's +0 error for them
    zr = np.random.default_rng(94)
    x1[zr.choice(n, n // 40, replace=False)] = dt(-0.0)
    x1[zr.choice(n, n // 40, replace=False)] = dt(0.0)
    print("case", fn, dts, "ept", ept or "default", flush=True)
    a0, a1 = gpu_call(tf, fn, x0, x1)
    rng = np.random.default_rng(92)
    starts = np.arange(0, n, 64)
    idx = starts + rng.integers(0, 64, size=starts.size)
    idx = idx[idx < n]
    p1 = x1.copy()
    p1[idx] = np.nan
    b0, b1 = gpu_call(tf, fn, x0, p1)
    keep = np.ones(n, bool)
    keep[idx] = False
    for name, a, b in (("z0", a0, b0), ("z1", a1, b1)):
        ok = same_bits(a[keep], b[keep])
        if not ok.all():
            i = np.flatnonzero(keep)[np.flatnonzero(~ok)[:5]]
            raise AssertionError("%s %s: %s differs at %d elements, e.g. idx %s x0 %s fast %s "
                                 "general %s" % (fn, dts, name, (~ok).sum(), i, x0[i], a[i], b[i]))
    if fn == "texpm1":
        # the drain really ran: some lanes had |x0| > ln 2
        assert (np.abs(x0) > 0.7).sum() > 100


@pytest.mark.parametrize("tables", ["lds", "global"])
@pytest.mark.parametrize("frac", [1.0, 0.5], ids=["all", "half"])
@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_texpm1_deferred_lanes_against_oracle(tf, dt, frac, tables):
    """texpm1 where every lane (or every other one) has |x0| > ln 2, so the
    wave queue fills on every tile and the drain rewrites the z1 of most
    lines: the result must still meet the parity bar everywhere."""
    import oracle
    from parity_util import compare
    dts = "f64" if dt == np.float64 else "f32"
    n = 256 * 4 * 33 + 45
    rng = np.random.default_rng(93)
    hi = 700.0 if dt == np.float64 else 85.0
    lo = -40.0 if dt == np.float64 else -20.0
    big = np.where(rng.random(n) < 0.5, rng.uniform(0.7, hi, n), -rng.uniform(0.7, -lo, n))
    small = rng.uniform(-0.69, 0.69, n)
    x0 = np.where(rng.random(n) < frac, big, small).astype(dt)
    x1 = (x0 * rng.uniform(-1, 1, n).astype(dt) * np.finfo(dt).eps).astype(dt)
    from paper_1502_05216_amd import _lib
    _lib.set_table_placement(tables)
    print("case texpm1", dts, "deferred fraction", frac, "tables", tables, flush=True)
    g0, g1 = gpu_call(tf, "texpm1", x0, x1)
    o0, o1 = getattr(oracle, "texpm1" + ("" if dt == np.float64 else "f"))(x0, x1)
    compare(g0, g1, o0, o1, "texpm1 %s deferred %.1f" % (dts, frac))


def _branch_point_args(fn, dt, n, seed):
    """Ordinary arguments only, packed at the logs' branch points: tlog near
    y0 = 1/2 and 2 (scaling on or off) and at powers of two (reduced a0 = -1/2);
    tlog1p near y0 = -1/2 and 1 (outer branch on or off), near 0 and just above
    -1.  Second parts coupled, zero of either sign, or half an ulp."""
    rng = np.random.default_rng(seed)
    if fn == "tlog":
        centres = [0.5, 2.0] + [2.0 ** k for k in rng.integers(-120, 120, 6)]
    else:
        centres = [-0.5, 1.0, 0.0, -1.0]
    per = n // len(centres) + 1
    parts = []
    for c in centres:
        k = rng.integers(-2000, 2000, per)
        v = np.full(per, c, dt)
        tgt = np.where(k > 0, np.inf, -np.inf).astype(dt)
        for _ in range(int(np.abs(k).max())):
            v = np.where(k != 0, np.nextafter(v, tgt), v)
            k = k - np.sign(k)
        parts.append(v)
    x0 = np.concatenate(parts)[:n].astype(dt)
    if fn == "tlog":
        x0 = np.abs(x0)
        x0[x0 == 0] = dt(1.0)
    else:
        x0[x0 <= -1] = np.nextafter(dt(-1.0), dt(0.0))
    rng.shuffle(x0)
    u = np.finfo(dt).eps / 2
    r = rng.uniform(-1, 1, n).astype(dt)
    x1 = (x0 * r * dt(u)).astype(dt)
    pick = rng.integers(0, 6, n)
    x1[pick == 0] = dt(0.0)
    x1[pick == 1] = dt(-0.0)
    half = (np.spacing(np.abs(x0)) / 2).astype(dt)
    x1 = np.where(pick == 2, np.where(r < 0, -half, half), x1).astype(dt)
    # the argument stays inside the domain (tlog1p: above -1)
    if fn == "tlog1p":
        x1 = np.where(x0 < -0.75, np.abs(x1), x1).astype(dt)
    return x0, x1


@pytest.mark.parametrize("tables", ["lds", "global"])
@pytest.mark.parametrize("ept", [0, 1, 4], ids=["default", "ept1", "ept4"])
@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", ["tlog", "tlog1p"])
def test_fast_body_at_branch_points(tf, fn, dt, ept, tables):
    """Whole waves of ordinary arguments at the logs' branch points run the
    fast body (its cheaper Newton sum, outer-branch sums and + n ln2); with
    one NaN second part in every 64 elements the same arguments run the
    general body.  Both must give the same bits, and meet the oracle's bar."""
    import oracle
    from paper_1502_05216_amd import _lib
    from parity_util import compare
    dts = "f64" if dt == np.float64 else "f32"
    if ept:
        _, bpc, pd = _lib.get_launch_config(fn, dts)
        _lib.set_launch_config(fn, dts, ept, bpc, pd)
    n = 256 * 4 * 24
    x0, x1 = _branch_point_args(fn, dt, n, seed=95)
    _lib.set_table_placement(tables)
    print("case branch points", fn, dts, "ept", ept or "default", tables, flush=True)
    a0, a1 = gpu_call(tf, fn, x0, x1)
    o0, o1 = getattr(oracle, fn + ("" if dt == np.float64 else "f"))(x0, x1)
    compare(a0, a1, o0, o1, "%s %s branch points (fast body)" % (fn, dts))
    p1 = x1.copy()
    p1[::64] = np.nan
    b0, b1 = gpu_call(tf, fn, x0, p1)
    keep = np.ones(n, bool)
    keep[::64] = False
    for name, a, b in (("z0", a0, b0), ("z1", a1, b1)):
        ok = same_bits(a[keep], b[keep])
        assert ok.all(), "%s %s: %s fast and general bodies differ at %d elements" % (
            fn, dts, name, (~ok).sum())


@pytest.mark.parametrize("tables", ["lds", "global"])
@pytest.mark.parametrize("mix", ["none", "quarter", "half", "all"])
@pytest.mark.parametrize("ept", [1, 2, 4])
@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_tlog1p_shared_seeds(tf, dt, ept, mix, tables):
    """tlog1p's fast waves take the Newton seed of an element from its main
    part when the seed's argument equals y0, and evaluate the other seeds
    packed 64 to a pass.  Waves where no element, a quarter, half or every
    element needs its own seed (y1 beyond half an ulp of y0, or the outer
    branch), at 1, 2 and 4 elements per thread (up to four passes): the fast
    body against the general body bit for bit, and against the oracle."""
    import oracle
    from paper_1502_05216_amd import _lib
    from parity_util import compare
    dts = "f64" if dt == np.float64 else "f32"
    _, bpc, pd = _lib.get_launch_config("tlog1p", dts)
    _lib.set_launch_config("tlog1p", dts, ept, bpc, pd)
    _lib.set_table_placement(tables)
    n = 256 * 4 * 20
    rng = np.random.default_rng(96 + ept)
    p = {"none": 0.0, "quarter": 0.25, "half": 0.5, "all": 1.0}[mix]
    need = rng.random(n) < p
    x0 = rng.uniform(-0.5, 1.0, n).astype(dt)                    # inner, seed shared
    x1 = (x0 * rng.uniform(-1, 1, n).astype(dt) * dt(np.finfo(dt).eps / 4)).astype(dt)
    outer = need & (rng.random(n) < 0.5)
    x0[outer] = rng.uniform(1.0, 300.0, outer.sum()).astype(dt)   # outer branch
    x1[outer] = (x0[outer] * dt(np.finfo(dt).eps / 4)).astype(dt)
    loose = need & ~outer                                         # inner, y1 > ulp(y0)/2
    x1[loose] = (np.spacing(np.abs(x0[loose])) * dt(0.75)).astype(dt)
    print("case tlog1p shared seeds", dts, "ept", ept, mix, tables, flush=True)
    a0, a1 = gpu_call(tf, "tlog1p", x0, x1)
    o0, o1 = getattr(oracle, "tlog1p" + ("" if dt == np.float64 else "f"))(x0, x1)
    compare(a0, a1, o0, o1, "tlog1p %s shared seeds ept %d %s" % (dts, ept, mix))
    p1 = x1.copy()
    p1[::64] = np.nan
    b0, b1 = gpu_call(tf, "tlog1p", x0, p1)
    keep = np.ones(n, bool)
    keep[::64] = False
    for name, a, b in (("z0", a0, b0), ("z1", a1, b1)):
        ok = same_bits(a[keep], b[keep])
        assert ok.all(), "tlog1p %s ept %d %s: %s fast and general bodies differ at %d" % (
            dts, ept, mix, name, (~ok).sum())
