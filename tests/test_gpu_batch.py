"""Batched ragged launch on the GPU: one hipGraph-captured persistent launch
over many arrays of mixed function, format and length must equal the plain
per-array calls bit for bit (which the plain parity tests tie to the oracle),
on every replay of the graph and for every configuration; a sample is also
checked against the oracle directly.  Sizes: a small batch with empty,
single-element and misaligned arrays, and the full 4096-array batch with
lengths 2^U[0, 20]."""
import numpy as np
import pytest

import oracle
from paper_1502_05216_amd import workloads
from parity_util import compare, same_bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    m.lib()
    return m


def _make(descs, misalign_every=0):
    d = torch.device("cuda:0")
    host = workloads.batch_inputs(descs)
    items, outs, refs = [], [], []
    for k, (fn, dt, x0, x1) in enumerate(host):
        if misalign_every and k % misalign_every == 1 and x0.size > 0:
            pad0 = np.concatenate([[dt(0.5)], x0])
            pad1 = np.concatenate([[dt(0.0)], x1])
            a0 = torch.from_numpy(pad0).to(d)[1:]
            a1 = torch.from_numpy(pad1).to(d)[1:]
        else:
            a0 = torch.from_numpy(np.ascontiguousarray(x0)).to(d)
            a1 = torch.from_numpy(np.ascontiguousarray(x1)).to(d)
        z0 = torch.full_like(a0, float("nan"))
        z1 = torch.full_like(a0, float("nan"))
        items.append((fn, a0, a1, z0, z1))
        outs.append((z0, z1))
    return host, items, outs


def _plain(tf, items):
    return [getattr(tf, fn)(a0, a1) for fn, a0, a1, _, _ in items]


def _equal(u, v):
    """Same bits, or both NaN."""
    it = torch.int64 if u.dtype == torch.float64 else torch.int32
    return bool(((u.view(it) == v.view(it)) | (torch.isnan(u) & torch.isnan(v))).all())


def _check_equal(items, outs, plain):
    for (fn, _, _, _, _), (z0, z1), (p0, p1) in zip(items, outs, plain):
        assert _equal(z0, p0) and _equal(z1, p1), fn


@pytest.mark.parametrize("config", [None, (2, 4, 1, 0), (2, 4, 8, 2), (4, 4, 4, 0),
                                    (1, 2, 16, 0)])
def test_small_batch_equals_plain(tf, config):
    from paper_1502_05216_amd.batch import BatchPlan
    rng = np.random.default_rng(3)
    lens = [0, 1, 2, 63, 64, 65, 511, 512, 513, 4097] + list(rng.integers(1, 40000, 54))
    descs = [(workloads.FUNCS[i % 4], np.float64 if (i // 4) % 3 else np.float32, int(n))
             for i, n in enumerate(lens)]
    host, items, outs = _make(descs, misalign_every=7)
    plain = _plain(tf, items)
    with BatchPlan(items, config) as plan:
        info = plan.info()
        assert info["elements"] == sum(lens)
        plan.launch()
        torch.cuda.synchronize()
        _check_equal(items, outs, plain)
        # replays, with eager work and synchronisation between them
        for r in range(3):
            for _, _, _, z0, z1 in items:
                z0.fill_(float("nan"))
                z1.fill_(7.0)
            torch.cuda.synchronize()
            plan.launch()
            torch.cuda.synchronize()
            _check_equal(items, outs, plain)
    # a few arrays straight against the oracle
    for k in (9, 17, 30):
        fn, dt, x0, x1 = host[k]
        sfx = "" if dt == np.float64 else "f"
        o0, o1 = getattr(oracle, fn + sfx)(x0, x1)
        compare(outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy(), o0, o1, "batch %s" % fn)


def test_full_batch_4096_arrays(tf):
    from paper_1502_05216_amd.batch import BatchPlan
    descs = workloads.batch_descriptors()
    print("case full batch", len(descs), sum(d[2] for d in descs), flush=True)
    host, items, outs = _make(descs)
    with BatchPlan(items) as plan:
        plan.launch()
        plan.launch()
        torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    for k in range(len(items)):
        fn, a0, a1, z0, z1 = items[k]
        p0, p1 = getattr(tf, fn)(a0, a1)
        assert _equal(z0, p0) and _equal(z1, p1), (k, fn)
    for k in rng.choice(len(items), 24, replace=False):
        fn, dt, x0, x1 = host[k]
        sfx = "" if dt == np.float64 else "f"
        idx = np.sort(rng.choice(x0.size, min(x0.size, 2000), replace=False))
        o0, o1 = getattr(oracle, fn + sfx)(x0[idx], x1[idx])
        it = torch.from_numpy(idx).to(outs[k][0].device)
        compare(outs[k][0][it].cpu().numpy(), outs[k][1][it].cpu().numpy(), o0, o1,
                "full batch %s" % fn)


def test_autotune_picks_a_candidate_with_plain_results(tf):
    """batch.autotune times every candidate on the caller's arrays and returns
    the fastest; a plan under it still equals the plain calls bit for bit."""
    from paper_1502_05216_amd.batch import BatchPlan, autotune
    rng = np.random.default_rng(5)
    lens = list(rng.integers(1, 30000, 40))
    descs = [(workloads.FUNCS[i % 4], np.float64 if i % 3 else np.float32, int(n))
             for i, n in enumerate(lens)]
    host, items, outs = _make(descs)
    plain = _plain(tf, items)
    cands = [(2, 4, 8, 0), (1, 2, 16, 2), (4, 4, 32, 0)]
    best, times = autotune(items, candidates=cands, reps=2)
    assert best in cands and set(times) == set(cands)
    assert all(t > 0 for t in times.values()) and times[best] == min(times.values())
    torch.cuda.synchronize()
    _check_equal(items, outs, plain)
    for _, _, _, z0, z1 in items:
        z0.fill_(float("nan"))
    with BatchPlan(items, config=best) as plan:
        plan.launch()
        torch.cuda.synchronize()
    _check_equal(items, outs, plain)


@pytest.mark.parametrize("config", [None, (1, 2, 1, 0), (4, 4, 8, 2)])
def test_batch_with_fully_deferred_texpm1(tf, config):
    """texpm1 arrays whose every lane has |x0| > ln 2 fill the per-wave queue on
    every tile; interleaved with the other functions and formats, the queue of
    the pair being left must be drained before the next pair's work, and the
    drained z1 rewrites must land after the whole-line stores: the batch still
    equals the plain calls bit for bit, on every replay."""
    from paper_1502_05216_amd.batch import BatchPlan
    d = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    items, outs = [], []
    for k in range(24):
        fn = ("texpm1", "tlog1p", "texpm1", "texp", "tlog", "texpm1")[k % 6]
        dt = np.float64 if k % 4 != 3 else np.float32
        n = int(rng.integers(1, 30000))
        if fn == "texpm1":
            hi = 700.0 if dt == np.float64 else 85.0
            lo = 40.0 if dt == np.float64 else 20.0
            x0 = np.where(rng.random(n) < 0.5, rng.uniform(0.7, hi, n),
                          -rng.uniform(0.7, lo, n)).astype(dt)
            x1 = (x0 * rng.uniform(-1, 1, n).astype(dt) * np.finfo(dt).eps).astype(dt)
        else:
            x0, x1 = workloads.twofold_inputs(fn, n, dt, seed=100 + k)
        a0 = torch.from_numpy(x0).to(d)
        a1 = torch.from_numpy(x1).to(d)
        z0 = torch.full_like(a0, float("nan"))
        z1 = torch.full_like(a0, float("nan"))
        items.append((fn, a0, a1, z0, z1))
        outs.append((z0, z1))
    plain = _plain(tf, items)
    print("case deferred batch", config, flush=True)
    with BatchPlan(items, config) as plan:
        for r in range(3):
            for _, _, _, z0, z1 in items:
                z0.fill_(float("nan"))
                z1.fill_(7.0)
            torch.cuda.synchronize()
            plan.launch()
            torch.cuda.synchronize()
            _check_equal(items, outs, plain)
