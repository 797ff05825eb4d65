"""GPU parity of the twofold arithmetic (tadd, tsub, tmul, tdiv, tsqrt,
trenorm), binary64 and binary32, through the C ABI, against the oracle: random
twofolds over many magnitudes with cancellations, special values (zeros,
infinities, NaN, subnormals) mixed in, ragged sizes, misaligned arrays, and a
2^24-element run on a sample.  z0 bit for bit (the correctly rounded 1x
operation), z1 within 4 ulp (in practice bit for bit).  trenorm takes two
independent numbers (x0, y0) as its pair, so either part may be the larger,
with cancellations among them."""
import numpy as np
import pytest

import oracle
from parity_util import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OPS = ("tadd", "tsub", "tmul", "tdiv", "tsqrt", "trenorm")
DTS = (np.float64, np.float32)


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    m.lib()
    return m


def sfx(dt):
    return "" if dt == np.float64 else "f"


def operands(n, dt, seed, specials=0.01):
    rng = np.random.default_rng(seed)
    lo, hi = (-300, 300) if dt == np.float64 else (-40, 40)
    eps = dt(2.0 ** (-53 if dt == np.float64 else -24))
    out = []
    for _ in range(2):
        s = np.where(rng.uniform(-1, 1, n) < 0, -1.0, 1.0)
        a0 = (s * np.exp2(rng.uniform(lo, hi, n))).astype(dt)
        a1 = ((a0 * rng.uniform(-1, 1, n).astype(dt)) * eps).astype(dt)
        out += [a0, a1]
    x0, x1, y0, y1 = out
    k = n // 8                                          # near cancellation
    y0[:k] = (-x0[:k] * (dt(1) + dt(2.0 ** -20) * rng.uniform(-1, 1, k).astype(dt))).astype(dt)
    y1[:k] = ((y0[:k] * rng.uniform(-1, 1, k).astype(dt)) * eps).astype(dt)
    ns = int(n * specials)
    if ns:
        fi = np.finfo(dt)
        sp = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, fi.smallest_subnormal, fi.tiny,
                       fi.max, -1.0, 1.0], dt)
        for arr in (x0, y0):
            idx = rng.choice(n, ns, replace=False)
            arr[idx] = sp[rng.integers(0, sp.size, ns)]
    return x0, x1, y0, y1


def run(tf, op, dt, arrs, misalign=False):
    d = torch.device("cuda:0")

    def dev(a):
        if misalign:
            return torch.from_numpy(np.concatenate([a[:1], a])).to(d)[1:]
        return torch.from_numpy(np.ascontiguousarray(a)).to(d)
    x0, x1, y0, y1 = arrs
    if op == "tsqrt":
        g0, g1 = tf.tsqrt(dev(x0), dev(x1))
        o0, o1 = getattr(oracle, "tsqrt" + sfx(dt))(x0, x1, threads=8)
    elif op == "trenorm":
        g0, g1 = tf.trenorm(dev(x0), dev(y0))
        o0, o1 = getattr(oracle, "trenorm" + sfx(dt))(x0, y0, threads=8)
    else:
        g0, g1 = getattr(tf, op)(dev(x0), dev(x1), dev(y0), dev(y1))
        o0, o1 = getattr(oracle, op + sfx(dt))(x0, x1, y0, y1, threads=8)
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy(), o0, o1


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("op", OPS)
def test_parity_random_with_specials(tf, op, dt):
    arrs = operands(100003, dt, 301)
    if op == "tsqrt":
        arrs = (np.abs(arrs[0]), arrs[1]) + arrs[2:]
        arrs[0][:100] = -arrs[0][:100]                  # negative arguments too
    print("case", op, np.dtype(dt).name, flush=True)
    g0, g1, o0, o1 = run(tf, op, dt, arrs)
    nd = compare(g0, g1, o0, o1, "%s %s" % (op, np.dtype(dt).name))
    print("%s %s: z1 not bit-identical at %d" % (op, np.dtype(dt).name, nd))


@pytest.mark.parametrize("op", OPS)
def test_sizes_and_misaligned(tf, op):
    for dt in DTS:
        for n in (1, 2, 63, 64, 65, 511, 513, 4097):
            arrs = operands(n, dt, 303 + n, specials=0.05)
            g0, g1, o0, o1 = run(tf, op, dt, arrs)
            compare(g0, g1, o0, o1, "%s %s n=%d" % (op, np.dtype(dt).name, n))
        arrs = operands(20001, dt, 307)
        g0, g1, o0, o1 = run(tf, op, dt, arrs, misalign=True)
        compare(g0, g1, o0, o1, "%s %s misaligned" % (op, np.dtype(dt).name))


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_full_size_sampled(tf, dt):
    n = 1 << 24
    idx = np.sort(np.random.default_rng(9).choice(n, 20000, replace=False))
    arrs = operands(n, dt, 311, specials=0.001)
    d = torch.device("cuda:0")
    dev = [torch.from_numpy(a).to(d) for a in arrs]
    sub = [a[idx] for a in arrs]
    for op in OPS:
        print("case full", op, np.dtype(dt).name, flush=True)
        if op == "tsqrt":
            g0, g1 = tf.tsqrt(dev[0].abs(), dev[1])
            o0, o1 = getattr(oracle, "tsqrt" + sfx(dt))(np.abs(sub[0]), sub[1])
        elif op == "trenorm":
            g0, g1 = tf.trenorm(dev[0], dev[2])
            o0, o1 = getattr(oracle, "trenorm" + sfx(dt))(sub[0], sub[2])
        else:
            g0, g1 = getattr(tf, op)(*dev)
            o0, o1 = getattr(oracle, op + sfx(dt))(*sub)
        torch.cuda.synchronize()
        it = torch.from_numpy(idx).to(d)
        compare(g0[it].cpu().numpy(), g1[it].cpu().numpy(), o0, o1,
                "%s %s full-size sample" % (op, np.dtype(dt).name))
