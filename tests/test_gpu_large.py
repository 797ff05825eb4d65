"""Arrays past 2^31 elements: element indices and byte offsets beyond 32 bits.

texp in binary32 on 2^31 + 4099 elements (8 GiB per array) and tlog in
binary64 on 2^30 + 777 elements (8 GiB per array), plus tadd in binary32 on
2^31 + 5 elements; inputs drawn on the device from a seeded generator, a
sample of indices (including the first and last elements and those around
2^31) checked against the oracle."""
import numpy as np
import pytest

import oracle
from parity_util import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    m.lib()
    return m


def _draw(n, dtype, lo, hi, seed, log2=False):
    d = torch.device("cuda:0")
    g = torch.Generator(device=d)
    g.manual_seed(seed)
    x0 = torch.empty(n, dtype=dtype, device=d).uniform_(lo, hi, generator=g)
    if log2:
        x0 = torch.exp2(x0)
    u = torch.empty(n, dtype=dtype, device=d).uniform_(-1.0, 1.0, generator=g)
    eps = 2.0 ** (-53 if dtype == torch.float64 else -24)
    x1 = (x0 * u) * eps
    del u
    return x0, x1


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    pts = [0, 1, n - 1, n - 2]
    for c in (1 << 31, 1 << 32):
        pts += [c + k for k in range(-3, 4) if 0 <= c + k < n]
    return np.unique(np.concatenate([np.array(pts, np.int64), rng.integers(0, n, 4000)]))


def _take(t, idx):
    return t[torch.from_numpy(idx).to(t.device)].cpu().numpy()


def test_texp_f32_beyond_2_31(tf):
    n = (1 << 31) + 4099
    print("case texp f32 n=%d" % n, flush=True)
    x0, x1 = _draw(n, torch.float32, -100.0, 88.0, 7)
    z0, z1 = tf.texp(x0, x1)
    torch.cuda.synchronize()
    idx = _sample(n, 1)
    a0, a1 = _take(x0, idx), _take(x1, idx)
    o0, o1 = oracle.texpf(a0, a1)
    compare(_take(z0, idx), _take(z1, idx), o0, o1, "texp f32 beyond 2^31")
    del x0, x1, z0, z1
    torch.cuda.empty_cache()


def test_tlog_f64_beyond_2_30(tf):
    n = (1 << 30) + 777
    print("case tlog f64 n=%d" % n, flush=True)
    x0, x1 = _draw(n, torch.float64, -1000.0, 1000.0, 8, log2=True)
    z0, z1 = tf.tlog(x0, x1)
    torch.cuda.synchronize()
    idx = _sample(n, 2)
    a0, a1 = _take(x0, idx), _take(x1, idx)
    o0, o1 = oracle.tlog(a0, a1)
    compare(_take(z0, idx), _take(z1, idx), o0, o1, "tlog f64 beyond 2^30")
    del x0, x1, z0, z1
    torch.cuda.empty_cache()


def test_tadd_f32_beyond_2_31(tf):
    n = (1 << 31) + 5
    print("case tadd f32 n=%d" % n, flush=True)
    x0, x1 = _draw(n, torch.float32, -1e3, 1e3, 9)
    y0 = x0.flip(0)
    y1 = x1.flip(0)
    z0, z1 = tf.tadd(x0, x1, y0, y1)
    torch.cuda.synchronize()
    idx = _sample(n, 3)
    o0, o1 = oracle.taddf(_take(x0, idx), _take(x1, idx), _take(y0, idx), _take(y1, idx))
    compare(_take(z0, idx), _take(z1, idx), o0, o1, "tadd f32 beyond 2^31")
    del x0, x1, y0, y1, z0, z1
    torch.cuda.empty_cache()
