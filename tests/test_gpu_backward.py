"""GPU backward kernels and the autograd chain against the oracle.

* tf_*_bwd through the C ABI equals the oracle's twofold adjoint bit for bit
  (same operations: twofold product/quotient with the FMA remainder), binary64
  and binary32, random operands, ragged sizes and special values.
* torch.autograd through TExp -> TExpm1 -> TLog1p (y = tlog1p(texpm1(texp(x)))
  = e^x): the forward results meet the parity bar (z0 bit for bit, z1 within
  4 ulp); the chained gradient, computed from forward second parts that may
  differ from the oracle's in their last bits, equals the oracle's chained
  gradient as a twofold value to 2^-98 with the same non-finite classes, and
  g e^x to 2^-94 where every intermediate is normal (mpmath, on a sample);
  elements with x > ln ln DBL_MAX overflow to y = inf and give NaN gradients
  on both sides.
"""
import mpmath
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


def _dev(*arrs):
    d = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in arrs]


def _np(*ts):
    return [t.detach().cpu().numpy() for t in ts]


def assert_twofold_close(g0, g1, o0, o1, rel, what):
    """Same non-finite classes; finite values g0 + g1 and o0 + o1 within rel
    of |o0| (the difference of main parts is exact when they are close)."""
    assert (np.isnan(g0) == np.isnan(o0)).all(), what
    assert (np.isinf(g0) == np.isinf(o0)).all() and (g0[np.isinf(o0)] == o0[np.isinf(o0)]).all(), what
    fin = np.isfinite(o0) & np.isfinite(o1)
    assert np.isfinite(g1[fin]).all(), what
    d = np.abs((g0[fin] - o0[fin]) + (g1[fin] - o1[fin]))
    bad = d > rel * np.abs(o0[fin])
    assert not bad.any(), "%s: %d of %d outside %g, e.g. gpu %r oracle %r" % (
        what, bad.sum(), fin.sum(), rel, g0[fin][bad][:3], o0[fin][bad][:3])


@pytest.mark.parametrize("n", [1, 77, 511, 100003])
@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("fn", ["texp", "texpm1", "tlog", "tlog1p"])
def test_backward_parity(tf, fn, dt, n):
    rng = np.random.default_rng(n)
    eps = dt(2.0 ** (-53 if dt == np.float64 else -24))
    s0 = rng.uniform(0.1, 50, n).astype(dt)
    s1 = ((s0 * rng.uniform(-1, 1, n).astype(dt)) * eps).astype(dt)
    g0 = rng.uniform(-1, 1, n).astype(dt)
    g1 = ((g0 * rng.uniform(-1, 1, n).astype(dt)) * eps).astype(dt)
    if n > 100:
        s0[:6] = np.array([0.0, -1.0, np.inf, np.nan, 1e-30, -0.5], dt)
    sfx = "" if dt == np.float64 else "f"
    o0, o1 = getattr(oracle, fn + sfx + "_bwd")(s0, s1, g0, g1)
    gx0, gx1 = getattr(tf, fn + "_bwd")(*_dev(s0, s1, g0, g1))
    torch.cuda.synchronize()
    assert same_bits(gx0.cpu().numpy(), o0).all()
    assert same_bits(gx1.cpu().numpy(), o1).all()


def test_autograd_chain(tf):
    from paper_1502_05216_amd.autograd import chain_exp_expm1_log1p
    n = 1 << 16
    x0, x1, g0, g1 = workloads.chain_inputs(n)
    X0, X1, G0, G1 = _dev(x0, x1, g0, g1)
    X0.requires_grad_(True)
    X1.requires_grad_(True)
    y0, y1 = chain_exp_expm1_log1p(X0, X1)
    torch.autograd.backward([y0, y1], [G0, G1])
    gx0 = X0.grad.cpu().numpy()
    gx1 = X1.grad.cpu().numpy()
    # oracle chain, forward then backward
    a0, a1 = oracle.texp(x0, x1)
    b0, b1 = oracle.texpm1(a0, a1)
    c0, c1 = oracle.tlog1p_bwd(b0, b1, g0, g1)
    d0, d1 = oracle.texpm1_bwd(b0, b1, c0, c1)
    e0, e1 = oracle.texp_bwd(a0, a1, d0, d1)
    assert_twofold_close(gx0, gx1, e0, e1, 2.0 ** -98, "chained gradient")
    o0, o1 = oracle.tlog1p(b0, b1)
    compare(*_np(y0, y1), o0, o1, "chain forward y")
    nan = ~np.isfinite(gx0)
    assert abs(int(nan.sum()) - int((x0 > 6.565).sum())) <= 2
    idx = np.flatnonzero(x0 < 6.2)[:400]
    worst = 0.0
    with mpmath.workprec(240):
        for i in idx:
            x = mpmath.mpf(float(x0[i])) + mpmath.mpf(float(x1[i]))
            g = mpmath.mpf(float(g0[i])) + mpmath.mpf(float(g1[i]))
            ref = g * mpmath.exp(x)
            got = mpmath.mpf(float(gx0[i])) + mpmath.mpf(float(gx1[i]))
            worst = max(worst, float(abs(got - ref) / abs(ref)))
    assert worst <= 2.0 ** -94


def test_chain_full_size_sampled(tf):
    """The cfg5 size, 2^24 elements, forward + backward; sampled check."""
    n = 1 << 24
    x0, x1, g0, g1 = workloads.chain_inputs(n)
    X0, X1, G0, G1 = _dev(x0, x1, g0, g1)
    a0, a1 = tf.texp(X0, X1)
    b0, b1 = tf.texpm1(a0, a1)
    y0, y1 = tf.tlog1p(b0, b1)
    c0, c1 = tf.tlog1p_bwd(b0, b1, G0, G1)
    d0, d1 = tf.texpm1_bwd(b0, b1, c0, c1)
    e0, e1 = tf.texp_bwd(a0, a1, d0, d1)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(1).choice(n, 20000, replace=False))
    it = torch.from_numpy(idx).to(X0.device)
    oa0, oa1 = oracle.texp(x0[idx], x1[idx])
    ob0, ob1 = oracle.texpm1(oa0, oa1)
    oc0, oc1 = oracle.tlog1p_bwd(ob0, ob1, g0[idx], g1[idx])
    od0, od1 = oracle.texpm1_bwd(ob0, ob1, oc0, oc1)
    oe0, oe1 = oracle.texp_bwd(oa0, oa1, od0, od1)
    compare(*_np(a0[it], a1[it]), oa0, oa1, "chain texp")
    compare(*_np(b0[it], b1[it]), ob0, ob1, "chain texpm1")
    assert_twofold_close(*_np(e0[it], e1[it]), oe0, oe1, 2.0 ** -98, "chained gradient")
