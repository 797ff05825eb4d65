"""GPU backward kernels and the autograd chain against the oracle.

* tf_*_bwd through the C ABI equals the oracle's twofold adjoint bit for bit
  (same operations: twofold product/quotient with the FMA remainder), binary64
  and binary32, random operands, ragged sizes and special values.
* tf_chain_bwd (one fused pass over a chain of up to 8 stages) equals the
  chained single-stage kernels and the oracle's chained adjoints bit for bit.
* torch.autograd through the fused chain node (y = tlog1p(texpm1(texp(x)))
  = e^x), which equals TExp -> TExpm1 -> TLog1p chained by autograd bit for
  bit: the forward results meet the parity bar (z0 bit for bit, z1 within
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


def _chain_case(tf, dt, names, n, share, misalign, seed):
    """Saved values and upstream gradient for a chain of `names` on n
    elements (host arrays, and device tensors: misaligned views if asked;
    stage j + 1 reuses stage j's arrays where share[j])."""
    rng = np.random.default_rng(seed)
    eps = dt(2.0 ** (-53 if dt == np.float64 else -24))

    def tw(lo, hi):
        a0 = rng.uniform(lo, hi, n).astype(dt)
        return a0, ((a0 * rng.uniform(-1, 1, n).astype(dt)) * eps).astype(dt)

    def dev(a):
        if misalign:
            return torch.from_numpy(np.concatenate([a[:1], a])).to(torch.device("cuda:0"))[1:]
        return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))

    host, devs = [], []
    for j in range(len(names)):
        if j > 0 and share[j - 1]:
            host.append(host[-1])
            devs.append(devs[-1])
            continue
        s0, s1 = tw(0.1, 50)
        if n > 100:
            s0[:5] = np.array([0.0, np.inf, np.nan, 1e-30, -0.5], dt)
        host.append((s0, s1))
        devs.append((dev(s0), dev(s1)))
    g0, g1 = tw(-1, 1)
    return host, devs, (g0, g1), (dev(g0), dev(g1))


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_chain_bwd_equals_stagewise(tf, dt):
    """tf_chain_bwd equals the chained single-stage backward kernels and the
    oracle's chained adjoints bit for bit: chains of 1..11 stages (longer
    than TF_CHAIN_MAX go in groups), stages sharing saved arrays, ragged and
    misaligned arrays, special saved values, gx aliasing g."""
    sfx = "" if dt == np.float64 else "f"
    rng = np.random.default_rng(31)
    cases = [(["tlog1p"], 77, False), (["texp", "texpm1", "tlog1p"], 100003, False),
             (list(rng.choice(list(tf.TWOFOLD), 8)), 4097, False),
             (list(rng.choice(list(tf.TWOFOLD), 5)), 20001, True),
             (["tlog", "texp"], 1, False), (list(rng.choice(list(tf.TWOFOLD), 11)), 5003, False)]
    for ci, (names, n, mis) in enumerate(cases):
        share = [names[j] in ("texp", "texpm1") and names[j + 1] in ("tlog", "tlog1p")
                 for j in range(len(names) - 1)]
        print("case", ci, names, n, "misaligned" if mis else "", flush=True)
        host, devs, g, G = _chain_case(tf, dt, names, n, share, mis, 100 + ci)
        f0, f1 = tf.chain_bwd(names, devs, *G)
        c = G
        for name, (s0, s1) in reversed(list(zip(names, devs))):
            c = getattr(tf, name + "_bwd")(s0, s1, *c)
        o = g
        for name, (s0, s1) in reversed(list(zip(names, host))):
            o = getattr(oracle, name + sfx + "_bwd")(s0, s1, *o)
        torch.cuda.synchronize()
        f0, f1, c0, c1 = _np(f0, f1, *c)
        assert same_bits(f0, c0).all() and same_bits(f1, c1).all(), (ci, names)
        assert same_bits(f0, o[0]).all() and same_bits(f1, o[1]).all(), (ci, names)
        if not mis:                                    # gx aliasing g
            A0, A1 = G[0].clone(), G[1].clone()
            tf.chain_bwd(names, devs, A0, A1, out=(A0, A1))
            torch.cuda.synchronize()
            a0, a1 = _np(A0, A1)
            assert same_bits(a0, f0).all() and same_bits(a1, f1).all(), (ci, names)


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
    # the fused chain node equals the single-stage Functions chained by autograd
    from paper_1502_05216_amd.autograd import TExp, TExpm1, TLog1p
    W0, W1 = [t.detach().clone().requires_grad_(True) for t in (X0, X1)]
    v0, v1 = TLog1p.apply(*TExpm1.apply(*TExp.apply(W0, W1)))
    torch.autograd.backward([v0, v1], [G0, G1])
    assert same_bits(W0.grad.cpu().numpy(), gx0).all()
    assert same_bits(W1.grad.cpu().numpy(), gx1).all()
    assert same_bits(v0.detach().cpu().numpy(), y0.detach().cpu().numpy()).all()
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
    f0, f1 = tf.chain_bwd(("texp", "texpm1", "tlog1p"), [(a0, a1), (b0, b1), (b0, b1)], G0, G1)
    torch.cuda.synchronize()
    assert same_bits(*_np(f0, e0)).all() and same_bits(*_np(f1, e1)).all()
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
