"""CPU pins for the cheaper forms the GPU kernels' fast bodies use in place of
the general twofold operations, swept densely around the branch points.

A wave whose lanes all hold ordinary arguments runs a fast body that writes
three steps of the logarithms with fewer operations than the oracle's general
form; the claim is that each gives the general form's bits on every argument
a fast wave can see.  Each form is emulated here in numpy (binary64 and
binary32 arithmetic, round to nearest; the fused products through the oracle's
exact two_prod or exact rationals) next to the general form, and both are
compared bit for bit, signed zeros included:

1. The end of the Newton step (section "Twofold logarithm > Newton inversion"):
   r1 = (m0 + s0) + (m1 + s1) for the twofold sum u = m + s followed by
   r1 = u0 + u1, where m = a s + a and s = e^-r0 - 1 for the 1x seed
   r0 = log1p(a0 + a1).  m0 and -s0 agree to a few ulps, so m0 + s0 is exact.
   Swept: a0 on both sides of -1/2 (z0 = 1/2 in tlog, y0 = -1/2 in tlog1p),
   of 0, of 1, random in [-1/2, 1], with coupled and zero second parts; s0 is
   moved by up to 4 ulps to cover any last-bit difference of the seed path.
2. tlog1p's outer branch: 1 + v as two fast two-sums for v0 > 1 or
   -1 <= v0 < -1/2 (1 + v0 exact there), against add_td then two_sum.
3. X + n ln2 as a fast two-sum for |X0| < 1, against add_tt, for every n a
   binary64 or binary32 argument can produce.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def bits(x):
    x = np.asarray(x)
    return x.view(np.uint64 if x.dtype == np.float64 else np.uint32)


def two_sum(a, b):
    s = a + b
    bp = s - a
    ap = s - bp
    return s, (a - ap) + (b - bp)


def fast_two_sum(a, b):
    s = a + b
    return s, b - (s - a)


def fma(a, b, c):
    """Correctly rounded a*b + c elementwise (exact rationals)."""
    dt = a.dtype.type
    out = np.empty_like(a)
    for i, (x, y, z) in enumerate(zip(a.tolist(), b.tolist(), c.tolist())):
        if dt == np.float64:
            out[i] = float(Fraction(x) * Fraction(y) + Fraction(z))
        else:
            out[i] = np.float32(_round_f32(Fraction(x) * Fraction(y) + Fraction(z)))
    return out


def _round_f32(q):
    """Round an exact rational to binary32 (nearest even, subnormals kept)."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    quantum = Fraction(2) ** (max(e, -126) - 23)
    m = q / quantum
    r = m.numerator // m.denominator
    rem = m - r
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and r % 2 == 1):
        r += 1
    return sign * float(r * quantum)


def two_prod(a, b):
    p = a * b
    return p, fma(a, b, -p)


def mul_tt(A, B):
    p, e = two_prod(A[0], B[0])
    return p, fma(A[0], B[1], fma(A[1], B[0], e))


def add_tt(A, B):
    s, t = two_sum(A[0], B[0])
    return s, t + (A[1] + B[1])


def ulps_away(x, k):
    """x moved by k units in the last place (k may be negative)."""
    out = x.copy()
    tgt = np.where(k > 0, np.inf, -np.inf).astype(x.dtype)
    for _ in range(int(np.abs(k).max())):
        move = np.abs(k) > 0
        out = np.where(move, np.nextafter(out, tgt), out)
        k = k - np.sign(k)
    return out


def newton_args(dt, n, seed):
    """Reduced twofold arguments a of the Newton step, dense at its branch points."""
    rng = np.random.default_rng(seed)
    u = np.finfo(dt).eps / 2
    parts = []
    for c in (-0.5, 0.0, 1.0):
        k = rng.integers(-3000, 3000, n // 8)
        a0 = ulps_away(np.full(k.size, c, dt), k)
        parts.append(a0)
    parts.append(rng.uniform(-0.5, 1.0, n // 4).astype(dt))
    parts.append((np.sign(rng.uniform(-1, 1, n // 8)) *
                  np.exp2(rng.uniform(-60, -1, n // 8))).astype(dt))
    sub = np.array([0.0, -0.0, np.finfo(dt).smallest_subnormal, -np.finfo(dt).smallest_subnormal,
                    np.finfo(dt).tiny, -0.5, 0.5, 1.0, -np.nextafter(dt(0.5), dt(0))], dt)
    a0 = np.concatenate(parts + [sub])
    a0 = a0[(a0 >= -0.5) & (a0 <= 1.0)]
    # second parts: coupled (|a1| <= ulp(a0)/2), zero of either sign, half-way
    r = rng.uniform(-1, 1, a0.size).astype(dt)
    a1 = (a0 * r * dt(u)).astype(dt)
    pick = rng.integers(0, 6, a0.size)
    a1 = np.where(pick == 0, dt(0.0), a1)
    a1 = np.where(pick == 1, dt(-0.0), a1)
    half = (np.spacing(np.abs(a0)) / 2).astype(dt)
    a1 = np.where(pick == 2, np.where(r < 0, -half, half), a1)
    # a = z - 1 with z in [1/2, 2] renormalised: keep a0 + a1 in [-1/2 - ulp, 1 + ulp]
    return a0, a1.astype(dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_newton_sum_as_two_plain_sums(dt):
    sfx = "" if dt == np.float64 else "f"
    a0, a1 = newton_args(dt, 6000 if dt == np.float64 else 4000, seed=5)
    r0 = getattr(oracle, "log1p_1x" + sfx)((a0 + a1).astype(dt))
    s0, s1 = getattr(oracle, "pexpm10" + sfx)(-r0)
    rng = np.random.default_rng(6)
    s0 = ulps_away(s0, rng.integers(-4, 5, s0.size))
    s1 = (s1 * rng.uniform(-1.0, 1.0, s1.size)).astype(dt)
    m = add_tt(mul_tt((a0, a1), (s0, s1)), (a0, a1))
    # general: u = add_tt(m, s), r1 = u0 + u1; fast: two plain sums
    u0, u1 = add_tt(m, (s0, s1))
    r1_gen = u0 + u1
    r1_fast = (m[0] + s0) + (m[1] + s1)
    exact = np.array([Fraction(float(x)) + Fraction(float(y)) == Fraction(float(x + y))
                      for x, y in zip(m[0], s0)])
    assert exact.all(), "m0 + s0 inexact at a0 = %r" % (a0[~exact][:4],)
    np.testing.assert_array_equal(bits(r1_fast), bits(r1_gen))
    # the sweep is sharp: the sum a s + a written as a fast two-sum (the cut
    # withdrawn because |a s| can round up to |a| = 1/2) differs somewhere here
    p = mul_tt((a0, a1), (s0, s1))
    st = fast_two_sum(p[0], a0)
    m_cut = (st[0], st[1] + (p[1] + a1))
    differs = (bits(m_cut[0]) != bits(m[0])) | (bits(m_cut[1]) != bits(m[1]))
    assert differs.any()


def outer_args(dt, n, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for c, lo, hi in ((-1.0, 0, 4000), (-0.5, -4000, 0), (1.0, 1, 4000)):
        k = rng.integers(lo, hi, n // 6)
        parts.append(ulps_away(np.full(k.size, c, dt), k))
    parts.append(rng.uniform(-1.0, -0.5, n // 6).astype(dt))
    parts.append(np.exp2(rng.uniform(0.0, 100.0, n // 6)).astype(dt))
    parts.append(np.array([-1.0, np.nextafter(dt(-0.5), dt(-1)), np.nextafter(dt(1), dt(2)),
                           np.finfo(dt).max, 2.0, 3.0], dt))
    v0 = np.concatenate(parts)
    v0 = v0[(v0 > 1) | ((v0 >= -1) & (v0 < -0.5))]
    half = (np.spacing(np.abs(v0)) / 2).astype(dt)
    r = rng.uniform(-1, 1, v0.size).astype(dt)
    v1 = (half * r).astype(dt)
    pick = rng.integers(0, 6, v0.size)
    v1 = np.where(pick == 0, dt(0.0), v1)
    v1 = np.where(pick == 1, dt(-0.0), v1)
    v1 = np.where(pick == 2, np.where(r < 0, -half, half), v1)
    v1 = np.where(v0 == -1, np.abs(v1), v1)          # the argument stays above -1
    return v0, v1.astype(dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_tlog1p_outer_one_plus_v_as_fast_two_sums(dt):
    v0, v1 = outer_args(dt, 60000, seed=8)
    with np.errstate(over="ignore"):
        one = dt(1.0)
        # general: w = add_td(v, 1) = two_sum(v0, 1) then t + v1; w = two_sum(w)
        s, t = two_sum(v0, np.full_like(v0, one))
        g0, g1 = two_sum(s, t + v1)
        # fast
        s2, t2 = fast_two_sum(v0, np.full_like(v0, one))
        f0, f1 = fast_two_sum(s2, t2 + v1)
    fin = np.isfinite(g0)
    assert fin.sum() > 0.99 * v0.size
    np.testing.assert_array_equal(bits(f0[fin]), bits(g0[fin]))
    np.testing.assert_array_equal(bits(f1[fin]), bits(g1[fin]))


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_plus_n_ln2_as_fast_two_sum(dt):
    if dt == np.float64:
        ln2_hi, ln2_lo, nmin, nmax = 0.6931471805599453, 2.3190468138462996e-17, -1075, 1025
    else:
        ln2_hi, ln2_lo, nmin, nmax = np.float32(0.6931472), np.float32(-1.9046542e-09), -150, 129
    assert Fraction(float(ln2_hi)) + Fraction(float(ln2_lo)) != 0
    rng = np.random.default_rng(9)
    n = np.concatenate([np.arange(nmin, nmax), rng.integers(nmin, nmax, 20000)]).astype(dt)
    x0 = rng.uniform(-1, 1, n.size).astype(dt)
    edge = np.array([0.0, -0.0, ln2_hi, -ln2_hi, np.nextafter(dt(1), dt(0)),
                     -np.nextafter(dt(1), dt(0)), np.finfo(dt).smallest_subnormal, 0.5, -0.5], dt)
    x0[: n.size // 4] = ulps_away(np.resize(edge, n.size // 4),
                                  rng.integers(-3, 4, n.size // 4)).astype(dt)
    x0 = np.where(np.abs(x0) < 1, x0, dt(0.5))
    x1 = (x0 * rng.uniform(-1, 1, n.size).astype(dt) * dt(np.finfo(dt).eps / 2)).astype(dt)
    x1[::7] = dt(-0.0)
    x1[3::7] = dt(0.0)
    hi = np.full_like(x0, ln2_hi)
    L0, e = two_prod(hi, n)
    L1 = e + np.full_like(x0, ln2_lo) * n
    g = add_tt((x0, x1), (L0, L1))                    # general
    s, t = fast_two_sum(L0, x0)                       # fast
    f = (s, t + (x1 + L1))
    np.testing.assert_array_equal(bits(f[0]), bits(g[0]))
    np.testing.assert_array_equal(bits(f[1]), bits(g[1]))

