"""Pins for the oracle's twofold arithmetic (section "Twofolds update": the
tadd / tmul / tdiv / tsqrt workload; subtraction by the corrected Algorithm 2.2
of section "Twofold bugs").

* Against exact rational arithmetic (fractions) on random twofolds of many
  magnitudes, cancellation included: |z0 + z1 - (x op y)| within a few units
  of 2^-106 (double) / 2^-48 (float) of the operands' size.
* The main part is the 1x operation on the main parts, bit for bit (numpy's
  IEEE +, -, *, /, sqrt).
* The corrected Algorithm 2.2 gives d + t = a - b exactly, and tsub(x, y) is
  tadd(x, -y) bit for bit (the correction is two_sum with b -> -b).
* Special values: the rule for non-finite main parts; sqrt of 0 and of
  negative numbers; division by zero.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

F = Fraction


def _tw(rng, n, dt, lo=-30, hi=30):
    s = np.where(rng.uniform(-1, 1, n) < 0, -1.0, 1.0)
    x0 = (s * np.exp2(rng.uniform(lo, hi, n))).astype(dt)
    eps = dt(2.0 ** (-53 if dt == np.float64 else -24))
    x1 = ((x0 * rng.uniform(-1, 1, n).astype(dt)) * eps).astype(dt)
    return x0, x1


def _sfx(dt):
    return "" if dt == np.float64 else "f"


def _val(a, b):
    return F(float(a)) + F(float(b))


def _bits(a):
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("op", ["tadd", "tsub", "tmul", "tdiv"])
def test_binary_ops_against_exact_rationals(op, dt):
    rng = np.random.default_rng(17)
    n = 3000
    x0, x1 = _tw(rng, n, dt)
    y0, y1 = _tw(rng, n, dt)
    if op in ("tadd", "tsub"):
        # near-cancellation: y close to -x (tadd) or x (tsub)
        k = n // 4
        sgn = dt(-1) if op == "tadd" else dt(1)
        y0[:k] = (sgn * x0[:k] * (dt(1) + dt(2.0 ** -20) * rng.uniform(-1, 1, k).astype(dt))
                  ).astype(dt)
        eps = dt(2.0 ** (-53 if dt == np.float64 else -24))
        y1[:k] = ((y0[:k] * rng.uniform(-1, 1, k).astype(dt)) * eps).astype(dt)
    z0, z1 = getattr(oracle, op + _sfx(dt))(x0, x1, y0, y1)
    unit = 2.0 ** (-106 if dt == np.float64 else -48)
    worst = 0.0
    for a, b, c, d, r0, r1 in zip(x0, x1, y0, y1, z0, z1):
        x, y = _val(a, b), _val(c, d)
        exact = {"tadd": x + y, "tsub": x - y, "tmul": x * y, "tdiv": x / y}[op]
        err = abs(_val(r0, r1) - exact)
        size = abs(F(float(a))) + abs(F(float(c))) if op in ("tadd", "tsub") else abs(exact)
        worst = max(worst, float(err / size) / unit)
    bound = {"tadd": 3, "tsub": 3, "tmul": 6, "tdiv": 12}[op]
    assert worst <= bound, (op, worst)
    main = {"tadd": x0 + y0, "tsub": x0 - y0, "tmul": x0 * y0, "tdiv": x0 / y0}[op]
    assert (_bits(z0) == _bits(main.astype(dt))).all()


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_tsqrt_against_exact_rationals(dt):
    rng = np.random.default_rng(19)
    x0, x1 = _tw(rng, 3000, dt)
    x0 = np.abs(x0)
    x1 = ((x0 * rng.uniform(-1, 1, x0.size).astype(dt)) *
          dt(2.0 ** (-53 if dt == np.float64 else -24))).astype(dt)
    z0, z1 = getattr(oracle, "tsqrt" + _sfx(dt))(x0, x1)
    unit = 2.0 ** (-106 if dt == np.float64 else -48)
    worst = 0.0
    for a, b, r0, r1 in zip(x0, x1, z0, z1):
        x = _val(a, b)
        z = _val(r0, r1)
        # |z - sqrt(x)| = |z^2 - x| / (z + sqrt(x)) ~ |z^2 - x| / (2 z)
        rel = float(abs(z * z - x) / (2 * z * z))
        worst = max(worst, rel / unit)
    assert worst <= 6, worst
    assert (_bits(z0) == _bits(np.sqrt(x0))).all()


def test_corrected_two_diff_is_exact_and_matches_tadd():
    rng = np.random.default_rng(23)
    for dt in (np.float64, np.float32):
        x0, x1 = _tw(rng, 5000, dt, -60, 60)
        y0, y1 = _tw(rng, 5000, dt, -60, 60)
        y0[:1000] = x0[:1000]                                 # exact cancellation
        y0[1000:2000] = np.nextafter(x0[1000:2000], dt(np.inf))
        sfx = _sfx(dt)
        d0, d1 = getattr(oracle, "tsub" + sfx)(x0, np.zeros_like(x0), y0, np.zeros_like(y0))
        for a, c, r0, r1 in zip(x0, y0, d0, d1):
            assert F(float(r0)) + F(float(r1)) == F(float(a)) - F(float(c))
        s0, s1 = getattr(oracle, "tsub" + sfx)(x0, x1, y0, y1)
        a0, a1 = getattr(oracle, "tadd" + sfx)(x0, x1, -y0, -y1)
        assert (_bits(s0) == _bits(a0)).all() and (_bits(s1) == _bits(a1)).all()


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_special_values(dt):
    inf, nan = np.inf, np.nan
    sfx = _sfx(dt)

    def bin_op(op, a, b, c, d):
        r = getattr(oracle, op + sfx)(*(np.array([v], dt) for v in (a, b, c, d)))
        return r[0][0], r[1][0]

    def sq(a, b=0.0):
        r = getattr(oracle, "tsqrt" + sfx)(np.array([a], dt), np.array([b], dt))
        return r[0][0], r[1][0]

    assert bin_op("tdiv", 1.0, 0.0, 0.0, 0.0) == (inf, 0.0)
    z0, z1 = bin_op("tdiv", 0.0, 0.0, 0.0, 0.0)
    assert np.isnan(z0) and np.isnan(z1)
    assert bin_op("tadd", inf, 0.0, 1.0, 0.0) == (inf, 0.0)
    z0, z1 = bin_op("tadd", inf, 0.0, -inf, 0.0)
    assert np.isnan(z0) and np.isnan(z1)
    assert bin_op("tmul", inf, 0.0, 2.0, 0.0) == (inf, 0.0)
    assert sq(0.0) == (0.0, 0.0)
    assert sq(4.0) == (2.0, 0.0)
    assert sq(inf) == (inf, 0.0)
    z0, z1 = sq(-1.0)
    assert np.isnan(z0) and np.isnan(z1)
    for op in ("tadd", "tsub", "tmul", "tdiv"):
        z0, z1 = bin_op(op, nan, 0.0, 1.0, 0.0)
        assert np.isnan(z0) and np.isnan(z1)


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_trenorm_exact_and_fast_form(dt):
    """trenorm: z0 + z1 = x0 + x1 exactly (rationals), z0 = RN(x0 + x1), |z1| <= ulp(z0)/2,
    for any pair (second part larger than the first, cancellation, zeros); where
    |x0| >= |x1| it equals the paper's three-operation fast renormalization bit for bit."""
    rng = np.random.default_rng(29)
    n = 4000
    x0, _ = _tw(rng, n, dt, -40, 40)
    x1, _ = _tw(rng, n, dt, -40, 40)                  # any magnitude relative to x0
    x1[:500] = -x0[:500]                                # exact cancellation
    x1[500:1000] = (-x0[500:1000] * (dt(1) + dt(2.0 ** -20))).astype(dt)
    x0[1000:1100] = dt(0)
    x1[1100:1200] = dt(0)
    sfx = _sfx(dt)
    z0, z1 = getattr(oracle, "trenorm" + sfx)(x0, x1)
    for a, b, r0, r1 in zip(x0, x1, z0, z1):
        assert _val(r0, r1) == _val(a, b)
    assert (_bits(z0) == _bits((x0 + x1).astype(dt))).all()
    assert (np.abs(z1) <= np.spacing(np.abs(z0)) / 2).all()
    big = np.abs(x0) >= np.abs(x1)
    s = (x0 + x1).astype(dt)
    t = (x1 - (s - x0)).astype(dt)
    assert (_bits(z0[big]) == _bits(s[big])).all() and (_bits(z1[big]) == _bits(t[big])).all()
    assert big.sum() > 1000 and (~big).sum() > 1000


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_trenorm_special_values(dt):
    inf, nan = np.inf, np.nan
    f = getattr(oracle, "trenorm" + _sfx(dt))
    z0, z1 = f(np.array([inf, 1.0, -inf, nan, inf, 0.0], dt), np.array([1.0, inf, 2.0, 0.0, -inf, -0.0], dt))
    assert z0[0] == inf and z1[0] == 0 and z0[1] == inf and z1[1] == 0
    assert z0[2] == -inf and z1[2] == 0
    assert np.isnan(z0[3]) and np.isnan(z1[3]) and np.isnan(z0[4]) and np.isnan(z1[4])
    assert z0[5] == 0 and z1[5] == 0
