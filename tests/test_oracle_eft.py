"""Pins for the oracle's error-free transforms (twofold arithmetic layer).

two_sum / fast_two_sum / two_prod return s + t equal to the exact sum or
product (checked with exact rationals), with s the rounded operation; the
fast form gives the same bits as two_sum whenever |a| >= |b| -- the property
that lets the method use it in Horner steps and renormalisation.
"""
from fractions import Fraction

import numpy as np

import oracle


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-60, 60, n))
    b = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-60, 60, n))
    adv_a = np.array([1.0, 1.0, 2.0 ** 1000, 0.0, -0.0, 1e-310, 3.0, 2.0 ** -1022, 1.0 + 2 ** -52,
                      0.1, 1e308])
    adv_b = np.array([2.0 ** -60, -1.0 + 2 ** -53, -(2.0 ** 1000) * (1 - 2 ** -53), 5.0, -0.0,
                      -1e-310, 2.0 ** -53, -(2.0 ** -1074), -(1.0 + 2 ** -51), 0.2, 1e307])
    return np.concatenate([a, adv_a]), np.concatenate([b, adv_b])


def test_two_sum_exact():
    a, b = _pairs(4000, 1)
    s, t = oracle.eft("two_sum", a, b)
    np.testing.assert_array_equal(s, a + b)
    for ai, bi, si, ti in zip(a, b, s, t):
        assert Fraction(si) + Fraction(ti) == Fraction(ai) + Fraction(bi)


def test_fast_two_sum_matches_two_sum_when_ordered():
    a, b = _pairs(4000, 2)
    swap = np.abs(a) < np.abs(b)
    a2 = np.where(swap, b, a)
    b2 = np.where(swap, a, b)
    s1, t1 = oracle.eft("two_sum", a2, b2)
    s2, t2 = oracle.eft("fast_two_sum", a2, b2)
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(t1, t2)


def test_two_prod_exact():
    a, b = _pairs(4000, 3)
    with np.errstate(over="ignore"):
        prod = np.abs(a * b)
    keep = (prod > 2.0 ** -900) & (prod < 2.0 ** 1000)   # exact away from under/overflow
    a, b = a[keep], b[keep]
    p, e = oracle.eft("two_prod", a, b)
    np.testing.assert_array_equal(p, a * b)
    for ai, bi, pi, ei in zip(a, b, p, e):
        assert Fraction(pi) + Fraction(ei) == Fraction(ai) * Fraction(bi)
