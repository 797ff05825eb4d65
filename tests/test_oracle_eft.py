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


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def test_fast_two_sum_plus_zero_form_equals_two_sum_bitwise():
    """The fast two-sum with its error written (a - s) + b, which the GPU
    kernels use where |a| >= |b| is guaranteed (the logs' first
    renormalisation on fast waves, the 1x expm1's reconstruction), gives
    two_sum's bits, signed zeros included.  The usual b - (s - a) gives -0
    where two_sum gives +0 (b = -0, a != 0).  Where |b| exceeds |a| across a
    power of two no three-operation form is exact, which is why the logs'
    Newton sum a s + a (|a s| can round up to |a| = 1/2) keeps two_sum."""
    a, b = _pairs(4000, 4)
    swap = np.abs(a) < np.abs(b)
    a2 = np.where(swap, b, a)
    b2 = np.where(swap, a, b)
    zeros_a = np.array([1.0, -1.0, 0.0, -0.0, 0.0, -0.0, 2.5, -2.5])
    zeros_b = np.array([-0.0, -0.0, -0.0, -0.0, 0.0, 0.0, 0.0, -0.0])
    A = np.concatenate([a2, zeros_a])
    B = np.concatenate([b2, zeros_b])
    s_ref, t_ref = oracle.eft("two_sum", A, B)
    s = A + B
    t = (A - s) + B
    np.testing.assert_array_equal(_bits(s), _bits(s_ref))
    np.testing.assert_array_equal(_bits(t), _bits(t_ref))
    # the usual form differs exactly on the signed zero
    t_usual = B[-8:-6] - (s[-8:-6] - A[-8:-6])
    assert np.all(np.signbit(t_usual)) and not np.any(np.signbit(t_ref[-8:-6]))
    # |b| just above |a| = 1/2 - 2^-54, one sign: the sum rounds to -1 and the
    # three-operation error is wrong
    a3, b3 = np.array([-(0.5 - 2.0 ** -54)]), np.array([-0.5])
    s3, t3_ref = oracle.eft("two_sum", a3, b3)
    t3 = (a3 - s3) + b3
    assert Fraction(float(s3[0])) + Fraction(float(t3_ref[0])) == Fraction(-(0.5 - 2.0 ** -54)) - Fraction(1, 2)
    assert t3[0] != t3_ref[0]
