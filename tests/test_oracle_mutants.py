"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a wrong sign, a dropped term, a transposed
operand, a wrong index or exponent) in a copy of oracle/tfo.cpp, builds it on
the CPU and runs a short battery of the same checks the pin tests make
(accuracy against mpmath, special values).  Every mutant must fail the battery,
and the unmodified source must pass it.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mpref
from paper_1502_05216_amd import workloads

SRC = open(oracle.SRC).read()

MUTANTS = {
    "mul_td sign": ("return {pe.x0, pe.x1 + A.x1 * c};", "return {pe.x0, pe.x1 - A.x1 * c};"),
    "mul_td dropped low product": ("return {pe.x0, pe.x1 + A.x1 * c};", "return {pe.x0, pe.x1};"),
    "two_sum sign": ("return {s, da + db};", "return {s, da - db};"),
    "mul_tt dropped term": ("fma(A.x0, B.x1, fma(A.x1, B.x0, pe.x1))", "fma(A.x1, B.x0, pe.x1)"),
    "Horner dropped term": ("for (int j = K::N - 2; j >= 0; --j)", "for (int j = K::N - 2; j >= 1; --j)"),
    "texp dropped z0*t1": ("T z1s = z0s * t1 + (s.v.x1 + (s.v.x0 - z0s));",
                           "T z1s = (s.v.x1 + (s.v.x0 - z0s));"),
    "Newton dropped s": ("add_tt(add_tt(mul_tt(a, s), a), s)", "add_tt(mul_tt(a, s), a)"),
    "pexpm10 transposed": ("mul_tt(C, Tt));", "mul_tt(C, C));"),
    "scaling sign": ("T z0s = ldexp(z0, -s.k);", "T z0s = ldexp(z0, s.k);"),
    "texpm1 dropped +1": ("z1 = (z0 + T(1)) * t1", "z1 = z0 * t1"),
    "expm1 scaled -1": ("two_sum(shi, -ldexp(T(1), -m))", "two_sum(shi, -ldexp(T(1), m))"),
    "log dropped z1": ("Tw<T> a = {z.x0 - T(1), z.x1};               /* exact (Sterbenz) */",
                       "Tw<T> a = {z.x0 - T(1), T(0)};"),
    "n ln2 low part": ("mul_td(Tw<T>{T(K::LN2_HI()), T(K::LN2_LO())}, from_int<T>(n))",
                       "mul_td(Tw<T>{T(K::LN2_HI()), T(0)}, from_int<T>(n))"),
    "log table index": ("T r = fma(z, T(K::LOG_INVC()[i]), T(-1)); /* exact */",
                        "T r = fma(z, T(K::LOG_INVC()[i ^ 1]), T(-1));"),
    "exp table low part": ("T y = s + fma(s, p, T(K::S_LO()[j]));", "T y = s + fma(s, p, T(0));"),
    # the other entry points of the interface
    "tlog0 correction sign": ("x1 = X.x1 + (X.x0 - u0);", "x1 = X.x1 + (u0 - X.x0);"),
    "plog0 dropped n ln2": ("return add_n_ln2(newton_log(a, log1x(z.x0)), n);",
                            "return newton_log(a, log1x(z.x0));"),
    "plog1p0 outer sign": ("return plog_coupled_core(two_sum(T(1), y0));",
                           "return plog_coupled_core(two_sum(T(1), -y0));"),
    "texp0 dropped v1": ("z1 = ldexp((s.v.x0 - z0s) + s.v.x1, s.k);",
                         "z1 = ldexp((s.v.x0 - z0s), s.k);"),
    "p-function not renormalised": ("Tw<T> r = fast_two_sum(z0, z1);", "Tw<T> r = {z0, z1};"),
    # twofold arithmetic
    "two_diff sign": ("template <class T> Tw<T> two_diff(T a, T b) { return two_sum(a, -b); }",
                      "template <class T> Tw<T> two_diff(T a, T b) { return two_sum(a, b); }"),
    "tdiv dropped y1": ("T q1 = ((r + A.x1) - q0 * B.x1) / B.x0;", "T q1 = (r + A.x1) / B.x0;"),
    "tsqrt remainder sign": ("T r = fma(-z0, z0, x.x0);", "T r = fma(z0, z0, -x.x0);"),
    "trenorm fast sum for any pair": ("Tw<T> r = rule_tw(two_sum(x0, x1));",
                                      "Tw<T> r = rule_tw(fast_two_sum(x0, x1));"),
    "plog1p outer 1 + y": ("Tw<T> w = add_td(y, T(1));\n        return plog_coupled_core",
                           "Tw<T> w = add_td(y, T(-1));\n        return plog_coupled_core"),
}


def battery_interface(o):
    """Accuracy of the other interface functions (and coupling of the
    p-functions' results) on a few hundred arguments each."""
    math_of = {"texp": "exp", "texpm1": "expm1", "tlog": "log", "tlog1p": "log1p"}
    for name in ("texp0", "pexp", "plog0", "tlog0", "plog1p0", "tlog1pp", "plog1p"):
        base = workloads.INTERFACE_BASE[name]
        x0, x1 = workloads.twofold_inputs(name, 300, np.float64, seed=8, edges=0.0,
                                          coupled=name in workloads.COUPLED)
        if name in workloads.DOTTED:
            x1 = np.zeros_like(x0)
            z0, z1 = getattr(o, name)(x0)
        else:
            z0, z1 = getattr(o, name)(x0, x1)
        if name.startswith("p"):
            fin = np.isfinite(z0)
            if not ((z0[fin] + z1[fin]) == z0[fin]).all():
                return False
        rel = []
        for a, b, c, d in zip(x0, x1, z0, z1):
            v = mpref.exact(math_of[base], a, b)
            if v is None or abs(v) < 2.0 ** -969:
                continue
            if not np.isfinite(c) or not np.isfinite(d):
                return False
            rel.append(mpref.rel_error(c, d, v))
        if max(rel) > 2.0 ** -93:
            return False
    return True


def battery_arith(o):
    """Twofold arithmetic against exact rationals on a few hundred operands."""
    from fractions import Fraction as F
    rng = np.random.default_rng(4)
    n = 300
    x0 = np.exp2(rng.uniform(-20, 20, n)) * np.where(rng.uniform(-1, 1, n) < 0, -1, 1)
    x1 = x0 * rng.uniform(-1, 1, n) * 2.0 ** -53
    y0 = np.exp2(rng.uniform(-20, 20, n)) * np.where(rng.uniform(-1, 1, n) < 0, -1, 1)
    y1 = y0 * rng.uniform(-1, 1, n) * 2.0 ** -53
    y0[:50] = -x0[:50] * (1 + 2.0 ** -30)
    y1[:50] = y0[:50] * rng.uniform(-1, 1, 50) * 2.0 ** -53
    v = lambda a, b: F(float(a)) + F(float(b))
    for op in ("tadd", "tsub", "tmul", "tdiv"):
        z0, z1 = getattr(o, op)(x0, x1, y0, y1)
        for a, b, c, d, r0, r1 in zip(x0, x1, y0, y1, z0, z1):
            x, y = v(a, b), v(c, d)
            ex = {"tadd": x + y, "tsub": x - y, "tmul": x * y, "tdiv": x / y}[op]
            size = abs(F(float(a))) + abs(F(float(c))) if op in ("tadd", "tsub") else abs(ex)
            if not np.isfinite(r1) or abs(v(r0, r1) - ex) > size * F(2) ** -100:
                return False
    xs = np.abs(x0)
    xs1 = xs * rng.uniform(-1, 1, n) * 2.0 ** -53
    z0, z1 = o.tsqrt(xs, xs1)
    for a, b, r0, r1 in zip(xs, xs1, z0, z1):
        z = v(r0, r1)
        if not np.isfinite(r1) or abs(z * z - v(a, b)) > abs(F(float(a))) * F(2) ** -100:
            return False
    # renormalization keeps the value exactly, whichever part is larger
    z0, z1 = o.trenorm(y1, x0)
    for a, b, r0, r1 in zip(y1, x0, z0, z1):
        if v(r0, r1) != v(a, b):
            return False
    return True


def battery(o):
    """True if the oracle build `o` passes a short version of the pins."""
    thr = {"texp": (-98, -95), "texpm1": (-98, -95), "tlog": (-98, -93), "tlog1p": (-98, -93)}
    for fn in ("texp", "texpm1", "tlog", "tlog1p"):
        x0, x1 = workloads.twofold_inputs(fn, 400, np.float64, seed=5, edges=0.0)
        z0, z1 = getattr(o, fn)(x0, x1)
        rel = []
        for a, b, c, d in zip(x0, x1, z0, z1):
            v = mpref.exact(fn, a, b)
            if v is None or abs(v) < 2.0 ** -969:
                continue
            if not np.isfinite(c) or not np.isfinite(d):
                return False
            rel.append(mpref.rel_error(c, d, v))
        rel = np.array(rel)
        if rel.mean() > 2.0 ** thr[fn][0] or rel.max() > 2.0 ** thr[fn][1]:
            return False
    for fn, name in (("exp", "exp1x"), ("expm1", "expm1_1x"), ("log", "log1x"),
                     ("log1p", "log1p_1x")):
        x, _ = workloads.twofold_inputs("t" + fn, 400, np.float64, seed=6, edges=0.0)
        z = getattr(o, name)(x)
        errs = [mpref.ulp_error(zi, mpref.exact(fn, xi), "D") for xi, zi in zip(x, z)
                if mpref.exact(fn, xi) is not None and abs(float(mpref.exact(fn, xi))) > 2.0 ** -1022]
        if max(errs) > 0.52 or np.mean(errs) > 0.3:
            return False
    return battery_interface(o) and battery_arith(o)


def test_unmodified_source_passes(tmp_path):
    path = oracle.build_variant(SRC, str(tmp_path / "libtfo_same.so"))
    assert battery(oracle.variant(path))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, name
    path = oracle.build_variant(SRC.replace(old, new, 1), str(tmp_path / "libtfo_mut.so"))
    assert not battery(oracle.variant(path)), name
