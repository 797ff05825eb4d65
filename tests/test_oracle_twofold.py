"""Pins for the oracle's twofold functions against mathematics, not itself.

* Accuracy (section "Accuracy"): relative error |z0 + z1 - f(x0 + x1)| / |f|
  against mpmath at 240 bits on random coupled arguments; average (L1) and
  maximum (L0) below the paper's thresholds: exp-family double 2^-98 / 2^-95,
  log-family double 2^-98 / 2^-93, float 2^-42 / 2^-38 (exp) and 2^-36 (log).
  (The paper's exp-family L1 is 2^-100; the 1x product z0*expm1(x1) caps texp
  near 2^-99 on x0 up to 745, so 2^-98 is the bar used here.)  Results whose
  z1 lies in the subnormal range (the paper's claim excludes them) are held to
  |z0 + z1 - f| <= 2^L0 |f| + one subnormal ulp (z1 rounds on the subnormal grid).
* p-functions pexp0/pexpm10: coupled, relative error <= 2^-104 (double).
* z0 is bitwise the 1x function of x0 (section "Method summary").
* Special values (sections "Exponent/Logarithm: Algorithm summary"): exact
  cases and the NaN/inf conventions.
* "Not worse than standard" (section "Conclusion").
* Round trips and the closed form tlog1p(texpm1(texp(x))) = e^x.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import mpref
from paper_1502_05216_amd import workloads

THR = {  # (L1, L0) as powers of two
    ("D", "exp"): (-98, -95), ("D", "log"): (-98, -93),
    ("F", "exp"): (-42, -38), ("F", "log"): (-42, -36),
}
SUB = {"D": (2.0 ** -969, 2.0 ** -1074), "F": (2.0 ** -102, 2.0 ** -149)}


def _call(fn, f, x0, x1):
    return getattr(oracle, fn + ("f" if f == "F" else ""))(x0, x1)


def _accuracy(fn, f, x0, x1):
    fam = "exp" if fn.startswith("texp") else "log"
    l0 = 2.0 ** THR[(f, fam)][1]
    z0, z1 = _call(fn, f, x0, x1)
    rel, sub_bad, n_sub = [], 0, 0
    for a, b, c, d in zip(x0, x1, z0, z1):
        v = mpref.exact(fn, a, b)
        if v is None or not np.isfinite(c):
            continue
        if abs(v) < SUB[f][0]:
            n_sub += 1
            if mpref.abs_error(c, d, v) > l0 * abs(float(v)) + SUB[f][1]:
                sub_bad += 1
            continue
        rel.append(mpref.rel_error(c, d, v))
    return np.array(rel), sub_bad, n_sub


@pytest.mark.parametrize("f", ["D", "F"])
@pytest.mark.parametrize("fn", ["texp", "texpm1", "tlog", "tlog1p"])
def test_accuracy_L1_L0(fn, f):
    dt = np.float64 if f == "D" else np.float32
    x0, x1 = workloads.twofold_inputs(fn, 3000, dt, seed=11 + len(fn), edges=0.0)
    rel, sub_bad, n_sub = _accuracy(fn, f, x0, x1)
    fam = "exp" if fn.startswith("texp") else "log"
    l1, l0 = THR[(f, fam)]
    assert rel.size > 2000
    assert rel.mean() <= 2.0 ** l1, math.log2(rel.mean())
    assert rel.max() <= 2.0 ** l0, math.log2(rel.max())
    assert sub_bad == 0, (sub_bad, n_sub)


@pytest.mark.parametrize("f", ["D", "F"])
def test_texp_near_underflow_and_overflow(f):
    """Arguments whose results are subnormal or near the overflow threshold."""
    dt = np.float64 if f == "D" else np.float32
    lo, hi = (-745.13, -700.0) if f == "D" else (-103.97, -85.0)
    rng = np.random.default_rng(7)
    x0 = np.concatenate([rng.uniform(lo, hi, 400),
                         rng.uniform(700.0 if f == "D" else 86.0,
                                     709.78 if f == "D" else 88.72, 200)]).astype(dt)
    x1 = ((x0 * rng.uniform(-1, 1, x0.size).astype(dt)) * dt(2.0 ** (-53 if f == "D" else -24)))
    rel, sub_bad, n_sub = _accuracy("texp", f, x0, x1.astype(dt))
    assert n_sub > 100 and sub_bad == 0
    assert rel.max() <= 2.0 ** THR[(f, "exp")][1]


@pytest.mark.parametrize("f", ["D", "F"])
def test_p_functions_coupled_and_accurate(f):
    dt = np.float64 if f == "D" else np.float32
    rng = np.random.default_rng(9)
    bound = -104 if f == "D" else -45
    # results above 2^-969 (2^-102): below, the low part is subnormal
    x = rng.uniform(-670, 709, 1500).astype(dt) if f == "D" else rng.uniform(-70, 88, 1500).astype(dt)
    for name, fn, xs in (("pexp0", "exp", x), ("pexpm10", "expm1", (x / dt(200)).astype(dt))):
        v0, v1 = getattr(oracle, name + ("f" if f == "F" else ""))(xs)
        np.testing.assert_array_equal((v0 + v1).astype(dt), v0)          # coupled
        worst = max(mpref.rel_error(a, b, mpref.exact(fn, xi)) for xi, a, b in zip(xs, v0, v1))
        assert worst <= 2.0 ** bound, (name, math.log2(worst))


@pytest.mark.parametrize("f", ["D", "F"])
@pytest.mark.parametrize("fn,onex", [("texp", "exp1x"), ("texpm1", "expm1_1x"),
                                     ("tlog", "log1x"), ("tlog1p", "log1p_1x")])
def test_main_part_is_the_1x_function(fn, onex, f):
    dt = np.float64 if f == "D" else np.float32
    sfx = "f" if f == "F" else ""
    x0, x1 = workloads.twofold_inputs(fn, 20000, dt, seed=21, edges=0.02)
    z0, _ = _call(fn, f, x0, x1)
    ref = getattr(oracle, onex + sfx)(x0)
    same = (z0.view(np.uint64 if f == "D" else np.uint32) == ref.view(np.uint64 if f == "D"
                                                                    else np.uint32))
    same |= np.isnan(z0) & np.isnan(ref)
    assert same.all()


@pytest.mark.parametrize("f", ["D", "F"])
def test_special_cases(f):
    dt = np.float64 if f == "D" else np.float32
    inf, nan = np.inf, np.nan

    def one(fn, a, b=0.0):
        z0, z1 = _call(fn, f, np.array([a], dt), np.array([b], dt))
        return z0[0], z1[0]

    for s in (0.0, -0.0):
        z0, z1 = one("texpm1", s)
        assert z0 == 0 and np.signbit(z0) == np.signbit(dt(s)) and z1 == 0
        z0, z1 = one("tlog1p", s)
        assert z0 == 0 and np.signbit(z0) == np.signbit(dt(s)) and z1 == 0
    z0, z1 = one("tlog", 1.0)
    assert z0 == 0 and not np.signbit(z0) and z1 == 0
    z0, z1 = one("texp", 0.0)
    assert z0 == 1 and abs(z1) <= (2.0 ** -104 if f == "D" else 2.0 ** -45)
    assert one("texp", inf) == (inf, 0.0)
    assert one("texp", -inf) == (0.0, 0.0)
    assert one("tlog", 0.0) == (-inf, 0.0)
    assert one("tlog", inf) == (inf, 0.0)
    assert one("tlog1p", -1.0) == (-inf, 0.0)
    assert one("texpm1", -inf) == (-1.0, 0.0)
    for fn in ("texp", "texpm1", "tlog", "tlog1p"):
        z0, z1 = one(fn, nan)
        assert np.isnan(z0) and np.isnan(z1)
    z0, z1 = one("tlog", -1.0)
    assert np.isnan(z0) and np.isnan(z1)
    z0, z1 = one("tlog1p", -2.0)
    assert np.isnan(z0) and np.isnan(z1)
    # argument out of the domain while y0 is inside: x0 a number, x1 NaN
    z0, z1 = one("tlog", 1e-30 if f == "F" else 1e-300, -1.0)
    assert np.isfinite(z0) and np.isnan(z1)
    z0, z1 = one("tlog1p", -0.75, -0.5)
    assert np.isfinite(z0) and np.isnan(z1)
    # non-finite second part propagates
    z0, z1 = one("texp", 1.0, inf)
    assert z1 == inf
    z0, z1 = one("texp", 1.0, nan)
    assert np.isnan(z1) and np.isfinite(z0)


def test_not_worse_than_standard():
    """|z0 + z1 - f| <= |z0 - f| on coupled arguments (double), allowing the
    paper's 2 warnings per million samples."""
    bad = tot = 0
    for fn in ("texp", "texpm1", "tlog", "tlog1p"):
        x0, x1 = workloads.twofold_inputs(fn, 1500, np.float64, seed=31, edges=0.0)
        z0, z1 = oracle.__dict__[fn](x0, x1)
        for a, b, c, d in zip(x0, x1, z0, z1):
            v = mpref.exact(fn, a, b)
            if v is None or abs(v) < 2.0 ** -969 or not np.isfinite(c):
                continue
            tot += 1
            if mpref.abs_error(c, d, v) > mpref.abs_error(c, 0.0, v):
                bad += 1
    assert tot > 5000 and bad <= max(2, 2e-6 * tot)


def test_round_trips_and_composition():
    rng = np.random.default_rng(41)
    x0 = rng.uniform(-600, 600, 1500)
    x1 = x0 * rng.uniform(-1, 1, x0.size) * 2.0 ** -53
    z0, z1 = oracle.texp(x0, x1)
    w0, w1 = oracle.tlog(z0, z1)
    err = np.array([float(abs(Fraction(a) + Fraction(b) - Fraction(c) - Fraction(d)))
                    for a, b, c, d in zip(w0, w1, x0, x1)])
    assert (err <= 2.0 ** -92 * np.maximum(1.0, np.abs(x0))).all()
    # y = tlog1p(texpm1(texp(x))) = e^x exactly in closed form (finite range)
    x0, x1, _, _ = workloads.chain_inputs(1500)
    keep = x0 < 6.5
    x0, x1 = x0[keep], x1[keep]
    a0, a1 = oracle.texp(x0, x1)
    b0, b1 = oracle.texpm1(a0, a1)
    c0, c1 = oracle.tlog1p(b0, b1)
    rel = [mpref.rel_error(c, d, mpref.exact("exp", a, b)) for a, b, c, d in zip(x0, x1, c0, c1)]
    assert max(rel) <= 2.0 ** -90


def test_edges_do_not_crash_and_follow_the_rule():
    """Every edge argument gives z1 NaN when z0 is NaN and z1 = +0 when z0 is
    infinite (the rule for non-finite main parts)."""
    for f, dt in (("D", np.float64), ("F", np.float32)):
        for fn in ("texp", "texpm1", "tlog", "tlog1p"):
            ev = workloads.edge_values(fn, dt)
            x0 = np.repeat(ev, 5)
            x1 = np.tile(np.array([0.0, np.inf, -np.inf, np.nan, 1e-30], dt), ev.size)
            z0, z1 = _call(fn, f, x0, x1)
            assert np.isnan(z1[np.isnan(z0)]).all()
            zi = z1[np.isinf(z0)]
            assert (zi == 0).all() and not np.signbit(zi).any()
