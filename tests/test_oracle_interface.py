"""Pins for the oracle's other entry points of the paper's interface (sections
"Twofold exponent: Algorithm summary", "Twofold logarithm: Algorithm summary",
"C/C++ interface"): functions of a dotted argument (pexp0 texp0 pexpm10
texpm10 plog0 tlog0 plog1p0 tlog1p0) and of a coupled argument (texpp pexp
texpm1p pexpm1 tlogp plog tlog1pp plog1p), binary64 and binary32.

* Accuracy against mpmath at 240 bits on random arguments of each function's
  range (coupled arguments for the coupled-argument functions): the paper's
  L1 / L0 bars, as for texp/texpm1/tlog/tlog1p.
* p-functions return coupled results (z0 + z1 rounds to z0); t-functions
  return the 1x function's value as the main part, bit for bit.
* Identities the paper states or implies: texpp is texp and texpm1p is
  texpm1 (no special algorithm for a coupled argument); pexp / pexpm1 are
  those results renormalised, so their sums are equal as exact rationals; on
  coupled arguments the renormalisation at the start of tlog and tlog1p is the
  identity, so tlogp and tlog1pp equal tlog and tlog1p bit for bit; with
  x1 = 0, texp(x0, 0) and texpm1(x0, 0) reduce to texp0 and texpm10.
* Special values: the domain ends of the 1x functions and the rule for
  non-finite main parts.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import mpref
from paper_1502_05216_amd import workloads

DOTTED = list(workloads.DOTTED)
COUPLED = list(workloads.COUPLED)
MATH = {"texp": "exp", "texpm1": "expm1", "tlog": "log", "tlog1p": "log1p"}
THR = {("D", "exp"): (-98, -95), ("D", "log"): (-98, -93),
       ("F", "exp"): (-42, -38), ("F", "log"): (-42, -36)}
SUB = {"D": 2.0 ** -969, "F": 2.0 ** -102}
ONEX = {"texp": "exp1x", "texpm1": "expm1_1x", "tlog": "log1x", "tlog1p": "log1p_1x"}


def _dt(f):
    return np.float64 if f == "D" else np.float32


def _sfx(f):
    return "" if f == "D" else "f"


def _call(name, f, x0, x1=None):
    fn = getattr(oracle, name + _sfx(f))
    return fn(x0) if name in DOTTED else fn(x0, x1)


def _inputs(name, n, f, seed, edges=0.0):
    return workloads.twofold_inputs(name, n, _dt(f), seed=seed, edges=edges,
                                    coupled=name in COUPLED)


def _bits(a):
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def _same(a, b):
    return (_bits(a) == _bits(b)) | (np.isnan(a) & np.isnan(b))


@pytest.mark.parametrize("f", ["D", "F"])
@pytest.mark.parametrize("name", DOTTED + COUPLED)
def test_accuracy_L1_L0(name, f):
    base = workloads.INTERFACE_BASE[name]
    fam = "exp" if base.startswith("texp") else "log"
    x0, x1 = _inputs(name, 1500, f, seed=61 + len(name))
    if name in DOTTED:
        x1 = np.zeros_like(x0)
    z0, z1 = _call(name, f, x0, x1)
    rel = []
    for a, b, c, d in zip(x0, x1, z0, z1):
        v = mpref.exact(MATH[base], a, b)
        if v is None or abs(v) < SUB[f] or not np.isfinite(c):
            continue
        rel.append(mpref.rel_error(c, d, v))
    rel = np.array(rel)
    l1, l0 = THR[(f, fam)]
    assert rel.size > 1000
    assert rel.mean() <= 2.0 ** l1, math.log2(rel.mean())
    assert rel.max() <= 2.0 ** l0, math.log2(rel.max())


@pytest.mark.parametrize("f", ["D", "F"])
@pytest.mark.parametrize("name", [n for n in DOTTED + COUPLED if n.startswith("p")])
def test_p_functions_are_coupled(name, f):
    x0, x1 = _inputs(name, 20000, f, seed=71, edges=0.01)
    z0, z1 = _call(name, f, x0, x1)
    fin = np.isfinite(z0) & np.isfinite(z1)
    assert fin.mean() > 0.9
    np.testing.assert_array_equal((z0[fin] + z1[fin]).astype(_dt(f)), z0[fin])


@pytest.mark.parametrize("f", ["D", "F"])
@pytest.mark.parametrize("name", [n for n in DOTTED + COUPLED if n.startswith("t")])
def test_t_functions_main_part_is_the_1x_function(name, f):
    x0, x1 = _inputs(name, 20000, f, seed=73, edges=0.02)
    z0, _ = _call(name, f, x0, x1)
    ref = getattr(oracle, ONEX[workloads.INTERFACE_BASE[name]] + _sfx(f))(x0)
    assert _same(z0, ref).all()


@pytest.mark.parametrize("f", ["D", "F"])
def test_identities(f):
    sfx = _sfx(f)
    # texpp / texpm1p are texp / texpm1, for any argument
    for name, base in (("texpp", "texp"), ("texpm1p", "texpm1")):
        x0, x1 = workloads.twofold_inputs(base, 20000, _dt(f), seed=81, edges=0.02)
        a = getattr(oracle, name + sfx)(x0, x1)
        b = getattr(oracle, base + sfx)(x0, x1)
        assert _same(a[0], b[0]).all() and _same(a[1], b[1]).all()
    # pexp / pexpm1: the same sums, renormalised
    for name, base in (("pexp", "texp"), ("pexpm1", "texpm1")):
        x0, x1 = _inputs(name, 3000, f, seed=83)
        p0, p1 = getattr(oracle, name + sfx)(x0, x1)
        t0, t1 = getattr(oracle, base + sfx)(x0, x1)
        fin = np.isfinite(t0) & np.isfinite(p0)
        for a, b, c, d in zip(p0[fin], p1[fin], t0[fin], t1[fin]):
            assert Fraction(float(a)) + Fraction(float(b)) == Fraction(float(c)) + Fraction(float(d))
    # coupled arguments: tlogp / tlog1pp equal tlog / tlog1p bit for bit
    for name, base in (("tlogp", "tlog"), ("tlog1pp", "tlog1p")):
        x0, x1 = _inputs(name, 20000, f, seed=85)
        ev = workloads.edge_values(base, _dt(f))
        x0 = np.concatenate([x0, ev])
        x1 = np.concatenate([x1, np.zeros_like(ev)])
        a = getattr(oracle, name + sfx)(x0, x1)
        b = getattr(oracle, base + sfx)(x0, x1)
        assert _same(a[0], b[0]).all() and _same(a[1], b[1]).all(), name
    # x1 = 0: texp and texpm1 reduce to texp0 and texpm10 (equal values)
    for name, base in (("texp0", "texp"), ("texpm10", "texpm1")):
        x0, _ = workloads.twofold_inputs(base, 20000, _dt(f), seed=87, edges=0.02)
        a = getattr(oracle, name + sfx)(x0)
        b = getattr(oracle, base + sfx)(x0, np.zeros_like(x0))
        assert _same(a[0], b[0]).all()
        assert ((a[1] == b[1]) | (np.isnan(a[1]) & np.isnan(b[1]))).all(), name


@pytest.mark.parametrize("f", ["D", "F"])
def test_special_values(f):
    dt = _dt(f)
    inf, nan = np.inf, np.nan

    def one(name, a, b=0.0):
        z0, z1 = _call(name, f, np.array([a], dt), np.array([b], dt))
        return z0[0], z1[0]

    for name in ("plog0", "tlog0", "plog", "tlogp"):
        assert one(name, 0.0) == (-inf, 0.0)
        assert one(name, inf) == (inf, 0.0)
        z0, z1 = one(name, -1.0)
        assert np.isnan(z0) and np.isnan(z1)
        z0, z1 = one(name, 1.0)
        assert z0 == 0 and z1 == 0
    for name in ("plog1p0", "tlog1p0", "plog1p", "tlog1pp"):
        assert one(name, -1.0) == (-inf, 0.0)
        assert one(name, inf) == (inf, 0.0)
        z0, z1 = one(name, -2.0)
        assert np.isnan(z0) and np.isnan(z1)
        z0, z1 = one(name, 0.0)
        assert z0 == 0 and z1 == 0
    for name in ("texpm10", "pexpm10", "texpm1p", "pexpm1"):
        z0, z1 = one(name, 0.0)
        assert z0 == 0 and z1 == 0
        assert one(name, -inf) == (-1.0, 0.0)
    for name in ("texp0", "texpp", "pexp"):
        assert one(name, inf) == (inf, 0.0)
        assert one(name, -inf) == (0.0, 0.0)
        z0, z1 = one(name, 0.0)
        assert z0 == 1 and abs(z1) <= (2.0 ** -104 if f == "D" else 2.0 ** -45)
    # pexp0 as the paper writes it: z0 = z1 = +inf above the range, 0 below
    assert one("pexp0", inf) == (inf, inf)
    assert one("pexp0", -inf) == (0.0, 0.0)
    for name in DOTTED + COUPLED:
        z0, z1 = one(name, nan)
        assert np.isnan(z0) and np.isnan(z1), name


@pytest.mark.parametrize("f", ["D", "F"])
def test_edges_follow_the_rule(f):
    """Non-finite main parts: z1 NaN when z0 is NaN; z1 = +0 when z0 is
    infinite (pexp0 and pexpm10 excepted above their range, where the paper
    makes both parts +inf)."""
    dt = _dt(f)
    for name in DOTTED + COUPLED:
        ev = workloads.edge_values(workloads.INTERFACE_BASE[name], dt)
        x0 = np.repeat(ev, 5)
        x1 = np.tile(np.array([0.0, np.inf, -np.inf, np.nan, 1e-30], dt), ev.size)
        z0, z1 = _call(name, f, x0, x1)
        assert np.isnan(z1[np.isnan(z0)]).all(), name
        if name not in ("pexp0", "pexpm10"):
            zi = z1[np.isinf(z0)]
            assert (zi == 0).all() and not np.signbit(zi).any(), name
