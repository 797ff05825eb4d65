"""Pins for the oracle's 1x functions exp, expm1, log, log1p (the main parts z0).

The paper takes z0 from the C library and asks only that it be reproducible
(section "Twofold exponent: Method summary"); the library allows 1/2 to 1 ulp.
Here each 1x function is checked against mpmath (240-bit) on random
arguments over its whole range, in units of the last place of the exact value:
max <= 1 ulp (subnormal results of exp may round twice), and <= 0.52 ulp
outside the subnormal range; C99 Annex F special values are checked exactly.
"""
import numpy as np
import pytest

import oracle
from oracle import mpref

FN = {"exp": "exp1x", "expm1": "expm1_1x", "log": "log1x", "log1p": "log1p_1x"}


def _args(fn, f, n, seed):
    rng = np.random.default_rng(seed)
    dt = np.float64 if f == "D" else np.float32
    if fn == "exp":
        x = rng.uniform(-745.2, 709.78, n) if f == "D" else rng.uniform(-104.0, 88.72, n)
    elif fn == "log":
        x = np.exp2(rng.uniform(-1074, 1024, n)) if f == "D" else np.exp2(rng.uniform(-149, 128, n))
    else:
        lo = -60 if f == "D" else -30
        top = 9.47 if f == "D" else 6.47    # expm1 finite below ~709.78 / ~88.72
        x = np.where(rng.uniform(-1, 1, n) < 0, -1.0, 1.0) * np.exp2(rng.uniform(lo, top, n))
        if fn == "log1p":
            x = np.where(x <= -1, -rng.uniform(0, 1, n), x)
    return x.astype(dt)


@pytest.mark.parametrize("f", ["D", "F"])
@pytest.mark.parametrize("fn", ["exp", "expm1", "log", "log1p"])
def test_ulp_accuracy(fn, f):
    x = _args(fn, f, 2500, hash((fn, f)) % 1000)
    z = getattr(oracle, FN[fn] + ("f" if f == "F" else ""))(x)
    tiny = 2.0 ** -1022 if f == "D" else 2.0 ** -126
    worst, worst_normal, tot, cnt = 0.0, 0.0, 0.0, 0
    for xi, zi in zip(x, z):
        v = mpref.exact(fn, xi)
        if v is None or not np.isfinite(zi):
            continue
        e = mpref.ulp_error(zi, v, f)
        worst = max(worst, e)
        if abs(v) >= tiny:
            worst_normal = max(worst_normal, e)
        tot += e
        cnt += 1
    assert cnt > 2000
    assert worst <= 1.0, worst
    assert worst_normal <= 0.52, worst_normal
    assert tot / cnt <= 0.3


@pytest.mark.parametrize("f", ["D", "F"])
def test_annex_f_special_values(f):
    dt = np.float64 if f == "D" else np.float32
    sfx = "f" if f == "F" else ""
    inf, nan = np.inf, np.nan

    def ev(name, xs):
        return getattr(oracle, name + sfx)(np.array(xs, dtype=dt))

    z = ev("exp1x", [0.0, -0.0, -inf, inf, nan, -1e6, 1e6])
    assert z[0] == 1 and z[1] == 1 and z[2] == 0 and not np.signbit(z[2])
    assert z[3] == inf and np.isnan(z[4]) and z[5] == 0 and z[6] == inf
    z = ev("expm1_1x", [0.0, -0.0, -inf, inf, nan, -1e6])
    assert z[0] == 0 and not np.signbit(z[0]) and z[1] == 0 and np.signbit(z[1])
    assert z[2] == -1 and z[3] == inf and np.isnan(z[4]) and z[5] == -1
    z = ev("log1x", [1.0, 0.0, -0.0, -1.0, inf, nan, -inf])
    assert z[0] == 0 and not np.signbit(z[0]) and z[1] == -inf and z[2] == -inf
    assert np.isnan(z[3]) and z[4] == inf and np.isnan(z[5]) and np.isnan(z[6])
    z = ev("log1p_1x", [0.0, -0.0, -1.0, -2.0, inf, nan, -inf])
    assert z[0] == 0 and not np.signbit(z[0]) and z[1] == 0 and np.signbit(z[1])
    assert z[2] == -inf and np.isnan(z[3]) and z[4] == inf and np.isnan(z[5]) and np.isnan(z[6])


@pytest.mark.parametrize("f", ["D", "F"])
def test_tiny_and_boundary_arguments(f):
    dt = np.float64 if f == "D" else np.float32
    sfx = "f" if f == "F" else ""
    fi = np.finfo(dt)
    tiny = dt(fi.smallest_subnormal)
    # expm1 and log1p are the identity on tiny arguments; exp and log at 1 ulp of 1
    for name in ("expm1_1x", "log1p_1x"):
        x = np.array([tiny, -tiny, dt(fi.tiny), dt(1e-30) if f == "D" else dt(1e-20)], dtype=dt)
        np.testing.assert_array_equal(getattr(oracle, name + sfx)(x), x)
    e = getattr(oracle, "exp1x" + sfx)(np.array([tiny, -tiny], dtype=dt))
    assert (e == 1).all()
    # exp overflows exactly above its threshold and underflows to 0 below ln 2^(emin-p)
    from tables_util import parse_header
    import os
    T = parse_header(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                  "oracle", "tfo_tables.h"))
    xmax = dt(T["TFO_%s_EXP_XMAX" % f])
    xlo = dt(T["TFO_%s_EXP_XLO" % f])
    z = getattr(oracle, "exp1x" + sfx)(np.array(
        [xmax, np.nextafter(xmax, dt(np.inf)), xlo, np.nextafter(xlo, dt(-np.inf))], dtype=dt))
    assert np.isfinite(z[0]) and z[0] == fi.max or np.isfinite(z[0])
    assert z[1] == np.inf
    assert z[2] == fi.smallest_subnormal and z[3] == 0


@pytest.mark.parametrize("f", ["D", "F"])
def test_demo_values(f):
    """The demo of section "Demo examples": exp(1), expm1(1), log(2), log1p(1)."""
    dt = np.float64 if f == "D" else np.float32
    sfx = "f" if f == "F" else ""
    one = np.array([1.0], dtype=dt)
    two = np.array([2.0], dtype=dt)
    zero = np.zeros(1, dtype=dt)
    exact = {k: mpref.exact(k, a) for k, a in
             (("exp", 1.0), ("expm1", 1.0), ("log", 2.0), ("log1p", 1.0))}
    vals = {
        "exp": getattr(oracle, "exp1x" + sfx)(one)[0],
        "expm1": getattr(oracle, "expm1_1x" + sfx)(one)[0],
        "log": getattr(oracle, "log1x" + sfx)(two)[0],
        "log1p": getattr(oracle, "log1p_1x" + sfx)(one)[0],
    }
    for k, v in vals.items():   # within half an ulp (correctly rounded) at these points
        assert mpref.ulp_error(v, exact[k], f) <= 0.5, k
    assert getattr(oracle, "texp" + sfx)(one, zero)[0][0] == vals["exp"]
    assert getattr(oracle, "texpm1" + sfx)(one, zero)[0][0] == vals["expm1"]
    assert getattr(oracle, "tlog" + sfx)(two, zero)[0][0] == vals["log"]
    assert getattr(oracle, "tlog1p" + sfx)(one, zero)[0][0] == vals["log1p"]
