"""High-precision reference values (mpmath) and error metrics for the oracle's
pins -- TEST INFRASTRUCTURE.

The exact argument of a twofold is the real sum x0 + x1 (evaluated exactly in
mpmath); the exact result f(x0 + x1) is evaluated at PREC bits.  Relative
error of a twofold result is |z0 + z1 - f| / |f|; 1x results are measured in
units of the last place (ulp) of the exact value in the target format.
"""
import math

import mpmath
from mpmath import mpf

PREC = 240

FMT = {"D": (53, -1022), "F": (24, -126)}

_F = {
    "texp": mpmath.exp,
    "texpm1": mpmath.expm1,
    "tlog": mpmath.log,
    "tlog1p": mpmath.log1p,
    "exp": mpmath.exp,
    "expm1": mpmath.expm1,
    "log": mpmath.log,
    "log1p": mpmath.log1p,
}


def exact(fn, x0, x1=0.0):
    """f(x0 + x1) at PREC bits (mpf), or None where the value is not finite/real."""
    with mpmath.workprec(PREC):
        x = mpf(float(x0)) + mpf(float(x1))
        f = _F[fn]
        if fn in ("tlog", "log") and x <= 0:
            return None
        if fn in ("tlog1p", "log1p") and x <= -1:
            return None
        try:
            v = f(x)
        except (OverflowError, ValueError):
            return None
        return v


def ulp_of(v, fmt):
    p, emin = FMT[fmt]
    if v == 0:
        return mpf(2) ** (emin - p + 1)
    e = int(mpmath.floor(mpmath.log(abs(v), 2)))
    while mpf(2) ** e > abs(v):
        e -= 1
    while mpf(2) ** (e + 1) <= abs(v):
        e += 1
    return mpf(2) ** (max(e, emin) - p + 1)


def ulp_error(z, v, fmt):
    """|z - v| in ulps of the exact value v (z a float of the format)."""
    with mpmath.workprec(PREC):
        return float(abs(mpf(float(z)) - v) / ulp_of(v, fmt))


def rel_error(z0, z1, v):
    """|z0 + z1 - v| / |v| for a twofold result."""
    with mpmath.workprec(PREC):
        s = mpf(float(z0)) + mpf(float(z1))
        if v == 0:
            return float(abs(s))
        return float(abs(s - v) / abs(v))


def abs_error(z0, z1, v):
    with mpmath.workprec(PREC):
        return float(abs(mpf(float(z0)) + mpf(float(z1)) - v))


def log2_or_neg(x):
    return math.log2(x) if x > 0 else -math.inf
