"""Helpers for table pins: parse a C header of hex-float arrays, and exact
round-to-nearest checks with Python's decimal/fractions (independent of the
mpmath used by the table generators)."""
import re
from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 80          # ~265 bits

_ARR = re.compile(r"static const (double|float|int) (\w+)\[(\d+)\] = \{(.*?)\};", re.S)
_SCAL = re.compile(r"static const (double|float) (\w+) = ([^;]+);")
_DEF = re.compile(r"#define (\w+) (-?\d+)")


def _num(tok, ty):
    tok = tok.strip()
    if ty == "int":
        return int(tok)
    if tok.endswith("f"):
        tok = tok[:-1]
    if tok in ("INFINITY", "-INFINITY"):
        return float(tok.replace("INFINITY", "inf"))
    if tok.startswith(("0x", "-0x")):
        return float.fromhex(tok)
    return float(tok)


def parse_header(path):
    src = open(path).read()
    out = {}
    for ty, name, n, body in _ARR.findall(src):
        vals = [_num(t, ty) for t in body.replace("\n", " ").split(",") if t.strip()]
        assert len(vals) == int(n), name
        out[name] = vals
    for ty, name, v in _SCAL.findall(src):
        out[name] = _num(v, ty)
    for name, v in _DEF.findall(src):
        out[name] = int(v)
    return out


def D(x):
    """Decimal of a float, exactly."""
    return Decimal(Fraction(x).numerator) / Decimal(Fraction(x).denominator)


def exp_(x):
    return Decimal(x).exp() if not isinstance(x, Decimal) else x.exp()


def ln2():
    return Decimal(2).ln()


def ulp(x, p, emin):
    """ulp of a binary float with p-bit significand at value x (exact Fraction)."""
    x = abs(Fraction(x))
    if x == 0:
        return Fraction(2) ** (emin - p + 1)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    if Fraction(2) ** (e + 1) <= x:
        e += 1
    return Fraction(2) ** (max(e, emin) - p + 1)


def is_rn(f, v, p, emin):
    """True if the float f is the p-bit round-to-nearest of the real v
    (v a Decimal or Fraction), up to an exact tie."""
    fv = Fraction(v) if not isinstance(v, Fraction) else v
    return abs(Fraction(f) - fv) <= ulp(fv if fv != 0 else f, p, emin) / 2


def is_twofold_rn(hi, lo, v, p, emin):
    """hi = RN(v) and lo = RN(v - hi)."""
    fv = Fraction(v)
    return is_rn(hi, fv, p, emin) and is_rn(lo, fv - Fraction(hi), p, emin)
