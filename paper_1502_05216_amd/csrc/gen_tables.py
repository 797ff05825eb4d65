"""Generates tf_tables.inc: the constants and range-reduction tables of the
HIP twofold library.

Every value is the round-to-nearest-even binary64/binary32 number of its
mathematical definition, computed with Python's decimal module at 90 digits
and rounded with exact integer arithmetic (fractions):

* pexp0 (section "Function pexp0()"): E = e^(2^L m) as Ehat 2^k, Ehat in [1,2)
  stored as a twofold (hi, lo), k integer; C = e^(n/32)/N! twofold;
  (L, N) = (2, 12) double, (1, 6) float; -744 <= 4m <= 708, -128 <= n <= 128
  (float -102 <= 2m <= 88, -64 <= n <= 64).
* the pexp0 table of the finer decomposition (build variant k6, the
  rebalancing of the section's closing remarks): K = 6, C6 = e^(n/64)/N6!
  with N6 = 11 (float 5), -256 <= n <= 256 (float -128 <= n <= 128); E is
  shared, since 2^L m is the same split.
* pexpm10 (section "Function pexpm10()"): e^(n/128) - 1, -89 <= n <= 89, and
  the twofold 1/N! (N = 10 double, 5 float).
* twofold ln 2 (n ln2 in plog).
* the 1x exp/expm1/log/log1p used for the main part z0:
  2^(j/32) twofolds (j < 32), RN(32/ln2), ln2/32 as L1 + L2, Taylor
  coefficients RN(1/k!) (k = 2..7 double, 2..4 float) and RN((-1)^(k+1)/k)
  (k = 2..9 double, 2..5 float); log cells i < 128 (top 7 significand bits)
  with invc = 1/c rounded to 8 significant bits (1 for i = 0, 127),
  -log(invc) split as hi (multiple of 2^-42, float 2^-16) + lo, and ln 2 split
  the same way; thresholds of exp/expm1 overflow and underflow.

Run:  python paper_1502_05216_amd/csrc/gen_tables.py
"""
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 90

FMTS = {"D": (53, -1022, 1023), "F": (24, -126, 127)}


def rn(v, p, emin):
    """Nearest p-bit binary float (ties to even) of the rational v, as Fraction."""
    v = Fraction(v)
    if v == 0:
        return Fraction(0)
    neg = v < 0
    a = -v if neg else v
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    q = max(e, emin) - (p - 1)
    s = a / Fraction(2) ** q
    n, rem = divmod(s.numerator, s.denominator)
    twice = 2 * rem
    if twice > s.denominator or (twice == s.denominator and n & 1):
        n += 1
    r = Fraction(n) * Fraction(2) ** q
    return -r if neg else r


def grid(v, g):
    """Nearest multiple of 2^-g (ties to even)."""
    s = Fraction(v) * 2 ** g
    n, rem = divmod(s.numerator, s.denominator)
    if 2 * rem > s.denominator or (2 * rem == s.denominator and n & 1):
        n += 1
    return Fraction(n, 2 ** g)


def exp_q(v):
    """e^v as a Fraction (90 significant digits)."""
    v = Fraction(v)
    return Fraction((Decimal(v.numerator) / Decimal(v.denominator)).exp())


LN2 = Fraction(Decimal(2).ln())


def ln_q(v):
    v = Fraction(v)
    return Fraction(Decimal(v.numerator).ln() - Decimal(v.denominator).ln())


def pair(v, f):
    p, emin, _ = FMTS[f]
    hi = rn(v, p, emin)
    lo = rn(Fraction(v) - hi, p, emin)
    return hi, lo


def to_float(fr):
    x = float(fr)
    assert Fraction(x) == fr
    return x


def nxt(x, f, up):
    if f == "D":
        return math.nextafter(x, math.inf if up else -math.inf)
    import struct
    b = struct.unpack("<I", struct.pack("<f", x))[0]
    if x == 0:
        b = 1 if up else 0x80000001
    elif (x > 0) == up:
        b += 1
    else:
        b -= 1
    return struct.unpack("<f", struct.pack("<I", b))[0]


def build(f):
    p, emin, emax = FMTS[f]
    t = {}
    L, K, N, N1 = (2, 5, 12, 10) if f == "D" else (1, 5, 6, 5)
    mlo, mhi = (-186, 177) if f == "D" else (-51, 44)
    nmax = 128 if f == "D" else 64
    t["int"] = dict(L=L, K=K, N=N, N1=N1, E_OFF=-mlo, E_CNT=mhi - mlo + 1, C_OFF=nmax,
                    C_CNT=2 * nmax + 1, CM1_OFF=89, CM1_CNT=179)
    E, EK = [], []
    for m in range(mlo, mhi + 1):
        v = exp_q(Fraction(2 ** L * m))
        k = v.numerator.bit_length() - v.denominator.bit_length()
        if Fraction(2) ** k > v:
            k -= 1
        elif Fraction(2) ** (k + 1) <= v:
            k += 1
        E.append(pair(v / Fraction(2) ** k, f))
        EK.append(k)
    t["E"], t["EK"] = E, EK
    t["C"] = [pair(exp_q(Fraction(n, 32)) / math.factorial(N), f) for n in range(-nmax, nmax + 1)]
    # finer decomposition: K = 6 halves |y| to 2^-7, one Taylor term fewer
    N6 = 11 if f == "D" else 5
    nmax6 = 2 * nmax
    t["int6"] = dict(K=6, N=N6, C_OFF=nmax6, C_CNT=2 * nmax6 + 1)
    t["C6"] = [pair(exp_q(Fraction(n, 64)) / math.factorial(N6), f)
               for n in range(-nmax6, nmax6 + 1)]
    t["CM1"] = [pair(exp_q(Fraction(n, 128)) - 1, f) for n in range(-89, 90)]
    t["S"] = [pair(exp_q(Fraction(j, 32) * LN2), f) for j in range(32)]
    scal = {}
    scal["LN2_HI"], scal["LN2_LO"] = pair(LN2, f)
    scal["RCP_HI"], scal["RCP_LO"] = pair(Fraction(1, math.factorial(N1)), f)
    scal["INV_L"] = rn(32 / LN2, p, emin)
    scal["L1"], scal["L2"] = pair(LN2 / 32, f)
    g = 42 if f == "D" else 16
    scal["LN2X_HI"] = grid(LN2, g)
    scal["LN2X_LO"] = rn(LN2 - scal["LN2X_HI"], p, emin)
    t["EXP_C"] = [rn(Fraction(1, math.factorial(k)), p, emin) for k in range(2, (7 if f == "D" else 4) + 1)]
    t["LOG_C"] = [rn(Fraction((-1) ** (k + 1), k), p, emin) for k in range(2, (9 if f == "D" else 5) + 1)]
    inv, lg = [], []
    for i in range(128):
        if i in (0, 127):
            ic = Fraction(1)
        else:
            c = 1 + Fraction(2 * i + 1, 256)
            if i >= 64:
                c /= 2
            ic = rn(1 / c, 8, -1000)
        lc = -ln_q(ic)
        hi = grid(lc, g)
        inv.append(ic)
        lg.append((hi, rn(lc - hi, p, emin)))
    t["LOG_INVC"], t["LOG"] = inv, lg
    # thresholds
    big = Fraction(2) ** (emax + 1) * (1 - Fraction(1, 2 ** (p + 1)))
    half_tiny = Fraction(2) ** (emin - p)
    x = to_float(rn(ln_q(big), p, emin))
    while exp_q(Fraction(x)) >= big:
        x = nxt(x, f, False)
    while exp_q(Fraction(nxt(x, f, True))) < big:
        x = nxt(x, f, True)
    scal["EXP_XMAX"] = Fraction(x)
    y = x
    while exp_q(Fraction(y)) - 1 >= big:
        y = nxt(y, f, False)
    while exp_q(Fraction(nxt(y, f, True))) - 1 < big:
        y = nxt(y, f, True)
    scal["EXPM1_XMAX"] = Fraction(y)
    x = to_float(rn(ln_q(half_tiny), p, emin))
    while not exp_q(Fraction(x)) > half_tiny:
        x = nxt(x, f, True)
    while exp_q(Fraction(nxt(x, f, False))) > half_tiny:
        x = nxt(x, f, False)
    scal["EXP_XLO"] = Fraction(x)
    scal["EXPM1_XNEG"] = Fraction(-40 if f == "D" else -20)
    scal["EXPM1_TINY"] = Fraction(1, 2 ** (30 if f == "D" else 14))
    scal["LOG1P_TINY"] = Fraction(1, 2 ** (60 if f == "D" else 30))
    t["scal"] = scal
    return t


def lit(fr, f):
    x = to_float(Fraction(fr))
    if x == 0:
        return "0.0" + ("f" if f == "F" else "")
    return x.hex() + ("f" if f == "F" else "")


def emit(tabs):
    o = ["// Generated by paper_1502_05216_amd/csrc/gen_tables.py (decimal, 90 digits,",
         "// round-to-nearest-even).  Do not edit by hand.",
         "#pragma once", ""]
    for f, t in tabs.items():
        ty = "double" if f == "D" else "float"
        two = "double2" if f == "D" else "float2"
        P = "TFH_" + f + "_"
        for k, v in t["int"].items():
            o.append("#define %s%s %d" % (P, k, v))
        for k, v in t["int6"].items():
            o.append("#define %sK6_%s %d" % (P, k, v))
        for k, v in t["scal"].items():
            o.append("#define %s%s %s" % (P, k, lit(v, f)))
        o.append("#define %sEXP_NC %d" % (P, len(t["EXP_C"])))
        o.append("#define %sLOG_NC %d" % (P, len(t["LOG_C"])))
        o.append("#define %sEXP_C_LIST %s" % (P, ", ".join(lit(c, f) for c in t["EXP_C"])))
        o.append("#define %sLOG_C_LIST %s" % (P, ", ".join(lit(c, f) for c in t["LOG_C"])))
        for name in ("E", "C", "C6", "CM1", "S", "LOG"):
            arr = t[name]
            o.append("__device__ const %s %s%s[%d] = {" % (two, P, name, len(arr)))
            for i in range(0, len(arr), 2):
                o.append("    " + " ".join("{%s, %s}," % (lit(h, f), lit(l, f)) for h, l in arr[i:i + 2]))
            o.append("};")
        o.append("__device__ const int %sEK[%d] = {" % (P, len(t["EK"])))
        for i in range(0, len(t["EK"]), 12):
            o.append("    " + ", ".join(str(k) for k in t["EK"][i:i + 12]) + ",")
        o.append("};")
        o.append("__device__ const %s %sLOG_INVC[128] = {" % (ty, P))
        for i in range(0, 128, 4):
            o.append("    " + ", ".join(lit(v, f) for v in t["LOG_INVC"][i:i + 4]) + ",")
        o.append("};")
        o.append("")
    return "\n".join(o) + "\n"


def main():
    tabs = {"D": build("D"), "F": build("F")}
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tf_tables.inc")
    with open(out, "w") as fh:
        fh.write(emit(tabs))
    print("wrote", out)


if __name__ == "__main__":
    main()
