"""Writes oracle/tfo_tables.h: every constant and table the oracle uses.

TEST INFRASTRUCTURE (part of the oracle).  Values are computed with mpmath at
256 bits and rounded to nearest-even with integer arithmetic, so each stored
number is the correctly rounded value of its mathematical definition:

* pexp0 tables (section "Function pexp0()"): E = e^(2^L m) stored as a
  normalised twofold Ehat in [1,2) plus the exponent k = floor(log2 e^(2^L m)),
  C = e^(n/2^K)/N!, with (L,K,N) = (2,5,12) for double and (1,5,6) for float;
  the index ranges are the paper's: -744 <= 4m <= 708 (364 entries),
  -128 <= n <= 128 (257); float -102 <= 2m <= 88 (96), -64 <= n <= 64 (129).
* pexpm10 table (section "Function pexpm10()"): e^(n/128) - 1 for
  -89 <= n <= 89 (179 entries, both formats), and the twofold 1/N! for N = 10
  (double) and N = 5 (float).
* twofold ln 2 for n*ln2 in plog (section "Logarithm: Algorithm summary").
* the constants of the project's 1x exp/expm1/log/log1p (the "standard
  library" part z0; the paper leaves its algorithm to the C library).

Run:  python oracle/gen_tables.py   (rewrites oracle/tfo_tables.h)
"""
import math
import os
import sys

import mpmath
from mpmath import mpf

mpmath.mp.prec = 256

FMT = {
    # name: (precision p, emax, emin) -- IEEE binary64 / binary32
    "D": (53, 1023, -1022),
    "F": (24, 127, -126),
}


def rn(x, p, emin):
    """Round the mpf x to the nearest p-bit binary float (ties to even),
    honouring the subnormal grid below 2^emin.  Returns an exact mpf."""
    if x == 0:
        return mpf(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = int(mpmath.floor(mpmath.log(a, 2)))
    # guard against log rounding at exact powers of two
    while mpf(2) ** e > a:
        e -= 1
    while mpf(2) ** (e + 1) <= a:
        e += 1
    q = max(e, emin) - (p - 1)              # exponent of one unit in the last place
    scaled = a / mpf(2) ** q                # exact in mpf (power of two)
    man, ex = scaled.man_exp                # scaled = man * 2^ex exactly
    if ex >= 0:
        n = man << ex
        return sign * mpf(n) * mpf(2) ** q
    n, rem = divmod(man, 1 << (-ex))
    half = 1 << (-ex - 1)
    if rem > half or (rem == half and (n & 1)):
        n += 1
    return sign * mpf(n) * mpf(2) ** q


def rn_grid(x, g):
    """Round x to the nearest multiple of 2^-g (ties to even)."""
    s = x * mpf(2) ** g
    fl = int(mpmath.floor(s))
    frac = s - fl
    if frac > 0.5 or (frac == 0.5 and (fl & 1)):
        fl += 1
    return mpf(fl) / mpf(2) ** g


def as_float(v):
    f = float(v)
    assert mpf(f) == v, "value not exactly representable"
    return f


def twofold(v, fmt):
    p, _, emin = FMT[fmt]
    hi = rn(v, p, emin)
    lo = rn(v - hi, p, emin)
    return as_float(hi), as_float(lo)


def lit(x, fmt):
    if x == 0:
        return "0.0f" if fmt == "F" else "0.0"
    if math.isinf(x):
        return ("INFINITY" if x > 0 else "-INFINITY")
    h = float(x).hex()
    return h + ("f" if fmt == "F" else "")


def next_up(x, fmt):
    if fmt == "D":
        return math.nextafter(x, math.inf)
    import numpy as np
    return float(np.nextafter(np.float32(x), np.float32(np.inf)))


def next_down(x, fmt):
    if fmt == "D":
        return math.nextafter(x, -math.inf)
    import numpy as np
    return float(np.nextafter(np.float32(x), np.float32(-np.inf)))


def threshold_max(f, bound, guess, fmt):
    """Largest x of the format with f(x) < bound, f increasing."""
    x = guess
    while f(mpf(x)) >= bound:
        x = next_down(x, fmt)
    while f(mpf(next_up(x, fmt))) < bound:
        x = next_up(x, fmt)
    return x


def threshold_min(f, bound, guess, fmt):
    """Smallest x of the format with f(x) > bound, f increasing."""
    x = guess
    while not f(mpf(x)) > bound:
        x = next_up(x, fmt)
    while f(mpf(next_down(x, fmt))) > bound:
        x = next_down(x, fmt)
    return x


def gen(fmt):
    p, emax, emin = FMT[fmt]
    out = {}
    L, K, N = (2, 5, 12) if fmt == "D" else (1, 5, 6)
    N1 = 10 if fmt == "D" else 5
    mlo, mhi = (-186, 177) if fmt == "D" else (-51, 44)
    nmax = 128 if fmt == "D" else 64
    out["L"], out["K"], out["N"], out["N1"] = L, K, N, N1
    out["E_OFF"], out["E_CNT"] = -mlo, mhi - mlo + 1
    out["C_OFF"], out["C_CNT"] = nmax, 2 * nmax + 1
    out["CM1_OFF"], out["CM1_CNT"] = 89, 179

    ehi, elo, ek = [], [], []
    for m in range(mlo, mhi + 1):
        v = mpmath.exp(mpf(2) ** L * m)
        k = int(mpmath.floor(mpmath.log(v, 2)))
        while mpf(2) ** k > v:
            k -= 1
        while mpf(2) ** (k + 1) <= v:
            k += 1
        h, l = twofold(v / mpf(2) ** k, fmt)
        assert 1 <= h < 2
        ehi.append(h); elo.append(l); ek.append(k)
    out["E_HI"], out["E_LO"], out["E_K"] = ehi, elo, ek

    fN = math.factorial(N)
    chi, clo = [], []
    for n in range(-nmax, nmax + 1):
        h, l = twofold(mpmath.exp(mpf(n) / 2 ** K) / fN, fmt)
        chi.append(h); clo.append(l)
    out["C_HI"], out["C_LO"] = chi, clo

    mhi_, mlo_ = [], []
    for n in range(-89, 90):
        h, l = twofold(mpmath.expm1(mpf(n) / 128), fmt)
        mhi_.append(h); mlo_.append(l)
    out["CM1_HI"], out["CM1_LO"] = mhi_, mlo_

    out["LN2_HI"], out["LN2_LO"] = twofold(mpmath.log(2), fmt)
    out["RCP_HI"], out["RCP_LO"] = twofold(mpf(1) / math.factorial(N1), fmt)
    # Horner coefficients N!/j! (j = 0..N-2) and N1!/j! (j = 1..N1-2): exact integers
    out["HORNER"] = [math.factorial(N) // math.factorial(j) for j in range(0, N - 1)]
    out["HORNER1"] = [math.factorial(N1) // math.factorial(j) for j in range(0, N1 - 1)]
    for c in out["HORNER"] + out["HORNER1"]:
        assert c < 2 ** p

    # ---- 1x exp / expm1 ----
    shi, slo = [], []
    for j in range(32):
        h, l = twofold(mpf(2) ** (mpf(j) / 32), fmt)
        shi.append(h); slo.append(l)
    out["S_HI"], out["S_LO"] = shi, slo
    ln2 = mpmath.log(2)
    out["INV_L"] = as_float(rn(32 / ln2, p, emin))
    l1 = rn(ln2 / 32, p, emin)
    out["L1"] = as_float(l1)
    out["L2"] = as_float(rn(ln2 / 32 - l1, p, emin))
    nexp = 7 if fmt == "D" else 4
    out["EXP_C"] = [as_float(rn(mpf(1) / math.factorial(k), p, emin)) for k in range(2, nexp + 1)]
    # ---- 1x log / log1p ----
    nlog = 9 if fmt == "D" else 5
    out["LOG_C"] = [as_float(rn(mpf((-1) ** (k + 1)) / k, p, emin)) for k in range(2, nlog + 1)]
    g = 42 if fmt == "D" else 16
    l2h = rn_grid(ln2, g)
    out["LN2X_HI"] = as_float(l2h)
    out["LN2X_LO"] = as_float(rn(ln2 - l2h, p, emin))
    invc, lhi, llo = [], [], []
    for i in range(128):
        if i in (0, 127):
            ic = mpf(1)
        else:
            c = 1 + (mpf(i) + mpf(1) / 2) / 128
            if i >= 64:
                c = c / 2
            ic = rn(1 / c, 8, -1000)
        lc = -mpmath.log(ic)
        h = rn_grid(lc, g)
        l = rn(lc - h, p, emin)
        invc.append(as_float(ic)); lhi.append(as_float(h)); llo.append(as_float(l))
        # reduced argument r = z*invc - 1 must stay below 2^-7 on the whole cell
        f0 = 1 + mpf(i) / 128
        f1 = 1 + mpf(i + 1) / 128
        if i >= 64:
            f0, f1 = f0 / 2, f1 / 2
        # (f1 is the open end of the cell, so equality there is allowed)
        assert abs(f0 * ic - 1) < mpf(2) ** -7 and abs(f1 * ic - 1) <= mpf(2) ** -7, (i, ic)
        # |log c| dominates |r| on the cell, so hi + r may use the fast two-sum
        if i not in (0, 127):
            assert abs(h) >= max(abs(f0 * ic - 1), abs(f1 * ic - 1)), (i, h)
    out["LOG_INVC"], out["LOG_HI"], out["LOG_LO"] = invc, lhi, llo

    # ---- thresholds ----
    big = mpf(2) ** (emax + 1) * (1 - mpf(2) ** (-p - 1))   # first value rounding to inf
    tiny_half = mpf(2) ** (emin - p)                            # half the least subnormal
    out["EXP_XMAX"] = threshold_max(mpmath.exp, big, as_float(rn(mpmath.log(big), p, emin)), fmt)
    out["EXPM1_XMAX"] = threshold_max(mpmath.expm1, big, out["EXP_XMAX"], fmt)
    out["EXP_XLO"] = threshold_min(mpmath.exp, tiny_half,
                                   as_float(rn(mpmath.log(tiny_half), p, emin)), fmt)
    out["EXPM1_XNEG"] = -40.0 if fmt == "D" else -20.0
    out["EXPM1_TINY"] = 2.0 ** -30 if fmt == "D" else 2.0 ** -14
    out["LOG1P_TINY"] = 2.0 ** -60 if fmt == "D" else 2.0 ** -30
    out["LN2_RN"] = out["LN2_HI"]
    return out


def emit(tabs):
    lines = [
        "/* Generated by oracle/gen_tables.py (mpmath, 256-bit, round-to-nearest-even).",
        " * Oracle-only data: TEST INFRASTRUCTURE.  Do not edit by hand. */",
        "#ifndef TFO_TABLES_H",
        "#define TFO_TABLES_H",
        "#include <math.h>",
        "",
    ]
    for fmt, t in tabs.items():
        ty = "double" if fmt == "D" else "float"
        pre = "TFO_" + fmt + "_"
        for key in ("L", "K", "N", "N1", "E_OFF", "E_CNT", "C_OFF", "C_CNT", "CM1_OFF", "CM1_CNT"):
            lines.append("#define %s%s %d" % (pre, key, t[key]))
        for key in ("LN2_HI", "LN2_LO", "RCP_HI", "RCP_LO", "INV_L", "L1", "L2", "LN2X_HI",
                    "LN2X_LO", "EXP_XMAX", "EXPM1_XMAX", "EXP_XLO", "EXPM1_XNEG", "EXPM1_TINY",
                    "LOG1P_TINY", "LN2_RN"):
            lines.append("static const %s %s%s = %s;" % (ty, pre, key, lit(t[key], fmt)))
        for key in ("E_HI", "E_LO", "C_HI", "C_LO", "CM1_HI", "CM1_LO", "S_HI", "S_LO", "EXP_C",
                    "LOG_C", "LOG_INVC", "LOG_HI", "LOG_LO"):
            arr = t[key]
            lines.append("static const %s %s%s[%d] = {" % (ty, pre, key, len(arr)))
            for i in range(0, len(arr), 4):
                lines.append("    " + ", ".join(lit(v, fmt) for v in arr[i:i + 4]) + ",")
            lines.append("};")
        for key in ("HORNER", "HORNER1"):
            arr = t[key]
            lines.append("static const %s %s%s[%d] = {%s};" % (
                ty, pre, key, len(arr), ", ".join(lit(float(v), fmt) for v in arr)))
        lines.append("static const int %sE_K[%d] = {" % (pre, len(t["E_K"])))
        for i in range(0, len(t["E_K"]), 12):
            lines.append("    " + ", ".join(str(v) for v in t["E_K"][i:i + 12]) + ",")
        lines.append("};")
        lines.append("")
    lines.append("#endif")
    return "\n".join(lines) + "\n"


def main():
    tabs = {"D": gen("D"), "F": gen("F")}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tfo_tables.h")
    with open(path, "w") as f:
        f.write(emit(tabs))
    print("wrote", path)


if __name__ == "__main__":
    sys.exit(main())
