"""Pins for the oracle's constant tables (oracle/tfo_tables.h).

Each entry is checked against its mathematical definition evaluated with
Python's decimal module (80 digits), independently of the mpmath generator:
hi = RN(v), lo = RN(v - hi).  Table sizes are the paper's (sections
"Function pexp0()" and "Function pexpm10()"): 364 / 257 / 179 entries for
double, 96 / 129 / 179 for float, i.e. about 10 KB + 2.8 KB (double) and
about 2 KB + 1.4 KB (float) of twofolds.
"""
import math
import os
from decimal import Decimal
from fractions import Fraction

import pytest

from tables_util import D, is_rn, is_twofold_rn, ln2, parse_header

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
T = parse_header(os.path.join(ROOT, "oracle", "tfo_tables.h"))
FMT = {"D": (53, -1022), "F": (24, -126)}


def tab(f, name):
    return T["TFO_%s_%s" % (f, name)]


@pytest.mark.parametrize("f,ne,nc,nm,bytes_ec,bytes_m", [
    ("D", 364, 257, 179, 9936, 2864),
    ("F", 96, 129, 179, 1800, 1432),
])
def test_table_sizes(f, ne, nc, nm, bytes_ec, bytes_m):
    w = 16 if f == "D" else 8
    assert len(tab(f, "E_HI")) == ne == len(tab(f, "E_LO")) == len(tab(f, "E_K"))
    assert len(tab(f, "C_HI")) == nc and len(tab(f, "CM1_HI")) == nm
    assert (ne + nc) * w == bytes_ec          # about 10 KB (double) / 2 KB (float), as stated
    assert nm * w == bytes_m                  # about 2.8 KB / 1.4 KB, as stated
    # index ranges: -744 <= 4m <= 708 (double), -102 <= 2m <= 88 (float)
    L = tab(f, "L")
    off = tab(f, "E_OFF")
    assert -off * 2 ** L == (-744 if f == "D" else -102)
    assert (ne - 1 - off) * 2 ** L == (708 if f == "D" else 88)


@pytest.mark.parametrize("f", ["D", "F"])
def test_E_table(f):
    p, emin = FMT[f]
    L = tab(f, "L")
    off = tab(f, "E_OFF")
    for idx, (h, l, k) in enumerate(zip(tab(f, "E_HI"), tab(f, "E_LO"), tab(f, "E_K"))):
        m = idx - off
        v = Fraction(Decimal(2 ** L * m).exp()) / Fraction(2) ** k
        assert 1 <= h < 2
        assert is_twofold_rn(h, l, v, p, emin), (f, m)


@pytest.mark.parametrize("f", ["D", "F"])
def test_C_tables(f):
    p, emin = FMT[f]
    N, K = tab(f, "N"), tab(f, "K")
    off = tab(f, "C_OFF")
    for idx, (h, l) in enumerate(zip(tab(f, "C_HI"), tab(f, "C_LO"))):
        n = idx - off
        v = Fraction((Decimal(n) / 2 ** K).exp()) / math.factorial(N)
        assert is_twofold_rn(h, l, v, p, emin), (f, n)
    for idx, (h, l) in enumerate(zip(tab(f, "CM1_HI"), tab(f, "CM1_LO"))):
        n = idx - 89
        v = Fraction((Decimal(n) / 128).exp() - 1)
        assert is_twofold_rn(h, l, v, p, emin), (f, n)
    # the corner entries n = +-89 lie just beyond ln 2
    assert 89 / 128 > math.log(2) > 88 / 128


@pytest.mark.parametrize("f", ["D", "F"])
def test_scalar_twofolds(f):
    p, emin = FMT[f]
    assert is_twofold_rn(tab(f, "LN2_HI"), tab(f, "LN2_LO"), Fraction(ln2()), p, emin)
    n1 = tab(f, "N1")
    assert is_twofold_rn(tab(f, "RCP_HI"), tab(f, "RCP_LO"), Fraction(1, math.factorial(n1)),
                         p, emin)
    N = tab(f, "N")
    assert tab(f, "HORNER") == [math.factorial(N) // math.factorial(j) for j in range(N - 1)]
    assert tab(f, "HORNER1") == [math.factorial(n1) // math.factorial(j) for j in range(n1 - 1)]
    assert tab(f, "N") == (12 if f == "D" else 6) and n1 == (10 if f == "D" else 5)
    assert tab(f, "K") == 5 and tab(f, "L") == (2 if f == "D" else 1)


@pytest.mark.parametrize("f", ["D", "F"])
def test_1x_exp_constants(f):
    p, emin = FMT[f]
    L2 = Fraction(ln2())
    for j, (h, l) in enumerate(zip(tab(f, "S_HI"), tab(f, "S_LO"))):
        v = Fraction((Decimal(j) / 32 * ln2()).exp())
        assert is_twofold_rn(h, l, v, p, emin), j
    assert is_rn(tab(f, "INV_L"), 32 / L2, p, emin)
    assert is_twofold_rn(tab(f, "L1"), tab(f, "L2"), L2 / 32, p, emin)
    for k, c in enumerate(tab(f, "EXP_C"), start=2):
        assert is_rn(c, Fraction(1, math.factorial(k)), p, emin)
    for k, c in enumerate(tab(f, "LOG_C"), start=2):
        assert is_rn(c, Fraction((-1) ** (k + 1), k), p, emin)


@pytest.mark.parametrize("f", ["D", "F"])
def test_1x_log_table(f):
    p, emin = FMT[f]
    g = 42 if f == "D" else 16
    hi = Fraction(tab(f, "LN2X_HI"))
    assert (hi * 2 ** g).denominator == 1                       # multiple of 2^-g
    assert abs(hi - Fraction(ln2())) <= Fraction(1, 2 ** (g + 1))
    assert is_rn(tab(f, "LN2X_LO"), Fraction(ln2()) - hi, p, emin)
    emax_bits = 11 if f == "D" else 8
    assert (hi * 2 ** g).numerator.bit_length() + emax_bits <= p      # e*LN2X_HI exact
    for i, (ic, h, l) in enumerate(zip(tab(f, "LOG_INVC"), tab(f, "LOG_HI"), tab(f, "LOG_LO"))):
        ic = Fraction(ic)
        # at most 8 significant bits, so z*invc - 1 is exact in the format
        num, den = ic.numerator, ic.denominator
        while num % 2 == 0:
            num //= 2
        assert num.bit_length() <= 8, i
        lo_z = 1 + Fraction(i, 128)
        hi_z = 1 + Fraction(i + 1, 128)
        if i >= 64:
            lo_z, hi_z = lo_z / 2, hi_z / 2
        assert abs(lo_z * ic - 1) < Fraction(1, 128) and abs(hi_z * ic - 1) <= Fraction(1, 128)
        if i in (0, 127):
            assert ic == 1 and h == 0 and l == 0
        v = -Fraction(Decimal(ic.numerator).ln() - Decimal(ic.denominator).ln())
        assert (Fraction(h) * 2 ** g).denominator == 1
        assert abs(Fraction(h) - v) <= Fraction(1, 2 ** (g + 1))
        assert is_rn(l, v - Fraction(h), p, emin), i


def _exp_dec(x):
    return Fraction(D(x).exp())


@pytest.mark.parametrize("f", ["D", "F"])
def test_thresholds(f):
    import numpy as np
    dt = np.float64 if f == "D" else np.float32
    p, emin = FMT[f]
    emax = 1023 if f == "D" else 127
    big = Fraction(2) ** (emax + 1) * (1 - Fraction(1, 2 ** (p + 1)))
    half_tiny = Fraction(2) ** (emin - p)
    xmax = tab(f, "EXP_XMAX")
    nxt = float(np.nextafter(dt(xmax), dt(np.inf)))
    assert _exp_dec(xmax) < big <= _exp_dec(nxt)
    assert tab(f, "EXPM1_XMAX") == xmax
    xlo = tab(f, "EXP_XLO")
    prv = float(np.nextafter(dt(xlo), dt(-np.inf)))
    assert _exp_dec(prv) <= half_tiny < _exp_dec(xlo)
    # 2^-p/2 below -1: expm1 rounds to -1 beyond EXPM1_XNEG
    assert _exp_dec(tab(f, "EXPM1_XNEG")) < Fraction(1, 2 ** (p + 2))
    assert tab(f, "LN2_RN") == tab(f, "LN2_HI")
