"""The C ABI library (no GPU needed): it loads, exports every function that
include/twofold_hip.h declares, and validates arguments before any HIP call
(n == 0 -> TF_OK, NULL array with n > 0 -> TF_EINVAL).  Also: the GPU
library's tables equal the oracle's, value for value -- two generators written
independently (decimal vs mpmath) from the same definitions."""
import ctypes
import math
import os
import re
from fractions import Fraction

import pytest

from tables_util import is_twofold_rn, parse_header

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1502_05216_amd", "libtwofold_hip.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1502_05216_amd import _build
        _build.build()
    from paper_1502_05216_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(lib):
    from paper_1502_05216_amd import declared_functions
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings_and_version(lib):
    for s in range(6):
        assert lib.tf_status_string(s)
    assert b"gfx950" in lib.tf_version()
    assert lib.tf_abi_version() == 1


@pytest.mark.parametrize("name", ["tf_texp", "tf_texpm1", "tf_tlog", "tf_tlog1p",
                                  "tf_texpf", "tf_texpm1f", "tf_tlogf", "tf_tlog1pf"])
def test_twofold_argument_validation(lib, name):
    fn = getattr(lib, name)
    # n == 0: nothing to do, no HIP call
    assert fn(None, None, None, None, 0, None) == 0
    # a NULL array with n > 0 is rejected before any HIP call
    fake = ctypes.c_void_p(0x1000)
    for k in range(4):
        args = [fake] * 4
        args[k] = None
        assert fn(*args, 10, None) == 1


@pytest.mark.parametrize("name", ["tf_exp1x", "tf_expm1_1x", "tf_log1x", "tf_log1p_1x",
                                  "tf_exp1xf", "tf_expm1_1xf", "tf_log1xf", "tf_log1p_1xf"])
def test_onex_argument_validation(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, 0, None) == 0
    assert fn(None, ctypes.c_void_p(0x1000), 5, None) == 1
    assert fn(ctypes.c_void_p(0x1000), None, 5, None) == 1


def _hip_tables():
    src = open(os.path.join(ROOT, "paper_1502_05216_amd", "csrc", "tf_tables.inc")).read()
    out = {}
    for name, body in re.findall(r"__device__ const \w+ (\w+)\[\d+\] = \{(.*?)\};", src, re.S):
        toks = [t for t in re.split(r"[,{}\s]+", body) if t]
        out[name] = [float.fromhex(t.rstrip("f")) if "0x" in t or "." in t else int(t)
                     for t in toks]
    for name, val in re.findall(r"#define (TFH_\w+) (\S+)$", src, re.M):
        if "LIST" in name:
            continue
        out[name] = float.fromhex(val.rstrip("f")) if "0x" in val or "." in val else int(val)
    for name, val in re.findall(r"#define (TFH_\w+_LIST) (.+)$", src, re.M):
        out[name] = [float.fromhex(v.strip().rstrip("f")) for v in val.split(",")]
    return out


@pytest.mark.parametrize("f", ["D", "F"])
def test_gpu_tables_equal_oracle_tables(f):
    H = _hip_tables()
    O = parse_header(os.path.join(ROOT, "oracle", "tfo_tables.h"))
    o = lambda k: O["TFO_%s_%s" % (f, k)]
    h = lambda k: H["TFH_%s_%s" % (f, k)]

    def inter(hi, lo):
        return [v for pair in zip(hi, lo) for v in pair]

    assert h("E") == inter(o("E_HI"), o("E_LO"))
    assert h("EK") == o("E_K")
    assert h("C") == inter(o("C_HI"), o("C_LO"))
    assert h("CM1") == inter(o("CM1_HI"), o("CM1_LO"))
    assert h("S") == inter(o("S_HI"), o("S_LO"))
    assert h("LOG") == inter(o("LOG_HI"), o("LOG_LO"))
    assert h("LOG_INVC") == o("LOG_INVC")
    assert h("EXP_C_LIST") == o("EXP_C") and h("LOG_C_LIST") == o("LOG_C")
    for k in ("LN2_HI", "LN2_LO", "RCP_HI", "RCP_LO", "INV_L", "L1", "L2", "LN2X_HI", "LN2X_LO",
              "EXP_XMAX", "EXPM1_XMAX", "EXP_XLO", "EXPM1_XNEG", "EXPM1_TINY", "LOG1P_TINY"):
        assert h(k) == o(k), k
    for k in ("L", "K", "N", "N1", "E_OFF", "E_CNT", "C_OFF", "C_CNT", "CM1_OFF", "CM1_CNT"):
        assert h(k) == o(k), k


@pytest.mark.parametrize("f", ["D", "F"])
def test_k6_variant_table_against_mpmath(f):
    """The C table of build variant k6 (pexp0 with K = 6): entry n is the
    round-to-nearest twofold of e^(n/64)/N6!, N6 = 11 (binary32 5), for
    |n| <= 256 (128), recomputed with mpmath at 240 bits; its sizes cover the
    decomposition's n < 2^(L+K)."""
    import mpmath
    H = _hip_tables()
    h = lambda k: H["TFH_%s_%s" % (f, k)]
    p, emin = (53, -1022) if f == "D" else (24, -126)
    assert h("K6_K") == 6 and h("K6_N") == (11 if f == "D" else 5)
    assert h("K6_C_OFF") == 2 ** (h("L") + 6) and h("K6_C_CNT") == 2 * h("K6_C_OFF") + 1
    c6 = h("C6")
    assert len(c6) == 2 * h("K6_C_CNT")
    with mpmath.workprec(240):
        fact = mpmath.factorial(h("K6_N"))
        for k, n in enumerate(range(-h("K6_C_OFF"), h("K6_C_OFF") + 1)):
            man, ex = (mpmath.exp(mpmath.mpf(n) / 64) / fact).man_exp
            v = Fraction(man) * Fraction(2) ** ex
            assert is_twofold_rn(c6[2 * k], c6[2 * k + 1], v, p, emin), n
    # the Taylor remainder of the shortened sum at |y| = 2^-7 stays far below
    # the twofold precision of the format: 2^-112.8 <= 2^-108 (binary32
    # 2^-51.5 <= 2^-50)
    n6 = h("K6_N")
    rem6 = Fraction(1, 2 ** (7 * (n6 + 1))) / math.factorial(n6 + 1)
    assert rem6 <= Fraction(1, 2 ** (2 * p + 2))


def test_batch_plan_validation(lib):
    """Descriptor and configuration checks run before any HIP call."""
    from paper_1502_05216_amd import batch
    L = batch._bind(lib)
    P = ctypes.c_void_p
    out = P()
    fake = 0x1000
    good = batch.BatchDesc(0, 0, 10, fake, fake, fake, fake)
    arr = (batch.BatchDesc * 1)(good)
    cfg = batch.BatchConfig(2, 4, 8, 0)
    for d in (batch.BatchDesc(4, 0, 10, fake, fake, fake, fake),      # func out of range
              batch.BatchDesc(0, 2, 10, fake, fake, fake, fake),      # dtype out of range
              batch.BatchDesc(1, 1, 10, fake, None, fake, fake)):     # NULL array, n > 0
        bad = (batch.BatchDesc * 1)(d)
        assert L.tf_batch_plan_create(bad, 1, ctypes.byref(cfg), ctypes.byref(out)) == 1
    for c in ((3, 4, 8, 0), (2, 4, 0, 0), (2, 4, 8, -1), (2, 2, 8, 0)):
        bc = batch.BatchConfig(*c)
        assert L.tf_batch_plan_create(arr, 1, ctypes.byref(bc), ctypes.byref(out)) == 1
    assert L.tf_batch_plan_create(None, 1, ctypes.byref(cfg), ctypes.byref(out)) == 1
    assert L.tf_batch_plan_create(arr, 1, ctypes.byref(cfg), None) == 1
    assert L.tf_batch_launch(None, None) == 1
    assert L.tf_batch_plan_destroy(None) == 1
    assert L.tf_batch_plan_info(None, None, None) == 1


@pytest.mark.parametrize("name", ["tf_" + n + s for n in ("pexp0", "texp0", "pexpm10", "texpm10",
                                                         "plog0", "tlog0", "plog1p0", "tlog1p0")
                                  for s in ("", "f")])
def test_dotted_argument_validation(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, None, 0, None) == 0
    fake = ctypes.c_void_p(0x1000)
    for k in range(3):
        args = [fake] * 3
        args[k] = None
        assert fn(*args, 10, None) == 1


@pytest.mark.parametrize("name", ["tf_" + n + s for n in ("texpp", "pexp", "texpm1p", "pexpm1",
                                                         "tlogp", "plog", "tlog1pp", "plog1p")
                                  for s in ("", "f")])
def test_coupled_argument_validation(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, None, None, 0, None) == 0
    fake = ctypes.c_void_p(0x1000)
    for k in range(4):
        args = [fake] * 4
        args[k] = None
        assert fn(*args, 10, None) == 1


@pytest.mark.parametrize("name", ["tf_" + n + s for n in ("tadd", "tsub", "tmul", "tdiv")
                                  for s in ("", "f")])
def test_arith_argument_validation(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, None, None, None, None, 0, None) == 0
    fake = ctypes.c_void_p(0x1000)
    for k in range(6):
        args = [fake] * 6
        args[k] = None
        assert fn(*args, 10, None) == 1


@pytest.mark.parametrize("name", ["tf_tsqrt", "tf_tsqrtf", "tf_trenorm", "tf_trenormf"])
def test_unary_arith_argument_validation(lib, name):
    fn = getattr(lib, name)
    assert fn(None, None, None, None, 0, None) == 0
    fake = ctypes.c_void_p(0x1000)
    for k in range(4):
        args = [fake] * 4
        args[k] = None
        assert fn(*args, 10, None) == 1


@pytest.mark.parametrize("name", ["tf_chain_bwd", "tf_chain_bwdf"])
def test_chain_bwd_argument_validation(lib, name):
    fn = getattr(lib, name)
    fake = ctypes.c_void_p(0x1000)

    def call(k, fns, n, s0=None, s1=None, g=(fake, fake, fake, fake)):
        m = max(len(fns), 1)
        f = (ctypes.c_int * m)(*fns)
        p0 = (ctypes.c_void_p * m)(*([fake] * m if s0 is None else s0))
        p1 = (ctypes.c_void_p * m)(*([fake] * m if s1 is None else s1))
        return fn(k, f, p0, p1, *g, n, None)

    # stage count outside [1, TF_CHAIN_MAX] and unknown function ids
    assert call(0, [0], 10) == 1
    assert call(9, [0] * 9, 10) == 1
    assert call(-1, [0], 10) == 1
    assert call(2, [0, 4], 10) == 1
    assert call(2, [-1, 1], 10) == 1
    # NULL host arrays
    assert fn(1, None, None, None, fake, fake, fake, fake, 10, None) == 1
    # n == 0 with a valid chain: nothing to do, no HIP call
    assert call(3, [0, 1, 3], 0, g=(None, None, None, None)) == 0
    assert call(8, [0, 1, 2, 3] * 2, 0, s0=[None] * 8, s1=[None] * 8,
                g=(None, None, None, None)) == 0
    # a NULL device array with n > 0, saved or gradient, before any HIP call
    assert call(2, [0, 2], 10, s0=[fake, None]) == 1
    assert call(2, [0, 2], 10, s1=[None, fake]) == 1
    for k in range(4):
        g = [fake] * 4
        g[k] = None
        assert call(2, [1, 3], 10, g=tuple(g)) == 1


def test_table_placement_setting(lib):
    """tf_set_table_placement takes TF_TABLES_AUTO / _LDS / _GLOBAL (0, 1, 2)
    and rejects anything else with TF_EINVAL, keeping the setting."""
    from paper_1502_05216_amd import _lib
    assert lib.tf_get_table_placement() == 0
    try:
        for mode, name in ((1, "lds"), (2, "global"), (0, "auto")):
            assert lib.tf_set_table_placement(mode) == 0
            assert lib.tf_get_table_placement() == mode
            assert _lib.get_table_placement() == name
        assert lib.tf_set_table_placement(2) == 0
        for bad in (-1, 3, 7):
            assert lib.tf_set_table_placement(bad) == 1
            assert lib.tf_get_table_placement() == 2
    finally:
        lib.tf_set_table_placement(0)
