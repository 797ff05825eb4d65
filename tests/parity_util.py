"""GPU-vs-oracle comparison helpers.

Bar: z0 identical bit for bit (NaNs compared by class, payloads differ
between machines); z1 within 4 ulp of the oracle's z1, where the ulp is
max(ulp(z1_oracle), u * ulp(z0_oracle)) with the unit roundoff u = 2^-53
(binary32 2^-24), so that z1 ~ 0 is handled; NaN and
infinity classes equal; signed zeros equal.  The GPU runs the same sequence of
IEEE operations as the oracle, so z1 is expected to be identical too and the
number of non-identical z1 is reported.
"""
import numpy as np


def uint_of(dt):
    return np.uint64 if np.dtype(dt) == np.float64 else np.uint32


def same_bits(a, b):
    ui = uint_of(a.dtype)
    return (a.view(ui) == b.view(ui)) | (np.isnan(a) & np.isnan(b))


def unit_roundoff(dt):
    """2^-53 for binary64, 2^-24 for binary32 (half the machine epsilon)."""
    return np.finfo(dt).eps / 2


def z1_ok(g0, g1, o0, o1):
    dt = o1.dtype
    u = unit_roundoff(dt)
    ok = same_bits(g1, o1)
    fin = np.isfinite(o1) & np.isfinite(g1) & np.isfinite(o0)
    with np.errstate(over="ignore", invalid="ignore"):
        tol = 4 * np.maximum(np.spacing(np.abs(o1)), u * np.spacing(np.abs(o0)))
        close = np.abs(g1.astype(np.float64) - o1.astype(np.float64)) <= tol
    ok |= fin & close & ~((o1 == 0) & (g1 == 0) & (np.signbit(o1) != np.signbit(g1)))
    return ok


def compare(g0, g1, o0, o1, what=""):
    """Assert the parity bar; return the number of z1 that are not bit-identical."""
    s0 = same_bits(g0, o0)
    if not s0.all():
        i = np.flatnonzero(~s0)[:5]
        raise AssertionError("%s: z0 differs at %d of %d elements, e.g. idx %s gpu %s oracle %s"
                             % (what, (~s0).sum(), s0.size, i, g0[i], o0[i]))
    ok1 = z1_ok(g0, g1, o0, o1)
    if not ok1.all():
        i = np.flatnonzero(~ok1)[:5]
        raise AssertionError("%s: z1 outside tolerance at %d of %d elements, e.g. idx %s "
                             "gpu %s oracle %s (z0 %s)" % (what, (~ok1).sum(), ok1.size, i, g1[i],
                                                          o1[i], o0[i]))
    return int((~same_bits(g1, o1)).sum())
