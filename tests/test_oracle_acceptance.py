"""The oracle's twofold functions under the paper's accuracy protocol (section
"Analysis > Accuracy") at the paper's scale: a million random arguments per
function and format (the benchmark's argument laws, 0.1% edge values) plus the
whole edge grid, against a binary128 etalon; see tests/accept_util.py for the
bars.  The etalon is pinned first against mpmath at 240 bits.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import mpref, qref
from paper_1502_05216_amd import workloads

from accept_util import N_ACCEPT, assert_accepted, describe, edge_grid, measure

FUNCS = ("texp", "texpm1", "tlog", "tlog1p")


@pytest.mark.parametrize("fn", FUNCS)
def test_quad_etalon_against_mpmath(fn):
    """The binary128 etalon agrees with mpmath at 240 bits to 2^-108 of the
    result, at the ends of each argument range too (so its split into an x0
    part and an x1 correction, and libquadmath's functions, are right)."""
    x0, x1 = workloads.twofold_inputs(fn, 400, np.float64, seed=3 + len(fn), edges=0.0)
    ends = {"texp": [-745.0, -700.5, 709.7, 1e-3, -1e-300], "texpm1": [-4.0, 4.0, 2.0 ** -60, -0.7],
            "tlog": [2.0 ** -1074, 1e300, 0.75, 1.5], "tlog1p": [-0.9999, 4.0, 2.0 ** -60, -0.5]}
    e0 = np.array(ends[fn])
    x0 = np.concatenate([x0, e0])
    x1 = np.concatenate([x1, e0 * 2.0 ** -53 * 0.7])
    x0, x1 = x0[x0 != 1.0], x1[x0 != 1.0]
    parts, ex = qref.evaluate(fn, x0, x1)
    worst = 0.0
    with mpmath.workprec(mpref.PREC):
        for a, b, p, e in zip(x0, x1, parts, ex):
            v = mpref.exact(fn, a, b)
            q = mpmath.fsum(mpmath.mpf(float(t)) for t in p) * mpmath.mpf(2) ** int(e)
            worst = max(worst, float(abs(q - v) / abs(v)))
    assert worst <= 2.0 ** -108, math.log2(worst)
    print("%s: etalon within 2^%.1f of mpmath" % (fn, math.log2(worst) if worst else -math.inf))


@pytest.mark.parametrize("fmt", ["D", "F"])
@pytest.mark.parametrize("fn", FUNCS)
def test_acceptance_million(fn, fmt):
    dt = np.float64 if fmt == "D" else np.float32
    x0, x1 = workloads.twofold_inputs(fn, N_ACCEPT, dt, seed=101 + len(fn), edges=0.001)
    g0, g1 = edge_grid(fn, dt)
    x0 = np.concatenate([x0, g0])
    x1 = np.concatenate([x1, g1])
    z0, z1 = getattr(oracle, fn + ("f" if fmt == "F" else ""))(x0, x1,
                                                              threads=oracle.default_threads())
    s = measure(fn, x0, x1, z0, z1)
    print(describe(s))
    assert s["measured"] > 0.8 * N_ACCEPT
    assert_accepted(s)


IFACE = workloads.DOTTED + workloads.COUPLED


@pytest.mark.parametrize("fmt", ["D", "F"])
@pytest.mark.parametrize("name", IFACE)
def test_acceptance_interface_functions(name, fmt):
    """The other 16 entry points under the same protocol: the dotted-argument
    functions on a million x0 (second part 0), the coupled-argument ones on a
    million coupled twofolds (x1 = x0 u 2^-54), each with its family's bars."""
    dt = np.float64 if fmt == "D" else np.float32
    sfx = "f" if fmt == "F" else ""
    base = workloads.INTERFACE_BASE[name]
    dotted = name in workloads.DOTTED
    x0, x1 = workloads.twofold_inputs(name, N_ACCEPT, dt, seed=201 + IFACE.index(name),
                                      edges=0.001, coupled=not dotted)
    if dotted:
        x1 = np.zeros_like(x0)
        z0, z1 = getattr(oracle, name + sfx)(x0, threads=oracle.default_threads())
    else:
        z0, z1 = getattr(oracle, name + sfx)(x0, x1, threads=oracle.default_threads())
    s = measure(base, x0, x1, z0, z1)
    print(name, describe(s))
    assert s["measured"] > 0.8 * N_ACCEPT
    assert_accepted(s)


def test_acceptance_catches_a_planted_mistake():
    """The protocol is sharp enough to see a one-ulp slip in the second part:
    z1 moved by 2^-50 of z0 on one element in 2^12 gives L1 far above 2^-98."""
    x0, x1 = workloads.twofold_inputs("tlog1p", 200_000, np.float64, seed=5, edges=0.0)
    z0, z1 = oracle.tlog1p(x0, x1, threads=oracle.default_threads())
    ok = measure("tlog1p", x0, x1, z0, z1)
    assert_accepted(ok)
    z1 = z1.copy()
    z1[::4096] += z0[::4096] * 2.0 ** -50
    bad = measure("tlog1p", x0, x1, z0, z1)
    assert bad["exceed"] > 2 and bad["L1"] > 2.0 ** -98
