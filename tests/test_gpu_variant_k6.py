"""GPU: build variant k6 (pexp0 with the finer decomposition K = 6: |y| <=
2^-7, one Taylor term fewer, a C table of twice the entries), the rebalancing
of table size against Horner length that the section "Function pexp0()"
closes with.

Its second parts differ from the oracle's (whose parameters are the paper's),
so it is validated against mathematics, as a flagged variant must be:

* the accuracy acceptance protocol (tests/accept_util.py: a million arguments
  plus the edge grid, L1 / L0 / at most 2 exceedances per million, against the
  binary128 etalon) for texp and texpm1 (whose |x0| > ln 2 lanes run pexp0),
  both formats, and for the coupled pexp;
* pexp0 renormalised: coupled, and within 2^-103.5 (binary32 2^-45) of mpmath,
  next to the default library's pexp0 on the same arguments (within 2^-104);
* main parts bit for bit those of the default library (z0 is the 1x function
  of x0 and does not depend on pexp0), and the logs, which do not use pexp0,
  bit for bit in both parts.
"""
import math

import numpy as np
import pytest

from oracle import mpref
from paper_1502_05216_amd import workloads

from accept_util import N_ACCEPT, assert_accepted, describe, edge_grid, measure
from parity_util import same_bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DTS = (np.float64, np.float32)


@pytest.fixture(scope="module")
def vlib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_05216_amd import _lib
    lib = _lib.variant("k6")
    assert b"pexp0 K=6" in lib.tf_version()
    return lib


def run(fn, x0, x1=None, lib=None):
    from paper_1502_05216_amd import _lib
    d = torch.device("cuda:0")
    X0 = torch.from_numpy(np.ascontiguousarray(x0)).to(d)
    if x1 is None:
        g0, g1 = _lib.dotted_call(fn, X0, lib=lib)
    else:
        g0, g1 = _lib.twofold_call(fn, X0, torch.from_numpy(np.ascontiguousarray(x1)).to(d),
                                   lib=lib)
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy()


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", ["texp", "texpm1", "pexp"])
def test_k6_acceptance_million(vlib, fn, dt):
    base = "texp" if fn == "pexp" else fn
    print("case k6 acceptance", fn, np.dtype(dt).name, flush=True)
    x0, x1 = workloads.twofold_inputs(fn, N_ACCEPT, dt, seed=111 + len(fn), edges=0.001,
                                      coupled=fn == "pexp")
    g0, g1 = edge_grid(base, dt)
    x0 = np.concatenate([x0, g0])
    x1 = np.concatenate([x1, g1])
    z0, z1 = run(fn, x0, x1, lib=vlib)
    s = measure(base, x0, x1, z0, z1)
    print(describe(s))
    assert s["measured"] > 0.8 * N_ACCEPT
    assert_accepted(s)


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_k6_pexp0_coupled_and_accurate(vlib, dt):
    rng = np.random.default_rng(131)
    bound = -103.5 if dt == np.float64 else -45
    x = (rng.uniform(-670, 709, 2000) if dt == np.float64 else rng.uniform(-70, 88, 2000))
    x = x.astype(dt)
    worst = {}
    for name, lib in (("k6", vlib), ("default", None)):
        v0, v1 = run("pexp0", x, lib=lib)
        np.testing.assert_array_equal((v0 + v1).astype(dt), v0)
        worst[name] = max(mpref.rel_error(a, b, mpref.exact("exp", xi))
                          for xi, a, b in zip(x, v0, v1))
        print("%s pexp0 %s: worst 2^%.2f" % (name, np.dtype(dt).name, math.log2(worst[name])))
    assert worst["k6"] <= 2.0 ** bound
    assert worst["default"] <= 2.0 ** (-104 if dt == np.float64 else -45)


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", ["texp", "texpm1", "tlog", "tlog1p"])
def test_k6_main_parts_and_logs_unchanged(vlib, fn, dt):
    print("case k6 against the default library", fn, np.dtype(dt).name, flush=True)
    x0, x1 = workloads.twofold_inputs(fn, 100003, dt, seed=141, edges=0.01)
    a0, a1 = run(fn, x0, x1, lib=vlib)
    b0, b1 = run(fn, x0, x1)
    assert same_bits(a0, b0).all()
    if fn in ("tlog", "tlog1p"):
        assert same_bits(a1, b1).all()
    else:
        # the two results agree to well within the accuracy bars: 2^-100 of
        # the value (binary32 2^-44), plus the rounding of the second part
        # itself (texp's z1 holds z0 expm1(x1), up to 2^-43.5 of z0, so its own
        # ulps weigh more than the twofold rounding of pexp0)
        fin = np.isfinite(b1) & np.isfinite(b0)
        rel = 2.0 ** (-100 if dt == np.float64 else -44)
        tol = (rel * np.abs(b0[fin].astype(np.float64))
               + 4.0 * np.spacing(np.maximum(np.abs(a1[fin]), np.abs(b1[fin]))).astype(np.float64)
               + 4.0 * np.finfo(dt).smallest_subnormal)
        bad = np.abs(a1[fin].astype(np.float64) - b1[fin]) > tol
        if bad.any():
            i = np.flatnonzero(fin)[np.flatnonzero(bad)[:6]]
            raise AssertionError("%s %s: %d second parts differ beyond the tolerance, e.g. x0 %r "
                                 "x1 %r z0 %r k6 %r default %r" % (fn, np.dtype(dt).name,
                                                                   bad.sum(), x0[i], x1[i],
                                                                   b0[i], a1[i], b1[i]))
        assert same_bits(a1[~fin], b1[~fin]).all()
