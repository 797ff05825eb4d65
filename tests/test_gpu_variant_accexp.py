"""GPU: build variant accexp (TF_TEXP_ACC=1), the accuracy-improved texp:
the second part e^x0 (1 + t1) - z0 in twofold, as v0 t1 (an exact FMA product,
v = pexp0(x0)) + v1 t1 + (v1 + (v0 - z0)) with t1 = x1 + x1^2/2 for a coupled
x1, where the method's step takes one rounded product z0 t1; the low part of
the sum is kept apart: texp adds it in one rounding, the coupled pexp carries
it through its renormalisation.

Its second parts differ from the oracle's (which follows the method's step), so
it is validated against mathematics, as a flagged variant must be:

* the accuracy acceptance protocol (tests/accept_util.py: a million arguments
  plus the edge grid, L1 / L0 / at most 2 exceedances per million, against the
  binary128 etalon) for texp and the coupled pexp, both formats;
* pexp's worst error on coupled arguments over the exp range against the
  etalon: the variant's is far below the default library's, which the
  method's step caps near 2^-96 (binary32 2^-42);
* main parts bit for bit those of the default library, and the functions that
  do not take texp's second part (texpm1, the logs) bit for bit in both parts.
"""
import math

import numpy as np
import pytest

from oracle import qref
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
    lib = _lib.variant("accexp")
    assert b"texp exact z0 t1" in lib.tf_version()
    return lib


def run(fn, x0, x1, lib=None):
    from paper_1502_05216_amd import _lib
    d = torch.device("cuda:0")
    g0, g1 = _lib.twofold_call(fn, torch.from_numpy(np.ascontiguousarray(x0)).to(d),
                               torch.from_numpy(np.ascontiguousarray(x1)).to(d), lib=lib)
    torch.cuda.synchronize()
    return g0.cpu().numpy(), g1.cpu().numpy()


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", ["texp", "pexp"])
def test_accexp_acceptance_million(vlib, fn, dt):
    print("case accexp acceptance", fn, np.dtype(dt).name, flush=True)
    x0, x1 = workloads.twofold_inputs(fn, N_ACCEPT, dt, seed=151 + len(fn), edges=0.001,
                                      coupled=fn == "pexp")
    g0, g1 = edge_grid("texp", dt)
    x0 = np.concatenate([x0, g0])
    x1 = np.concatenate([x1, g1])
    z0, z1 = run(fn, x0, x1, lib=vlib)
    s = measure("texp", x0, x1, z0, z1)
    print(describe(s))
    assert s["measured"] > 0.8 * N_ACCEPT
    assert_accepted(s)


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
def test_accexp_pexp_more_accurate(vlib, dt):
    """Coupled arguments over the range of normal second parts, where the
    second part z0 x1 reaches 2^-43.5 of z0 (binary32 2^-18.5): the default
    pexp's error is capped by the method's step (the dropped (v - z0) t1 and
    the rounded product), the variant's is not."""
    rng = np.random.default_rng(161)
    n = 200_000
    # results above 2^-969 (binary32 2^-102): second parts in the normal range
    hi, lo = (700.0, -670.0) if dt == np.float64 else (88.0, -70.0)
    x0 = rng.uniform(lo, hi, n).astype(dt)
    half_ulp = np.finfo(dt).eps / 2
    x1 = (x0 * rng.uniform(-1, 1, n).astype(dt) * dt(half_ulp)).astype(dt)
    x1[(x0 + x1) != x0] = dt(0)
    worst = {}
    for name, lib in (("accexp", vlib), ("default", None)):
        z0, z1 = run("pexp", x0, x1, lib=lib)
        np.testing.assert_array_equal((z0 + z1).astype(dt), z0)       # coupled
        rel, cls = qref.check("texp", x0, x1, z0, z1, 1.0)
        ok = cls == 0
        assert ok.sum() > 0.99 * n
        worst[name] = float(rel[ok].max())
        print("%s pexp %s: worst 2^%.2f, mean 2^%.2f" % (
            name, np.dtype(dt).name, math.log2(worst[name]), math.log2(float(rel[ok].mean()))))
    assert worst["accexp"] <= 2.0 ** (-102 if dt == np.float64 else -44)
    assert worst["accexp"] < worst["default"] / 8


@pytest.mark.parametrize("dt", DTS, ids=["f64", "f32"])
@pytest.mark.parametrize("fn", ["texp", "texpm1", "tlog", "tlog1p"])
def test_accexp_main_parts_and_others_unchanged(vlib, fn, dt):
    print("case accexp against the default library", fn, np.dtype(dt).name, flush=True)
    x0, x1 = workloads.twofold_inputs(fn, 100003, dt, seed=171, edges=0.01)
    a0, a1 = run(fn, x0, x1, lib=vlib)
    b0, b1 = run(fn, x0, x1)
    assert same_bits(a0, b0).all()
    if fn != "texp":
        assert same_bits(a1, b1).all()
    else:
        # the two second parts agree to within the rounding of the default's
        # product: a few units in the last place of z1
        fin = np.isfinite(b1) & np.isfinite(b0)
        tol = (4.0 * np.spacing(np.maximum(np.abs(a1[fin]), np.abs(b1[fin]))).astype(np.float64)
               + 2.0 ** (-104 if dt == np.float64 else -46) * np.abs(b0[fin].astype(np.float64))
               + 4.0 * np.finfo(dt).smallest_subnormal)
        bad = np.abs(a1[fin].astype(np.float64) - b1[fin]) > tol
        assert not bad.any(), (fn, np.dtype(dt).name, int(bad.sum()))
        assert same_bits(a1[~fin], b1[~fin]).all()
