"""The batched launch that allocates nothing (tf_batch_run_noalloc) through the
C ABI, against the batched launch of a plan (tf_batch_plan_create +
tf_batch_launch) with the same configuration: outputs equal bit for bit, on
two calls in a row, the second with a smaller input (the static scratch keeps
the first call's contents: its descriptors and chunk list must not leak into
the second), in two configurations; capacity and argument errors enqueue
nothing and leave the outputs untouched."""
import ctypes

import numpy as np
import pytest

from paper_1502_05216_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as m
    m.lib()
    return m


def _items(descs, seed, misalign_every=0):
    d = torch.device("cuda:0")
    items = []
    for k, (fn, dt, x0, x1) in enumerate(workloads.batch_inputs(descs, seed=seed)):
        if misalign_every and k % misalign_every == 1 and x0.size > 0:
            a0 = torch.from_numpy(np.concatenate([[dt(0.5)], x0])).to(d)[1:]
            a1 = torch.from_numpy(np.concatenate([[dt(0.0)], x1])).to(d)[1:]
        else:
            a0 = torch.from_numpy(np.ascontiguousarray(x0)).to(d)
            a1 = torch.from_numpy(np.ascontiguousarray(x1)).to(d)
        items.append((fn, a0, a1, torch.full_like(a0, float("nan")),
                      torch.full_like(a0, float("nan"))))
    return items


def _twin(items):
    """The same arguments with fresh (NaN-filled) outputs."""
    return [(fn, a0, a1, torch.full_like(a0, float("nan")), torch.full_like(a0, float("nan")))
            for fn, a0, a1, _, _ in items]


def _equal(u, v):
    it = torch.int64 if u.dtype == torch.float64 else torch.int32
    return bool(((u.view(it) == v.view(it)) | (torch.isnan(u) & torch.isnan(v))).all())


def _check(items, ref, what):
    for k, ((fn, _, _, z0, z1), (_, _, _, r0, r1)) in enumerate(zip(items, ref)):
        assert _equal(z0, r0) and _equal(z1, r1), "%s: array %d (%s, n=%d)" % (
            what, k, fn, z0.numel())


@pytest.mark.parametrize("config", [(2, 4, 32, 0), (1, 2, 8, 2)])
def test_noalloc_equals_plan_two_calls(tf, config):
    from paper_1502_05216_amd.batch import BatchPlan, run_noalloc
    # first call: 1500 arrays (lengths 2^U[0, 20], mixed function and format,
    # empty and misaligned arrays among them); second call: 200 other arrays
    big = workloads.batch_descriptors(count=1500, seed=workloads.SEED + 11)
    big[3] = (big[3][0], big[3][1], 0)
    small = workloads.batch_descriptors(count=200, seed=workloads.SEED + 12, max_log2=14)
    for call, (descs, seed, mis) in enumerate(((big, 5, 7), (small, 6, 0))):
        print("case noalloc config %s call %d: %d arrays" % (config, call, len(descs)),
              flush=True)
        items = _items(descs, seed, misalign_every=mis)
        ref = _twin(items)
        with BatchPlan(ref, config=config) as plan:
            plan.launch()
            run_noalloc(items, config=config)
            torch.cuda.synchronize()
        _check(items, ref, "config %s call %d" % (config, call))
        # both launches ran (not two untouched NaN fills): nearly every main
        # part is a number (edge arguments give a few NaNs)
        total = sum(it[3].numel() for it in items)
        finite = sum(int((~torch.isnan(it[3])).sum()) for it in items)
        assert finite >= 0.99 * total, (finite, total)


def test_noalloc_c_abi_limits(tf):
    from paper_1502_05216_amd import _lib
    from paper_1502_05216_amd.batch import (MAX_ARRAYS_NOALLOC, BatchConfig, BatchDesc, _bind,
                                            run_noalloc)
    lib = _bind(_lib.lib())
    d = torch.device("cuda:0")
    x = torch.ones(4097, dtype=torch.float64, device=d)
    z0 = torch.full_like(x, float("nan"))
    z1 = torch.full_like(x, float("nan"))
    one = BatchDesc(0, 0, x.numel(), x.data_ptr(), x.data_ptr(), z0.data_ptr(), z1.data_ptr())
    stream = _lib._stream()
    cfg = BatchConfig(2, 4, 1, 0)          # 512-element chunks
    # too many arrays
    arr = (BatchDesc * (MAX_ARRAYS_NOALLOC + 1))(*([one] * (MAX_ARRAYS_NOALLOC + 1)))
    assert lib.tf_batch_run_noalloc(arr, MAX_ARRAYS_NOALLOC + 1, ctypes.byref(cfg),
                                    stream) == _lib.TF_ECAPACITY
    # too many chunks: 8192 arrays of 4097 elements in 512-element chunks (9 each)
    assert lib.tf_batch_run_noalloc(arr, MAX_ARRAYS_NOALLOC, ctypes.byref(cfg),
                                    stream) == _lib.TF_ECAPACITY
    # bad descriptor, bad configuration
    bad = (BatchDesc * 1)(BatchDesc(4, 0, 1, x.data_ptr(), x.data_ptr(), z0.data_ptr(),
                                    z1.data_ptr()))
    assert lib.tf_batch_run_noalloc(bad, 1, None, stream) == _lib.TF_EINVAL
    assert lib.tf_batch_run_noalloc(arr, 1, ctypes.byref(BatchConfig(3, 4, 32, 0)),
                                    stream) == _lib.TF_EINVAL
    assert lib.tf_batch_run_noalloc(None, 0, None, stream) == _lib.TF_OK
    torch.cuda.synchronize()
    assert bool(torch.isnan(z0).all()) and bool(torch.isnan(z1).all())
    # within the limits the same descriptor runs
    run_noalloc([("texp", x, x, z0, z1)])
    torch.cuda.synchronize()
    r0, r1 = tf.texp(x, x)
    assert _equal(z0, r0) and _equal(z1, r1)
