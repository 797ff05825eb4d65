"""The plain entry points under HIP graph capture.

They allocate nothing and issue no memset, so a caller may capture them into
a graph (torch.cuda.CUDAGraph records the launches on its capture stream).
A graph of the four twofold functions in both formats, an interface function,
twofold arithmetic and the fused chain backward is replayed several times,
with eager work and synchronisation between the replays that overwrites the
outputs, and every replay must reproduce the eager results bit for bit.
"""
import numpy as np
import pytest

from paper_1502_05216_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bits_equal(a, b):
    it = torch.int64 if a.dtype == torch.float64 else torch.int32
    return bool(((a.view(it) == b.view(it)) | (torch.isnan(a) & torch.isnan(b))).all())


def test_capture_and_replay():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1502_05216_amd as tf
    tf.lib()
    d = torch.device("cuda:0")
    n = 3 * 256 * 4 * 9 + 77                       # several tiles and a ragged tail
    ins = {}
    for dt in (np.float64, np.float32):
        for fn in tf.TWOFOLD + ("plog",):
            a, b = workloads.twofold_inputs(fn, n, dt, seed=41, edges=0.01,
                                            coupled=fn == "plog")
            ins[(fn, dt)] = (torch.from_numpy(a).to(d), torch.from_numpy(b).to(d))
    x0, x1 = ins[("texp", np.float64)]
    g0 = torch.linspace(-1, 1, n, dtype=torch.float64, device=d)
    g1 = g0 * 2.0 ** -60
    outs = {k: (torch.empty_like(v[0]), torch.empty_like(v[0])) for k, v in ins.items()}
    arith = (torch.empty_like(x0), torch.empty_like(x0))
    chain = (torch.empty_like(x0), torch.empty_like(x0))
    saved = [(torch.empty_like(x0), torch.empty_like(x0)) for _ in range(2)]

    def work():
        for (fn, dt), (a, b) in ins.items():
            getattr(tf, fn)(a, b, out=outs[(fn, dt)])
        tf.tadd(x0, x1, *outs[("texp", np.float64)], out=arith)
        tf.texp(x0, x1, out=saved[0])
        tf.texpm1(*saved[0], out=saved[1])
        tf.chain_bwd(("texp", "texpm1", "tlog1p"), (saved[0], saved[1], saved[1]), g0, g1,
                     out=chain)

    def snapshot():
        res = [t.clone() for pair in outs.values() for t in pair]
        return res + [t.clone() for t in arith + chain]

    def clobber():
        for pair in list(outs.values()) + [arith, chain] + saved:
            for t in pair:
                t.fill_(float("nan"))

    work()                                        # eager reference (also warms the library)
    torch.cuda.synchronize()
    ref = snapshot()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            work()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for replay in range(4):
        clobber()                                 # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = snapshot()
        assert all(_bits_equal(a, b) for a, b in zip(got, ref)), "replay %d" % replay
        # eager calls after a replay still agree
        work()
        torch.cuda.synchronize()
        assert all(_bits_equal(a, b) for a, b in zip(snapshot(), ref)), "eager %d" % replay
