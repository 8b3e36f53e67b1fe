"""The library keeps at most 32 captured graphs.  Calls on two streams, each
asking for a new graph, push older graphs out while the other stream may still
be replaying its own; every result must equal the direct launches'."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_graph_cache_eviction_across_streams():
    import paper_2004_04049_amd as h
    h.lib()
    n = 64
    dev = torch.device("cuda:0")
    t = torch.from_numpy(synth.blob_target(n, n, synth.SEED_GS_512)).to(dev)
    lut = h.Lut(4096, synth.SEED_LUT)
    iters = list(range(1, 41))   # 40 graph keys (n_iter is part of the key): 8 evictions
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def run(graphs):
        h.set_graphs(graphs)
        outs = [torch.empty((n, n), dtype=torch.complex64, device=dev) for _ in iters]
        try:
            for i, k in enumerate(iters):
                # no host outputs: the call only enqueues, so the streams overlap
                h.gs_iterate(t, k, lut, 0, field=outs[i], want_nmse=False, want_final=False,
                             stream=streams[i % 2])
            torch.cuda.synchronize()
        finally:
            h.set_graphs(True)
        return [o.cpu() for o in outs]

    direct = run(False)
    for _ in range(2):   # second pass: the survivors are replayed, the evicted re-captured
        graphed = run(True)
        for k, a, b in zip(iters, direct, graphed):
            assert torch.equal(a, b), f"n_iter {k}"


@pytest.mark.parametrize("graphs", [False, True])
def test_concurrent_threads(graphs):
    """Two host threads, each on its own stream (ctypes releases the GIL),
    with graph replay off and on: with it on, one thread captures new graphs
    (the library keeps its other calls out of a capture) and evicts old ones
    while the other looks its own up and launches it.  The results equal those
    of one thread's direct calls."""
    import threading
    import paper_2004_04049_amd as h
    h.lib()
    n = 64
    dev = torch.device("cuda:0")
    t = torch.from_numpy(synth.blob_target(n, n, synth.SEED_GS_512)).to(dev)
    lut = h.Lut(4096, synth.SEED_LUT)
    work = [list(range(1, 31)), list(range(31, 61))]   # 60 keys in all
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[torch.empty((n, n), dtype=torch.complex64, device=dev) for _ in w] for w in work]
    errs = []

    def worker(j):
        try:
            for _ in range(2):   # the second round replays survivors, re-captures the evicted
                for i, k in enumerate(work[j]):
                    h.gs_iterate(t, k, lut, 0, field=outs[j][i], want_nmse=False, want_final=False,
                                 stream=streams[j])
        except Exception as e:   # noqa: BLE001 (reported below)
            errs.append(e)

    h.set_graphs(graphs)
    try:
        th = [threading.Thread(target=worker, args=(j,)) for j in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        torch.cuda.synchronize()
        assert not errs, errs
        h.set_graphs(False)   # the same calls from this thread alone
        for j in range(2):
            for k, got in zip(work[j], outs[j]):
                f = torch.empty((n, n), dtype=torch.complex64, device=dev)
                h.gs_iterate(t, k, lut, 0, field=f, want_nmse=False, want_final=False, stream=streams[j])
                torch.cuda.synchronize()
                assert torch.equal(f.cpu(), got.cpu()), f"thread {j} n_iter {k}"
    finally:
        h.set_graphs(True)
