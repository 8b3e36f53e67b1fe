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
