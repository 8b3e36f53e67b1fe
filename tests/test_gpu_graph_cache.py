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


def test_concurrent_threads_batched_entry_points():
    """One thread captures and replays batched OSPR graphs while another does
    the same with batched GS; both equal one thread's direct calls."""
    import threading
    import paper_2004_04049_amd as h
    h.lib()
    dev = torch.device("cuda:0")
    lut = h.Lut(10007, synth.SEED_LUT)
    layouts = [[(64, 2), (128, 3), (64, 4)], [(128, 2), (64, 3)], [(64, 1), (64, 2), (128, 2), (64, 3)],
               [(128, 4)], [(64, 5), (128, 1)], [(128, 3), (128, 2), (64, 2)]]
    o_targets = [[torch.from_numpy(synth.blob_target(n, n, 700 + 10 * i + f)).to(dev) for f, (n, _) in enumerate(lay)]
                 for i, lay in enumerate(layouts)]
    g_iters = list(range(1, 11))
    g_targets = [torch.from_numpy(synth.blob_target(64, 64, 900 + f)).to(dev) for f in range(3)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def ospr_calls(out):
        for _ in range(2):
            for i, lay in enumerate(layouts):
                nm = torch.zeros((len(lay), 2), dtype=torch.float64, device=dev)
                bits, _, _ = h.ospr_generate_batched(o_targets[i], [k for _, k in lay], lut, 3 * i, nmse_out=nm,
                                                     stream=streams[0])
                out[i] = (bits, nm)

    def gs_calls(out):
        for _ in range(2):
            for k in g_iters:
                fl = [torch.empty((64, 64), dtype=torch.complex64, device=dev) for _ in g_targets]
                h.gs_iterate_batched(g_targets, k, lut, 5 * k, fields=fl, want_nmse=False, stream=streams[1])
                out[k] = fl

    def snapshot(o_out, g_out):
        torch.cuda.synchronize()
        return ({i: ([b.cpu() for b in bits], nm.cpu()) for i, (bits, nm) in o_out.items()},
                {k: [f.cpu() for f in fl] for k, fl in g_out.items()})

    h.set_graphs(False)
    try:
        o_ref, g_ref = {}, {}
        ospr_calls(o_ref)
        gs_calls(g_ref)
        o_ref, g_ref = snapshot(o_ref, g_ref)
    finally:
        h.set_graphs(True)
    o_out, g_out, errs = {}, {}, []

    def run(fn, out):
        try:
            fn(out)
        except Exception as e:   # noqa: BLE001 (reported below)
            errs.append(e)
    th = [threading.Thread(target=run, args=(ospr_calls, o_out)), threading.Thread(target=run, args=(gs_calls, g_out))]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errs, errs
    o_got, g_got = snapshot(o_out, g_out)
    for i in o_ref:
        for a, b in zip(o_ref[i][0], o_got[i][0]):
            assert torch.equal(a, b), f"OSPR layout {i}: bits"
        assert torch.equal(o_ref[i][1], o_got[i][1]), f"OSPR layout {i}: NMSE"
    for k in g_ref:
        for a, b in zip(g_ref[k], g_got[k]):
            assert torch.equal(a, b), f"GS n_iter {k}"
