"""Batched GS (holo_gs_iterate_batched): frames of one size iterating
together equal holo_gs_iterate calls frame by frame, with the pool cursor
continuing across pool-seeded frames; one frame against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    return h


def _singles(holo, targets, n_iter, lut, cursor, inits, want_codes):
    out, c = [], cursor
    for t, ip, wc in zip(targets, inits, want_codes):
        ny, nx = t.shape
        codes = torch.empty((ny, nx), dtype=torch.uint8, device="cuda") if wc else None
        recon = torch.empty((ny, nx), dtype=torch.float32, device="cuda") if wc else None
        r = holo.gs_iterate(t, n_iter, lut if ip is None else None, c, init_phasor=ip, codes=codes, recon=recon,
                            want_final=wc, want_err=True)
        c = r["cursor"]
        r["recon"] = recon
        out.append(r)
    return out, c


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("n,n_iter", [(256, 6), (512, 3)])
def test_batched_gs_equals_single_calls(holo, n, n_iter, graphs):
    print(f"batched GS {n}^2 x 4, {n_iter} iterations, graphs {graphs}", flush=True)
    targets = [torch.from_numpy(synth.blob_target(n, n, 500 + f)).cuda() for f in range(4)]
    lut = holo.Lut(4096, 1)
    seed = holo.gs_iterate(targets[3], 2, lut, 99)["field"].clone()
    inits = [None, None, seed, None]              # frame 2 resumes from a caller field
    want_codes = [True, False, True, True]
    holo.set_graphs(graphs)
    try:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            codes = [torch.empty((n, n), dtype=torch.uint8, device="cuda") if w else None for w in want_codes]
            recons = [torch.empty((n, n), dtype=torch.float32, device="cuda") if w else None for w in want_codes]
            for rep in range(2):                  # a second call replays the captured graph
                rb = holo.gs_iterate_batched(targets, n_iter, lut, 1000 + rep, init_phasors=inits, codes=codes,
                                             recons=recons, want_err=True)
                singles, c = _singles(holo, targets, n_iter, lut, 1000 + rep, inits, want_codes)
                assert rb["cursor"] == c == 1000 + rep + 3 * n * n
                for f, r in enumerate(singles):
                    np.testing.assert_array_equal(rb["nmse"][f], r["nmse"])
                    np.testing.assert_array_equal(rb["err"][f], r["err"])
                    assert torch.equal(rb["fields"][f], r["field"]), f
                    if want_codes[f]:
                        assert torch.equal(codes[f], r["codes"]), f
                        assert torch.equal(recons[f], r["recon"]), f
        torch.cuda.synchronize()
    finally:
        holo.set_graphs(True)


def test_batched_gs_final_nmse_and_oracle(holo, orc):
    n, n_iter = 128, 5
    targets = [synth.blob_target(n, n, 520 + f) for f in range(3)]
    lut = holo.Lut(4096, 1)
    tt = [torch.from_numpy(t).cuda() for t in targets]
    rb = holo.gs_iterate_batched(tt, n_iter, lut, 0, want_final=True)
    c = 0
    phi = orc.lut_phases(4096, 1)
    for f, t in enumerate(targets):
        r = holo.gs_iterate(tt[f], n_iter, lut, c)
        np.testing.assert_array_equal(rb["nmse_final2"][f], r["nmse_final2"])
        g = orc.gs(t, n_iter, orc.lut_phasor_field(phi, 4096, c, 0, n, n))
        np.testing.assert_allclose(rb["nmse"][f], g["nmse"], rtol=1e-4)
        c = r["cursor"]
    assert rb["cursor"] == c


def test_batched_gs_1024_fifty_iterations(holo):
    # the benchmark size under the GS plan in force, two frames
    n, n_iter = 1024, 50
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_GS_512 + f)).cuda() for f in range(2)]
    lut = holo.Lut(4096, 1)
    rb = holo.gs_iterate_batched(targets, n_iter, lut, 0)
    c = 0
    for f in range(2):
        r = holo.gs_iterate(targets[f], n_iter, lut, c)
        c = r["cursor"]
        np.testing.assert_array_equal(rb["nmse"][f], r["nmse"])
        assert torch.equal(rb["fields"][f], r["field"])
