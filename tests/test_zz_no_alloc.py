"""holo_gs_iterate_noalloc against holo_gs_iterate (GPU, through the C ABI).

The allocation-free variant runs the same kernels and launch plan on the
library's fixed scratch, so every output must equal the workspace path's bit
for bit: the final replay field, the 8-level codes, the per-iteration NMSE and
amplitude error, the replay NMSE pair and intensity.  Two calls in a row, the
second on a smaller frame (the scratch keeps the first call's contents), then
a third on a caller phasor; NMSE also against the FP64 oracle (1e-4).  Sizes
beyond the fixed scratch are rejected on the host before anything runs.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

HOLO_EUNSUPPORTED = -2


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    assert torch.cuda.is_available()
    return h


def _both(h, t, n_iter, lut, cursor, init=None):
    ny, nx = t.shape
    ref = h.gs_iterate(t, n_iter, lut, cursor, init_phasor=init, want_err=True,
                       recon=torch.empty((ny, nx), dtype=torch.float32, device="cuda"))
    f = torch.empty((ny, nx), dtype=torch.complex64, device="cuda")
    c = torch.empty((ny, nx), dtype=torch.uint8, device="cuda")
    rc = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    nm = torch.empty(n_iter, dtype=torch.float64, device="cuda")
    er = torch.empty(n_iter, dtype=torch.float64, device="cuda")
    f2 = torch.empty(2, dtype=torch.float64, device="cuda")
    cur = h.gs_iterate_noalloc(t, n_iter, lut, cursor, init_phasor=init, field=f, codes=c, nmse=nm, err=er,
                               final2=f2, recon=rc)
    torch.cuda.synchronize()
    assert cur == ref["cursor"]
    assert torch.equal(f, ref["field"])
    assert torch.equal(c, ref["codes"])
    assert np.array_equal(nm.cpu().numpy(), ref["nmse"])
    assert np.array_equal(er.cpu().numpy(), ref["err"])
    assert np.array_equal(f2.cpu().numpy(), ref["nmse_final2"])
    return ref, f, rc


def test_noalloc_matches_gs_iterate_two_calls(holo, orc):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lut = holo.Lut(4096, synth.SEED_LUT)
        t1 = synth.blob_target(1024, 1024, synth.SEED_GS_512)
        print("noalloc GS 1024x1024 x8", flush=True)
        _both(holo, torch.from_numpy(t1).cuda(), 8, lut, 0)
        t2 = synth.blob_target(256, 128, 41)
        print("noalloc GS 256x128 x5 (smaller, second call)", flush=True)
        ref, f, _ = _both(holo, torch.from_numpy(t2).cuda(), 5, lut, 12345)
        init = orc.lut_phasor_field(orc.lut_phases(4096, synth.SEED_LUT), 4096, 12345, 0, 256, 128)
        g = orc.gs(t2, 5, init)
        np.testing.assert_allclose(ref["nmse"], g["nmse"], rtol=1e-4)
        print("noalloc GS 256x128 x3 resumed from the field", flush=True)
        _both(holo, torch.from_numpy(t2).cuda(), 3, None, 0, init=f)


def test_noalloc_rejects_sizes_beyond_scratch(holo):
    t = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda")
    lut = holo.Lut(4096, 1)
    with pytest.raises(holo.HoloError) as e:
        holo.gs_iterate_noalloc(t, 2, lut, 0)
    assert e.value.status == HOLO_EUNSUPPORTED and "scratch" in str(e.value)
    t = torch.zeros((1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(holo.HoloError) as e:
        holo.gs_iterate_noalloc(t, 5000, lut, 0)
    assert e.value.status == HOLO_EUNSUPPORTED
