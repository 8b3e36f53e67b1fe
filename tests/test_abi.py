"""The C-ABI library: it loads, exports every symbol include/holo.h declares,
and rejects invalid arguments with the documented status codes before
touching a device.  CPU only (no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    syms = []
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            syms += re.findall(r"HOLO_API\s+[\w\s\*]+?\b(holo_\w+)\s*\(", txt)
    return sorted(set(syms))


@pytest.fixture(scope="module")
def lib():
    import paper_2004_04049_amd as h
    if not os.path.exists(h.LIB_PATH):
        pytest.fail("libholo.so is not built (run __graft_entry__.build())")
    return h.lib()


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    import paper_2004_04049_amd as h
    assert set(h.SIGNATURES) >= set(syms)


def test_lut_check_rules(lib):
    import paper_2004_04049_amd as h
    assert h.lut_check(10007, 1024, 1024, 24) == h.LUT_LT_FULL
    w = h.lut_check(256, 256, 256, 24)
    assert w & h.LUT_NOT_PRIME and w & h.LUT_LE_MAXDIM and w & h.LUT_DIVIDES_FRAME
    assert h.lut_check(23, 64, 64, 24) & h.LUT_LE_NSF
    assert h.lut_check(0, 64, 64, 8) & h.LUT_FLAT
    assert h.lut_check(1024 * 1024 * 24 + 7, 1024, 1024, 24) & h.LUT_LT_FULL == 0


def test_invalid_arguments_rejected_before_device_work(lib):
    import paper_2004_04049_amd as h
    cur = C.c_uint64(0)
    P = C.c_void_p
    fake = P(16)
    st = lib.holo_ospr_generate(None, 64, 64, 8, fake, C.byref(cur), fake, None, None, 0, 0, None)
    assert st == h.HOLO_EINVAL
    st = lib.holo_ospr_generate(fake, 64, 64, 0, fake, C.byref(cur), fake, None, None, 0, 0, None)
    assert st == h.HOLO_EINVAL
    assert b"n_sf" in lib.holo_last_error()
    st = lib.holo_ospr_generate(fake, 100, 64, 8, fake, C.byref(cur), fake, None, None, 0, 0, None)
    assert st == h.HOLO_EUNSUPPORTED
    st = lib.holo_ospr_generate(fake, 4096, 64, 8, fake, C.byref(cur), fake, None, None, 0, 0, None)
    assert st == h.HOLO_EUNSUPPORTED
    st = lib.holo_gs_iterate(fake, 64, 64, 0, fake, C.byref(cur), None, None, None, None, None, None, None, 0, 0,
                             None)
    assert st == h.HOLO_EINVAL
    st = lib.holo_gs_iterate(fake, 64, 64, 5, fake, C.byref(cur), None, None, None, None, None, fake, None, 0, 0,
                             None)
    assert st == h.HOLO_EINVAL   # nmse_final2 without codes
    st = lib.holo_reconstruct_nmse(fake, 4, 64, 64, 1, fake, None, None, 0, None)
    assert st == h.HOLO_EINVAL
    st = lib.holo_fft2(fake, fake, 64, 64, 2, 0, None)
    assert st == h.HOLO_EINVAL
    # matrix-core stages: sides of 256 and more; unknown precisions rejected
    st = lib.holo_fft2(fake, fake, 128, 256, -1, h.BF16, None)
    assert st == h.HOLO_EUNSUPPORTED
    st = lib.holo_fft2(fake, fake, 256, 256, -1, 3, None)
    assert st == h.HOLO_EINVAL
    st = lib.holo_ospr_generate(fake, 256, 128, 8, fake, C.byref(cur), fake, None, None, h.FP16, 0, None)
    assert st == h.HOLO_EUNSUPPORTED
    assert cur.value == 0
    # phase sources: table offsets are 32-bit byte offsets; a code table needs entries
    out = P()
    assert lib.holo_lut_build(1 << 29, 1, C.byref(out)) == h.HOLO_EUNSUPPORTED
    assert lib.holo_lut_build_codes(0, 1, C.byref(out)) == h.HOLO_EINVAL
    assert lib.holo_lut_build_codes(1 << 31, 1, C.byref(out)) == h.HOLO_EUNSUPPORTED
    assert lib.holo_lut_prng(1, None) == h.HOLO_EINVAL
    assert lib.holo_lut_mseq(1, None) == h.HOLO_EINVAL
    assert lib.holo_lut_kind(None) == -1
    assert lib.holo_phase_mask(fake, 0, 64, 64, 1, None, None) == h.HOLO_EINVAL
    assert lib.holo_phase_mask(fake, 0, 64, 64, 0, fake, None) == h.HOLO_EINVAL
    assert lib.holo_phase_mask(fake, 0, 100, 64, 1, fake, None) == h.HOLO_EUNSUPPORTED


def test_plan_points_per_thread_rules(lib, tmp_path):
    """OSPR plans take 8 or 16 points per thread (0: heuristic), GS plans also
    4; plan_set and plan_load refuse the others."""
    import paper_2004_04049_amd as h
    try:
        h.plan_set(h.PLAN_OSPR, 256, 128, 4, [0, 0, 0, 0, -1, 0, 8])
        assert h.plan_get(h.PLAN_OSPR, 256, 128, 4)[6] == 8
        with pytest.raises(h.HoloError) as e:
            h.plan_set(h.PLAN_OSPR, 256, 128, 4, [0, 0, 0, 0, -1, 0, 4])
        assert e.value.status == h.HOLO_EINVAL
        h.plan_set(h.PLAN_GS, 256, 128, 1, [0, 0, 0, 0, -1, 0, 4])
        with pytest.raises(h.HoloError):
            h.plan_set(h.PLAN_GS, 256, 128, 1, [0, 0, 0, 0, -1, 0, 12])
        bad = tmp_path / "plans.json"
        bad.write_text('[{"kind": 0, "nx": 64, "ny": 64, "n_sf": 2, "cfg": [0, 0, 0, 0, -1, 0, 4]}]')
        with pytest.raises(h.HoloError):
            h.plan_load(str(bad))
        bad.write_text('[{"kind": 3, "nx": 64, "ny": 64, "n_sf": 2, "cfg": [0, 0, 0, 0, -1, 0, 8]}]')
        with pytest.raises(h.HoloError):
            h.plan_load(str(bad))
        bad.write_text('[{"kind": 0, "nx": 64, "ny": 64, "n_sf": -1, "cfg": [0, 0, 0, 0, -1, 0, 8]}]')
        with pytest.raises(h.HoloError) as e:   # as plan_set: n_sf >= 0
            h.plan_load(str(bad))
        assert e.value.status == h.HOLO_EINVAL
        good = tmp_path / "good.json"
        h.plan_save(str(good))
        h.plan_set(h.PLAN_OSPR, 256, 128, 4, h.DEFAULT_PLAN)
        h.plan_load(str(good))
        assert h.plan_get(h.PLAN_OSPR, 256, 128, 4)[6] == 8
    finally:
        h.plan_set(h.PLAN_OSPR, 256, 128, 4, h.DEFAULT_PLAN)
        h.plan_set(h.PLAN_GS, 256, 128, 1, h.DEFAULT_PLAN)


def test_plan_for_every_subframe_count(lib):
    """An OSPR plan stored under n_sf = 0 serves the size's sub-frame counts
    that have no plan of their own; GS plans ignore n_sf."""
    import paper_2004_04049_amd as h
    try:
        h.plan_set(h.PLAN_OSPR, 512, 256, 0, [8, 2, 4, 0, 16, 0, 8])
        h.plan_set(h.PLAN_OSPR, 512, 256, 7, [16, 1, 2, 0, 0, 3, 16])
        assert h.plan_get(h.PLAN_OSPR, 512, 256, 5) == [8, 2, 4, 0, 16, 0, 8]
        assert h.plan_get(h.PLAN_OSPR, 512, 256, 7) == [16, 1, 2, 0, 0, 3, 16]
        assert h.plan_get(h.PLAN_OSPR, 256, 512, 5) == h.DEFAULT_PLAN
        with pytest.raises(h.HoloError):
            h.plan_set(h.PLAN_OSPR, 512, 256, -1, h.DEFAULT_PLAN)
    finally:
        h.plan_set(h.PLAN_OSPR, 512, 256, 0, h.DEFAULT_PLAN)
        h.plan_set(h.PLAN_OSPR, 512, 256, 7, h.DEFAULT_PLAN)


def test_batched_gs_invalid_arguments(lib):
    import paper_2004_04049_amd as h
    cur = C.c_uint64(0)
    fake = C.c_void_p(16)
    fr = (h.HoloGsFrame * 2)()
    fr[0] = h.HoloGsFrame(16, None, None, None, None)
    fr[1] = h.HoloGsFrame(None, None, None, None, None)
    arr = C.cast(fr, C.c_void_p)
    assert lib.holo_gs_iterate_batched(None, 1, 64, 64, 3, fake, C.byref(cur), None, None, None, 0, None) == h.HOLO_EINVAL
    assert lib.holo_gs_iterate_batched(arr, 0, 64, 64, 3, fake, C.byref(cur), None, None, None, 0, None) == h.HOLO_EINVAL
    assert lib.holo_gs_iterate_batched(arr, 1, 64, 64, 0, fake, C.byref(cur), None, None, None, 0, None) == h.HOLO_EINVAL
    assert lib.holo_gs_iterate_batched(arr, 2, 64, 64, 3, fake, C.byref(cur), None, None, None, 0, None) == h.HOLO_EINVAL
    assert b"frame 1" in lib.holo_last_error()
    fr[1] = h.HoloGsFrame(16, None, None, None, 16)     # recon without codes
    assert lib.holo_gs_iterate_batched(arr, 2, 64, 64, 3, fake, C.byref(cur), None, None, None, 0, None) == h.HOLO_EINVAL
    assert lib.holo_gs_iterate_batched(arr, 1, 100, 64, 3, fake, C.byref(cur), None, None, None, 0, None) == \
        h.HOLO_EUNSUPPORTED
