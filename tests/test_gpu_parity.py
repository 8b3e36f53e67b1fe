"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Tolerances (in unitary units of Eq. (1)/(2), targets in [0, 1]):
  * binary holograms: bit-exact except pixels with |Re H_oracle| < 1e-5;
  * NMSE values: 1e-4 relative;
  * transforms / time-averaged intensities: relative L2 error < 1e-5
    (FP32 radix-16 transforms: about log2(N) * 2^-24 per element).
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

TIE = 1e-5
NMSE_RTOL = 1e-4


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    assert torch.cuda.is_available()
    return h


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _check_bits(h, orc, bits_gpu, ref, n):
    got = h.unpack_bits(bits_gpu, n)
    want = orc.unpack_bits(ref["bits"], n)
    reh = ref["reH"].reshape(got.shape[0], -1)
    decided = np.abs(reh) >= TIE
    mism = (got != want) & decided
    assert int(mism.sum()) == 0, f"{int(mism.sum())} decided pixels differ"
    return int((~decided).sum())


@pytest.mark.parametrize("nx,ny", [(16, 16), (64, 32), (32, 128), (256, 256), (1024, 1024), (2048, 64), (64, 2048)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft2_matches_oracle(holo, orc, nx, ny, sign):
    rng = np.random.default_rng(nx + 7 * ny)
    f = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    print(f"fft2 {nx}x{ny} sign {sign}", flush=True)
    got = holo.fft2(torch.from_numpy(f).cuda(), sign).cpu().numpy()
    want = orc.fft2(f.astype(np.complex128), sign)
    assert _rel_l2(got, want) < 1e-6


def _ospr_case(holo, orc, nx, ny, nsf, n_lut, cursor, target, want_recon=True):
    print(f"ospr {nx}x{ny} nsf={nsf} lut={n_lut} cursor={cursor}", flush=True)
    lut = holo.Lut(n_lut, 1)
    phi = orc.lut_phases(n_lut, 1)
    assert np.array_equal(lut.phases(), phi)           # bit-exact FP64 phases
    t = torch.from_numpy(target).cuda()
    recon = torch.empty((ny, nx), dtype=torch.float32, device="cuda") if want_recon else None
    bits, nm, cur = holo.ospr_generate(t, nsf, lut, cursor, recon=recon)
    torch.cuda.synchronize()
    ref = orc.ospr(target, nsf, phi, n_lut, cursor)
    assert cur == cursor + nsf * nx * ny
    ties = _check_bits(holo, orc, bits, ref, nx * ny)
    np.testing.assert_allclose(nm, ref["nmse2"], rtol=NMSE_RTOL)
    # A pixel with |Re H| below the tie threshold may legitimately binarise
    # either way, and one flipped pixel moves every replay value by ~2/sqrt(N);
    # so the reconstruction is checked against the oracle's replay of the
    # GPU's own holograms (unique given the bits).
    own = orc.reconstruct(bits.cpu().numpy().view(np.uint32), 2, nx, ny, nsf)
    np.testing.assert_allclose(nm, orc.nmse_pair(own, target), rtol=NMSE_RTOL)
    if want_recon:
        assert _rel_l2(recon.cpu().numpy().astype(np.float64), own) < 1e-5
    return bits, ref, ties


def test_ospr_uniform_64_lut256(holo, orc):
    # 64x64 uniform target, 8 sub-frames, 256-entry LUT (which divides the
    # frame, so every sub-frame is the same hologram)
    t = synth.uniform_target(64, 64, synth.SEED_UNIFORM_64)
    bits, ref, _ = _ospr_case(holo, orc, 64, 64, 8, 256, 0, t)
    b = bits.cpu().numpy()
    assert all(np.array_equal(b[k], b[0]) for k in range(8))


@pytest.mark.parametrize("nx,ny,nsf,n_lut,cursor", [
    (128, 32, 5, 10007, 123456789012),      # ragged sub-frame count, non-square
    (32, 256, 3, 1, 7),                     # single-entry LUT
    (64, 64, 2, 0, 0),                      # flat phase
    (16, 16, 1, 17, 2 ** 63 + 5),           # smallest size, huge cursor
    (512, 512, 9, 65537, 3),
    # multi-wave column blocks on grids of several blocks per CU
    (1024, 512, 6, 65537, 17),
    (128, 1024, 6, 10007, 5),
])
def test_ospr_small_cases(holo, orc, nx, ny, nsf, n_lut, cursor):
    t = synth.blob_target(nx, ny, 5)
    _ospr_case(holo, orc, nx, ny, nsf, n_lut, cursor, t)


@pytest.mark.parametrize("n_lut", [2 ** 16, 10007, 2 ** 20, 1024 * 1024 * 24])
def test_ospr_1024_full_size(holo, orc, n_lut):
    # the benchmark's frame; 2^20 and the non-repeating table (every pixel of
    # every sub-frame its own entry) reach the largest pool offsets
    t = synth.blob_target(1024, 1024, synth.SEED_OSPR_1024)
    _, _, ties = _ospr_case(holo, orc, 1024, 1024, 24, n_lut, 0, t, want_recon=True)
    assert ties < 24 * 1024 * 1024 * 1e-3


def test_ospr_1024_partial_subframe_group(holo, orc):
    # the row pass serves up to 8 sub-frames per block at this size; 12
    # sub-frames leave a last group of 4
    t = synth.blob_target(1024, 1024, 23)
    _ospr_case(holo, orc, 1024, 1024, 12, 10007, 7, t)


def test_ospr_subframes_past_32bit_offsets(holo, orc):
    # 1100 sub-frames at 1024^2: the half spectra the replay pass reads span
    # ~4.7 GB, past 32-bit byte offsets.  A 256-entry LUT divides the frame, so
    # every sub-frame is the same hologram and the time average equals the
    # replay of one sub-frame: the NMSE pair must equal the one-sub-frame
    # frame's (GPU and oracle) and every sub-frame's bits the first one's.
    nx = ny = 1024
    t = synth.blob_target(nx, ny, 24)
    tt = torch.from_numpy(t).cuda()
    lut = holo.Lut(256, 1)
    print("ospr 1024x1024 nsf=1 lut=256", flush=True)
    b1, nm1, _ = holo.ospr_generate(tt, 1, lut, 0)
    ref = orc.ospr(t, 1, orc.lut_phases(256, 1), 256, 0)
    _check_bits(holo, orc, b1, ref, nx * ny)
    np.testing.assert_allclose(nm1, ref["nmse2"], rtol=NMSE_RTOL)
    print("ospr 1024x1024 nsf=1100 lut=256", flush=True)
    bits, nm, cur = holo.ospr_generate(tt, 1100, lut, 0)
    torch.cuda.synchronize()
    assert cur == 1100 * nx * ny
    assert bool((bits == b1[0]).all())
    np.testing.assert_allclose(nm, nm1, rtol=1e-5)
    del bits
    torch.cuda.empty_cache()


def test_ospr_2048_tall_and_wide(holo, orc):
    t = synth.blob_target(2048, 128, 21)
    _ospr_case(holo, orc, 2048, 128, 3, 10007, 11, t)
    t = synth.blob_target(128, 2048, 22)
    _ospr_case(holo, orc, 128, 2048, 3, 10007, 11, t)


@pytest.mark.parametrize("pts", [8, 16])
@pytest.mark.parametrize("nx,ny,nsf,n_lut,cursor,plan", [
    (16, 16, 3, 17, 5, [0, 0, 0, 0, -1, 0]),
    (128, 32, 5, 10007, 123456789012, [0, 0, 0, 0, -1, 0]),
    (256, 256, 6, 10007, 3, [8, 2, 2, 0, 16, 0]),
    (512, 1024, 4, 65537, 17, [16, 1, 4, 0, 16, 3]),   # chunks of 3 over 4 sub-frames
    (1024, 1024, 24, 65536, 0, [8, 1, 0, 0, 16, 0]),   # the benchmark frame
    (2048, 128, 3, 10007, 11, [8, 1, 2, 0, 16, 0]),
    (128, 2048, 3, 10007, 11, [16, 1, 2, 0, 16, 0]),   # 2048-point columns: 8 points -> 8-column tiles
])
def test_ospr_points_per_thread(holo, orc, nx, ny, nsf, n_lut, cursor, plan, pts):
    """Both radix factorisations of the row, column and reconstruction passes
    (8 points per thread: radix-8 stages, then one radix-2/4 stage; 16:
    radix-16 stages, then one radix-2/4/8 stage) for all three passes, as a
    plan selects them (the default mixes them per pass), against the oracle
    with the same bars."""
    t = synth.blob_target(nx, ny, 7)
    holo.plan_set(holo.PLAN_OSPR, nx, ny, nsf, plan + [pts])
    try:
        _ospr_case(holo, orc, nx, ny, nsf, n_lut, cursor, t)
    finally:
        holo.plan_set(holo.PLAN_OSPR, nx, ny, nsf, holo.DEFAULT_PLAN)


def test_ospr_cursor_chaining_bit_exact(holo):
    t = torch.from_numpy(synth.blob_target(256, 256, 3)).cuda()
    lut = holo.Lut(10007, 1)
    b8, _, c8 = holo.ospr_generate(t, 8, lut, 99)
    b4a, _, c4 = holo.ospr_generate(t, 4, lut, 99)
    b4b, _, c4b = holo.ospr_generate(t, 4, lut, c4)
    assert c8 == c4b
    assert torch.equal(b8, torch.cat([b4a, b4b]))


def test_reconstruct_from_oracle_holograms(holo, orc):
    nx, ny, nsf = 256, 128, 6
    t = synth.blob_target(nx, ny, 9)
    phi = orc.lut_phases(10007, 1)
    ref = orc.ospr(t, nsf, phi, 10007, 0)
    bits = torch.from_numpy(ref["bits"].view(np.int32)).cuda()
    nm = holo.reconstruct_nmse(bits, 2, nx, ny, nsf, torch.from_numpy(t).cuda())
    np.testing.assert_allclose(nm, ref["nmse2"], rtol=NMSE_RTOL)
    # 8-level codes
    codes = np.random.default_rng(1).integers(0, 8, (2, ny, nx), dtype=np.uint8)
    recon = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    nm8 = holo.reconstruct_nmse(torch.from_numpy(codes).cuda(), 8, nx, ny, 2, torch.from_numpy(t).cuda(), recon)
    iv = orc.reconstruct(codes.reshape(2, -1), 8, nx, ny, 2)
    np.testing.assert_allclose(nm8, orc.nmse_pair(iv, t), rtol=NMSE_RTOL)
    assert _rel_l2(recon.cpu().numpy().astype(np.float64), iv) < 1e-5


def _gs_case(holo, orc, nx, ny, n_iter, n_lut, seed):
    print(f"gs {nx}x{ny} iters={n_iter} lut={n_lut}", flush=True)
    t = synth.blob_target(nx, ny, seed)
    lut = holo.Lut(n_lut, 1)
    r = holo.gs_iterate(torch.from_numpy(t).cuda(), n_iter, lut, 0, want_err=True)
    phi = orc.lut_phases(n_lut, 1)
    init = orc.lut_phasor_field(phi, n_lut, 0, 0, nx, ny)
    ref = orc.gs(t, n_iter, init)
    assert r["cursor"] == nx * ny
    np.testing.assert_allclose(r["nmse"], ref["nmse"], rtol=NMSE_RTOL)
    np.testing.assert_allclose(r["err"], ref["err"], rtol=1e-3)
    return t, r, ref


# Error model of a 50-iteration GS trajectory.  GS is sensitive to its
# starting point: the FP64 oracle itself, with its seed phases perturbed by
# GS_EPS = 2^-22 (about the relative rounding error of one FP32 transform of
# 1024 points, log2(N)/2 * 2^-24), ends 50 iterations later with replay fields
# 0.5-1% (512^2) and 2.5-3.5% (1024^2) apart in relative L2, as many 8-level
# codes changed, and per-iteration NMSE up to ~3e-4 relative apart; an
# independent FP32 FFT (pocketfft) lands in the same range.  An FP32 run rounds
# at every iteration, not once, so its trajectory cannot match the FP64 one to
# 1e-4 after many iterations, whatever its arithmetic.  The bars therefore are:
#   * iterations 1..10 from the LUT seed, where the spread is still below 3e-5:
#     NMSE 1e-4 and amplitude error 1e-3 relative;
#   * every later iteration checked from the GPU's own state: the oracle
#     restarts from the GPU's field every 10 iterations and both run 10 more
#     (NMSE 1e-4, amplitude error 1e-3) -- this checks each iteration's
#     arithmetic independently of the trajectory's sensitivity;
#   * the free 50-iteration run against the FP64 envelope measured here (two
#     perturbation seeds): field and code mismatch within 2x, per-iteration
#     NMSE within 5x (the envelope perturbs once, the GPU every iteration);
#   * the replay NMSE of the GPU's own codes against the oracle's replay of
#     those codes: 1e-4 (exact given the codes).
GS_EPS = 2.0 ** -22
GS_WINDOW = 10


def _gs_envelope(orc, t, init, ref, n_iter, seeds=(100, 101)):
    env = {"field": 0.0, "codes": 0.0, "nmse": 0.0}
    for sd in seeds:
        rng = np.random.default_rng(sd)
        p = init * np.exp(1j * GS_EPS * rng.standard_normal(init.shape))
        r = orc.gs(t, n_iter, p)
        env["field"] = max(env["field"], _rel_l2(r["field"], ref["field"]))
        env["codes"] = max(env["codes"], float(np.mean(r["codes"] != ref["codes"])))
        env["nmse"] = max(env["nmse"], float(np.max(np.abs(r["nmse"] - ref["nmse"]) / ref["nmse"])))
    return env


@pytest.mark.parametrize("n,plan", [(512, None), (1024, [4, 1, 0, 0, 0, 0, 8]), (1024, [0, 0, 0, 0, -1, 0, 16])])
def test_gs_50_iterations(holo, orc, n, plan):
    # n^2, 50 iterations, 4096-entry LUT seed, 8 levels at the end; 1024^2
    # under the benchmark's tuned plan and with 16 points per thread
    n_iter = 50
    if plan is not None:
        holo.plan_set(holo.PLAN_GS, n, n, 1, plan)
    try:
        print(f"gs {n}x{n} x{n_iter} plan {plan}", flush=True)
        t = synth.blob_target(n, n, synth.SEED_GS_512)
        tt = torch.from_numpy(t).cuda()
        lut = holo.Lut(4096, 1)
        init = orc.lut_phasor_field(orc.lut_phases(4096, 1), 4096, 0, 0, n, n)
        r = holo.gs_iterate(tt, n_iter, lut, 0, want_err=True)
        ref = orc.gs(t, n_iter, init)
        assert r["cursor"] == n * n
        head = slice(0, GS_WINDOW)
        np.testing.assert_allclose(r["nmse"][head], ref["nmse"][head], rtol=1e-4)
        np.testing.assert_allclose(r["err"][head], ref["err"][head], rtol=1e-3)
        # windows from the GPU's own state
        f = holo.gs_iterate(tt, GS_WINDOW, lut, 0)["field"]
        for k0 in range(GS_WINDOW, n_iter, GS_WINDOW):
            print(f"gs {n}x{n} window from iteration {k0}", flush=True)
            state = f.cpu().numpy().astype(np.complex128)
            w = holo.gs_iterate(tt, GS_WINDOW, None, 0, init_phasor=f.clone(), want_err=True)
            wr = orc.gs(t, GS_WINDOW, state)
            np.testing.assert_allclose(w["nmse"], wr["nmse"], rtol=1e-4)
            np.testing.assert_allclose(w["err"], wr["err"], rtol=1e-3)
            f = w["field"]
        # the free run against the FP64 envelope
        env = _gs_envelope(orc, t, init, ref, n_iter)
        fld = _rel_l2(r["field"].cpu().numpy(), ref["field"])
        codes = r["codes"].cpu().numpy()
        mism = float(np.mean(codes != ref["codes"]))
        dn = float(np.max(np.abs(r["nmse"] - ref["nmse"]) / ref["nmse"]))
        print(f"gs {n}x{n}: field {fld:.2e} (envelope {env['field']:.2e}), codes {mism:.2e} "
              f"({env['codes']:.2e}), NMSE {dn:.2e} ({env['nmse']:.2e})", flush=True)
        assert fld < 2 * env["field"]
        assert mism < 2 * env["codes"]
        assert dn < 5 * env["nmse"]
        own = orc.reconstruct(codes[None], 8, n, n, 1)
        np.testing.assert_allclose(r["nmse_final2"], orc.nmse_pair(own, t), rtol=NMSE_RTOL)
    finally:
        if plan is not None:
            holo.plan_set(holo.PLAN_GS, n, n, 1, holo.DEFAULT_PLAN)


def test_gs_quantiser_exact_after_one_iteration(holo, orc):
    # After one iteration H_1 = F^{-1}{T * phasor} differs from FP64 by FP32
    # rounding only: codes must agree except within 1e-4 rad of a boundary.
    nx, ny = 256, 128
    t = synth.blob_target(nx, ny, 8)
    lut = holo.Lut(10007, 1)
    r = holo.gs_iterate(torch.from_numpy(t).cuda(), 1, lut, 0)
    init = orc.lut_phasor_field(orc.lut_phases(10007, 1), 10007, 0, 0, nx, ny)
    ref = orc.gs(t, 1, init)
    h1 = np.fft.ifft2(t.astype(np.float64) * init, norm="ortho")
    th = np.mod(np.angle(h1), 2 * np.pi)
    dist = np.abs(np.mod(th * 8 / (2 * np.pi), 1.0) - 0.5) * (2 * np.pi / 8)
    decided = (dist > 1e-4) & (np.abs(h1) > 1e-6)
    got = r["codes"].cpu().numpy()
    assert np.array_equal(got[decided], ref["codes"][decided])
    assert decided.mean() > 0.99


@pytest.mark.parametrize("nx,ny", [(16, 64), (128, 32), (1024, 1024)])
def test_gs_other_sizes(holo, orc, nx, ny):
    _gs_case(holo, orc, nx, ny, 6, 10007, 4)


@pytest.mark.parametrize("pts", [4, 8, 16])
@pytest.mark.parametrize("nx,ny", [(1024, 512), (64, 2048), (256, 16)])
def test_gs_points_per_thread(holo, orc, pts, nx, ny):
    # every points-per-thread factorisation of the GS transforms meets the
    # same oracle bar (plans are restored afterwards)
    holo.plan_set(holo.PLAN_GS, nx, ny, 1, [0, 0, 0, 0, -1, 0, pts])
    try:
        _gs_case(holo, orc, nx, ny, 5, 10007, 6)
    finally:
        holo.plan_set(holo.PLAN_GS, nx, ny, 1, holo.DEFAULT_PLAN)


def test_gs_fixed_point_and_resume(holo, orc):
    nx, ny = 64, 32
    rng = np.random.default_rng(3)
    hs = np.exp(1j * rng.uniform(0, 2 * np.pi, (ny, nx)))
    F = np.fft.fft2(hs, norm="ortho")
    t = torch.from_numpy(np.abs(F).astype(np.float32)).cuda()
    init = torch.from_numpy((F / np.abs(F)).astype(np.complex64)).cuda()
    r = holo.gs_iterate(t, 1, None, 0, init_phasor=init)
    assert r["nmse"][0] < 1e-8
    # resume: 3 iterations == 2, then 1 more seeded with the returned field
    tb = torch.from_numpy(synth.blob_target(nx, ny, 2)).cuda()
    lut = holo.Lut(101, 1)
    a = holo.gs_iterate(tb, 3, lut, 0)
    b = holo.gs_iterate(tb, 2, lut, 0)
    c = holo.gs_iterate(tb, 1, None, 0, init_phasor=b["field"].clone())
    np.testing.assert_allclose(c["nmse"][0], a["nmse"][2], rtol=1e-5)


def test_autotuned_plan_reproduces_default(holo):
    # the autotuner only keeps plans whose holograms equal the default plan's;
    # check the chosen plan end to end, and the plan save/load round trip
    import os
    import tempfile
    nx, ny, nsf = 256, 128, 6
    t = torch.from_numpy(synth.blob_target(nx, ny, 31)).cuda()
    lut = holo.Lut(10007, 1)
    holo.plan_set(holo.PLAN_OSPR, nx, ny, nsf, holo.DEFAULT_PLAN)
    b0, nm0, _ = holo.ospr_generate(t, nsf, lut, 5)
    chosen = holo.autotune_ospr(t, nsf, lut, reps=2)
    assert holo.plan_get(holo.PLAN_OSPR, nx, ny, nsf) == chosen
    b1, nm1, _ = holo.ospr_generate(t, nsf, lut, 5)
    assert torch.equal(b0, b1)
    np.testing.assert_allclose(nm1, nm0, rtol=1e-6)
    gchosen = holo.autotune_gs(t, lut, reps=2)
    path = os.path.join(tempfile.mkdtemp(), "plans.json")
    holo.plan_save(path)
    holo.plan_set(holo.PLAN_GS, nx, ny, 1, holo.DEFAULT_PLAN)
    holo.plan_load(path)
    assert holo.plan_get(holo.PLAN_GS, nx, ny, 1) == gchosen


def test_gs_graph_replay_matches_eager(holo):
    # GS calls are captured into a HIP graph on non-default streams and
    # replayed; every replay, with other eager work in between, must equal
    # the directly launched result.
    nx, ny = 256, 256
    t = torch.from_numpy(synth.blob_target(nx, ny, 17)).cuda()
    lut = holo.Lut(4096, 1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        holo.set_graphs(False)
        ref = holo.gs_iterate(t, 12, lut, 0)
        ref_codes = ref["codes"].clone()
        holo.set_graphs(True)
        field = torch.empty((ny, nx), dtype=torch.complex64, device="cuda")
        codes = torch.empty((ny, nx), dtype=torch.uint8, device="cuda")
        for rep in range(4):
            r = holo.gs_iterate(t, 12, lut, 0, field=field, codes=codes)
            np.testing.assert_array_equal(r["nmse"], ref["nmse"])
            assert torch.equal(codes, ref_codes)
            holo.ospr_generate(t, 3, lut, rep)        # eager work between replays
            torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["table", "prng", "mseq"])
def test_gs_graph_serves_every_cursor(holo, kind):
    # one captured GS graph per frame shape: the pool start is a device word
    # written before each replay, so successive frames (cursor += N, which a
    # 10007-entry pool sees at a new offset every time) replay the same graph
    # and still equal direct launches at their own cursors
    nx, ny = 256, 128
    t = torch.from_numpy(synth.blob_target(nx, ny, 18)).cuda()
    lut = {"table": lambda: holo.Lut(10007, 2), "prng": lambda: holo.Lut.prng(2),
           "mseq": lambda: holo.Lut.mseq(2)}[kind]()
    s = torch.cuda.Stream()
    cursors = [0, nx * ny, 5 * nx * ny + 17, (1 << 33) + 3]
    with torch.cuda.stream(s):
        holo.set_graphs(False)
        refs = [holo.gs_iterate(t, 6, lut, c) for c in cursors]
        refs = [(r["nmse"].copy(), r["codes"].clone(), r["cursor"]) for r in refs]
        holo.set_graphs(True)
        field = torch.empty((ny, nx), dtype=torch.complex64, device="cuda")
        codes = torch.empty((ny, nx), dtype=torch.uint8, device="cuda")
        for c, (nm, cd, cur) in zip(cursors, refs):
            r = holo.gs_iterate(t, 6, lut, c, field=field, codes=codes)
            np.testing.assert_array_equal(r["nmse"], nm)
            assert torch.equal(codes, cd) and r["cursor"] == cur
        torch.cuda.synchronize()


@pytest.mark.parametrize("plan", [
    [16, 2, 4, 0, 16, 5, 0],     # chunks of 5 over 13 sub-frames (ragged last chunk)
    [8, 1, 2, 0, 0, 4, 0],       # no padding
    [8, 8, 8, 4, 64, 0, 0],
])
def test_launch_plans_give_identical_holograms(holo, plan):
    nx, ny, nsf = 256, 512, 13
    t = torch.from_numpy(synth.blob_target(nx, ny, 41)).cuda()
    lut = holo.Lut(10007, 1)
    holo.plan_set(holo.PLAN_OSPR, nx, ny, nsf, holo.DEFAULT_PLAN)
    b0, nm0, c0 = holo.ospr_generate(t, nsf, lut, 77)
    holo.plan_set(holo.PLAN_OSPR, nx, ny, nsf, plan)
    b1, nm1, c1 = holo.ospr_generate(t, nsf, lut, 77)
    holo.plan_set(holo.PLAN_OSPR, nx, ny, nsf, holo.DEFAULT_PLAN)
    assert c0 == c1
    assert torch.equal(b0, b1)
    # the sub-frame grouping of the reconstruction pass changes only the FP32
    # summation order of the time average
    np.testing.assert_allclose(nm1, nm0, rtol=1e-6)


@pytest.mark.parametrize("pts,per_size", [(0, False), (8, False), (16, False), (8, True)])
def test_batched_equals_sequential_calls(holo, orc, pts, per_size):
    # a seeded batch of uneven frames in one (graph-replayed) call equals one
    # holo_ospr_generate call per frame with the cursor chained in batch order
    # (with the default plans, with every frame's plan at 8 or at 16 points
    # per thread, and with one plan per size stored for every sub-frame count)
    layout = synth.batch_layout(10, synth.SEED_BATCH, sizes=(64, 128, 256, 512), n_sf_range=(3, 9))
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_BATCH_TARGET0 + f)).cuda()
               for f, (n, _) in enumerate(layout)]
    nsfs = [k for _, k in layout]
    lut = holo.Lut(10007, 1)
    keys = sorted({(n, 0) for n, _ in layout}) if per_size else layout
    for n, k in keys:
        holo.plan_set(holo.PLAN_OSPR, n, n, k, [8, 2, 2, 0, 16, 2, pts] if per_size else [0, 0, 0, 0, -1, 0, pts])
    try:
        _batched_vs_sequential(holo, orc, layout, targets, nsfs, lut)
    finally:
        for n, k in keys:
            holo.plan_set(holo.PLAN_OSPR, n, n, k, holo.DEFAULT_PLAN)


def test_batched_grouped_ragged_frames(holo, orc):
    # many frames of one size with different sub-frame counts (ragged block
    # counts within one grouped launch), replay images on some frames only;
    # equal to single-frame calls, and one frame against the oracle
    nsfs = [1, 7, 3, 12, 2, 9, 5, 1, 4, 11, 6, 8]
    n = 128
    targets = [torch.from_numpy(synth.blob_target(n, n, 400 + f)).cuda() for f in range(len(nsfs))]
    recons = [torch.empty((n, n), dtype=torch.float32, device="cuda") if f % 3 == 0 else None
              for f in range(len(nsfs))]
    lut = holo.Lut(10007, 1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bits, nm, cur = holo.ospr_generate_batched(targets, nsfs, lut, 77, recons=recons)
        c = 77
        for f, (t, k) in enumerate(zip(targets, nsfs)):
            r1 = torch.empty_like(t) if recons[f] is not None else None
            b1, nm1, c = holo.ospr_generate(t, k, lut, c, recon=r1)
            assert torch.equal(bits[f], b1), f
            np.testing.assert_array_equal(nm[f], nm1)
            if r1 is not None:
                assert torch.equal(recons[f], r1), f
        assert cur == c
    torch.cuda.synchronize()
    f = 3
    ref = orc.ospr(targets[f].cpu().numpy(), nsfs[f], orc.lut_phases(10007, 1), 10007, 77 + n * n * sum(nsfs[:f]))
    _check_bits(holo, orc, bits[f], ref, n * n)
    np.testing.assert_allclose(nm[f], ref["nmse2"], rtol=NMSE_RTOL)


def test_batched_graph_follows_plan_changes(holo):
    # the same tensors through the batched call before and after a plan
    # change that only switches the points per thread: the second call must
    # run the new plan (its own graph), as the single-frame calls do
    layout = [(256, 5), (512, 3)]
    targets = [torch.from_numpy(synth.blob_target(n, n, 60 + f)).cuda() for f, (n, _) in enumerate(layout)]
    nsfs = [k for _, k in layout]
    lut = holo.Lut(10007, 1)
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            for pts in (16, 8, 16):
                for n, k in layout:
                    holo.plan_set(holo.PLAN_OSPR, n, n, k, [0, 0, 0, 0, -1, 0, pts])
                bits, nm, _ = holo.ospr_generate_batched(targets, nsfs, lut, 11)
                c = 11
                for f, (t, k) in enumerate(zip(targets, nsfs)):
                    b1, nm1, c = holo.ospr_generate(t, k, lut, c)
                    assert torch.equal(bits[f], b1), (pts, f)
                    np.testing.assert_array_equal(nm[f], nm1)
        torch.cuda.synchronize()
    finally:
        for n, k in layout:
            holo.plan_set(holo.PLAN_OSPR, n, n, k, holo.DEFAULT_PLAN)


def _batched_vs_sequential(holo, orc, layout, targets, nsfs, lut):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep, cursor in enumerate((123, 10 ** 12 + 7, 5)):
            bits, nm, cur = holo.ospr_generate_batched(targets, nsfs, lut, cursor)
            c = cursor
            for f, (t, k) in enumerate(zip(targets, nsfs)):
                b1, nm1, c = holo.ospr_generate(t, k, lut, c)
                assert torch.equal(bits[f], b1), (rep, f)
                np.testing.assert_array_equal(nm[f], nm1)
            assert cur == c
    torch.cuda.synchronize()
    # and one frame of the batch against the oracle
    f = 1
    n = layout[f][0]
    t = targets[f].cpu().numpy()
    ref = orc.ospr(t, nsfs[f], orc.lut_phases(10007, 1), 10007, 5 + sum(k * m * m for m, k in layout[:f]))
    _check_bits(holo, orc, bits[f], ref, n * n)
    np.testing.assert_allclose(nm[f], ref["nmse2"], rtol=NMSE_RTOL)


def test_lut_study_orders_pool_lengths(holo):
    # the LUT-length study on a small case: a pool no longer than the
    # sub-frame count (2 <= 24) is far worse than the paper's 10007, and the
    # non-repeating reference is the best of the three
    from paper_2004_04049_amd import lut_study
    targets = [torch.from_numpy(synth.blob_target(64, 64, synth.SEED_LUT_STUDY0 + i)).cuda() for i in range(2)]
    holo.set_graphs(False)
    try:
        res = lut_study.sweep(targets, 24, [2, 10007], 3)
    finally:
        holo.set_graphs(True)
    sm = lut_study.summarize(res, 64, 24)
    added = {r["n_lut"]: r["added_sym_pct"] for r in sm["rows"]}
    print(sm["nonrepeating"], added)
    assert added[2] > 10 * max(added[10007], 1.0)
    assert added[10007] > -5.0
