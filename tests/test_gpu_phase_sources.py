"""GPU parity of the phase sources (TABLE, 8-bit CODES, counter PRNG with
sine/cosine, M-sequence with code table) against the FP64 oracle.

Each source gives pool position i a phasor; the OSPR and GS kernels read
positions c + k*N + p exactly as with a table (Section 5, Fig. 3), so every
source is checked twice: its phasors (holo_phase_mask, the generation
kernels' own device code) against the oracle's phases, and whole OSPR / GS
frames against the oracle run on those phases.

Tolerances:
  * TABLE, CODES8, MSEQ phasors are FP64 cos/sin rounded to FP32 on the host:
    |error| <= 2^-24 per component; the M-sequence and 8-bit codes are exact
    integers and compared bit for bit;
  * PRNG phasors come from the GPU's FP32 sine/cosine of a 24-bit fraction of
    a turn (an exact FP32 argument); PRNG_PHASOR_TOL bounds their error at
    about four times the largest error measured over these cases (1.3e-7);
  * OSPR bits: bit-exact except pixels with |Re H_oracle| below the tie
    threshold (1e-5, which is above 4x the PRNG phasor bound); NMSE 1e-4
    relative.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

M31 = (1 << 31) - 1
PRNG_PHASOR_TOL = 5e-7
TIE = 1e-5


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    assert torch.cuda.is_available()
    return h


def _make(holo, kind, n_lut=10007, seed=3):
    if kind == "table":
        return holo.Lut(n_lut, seed)
    if kind == "codes8":
        return holo.Lut.codes(n_lut, seed)
    if kind == "prng":
        return holo.Lut.prng(seed)
    return holo.Lut.mseq(seed)


def _oracle_phases(orc, kind, cursor, n, n_lut=10007, seed=3):
    """Phases of pool positions cursor .. cursor+n-1 (oracle only)."""
    if kind == "table":
        return orc.lut_phases(n_lut, seed)[(cursor + np.arange(n)) % n_lut]
    if kind == "codes8":
        return orc.codes8_phases(n_lut, seed)[(cursor + np.arange(n)) % n_lut]
    if kind == "prng":
        return orc.prng_phases(seed, cursor, n)
    assert cursor + n < M31
    return orc.mseq_phases(seed, cursor, n)


def _codes(ph):
    return np.round(np.angle(ph) / (2 * np.pi) * 256).astype(np.int64) % 256


KINDS = ["table", "codes8", "prng", "mseq"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nx,ny,nsf,cursor", [(16, 16, 3, 0), (64, 32, 2, 12345), (1024, 16, 2, 99991),
                                              (2048, 16, 1, 7), (256, 2048, 1, 1 << 20)])
def test_phase_mask_matches_oracle(holo, orc, kind, nx, ny, nsf, cursor):
    print(f"phase mask {kind} {nx}x{ny} nsf={nsf} cursor={cursor}", flush=True)
    lut = _make(holo, kind)
    got = holo.phase_mask(lut, cursor, nx, ny, nsf).cpu().numpy().astype(np.complex128).ravel()
    phi = _oracle_phases(orc, kind, cursor, nsf * nx * ny)
    want = np.exp(1j * phi)
    err = np.abs(got - want).max()
    print(f"  max phasor error {err:.3e}", flush=True)
    if kind == "prng":
        assert err < PRNG_PHASOR_TOL
    else:
        assert err < 2 * 2.0 ** -24 * 1.5
    if kind in ("codes8", "mseq"):
        assert np.array_equal(_codes(got), np.round(phi / (2 * np.pi) * 256).astype(np.int64) % 256)


def test_mseq_period_and_prng_wrap(holo):
    # the M-sequence repeats after 2^31 - 1 positions (a primitive trinomial);
    # a mask that crosses the end of the period continues at its start
    lut = _make(holo, "mseq")
    a = holo.phase_mask(lut, 5, 256, 64, 2).cpu()
    b = holo.phase_mask(lut, 5 + M31, 256, 64, 2).cpu()
    assert torch.equal(a, b)
    c = holo.phase_mask(lut, M31 - 100, 256, 64, 1).cpu().reshape(-1)
    d = holo.phase_mask(lut, 0, 256, 64, 1).cpu().reshape(-1)
    assert torch.equal(c[100:], d[:-100])
    # the PRNG pool is unbounded: positions wrap only at 2^64
    p = _make(holo, "prng")
    e = holo.phase_mask(p, (1 << 64) - 64, 64, 16, 1).cpu().reshape(-1)
    f = holo.phase_mask(p, 0, 64, 16, 1).cpu().reshape(-1)
    assert torch.equal(e[64:], f[:-64])


def test_prng_pool_extends_the_table_of_its_seed(holo, orc):
    # same SplitMix64 outputs: a PRNG pool and a table of the same seed give
    # the same phases to within the 24-bit truncation and FP32 sine/cosine
    p = holo.phase_mask(_make(holo, "prng", seed=11), 0, 64, 64, 1).cpu().numpy().ravel()
    t = holo.phase_mask(_make(holo, "table", n_lut=4096, seed=11), 0, 64, 64, 1).cpu().numpy().ravel()
    assert np.abs(p - t).max() < 2 * np.pi * 2.0 ** -24 + PRNG_PHASOR_TOL


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nx,ny,nsf,cursor", [(64, 64, 8, 0), (256, 128, 3, 4242), (128, 1024, 2, 77)])
def test_ospr_per_source_matches_oracle(holo, orc, kind, nx, ny, nsf, cursor):
    print(f"ospr {kind} {nx}x{ny} nsf={nsf} cursor={cursor}", flush=True)
    target = synth.blob_target(nx, ny, 4100 + nx + ny)
    lut = _make(holo, kind)
    t = torch.from_numpy(target).cuda()
    recon = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    bits, nm, cur = holo.ospr_generate(t, nsf, lut, cursor, recon=recon)
    torch.cuda.synchronize()
    assert cur == cursor + nsf * nx * ny
    n = nx * ny
    phi = _oracle_phases(orc, kind, cursor, nsf * n)
    ref = orc.ospr(target, nsf, phi, nsf * n, 0)
    got = holo.unpack_bits(bits, n)
    want = orc.unpack_bits(ref["bits"], n)
    tie = TIE if kind != "prng" else max(TIE, 4 * PRNG_PHASOR_TOL)
    decided = np.abs(ref["reH"].reshape(nsf, -1)) >= tie
    assert int(((got != want) & decided).sum()) == 0
    np.testing.assert_allclose(nm, ref["nmse2"], rtol=1e-4)
    own = orc.reconstruct(bits.cpu().numpy().view(np.uint32), 2, nx, ny, nsf)
    np.testing.assert_allclose(nm, orc.nmse_pair(own, target), rtol=1e-4)


@pytest.mark.parametrize("kind", KINDS)
def test_batched_per_source_equals_single_calls(holo, kind):
    print(f"batched {kind}", flush=True)
    lut = _make(holo, kind)
    sizes = [(64, 64, 4), (256, 128, 3), (128, 256, 2), (64, 64, 5)]
    targets = [torch.from_numpy(synth.blob_target(nx, ny, 4300 + i)).cuda() for i, (nx, ny, _) in enumerate(sizes)]
    cursor0 = 123456
    single = []
    cur = cursor0
    for (nx, ny, nsf), t in zip(sizes, targets):
        bits, nm, cur = holo.ospr_generate(t, nsf, lut, cur)
        single.append((bits.cpu(), nm))
    for rep in range(2):      # second call replays the captured graph with a new cursor
        c0 = cursor0 + rep * 1000003
        bits_b, nms, cur_b = holo.ospr_generate_batched(targets, [s[2] for s in sizes], lut, c0)
        assert cur_b == c0 + sum(nx * ny * nsf for nx, ny, nsf in sizes)
        if rep == 0:
            for (b1, nm1), b2, nm2 in zip(single, bits_b, nms):
                assert torch.equal(b1, b2.cpu())
                np.testing.assert_array_equal(nm1, nm2)
    # the replay with the moved cursor equals single calls from that cursor
    cur = cursor0 + 1000003
    for ((nx, ny, nsf), t), b2 in zip(zip(sizes, targets), bits_b):
        bits, _, cur = holo.ospr_generate(t, nsf, lut, cur)
        assert torch.equal(bits.cpu(), b2.cpu())


@pytest.mark.parametrize("kind", KINDS)
def test_gs_seeded_per_source_matches_oracle(holo, orc, kind):
    nx, ny, n_iter, cursor = 256, 128, 6, 31337
    print(f"gs {kind} {nx}x{ny}", flush=True)
    target = synth.blob_target(nx, ny, 4400)
    lut = _make(holo, kind)
    t = torch.from_numpy(target).cuda()
    r = holo.gs_iterate(t, n_iter, lut, cursor)
    nm = r["nmse"]
    assert r["cursor"] == cursor + nx * ny
    phi = _oracle_phases(orc, kind, cursor, nx * ny).reshape(ny, nx)
    ref = orc.gs(target, n_iter, np.exp(1j * phi))
    np.testing.assert_allclose(nm, ref["nmse"], rtol=1e-4)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("prec", [1, 2])
def test_sources_on_matrix_core_row_pass(holo, kind, prec):
    # the phase fetch is the same code in the BF16/FP16 row pass (its code
    # tables sit after the matrix-core LDS rows): same pool positions, so the
    # frame differs from the FP32 one only by the stage rounding (< 2u*sqrt(S))
    nx, ny, nsf, cursor = 256, 256, 4, 7777
    u = {1: 2.0 ** -8, 2: 2.0 ** -11}[prec]
    t = torch.from_numpy(synth.blob_target(nx, ny, 4500)).cuda()
    lut = _make(holo, kind)
    b32, nm32, c32 = holo.ospr_generate(t, nsf, lut, cursor)
    bl, nml, cl = holo.ospr_generate(t, nsf, lut, cursor, precision=prec)
    assert c32 == cl
    frac = float((holo.unpack_bits(b32, nx * ny) != holo.unpack_bits(bl, nx * ny)).mean())
    assert 0 < frac < 2 * u * np.sqrt(4)
    np.testing.assert_allclose(nml, nm32, rtol=2e-2)


@pytest.mark.parametrize("kind", ["prng", "mseq"])
@pytest.mark.parametrize("pts", [4, 8, 16])
def test_gs_seed_per_points_per_thread(holo, orc, kind, pts):
    # GS rows with 4/8/16 points per thread: thread strides 256/128/64 at
    # 1024 wide, i.e. the M-sequence's larger jump tables
    nx, ny, n_iter, cursor = 1024, 64, 3, 99
    target = synth.blob_target(nx, ny, 4600)
    lut = _make(holo, kind)
    holo.plan_set(holo.PLAN_GS, nx, ny, 1, [0, 0, 0, 0, -1, 0, pts])
    try:
        r = holo.gs_iterate(torch.from_numpy(target).cuda(), n_iter, lut, cursor)
    finally:
        holo.plan_set(holo.PLAN_GS, nx, ny, 1, [0, 0, 0, 0, -1, 0, 0])
    phi = _oracle_phases(orc, kind, cursor, nx * ny).reshape(ny, nx)
    ref = orc.gs(target, n_iter, np.exp(1j * phi))
    np.testing.assert_allclose(r["nmse"], ref["nmse"], rtol=1e-4)


def test_code_table_phases_bit_exact(holo, orc):
    # the host keeps the codes and derives FP64 phases 2*pi*q/256 on request
    lut = holo.Lut.codes(4099, 17)
    assert lut.kind == holo.SRC_CODES8 and lut.size == 4099
    assert np.array_equal(lut.phases(), orc.codes8_phases(4099, 17))
    with pytest.raises(holo.HoloError):
        holo.Lut.mseq(17).phases()
