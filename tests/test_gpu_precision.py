"""BF16 / FP16 matrix-core DFT stages against the FP64 oracle.

Error model: every radix-16 stage rounds its input to the operand format once
(round to nearest, relative error at most u per real component, RMS below
u/sqrt(3); u = 2^-8 for BF16 with 8 significant bits, 2^-11 for FP16 with
11); the split DFT matrix (hi + lo), the FP32 accumulation and the FP32 last
radix-2/4/8 stage add O(u^2).  The stages are (scaled) unitary, so
independent stage errors add in quadrature: the relative L2 error of a 2D
transform with S radix-16 stages in all is below u * sqrt(S / 3).  Bound
used: u * sqrt(S).

Binarisation flips a pixel when the error of Re H exceeds |Re H|; with Re H
roughly Gaussian that is a fraction ~ sqrt(2/pi) * (relative error of H) of
the pixels.  Bound used: 2x the transform bound of the hologram path (K1 rows
+ K2 columns).  NMSE moves by far less than its own value: bound 2e-2
relative (BF16), 5e-3 (FP16)."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

U = {1: 2.0 ** -8, 2: 2.0 ** -11}
NAME = {1: "bf16", 2: "fp16"}
NMSE_TOL = {1: 2e-2, 2: 5e-3}


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    return h


def _stages(n):
    """Radix-16 stages of a length-n transform (the ones that round)."""
    return int(math.log2(n)) // 4


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("nx,ny", [(256, 256), (512, 1024), (2048, 256), (256, 2048), (1024, 1024)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft2_precision_error(holo, orc, prec, nx, ny, sign):
    rng = np.random.default_rng(nx + 3 * ny + prec)
    f = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    print(f"fft2 {NAME[prec]} {nx}x{ny} sign {sign}", flush=True)
    got = holo.fft2(torch.from_numpy(f).cuda(), sign, precision=prec).cpu().numpy()
    want = orc.fft2(f.astype(np.complex128), sign)
    s = _stages(nx) + _stages(ny)
    err = _rel_l2(got, want)
    bound = U[prec] * math.sqrt(s)
    print(f"  rel L2 {err:.3e} (model {U[prec] * math.sqrt(s / 3):.3e}, bound {bound:.3e})")
    assert err < bound
    # the matrix-core path is not a copy of the FP32 one
    assert err > 1e-6


def test_fft2_precision_impulse_and_constant(holo):
    """An impulse transforms to a constant and back; exact DFT-matrix entries
    (0, +-1) must hold through the split operands."""
    n = 256
    x = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    x[0, 0] = 1.0
    for prec in (1, 2):
        y = holo.fft2(x, -1, precision=prec).cpu().numpy()
        np.testing.assert_allclose(y, np.full((n, n), 1.0 / n), rtol=0, atol=U[prec] / n)
        z = holo.fft2(torch.from_numpy(y).cuda(), 1, precision=prec).cpu().numpy()
        e = np.zeros((n, n))
        e[0, 0] = 1.0
        np.testing.assert_allclose(z, e, atol=2 * U[prec])


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("nx,ny,nsf,n_lut", [(256, 256, 6, 10007), (1024, 1024, 4, 65536), (2048, 512, 3, 10007)])
def test_ospr_precision_vs_oracle(holo, orc, prec, nx, ny, nsf, n_lut):
    print(f"ospr {NAME[prec]} {nx}x{ny} nsf={nsf} lut={n_lut}", flush=True)
    target = synth.blob_target(nx, ny, 31)
    lut = holo.Lut(n_lut, 1)
    t = torch.from_numpy(target).cuda()
    recon = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    bits, nm, _ = holo.ospr_generate(t, nsf, lut, 5, recon=recon, precision=prec)
    ref = orc.ospr(target, nsf, orc.lut_phases(n_lut, 1), n_lut, 5)
    got = holo.unpack_bits(bits, nx * ny)
    want = orc.unpack_bits(ref["bits"], nx * ny)
    mism = float(np.mean(got != want))
    s = _stages(nx) + _stages(ny)
    bound = 2 * U[prec] * math.sqrt(s)
    nrel = abs(nm[0] - ref["nmse2"][0]) / ref["nmse2"][0]
    own = orc.reconstruct(bits.cpu().numpy().view(np.uint32), 2, nx, ny, nsf)
    rerr = _rel_l2(recon.cpu().numpy().astype(np.float64), own)
    print(f"  bit mismatch {mism:.2e} (bound {bound:.2e}); NMSE {nm[0]:.6f} vs {ref['nmse2'][0]:.6f} "
          f"(rel {nrel:.2e}); replay of own bits rel L2 {rerr:.2e}")
    assert 0 < mism < bound
    assert nrel < NMSE_TOL[prec]
    assert abs(nm[1] - ref["nmse2"][1]) / ref["nmse2"][1] < NMSE_TOL[prec]
    # the replay pass (reconstruction transforms on the matrix cores too)
    assert rerr < U[prec] * math.sqrt(s)


@pytest.mark.parametrize("prec", [1, 2])
def test_batched_precision_matches_single_frames(holo, prec):
    sizes = [(256, 8), (1024, 5), (512, 12), (2048, 3), (256, 24)]
    targets = [torch.from_numpy(synth.blob_target(n, n, 1000 + f)).cuda() for f, (n, _) in enumerate(sizes)]
    nsfs = [k for _, k in sizes]
    lut = holo.Lut(10007, 1)
    bits, nm, cur = holo.ospr_generate_batched(targets, nsfs, lut, 77, precision=prec)
    torch.cuda.synchronize()
    c = 77
    for f, (n, k) in enumerate(sizes):
        b1, nm1, c = holo.ospr_generate(targets[f], k, lut, c, precision=prec)
        assert torch.equal(bits[f], b1), f"frame {f}"
        np.testing.assert_allclose(nm[f], nm1, rtol=1e-12)
    assert cur == c


def test_benchmark_batch_per_frame_vs_oracle(holo, orc):
    """The benchmark's 64-frame batch (sizes and sub-frame counts from seed 14,
    targets 1000+f, LUT 10007 chained from cursor 0) in FP32, BF16 and FP16;
    for the first frame of each size (a stated subset: the FP64 oracle at
    2048^2 costs seconds per sub-frame) the per-frame errors against the
    oracle: bit mismatch, relative NMSE difference, relative L2 error of the
    time-averaged replay.  FP32: bit-exact outside the tie band, NMSE 1e-4.
    BF16/FP16: the bounds of the single-frame test above."""
    layout = synth.batch_layout(64, synth.SEED_BATCH)
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_BATCH_TARGET0 + f)).cuda()
               for f, (n, _) in enumerate(layout)]
    nsfs = [k for _, k in layout]
    offs = np.cumsum([0] + [k * n * n for n, k in layout])
    first = {}
    for f, (n, _) in enumerate(layout):
        first.setdefault(n, f)
    lut = holo.Lut(10007, 1)
    phi = orc.lut_phases(10007, 1)
    runs = {}
    for prec in (0, 1, 2):
        recons = [torch.empty_like(t) for t in targets]
        print(f"batch of 64, precision {prec}", flush=True)
        bits, nm, _ = holo.ospr_generate_batched(targets, nsfs, lut, 0, recons=recons, precision=prec)
        torch.cuda.synchronize()
        runs[prec] = ([bits[f].cpu().numpy() for f in first.values()], np.asarray(nm),
                      [recons[f].cpu().numpy() for f in first.values()])
    print("frame size n_sf | precision: bit mismatch, NMSE rel, replay rel L2 (vs FP64 oracle)")
    for i, (n, f) in enumerate(sorted(first.items())):
        k = layout[f][1]
        t = targets[f].cpu().numpy()
        print(f"oracle frame {f} ({n}x{n}, {k} sub-frames)", flush=True)
        ref = orc.ospr(t, k, phi, 10007, int(offs[f]))
        want = orc.unpack_bits(ref["bits"], n * n)
        decided = np.abs(ref["reH"].reshape(k, -1)) >= 1e-5
        line = f"{f:3d} {n:4d} {k:2d} |"
        for prec in (0, 1, 2):
            j = list(first.values()).index(f)
            got = holo.unpack_bits(torch.from_numpy(runs[prec][0][j]).cuda(), n * n)
            mism = float(np.mean(got != want))
            nrel = abs(runs[prec][1][f, 0] - ref["nmse2"][0]) / ref["nmse2"][0]
            rrel = _rel_l2(runs[prec][2][j].astype(np.float64), ref["ibar"])
            line += f" {NAME.get(prec, 'fp32')}: {mism:.2e} {nrel:.1e} {rrel:.1e} |"
            if prec == 0:
                assert not np.any((got != want) & decided)
                assert nrel < 1e-4
            else:
                s = 2 * _stages(n)
                assert mism < 2 * U[prec] * math.sqrt(s)
                assert nrel < NMSE_TOL[prec]
        print(line, flush=True)
