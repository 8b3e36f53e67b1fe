"""Pins for the oracle's quantisers, OSPR, reconstruction, NMSE and GS, from
the paper's definitions (Section 2 nearest-value rule, Section 3 time
averaging), closed forms and invariants.  CPU only."""
import numpy as np
import pytest

import synth


# ---------------------------------------------------------------- quantisers
def test_binarise_is_nearest_of_plus_minus_one(orc):
    rng = np.random.default_rng(0)
    for re, im in rng.standard_normal((500, 2)):
        h = complex(re, im)
        nearest = 1 if abs(h - (-1)) < abs(h - 1) else 0
        assert orc.binarise(re) == nearest
    assert orc.binarise(0.0) == 0 and orc.binarise(-0.0) == 0
    assert orc.binarise(-1e-300) == 1


def test_quant8_is_nearest_of_eight_phasors(orc):
    rng = np.random.default_rng(1)
    levels = np.exp(2j * np.pi * np.arange(8) / 8)
    for re, im in rng.standard_normal((2000, 2)):
        h = complex(re, im)
        d = abs(h - levels)
        if np.sort(d)[1] - d.min() < 1e-9:
            continue
        assert orc.quant8(re, im) == int(np.argmin(d))
    assert orc.quant8(0.0, 0.0) == 0
    assert orc.quant8(-1.0, -1e-12) == 4


# ---------------------------------------------------------------- NMSE
def test_nmse_worked_values(orc):
    assert orc.nmse([1, 1], [1, 0]) == pytest.approx(0.5, abs=1e-15)
    assert orc.nmse([1, 0], [0, 1]) == pytest.approx(1.0, abs=1e-15)
    assert orc.nmse_direct([1, 1], [1, 0]) == pytest.approx(0.5, abs=1e-15)


def test_nmse_properties(orc):
    rng = np.random.default_rng(2)
    w = rng.random(300)
    i = rng.random(300)
    assert orc.nmse(w, w) == pytest.approx(0.0, abs=1e-14)
    assert orc.nmse(7.5 * w, w) == pytest.approx(0.0, abs=1e-14)
    v = orc.nmse(i, w)
    assert 0.0 <= v <= 1.0
    assert v == pytest.approx(orc.nmse_direct(i, w), rel=1e-12)
    assert orc.nmse(3 * i, w) == pytest.approx(v, rel=1e-12)


# ---------------------------------------------------------------- reconstruction
def test_reconstruct_eight_level_map_is_a_plane_wave(orc):
    # Codes m = x mod 8 mean H'(x, y) = exp(+i*2*pi*x/8).  Under Eq. (1)
    # (forward kernel exp(-i*2*pi*u*x/nx)) that plane wave puts all of the
    # replay intensity N at (u, v) = (+nx/8, 0).  A conjugated code map
    # (exp(-i*2*pi*m/8)) would put it at u = -nx/8, a wrong step size at
    # another order: only the map exp(+i*2*pi*m/8) passes.
    for nx, ny in ((16, 8), (64, 16), (32, 32)):
        n = nx * ny
        x = np.tile(np.arange(nx), (ny, 1))
        codes = (x % 8).astype(np.uint8).reshape(1, n)
        iv = orc.reconstruct(codes, 8, nx, ny, 1)
        expect = np.zeros((ny, nx))
        expect[0, nx // 8] = n
        np.testing.assert_allclose(iv, expect, atol=1e-9 * n)
        # codes m = 2y mod 8: exp(+i*pi*y/2), all intensity at v = +ny/4
        y = np.tile(np.arange(ny)[:, None], (1, nx))
        codes = ((2 * y) % 8).astype(np.uint8).reshape(1, n)
        iv = orc.reconstruct(codes, 8, nx, ny, 1)
        expect = np.zeros((ny, nx))
        expect[ny // 4, 0] = n
        np.testing.assert_allclose(iv, expect, atol=1e-9 * n)


def test_reconstruct_flat_hologram_is_a_delta(orc):
    nx, ny = 16, 8
    n = nx * ny
    i2 = orc.reconstruct(np.zeros((1, (n + 31) // 32), np.uint32), 2, nx, ny, 1)
    i8 = orc.reconstruct(np.full((1, n), 3, np.uint8), 8, nx, ny, 1)
    for iv in (i2, i8):
        expect = np.zeros((ny, nx))
        expect[0, 0] = n
        np.testing.assert_allclose(iv, expect, atol=1e-9)


# ---------------------------------------------------------------- OSPR
def _ospr(orc, t, nsf, L, seed=1, cursor=0):
    phi = orc.lut_phases(L, seed) if L else np.zeros(0)
    return orc.ospr(t, nsf, phi, L, cursor)


def test_ospr_square_wave_grating(orc):
    # A single-pixel target at (u0, 0) with one LUT phase pi/P gives a tilted
    # plane wave; binarising its real part gives a +-1 square wave of period
    # P = nx/u0 along x.  The power in each first order is then the Fourier
    # coefficient of that square wave, |(1/P) sum_n s_n e^{-2 pi i n/P}|^2 * N,
    # which tends to 4/pi^2 as P grows (the classic binary grating).
    nx, ny = 64, 16
    n = nx * ny
    for u0 in (1, 2, 4, 8):
        P = nx // u0
        t = np.zeros((ny, nx), np.float32)
        t[0, u0] = 1.0
        r = orc.ospr(t, 1, np.array([np.pi / P]), 1, 0)
        s = np.where(np.cos(2 * np.pi * (np.arange(P) + 0.5) / P) < 0, -1.0, 1.0)
        c1 = abs(np.sum(s * np.exp(-2j * np.pi * np.arange(P) / P)) / P) ** 2
        ib = r["ibar"]
        assert ib[0, u0] == pytest.approx(c1 * n, rel=1e-10)
        assert ib[0, (-u0) % nx] == pytest.approx(c1 * n, rel=1e-10)
        assert ib.sum() == pytest.approx(n, rel=1e-12)
        assert np.all(ib[1:, :] < 1e-9)  # constant along y: only the v = 0 row lights up


def test_ospr_first_order_efficiency_limit(orc):
    nx, ny = 256, 4
    t = np.zeros((ny, nx), np.float32)
    t[0, 1] = 1.0
    r = orc.ospr(t, 1, np.array([np.pi / nx]), 1, 0)
    assert r["ibar"][0, 1] / (nx * ny) == pytest.approx(4 / np.pi ** 2, rel=1e-3)


def test_ospr_parseval_and_centro_symmetry(orc):
    nx, ny = 32, 16
    t = synth.blob_target(nx, ny, 5)
    r = _ospr(orc, t, 6, 101)
    ib = r["ibar"]
    assert ib.sum() == pytest.approx(nx * ny, rel=1e-12)
    mirror = np.roll(np.roll(ib[::-1, ::-1], 1, axis=0), 1, axis=1)
    np.testing.assert_allclose(ib, mirror, rtol=1e-10, atol=1e-10)


def test_ospr_matches_brute_force_steps(orc):
    # tiny non-square case rebuilt step by step from the brute-force DFT
    nx, ny, nsf, L, c = 8, 4, 3, 7, 5
    n = nx * ny
    t = synth.uniform_target(nx, ny, 11)
    phi = orc.lut_phases(L, 1)
    r = orc.ospr(t, nsf, phi, L, c)
    ib = np.zeros((ny, nx))
    for k in range(nsf):
        ph = np.array([phi[(c + k * n + p) % L] for p in range(n)]).reshape(ny, nx)
        h = orc.dft2_brute(t.astype(np.float64) * np.exp(1j * ph), +1)
        np.testing.assert_allclose(r["reH"][k], h.real, atol=1e-12)
        b = (h.real < 0).astype(np.uint8).ravel()
        assert np.array_equal(orc.unpack_bits(r["bits"][k], n), b)
        ib += abs(orc.dft2_brute((1.0 - 2.0 * b).reshape(ny, nx), -1)) ** 2 / nsf
    np.testing.assert_allclose(r["ibar"], ib, atol=1e-10)
    w = t.astype(np.float64) ** 2
    assert r["nmse2"][0] == pytest.approx(orc.nmse(ib, w), rel=1e-10)
    ws = 0.5 * (w + np.roll(np.roll(w[::-1, ::-1], 1, 0), 1, 1))
    assert r["nmse2"][1] == pytest.approx(orc.nmse(ib, ws), rel=1e-10)


def test_ospr_divisor_lut_gives_identical_subframes(orc):
    # I2 at the level of holograms: N_LUT | N => every sub-frame identical and
    # the average equals one sub-frame's intensity.
    nx = ny = 64
    t = synth.uniform_target(nx, ny, 11)
    r = _ospr(orc, t, 8, 256)
    assert all(np.array_equal(r["bits"][k], r["bits"][0]) for k in range(8))
    one = orc.reconstruct(r["bits"][:1], 2, nx, ny, 1)
    np.testing.assert_allclose(r["ibar"], one, rtol=1e-12, atol=1e-9)


def test_ospr_more_subframes_lower_error(orc):
    # Section 3: independent sub-frames averaged in time lower the error.
    nx = ny = 64
    t = synth.blob_target(nx, ny, 12)
    e1 = _ospr(orc, t, 1, 10007)["nmse2"][1]
    e8 = _ospr(orc, t, 8, 10007)["nmse2"][1]
    assert e8 < 0.6 * e1
    # and a LUT dividing the frame gives no benefit from averaging
    d1 = _ospr(orc, t, 1, 256)["nmse2"][1]
    d8 = _ospr(orc, t, 8, 256)["nmse2"][1]
    assert d8 == pytest.approx(d1, rel=1e-9)


def test_ospr_flat_phase_and_chaining(orc):
    nx = ny = 16
    t = synth.blob_target(nx, ny, 3)
    a = _ospr(orc, t, 4, 0)
    assert all(np.array_equal(a["bits"][k], a["bits"][0]) for k in range(4))
    # one frame of 4 sub-frames == two frames of 2 with the cursor carried on
    phi = orc.lut_phases(37, 1)
    f = orc.ospr(t, 4, phi, 37, 10)
    g1 = orc.ospr(t, 2, phi, 37, 10)
    g2 = orc.ospr(t, 2, phi, 37, 10 + 2 * nx * ny)
    assert np.array_equal(f["bits"], np.concatenate([g1["bits"], g2["bits"]]))


# ---------------------------------------------------------------- GS
def test_gs_fixed_point(orc):
    # a phase-only H* and T = |F{H*}| with the init phase of F{H*}: the first
    # iteration returns H* itself and a zero error.
    nx, ny = 16, 8
    rng = np.random.default_rng(3)
    hs = np.exp(1j * rng.uniform(0, 2 * np.pi, (ny, nx)))
    F = np.fft.fft2(hs, norm="ortho")
    t = np.abs(F).astype(np.float32)
    init = F / np.abs(F)
    r = orc.gs(t, 2, init)
    assert r["nmse"][0] < 1e-12
    assert r["err"][0] < 1e-10


@pytest.mark.parametrize("scale", [3.0, 0.37])
def test_gs_amplitude_error_scale_at_scaled_fixed_point(orc, scale):
    # The amplitude error compares |R'| with Te = T*sqrt(N/sum T^2), the
    # target rescaled to the replay energy of a unit-modulus hologram
    # (Parseval: sum |R'|^2 = N).  With T = c*|F{H*}| for a phase-only H*
    # (sum T^2 = c^2 N) the first iteration returns H* again and |R'| =
    # |F{H*}| = T/c = Te, so E and NMSE vanish for every c.  A missing or
    # inverted square root, or a scale taken from the wrong sum, leaves
    # E = (1 - c^{+-1})^2 N or similar, far from zero.
    nx, ny = 16, 8
    n = nx * ny
    rng = np.random.default_rng(4)
    hs = np.exp(1j * rng.uniform(0, 2 * np.pi, (ny, nx)))
    F = np.fft.fft2(hs, norm="ortho")
    t = (scale * np.abs(F)).astype(np.float32)
    init = F / np.abs(F)
    r = orc.gs(t, 2, init)
    # T was rounded to FP32, so |R'| = T/c only to FP32 relative precision
    assert r["nmse"][0] < 1e-12
    assert r["err"][0] < 1e-10 * n
    # the same field scaled: E is measured in replay units, so it must not
    # grow with the target's scale
    assert r["err"][1] < 1e-10 * n


def test_gs_error_reduction_and_parseval(orc):
    nx, ny = 32, 32
    t = synth.blob_target(nx, ny, 13)
    phi = orc.lut_phases(97, 1)
    init = orc.lut_phasor_field(phi, 97, 0, 0, nx, ny)
    r = orc.gs(t, 30, init)
    e = r["err"]
    assert np.all(np.diff(e) <= 1e-12 * e[0])   # Fienup's error-reduction property
    assert r["nmse"][-1] < r["nmse"][0]
    assert np.sum(abs(r["field"]) ** 2) == pytest.approx(nx * ny, rel=1e-12)


def test_gs_codes_are_quantised_final_hologram(orc):
    nx, ny = 16, 16
    t = synth.blob_target(nx, ny, 7)
    phi = orc.lut_phases(31, 1)
    init = orc.lut_phasor_field(phi, 31, 0, 0, nx, ny)
    r = orc.gs(t, 5, init)
    # H_5 = F^{-1}{R_4}; R_4 = T * R'_4/|R'_4| -- rebuild it with numpy from the
    # previous run's replay field and quantise by brute force.
    r4 = orc.gs(t, 4, init)
    rp = r4["field"]
    h = np.fft.ifft2(t * rp / np.abs(rp), norm="ortho")
    lv = np.exp(2j * np.pi * np.arange(8) / 8)
    d = np.abs(h.ravel()[:, None] / np.abs(h.ravel()[:, None]) - lv[None, :])
    want = np.argmin(d, axis=1).reshape(ny, nx)
    assert np.array_equal(r["codes"], want)
    iv = orc.reconstruct(r["codes"][None], 8, nx, ny, 1)
    assert r["nmse_final2"][0] == pytest.approx(orc.nmse(iv, t.astype(float) ** 2), rel=1e-12)
