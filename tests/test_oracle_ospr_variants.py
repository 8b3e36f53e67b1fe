"""Pins for the oracle's OSPR variants (not from the paper: two binary
sub-frames per randomised field, from Re H and Im H; eight phase levels per
sub-frame).  Each is tied to the pinned binary OSPR oracle or to brute force.
CPU only."""
import numpy as np

import synth


def _phases(orc, n_lut, seed=2):
    return orc.lut_phases(n_lut, seed)


def test_pairs_are_the_binary_frames_of_re_and_im(orc):
    nx, ny, n_sf = 32, 16, 6
    t = synth.blob_target(nx, ny, 71)
    phi = _phases(orc, 1009)
    n = nx * ny
    pair = orc.ospr_mode(t, n_sf, phi, 1009, 77, 1)
    # the Re sub-frames are the binary frame's sub-frames drawn from the same
    # pool positions (field j reads the pool at sub-frame index j)
    re = orc.ospr(t, n_sf // 2, phi, 1009, 77)
    # Im H = Re(H * exp(-i pi/2)) and H is linear in R: the Im sub-frames are
    # the binary frame of the phases shifted by -pi/2
    im = orc.ospr(t, n_sf // 2, phi - np.pi / 2, 1009, 77)
    got = orc.unpack_bits(pair["holo"], n)
    want_re = orc.unpack_bits(re["bits"], n)
    want_im = orc.unpack_bits(im["bits"], n)
    hv = pair["hval"].reshape(n_sf, -1)
    np.testing.assert_allclose(hv[0::2], re["reH"].reshape(n_sf // 2, -1), atol=1e-12)
    np.testing.assert_allclose(hv[1::2], im["reH"].reshape(n_sf // 2, -1), atol=1e-12)
    clear = np.abs(hv) > 1e-9
    assert np.array_equal(got[0::2][clear[0::2]], want_re[clear[0::2]])
    assert np.array_equal(got[1::2][clear[1::2]], want_im[clear[1::2]])
    # the time average is the mean of the two binary frames' averages
    np.testing.assert_allclose(pair["ibar"], 0.5 * (re["ibar"] + im["ibar"]), rtol=1e-9, atol=1e-12)


def test_pairs_replay_invariants(orc):
    nx, ny, n_sf = 64, 32, 4
    t = synth.blob_target(nx, ny, 72)
    phi = _phases(orc, 4099)
    r = orc.ospr_mode(t, n_sf, phi, 4099, 0, 1)
    ib = r["ibar"]
    # unitary transform of +-1 holograms: sum of each replay intensity = N
    assert abs(ib.sum() - nx * ny) < 1e-8 * nx * ny
    # binary holograms replay centro-symmetrically
    mirror = np.roll(np.roll(ib[::-1, ::-1], 1, axis=0), 1, axis=1)
    np.testing.assert_allclose(ib, mirror, rtol=1e-9, atol=1e-12)


def test_eight_level_codes_are_nearest_levels(orc):
    nx, ny, n_sf = 32, 32, 3
    t = synth.blob_target(nx, ny, 73)
    phi = _phases(orc, 2003)
    r = orc.ospr_mode(t, n_sf, phi, 2003, 5, 2)
    h = r["hval"]
    # brute force: the level exp(i*2*pi*m/8) closest to H/|H|
    lv = np.exp(2j * np.pi * np.arange(8) / 8)
    u = h / np.abs(h)
    dist = np.abs(u[..., None] - lv)
    want = np.argmin(dist, axis=-1)
    srt = np.sort(dist, axis=-1)
    clear = (srt[..., 1] - srt[..., 0]) > 1e-9
    assert np.array_equal(r["holo"][clear], want[clear])
    # the fields are the binary frame's H (same pool positions)
    ref = orc.ospr(t, n_sf, phi, 2003, 5)
    np.testing.assert_allclose(h.real, ref["reH"], atol=1e-12)
    # phase-only holograms of unit modulus: each replay sums to N
    assert abs(r["ibar"].sum() - nx * ny) < 1e-8 * nx * ny
    # and the average equals the replay of the codes, sub-frame by sub-frame
    np.testing.assert_allclose(r["ibar"], orc.reconstruct(r["holo"], 8, nx, ny, n_sf), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r["nmse2"], orc.nmse_pair(r["ibar"], t), rtol=1e-12)


def test_eight_levels_beat_binary(orc):
    # eight phase levels carry more of the field than a sign bit: lower error
    nx, ny, n_sf = 64, 64, 8
    t = synth.blob_target(nx, ny, 74)
    phi = _phases(orc, 100003)
    b = orc.ospr(t, n_sf, phi, 100003, 0)
    m = orc.ospr_mode(t, n_sf, phi, 100003, 0, 2)
    assert m["nmse2"][0] < b["nmse2"][0]
