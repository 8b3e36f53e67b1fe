"""Pins for the oracle's LUT generation and cyclic indexing (Section 4 pool,
Section 5 / Fig. 3 access order, Section 5.1 hard limits).  CPU only."""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_ints(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [int(l) for l in f if l.strip() and not l.startswith("#")]


def test_splitmix64_published_vector(orc):
    want = _golden_ints("splitmix64_seed1234567.txt")
    got = [int(x) for x in orc.splitmix64(1234567, len(want))]
    assert got == want
    # the input generator's independent vectorised SplitMix64 agrees too
    assert [int(x) for x in synth.splitmix64_stream(1234567, len(want))] == want


def test_lut_phases_definition(orc):
    n = 1000
    phi = orc.lut_phases(n, 1)
    x = np.array([int(v) for v in synth.splitmix64_stream(1, n)], dtype=object)
    u = np.array([float(v >> 11) * 2.0 ** -53 for v in x])
    # one correctly rounded multiply by fp64(2*pi): bit-exact
    assert np.array_equal(phi, (2 * np.pi) * u)
    assert phi.min() >= 0.0 and phi.max() < 2 * np.pi
    # roughly uniform on [0, 2*pi)
    h, _ = np.histogram(phi, bins=8, range=(0, 2 * np.pi))
    assert h.min() > 90 and h.max() < 160


def test_index_is_sequential_cycle(orc):
    # the pool is read sequentially across sub-frames and frames: flattening
    # (k, p) to k*N + p gives consecutive entries starting at the cursor.
    nx, ny, L, c = 4, 2, 7, 12
    n = nx * ny
    seq = [orc.lut_index(c, k, n, p, L) for k in range(3) for p in range(n)]
    assert seq == [(c + j) % L for j in range(3 * n)]
    # 64-bit cursors near the top of the range do not overflow
    big = 2 ** 64 - 5
    assert orc.lut_index(big, 2, 2 ** 20, 7, 10007) == (big + 2 * 2 ** 20 + 7) % 10007


def test_I1_lut_as_long_as_a_row_repeats_every_row(orc):
    # Section 5.2: N_LUT = 256 at 256x256 gives every row the same phases.
    nx, ny = 32, 8
    phi = orc.lut_phases(nx, 1)
    f = orc.lut_phasor_field(phi, nx, 5, 0, nx, ny)
    for y in range(1, ny):
        assert np.array_equal(f[y], f[0])


def test_I2_divisor_lut_repeats_subframes_and_I5_flat(orc):
    nx, ny, L = 16, 16, 64
    phi = orc.lut_phases(L, 1)
    f0 = orc.lut_phasor_field(phi, L, 3, 0, nx, ny)
    for k in (1, 2, 5):
        assert np.array_equal(orc.lut_phasor_field(phi, L, 3, k, nx, ny), f0)
    flat = orc.lut_phasor_field(np.zeros(1), 0, 3, 1, nx, ny)
    assert np.array_equal(flat, np.ones((ny, nx), complex))


def test_I3_prime_lut_gives_distinct_indices_per_pixel(orc):
    # Section 5.1: N_LUT > N_SF (prime, not dividing the frame) keeps a pixel's
    # sub-frame phases apart.
    nx, ny, L, nsf = 16, 16, 31, 24
    n = nx * ny
    for p in range(0, n, 17):
        idx = {orc.lut_index(9, k, n, p, L) for k in range(nsf)}
        assert len(idx) == nsf
    # and with N_LUT <= N_SF some pixel must repeat (pigeonhole)
    L2 = 23
    idx = {orc.lut_index(9, k, n, 0, L2) for k in range(nsf)}
    assert len(idx) < nsf


def test_I4_chaining_equals_one_long_frame(orc):
    # a frame of K sub-frames at cursor c reads exactly what K frames of one
    # sub-frame read with the cursor advanced by N each time.
    nx, ny, L = 8, 4, 13
    n = nx * ny
    a = [orc.lut_index(5, k, n, p, L) for k in range(4) for p in range(n)]
    b = [orc.lut_index(5 + k * n, 0, n, p, L) for k in range(4) for p in range(n)]
    assert a == b
