"""Pins for the oracle's transforms (Eq. (1)-(2)): an independent library FFT,
closed forms and identities.  CPU only."""
import numpy as np
import pytest

SIZES = [(8, 8), (16, 4), (4, 32), (32, 16)]


def _rand_field(nx, ny, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))


@pytest.mark.parametrize("nx,ny", SIZES)
def test_fft_matches_numpy_ortho(orc, nx, ny):
    # numpy's pocketfft is an independent implementation of the same unitary pair.
    f = _rand_field(nx, ny, 1)
    np.testing.assert_allclose(orc.fft2(f, -1), np.fft.fft2(f, norm="ortho"), rtol=0, atol=1e-13)
    np.testing.assert_allclose(orc.fft2(f, +1), np.fft.ifft2(f, norm="ortho"), rtol=0, atol=1e-13)


@pytest.mark.parametrize("nx,ny", [(8, 8), (4, 16), (16, 2)])
def test_brute_force_matches_numpy_and_fft(orc, nx, ny):
    f = _rand_field(nx, ny, 2)
    for s in (-1, +1):
        b = orc.dft2_brute(f, s)
        ref = np.fft.fft2(f, norm="ortho") if s < 0 else np.fft.ifft2(f, norm="ortho")
        np.testing.assert_allclose(b, ref, rtol=0, atol=1e-12)
        np.testing.assert_allclose(orc.fft2(f, s), b, rtol=0, atol=1e-12)


def test_large_size_matches_numpy(orc):
    f = _rand_field(256, 128, 3)
    np.testing.assert_allclose(orc.fft2(f, +1), np.fft.ifft2(f, norm="ortho"), rtol=0, atol=1e-12)


@pytest.mark.parametrize("nx,ny", SIZES)
def test_delta_and_constant(orc, nx, ny):
    n = nx * ny
    d = np.zeros((ny, nx), complex)
    d[0, 0] = 1.0
    for s in (-1, 1):
        np.testing.assert_allclose(orc.fft2(d, s), np.full((ny, nx), 1 / np.sqrt(n)), atol=1e-15)
        c = orc.fft2(np.ones((ny, nx)), s)
        expect = np.zeros((ny, nx))
        expect[0, 0] = np.sqrt(n)
        np.testing.assert_allclose(c, expect, atol=1e-12)


@pytest.mark.parametrize("nx,ny", SIZES)
def test_shift_theorem_sign(orc, nx, ny):
    # Eq. (1): a delta at (x0, y0) transforms to exp(-2*pi*i*(u x0/Nx + v y0/Ny))/sqrt(N).
    x0, y0 = 3 % nx, 1 % ny
    d = np.zeros((ny, nx), complex)
    d[y0, x0] = 1.0
    v, u = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ph = 2 * np.pi * (u * x0 / nx + v * y0 / ny)
    np.testing.assert_allclose(orc.fft2(d, -1), np.exp(-1j * ph) / np.sqrt(nx * ny), atol=1e-14)
    np.testing.assert_allclose(orc.fft2(d, +1), np.exp(+1j * ph) / np.sqrt(nx * ny), atol=1e-14)


@pytest.mark.parametrize("nx,ny", SIZES)
def test_parseval_and_round_trip(orc, nx, ny):
    f = _rand_field(nx, ny, 4)
    F = orc.fft2(f, -1)
    assert abs(np.sum(abs(F) ** 2) - np.sum(abs(f) ** 2)) < 1e-10 * np.sum(abs(f) ** 2)
    np.testing.assert_allclose(orc.fft2(F, +1), f, atol=1e-13)
