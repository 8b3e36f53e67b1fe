"""Seeded synthetic inputs shared by the product tests, the benchmark and the
oracle tests.

This module generates *inputs only* (target amplitudes, batch layouts); it holds
none of the hologram method's arithmetic.  The paper measures on six 256x256
USC-SIPI photographs (Section 5), which are not available here; seeded
blob-and-rectangle targets of the same sizes stand in for them.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014),
written here from its published definition, in vectorised numpy uint64
arithmetic (which wraps modulo 2^64 like the definition requires).
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_stream(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+n-1 of SplitMix64 seeded with `seed` (state after
    j+1 steps is seed + (j+1)*gamma mod 2^64)."""
    with np.errstate(over="ignore"):
        j = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + j * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class _Stream:
    """Sequential uniform draws u = (x >> 11) * 2^-53 from one SplitMix64 stream."""

    def __init__(self, seed: int):
        self.seed = seed
        self.pos = 0

    def u(self) -> float:
        x = int(splitmix64_stream(self.seed, 1, self.pos)[0])
        self.pos += 1
        return (x >> 11) * 2.0 ** -53


def uniform_target(nx: int, ny: int, seed: int) -> np.ndarray:
    """T_p = (x_p >> 40) * 2^-24 in [0, 1), exact in float32 (raster order)."""
    x = splitmix64_stream(seed, nx * ny)
    return ((x >> np.uint64(40)).astype(np.float64) * 2.0 ** -24).astype(np.float32).reshape(ny, nx)


def blob_target(nx: int, ny: int, seed: int, n_blobs: int = 20, n_rects: int = 10) -> np.ndarray:
    """Sum of `n_blobs` Gaussian blobs and `n_rects` rectangles, normalised to
    [0, 1] by its maximum, evaluated in float64 at integer pixel centres and
    rounded once to float32.  All draws come from one stream, blobs first:
      blob: cx = u*nx, cy = u*ny, sigma = (0.01 + 0.09u)*nx, a = 0.2 + 0.8u
      rect: x0 = floor(u*nx), y0 = floor(u*ny), w = floor((0.05+0.25u)*nx),
            h = floor((0.05+0.25u)*ny), a = 0.2 + 0.8u (clipped, no wrap)."""
    st = _Stream(seed)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    s = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(n_blobs):
        cx = st.u() * nx
        cy = st.u() * ny
        sig = (0.01 + 0.09 * st.u()) * nx
        a = 0.2 + 0.8 * st.u()
        # the Gaussian is separable: exp(-(dx^2 + dy^2)/2s^2) = gy(y) * gx(x)
        gx = np.exp(-((xs - cx) ** 2) / (2.0 * sig * sig))
        gy = a * np.exp(-((ys - cy) ** 2) / (2.0 * sig * sig))
        s += np.multiply.outer(gy, gx)
    for _ in range(n_rects):
        x0 = int(st.u() * nx)
        y0 = int(st.u() * ny)
        w = int((0.05 + 0.25 * st.u()) * nx)
        h = int((0.05 + 0.25 * st.u()) * ny)
        a = 0.2 + 0.8 * st.u()
        s[y0:min(y0 + h, ny), x0:min(x0 + w, nx)] += a
    m = s.max()
    return (s / m if m > 0 else s).astype(np.float32)


def batch_layout(n_frames: int, seed: int, sizes=(256, 512, 1024, 2048), n_sf_range=(8, 24)):
    """Per-frame (size, n_sf): size uniform over `sizes`, n_sf uniform over the
    inclusive integer range, drawn alternately from one stream."""
    st = _Stream(seed)
    out = []
    lo, hi = n_sf_range
    for _ in range(n_frames):
        s = sizes[min(int(st.u() * len(sizes)), len(sizes) - 1)]
        k = lo + min(int(st.u() * (hi - lo + 1)), hi - lo)
        out.append((s, k))
    return out


# Seeds of the standard workloads.
SEED_LUT = 1
SEED_UNIFORM_64 = 11
SEED_OSPR_1024 = 12
SEED_GS_512 = 13
SEED_BATCH = 14
SEED_BATCH_TARGET0 = 1000
SEED_CNN_TRAIN0 = 100000
SEED_CNN_HELDOUT0 = 200000
SEED_LUT_STUDY0 = 300000
