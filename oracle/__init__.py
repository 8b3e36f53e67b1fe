"""FP64 CPU oracle for LUT phase randomisation in GS / OSPR holography.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this package; the product library never does.
It shares no code with the HIP path and imports nothing from it.

This module is a thin numpy/ctypes wrapper around ``holo_oracle.c``,
``cnn_oracle.c`` and ``phase_oracle.c``, which hold all the arithmetic.  Conventions follow
Eq. (1)-(2) of the paper: unitary DFT pair, forward kernel e^{-}, row-major
[ny][nx] images with raster index p = y*nx + x.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["holo_oracle.c", "cnn_oracle.c", "phase_oracle.c"]
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP over outer loops)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp", *srcs, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    u64, i64, i32, dbl = C.c_uint64, C.c_int64, C.c_int, C.c_double
    sig = {
        "orc_splitmix64_next": (u64, [P]),
        "orc_lut_phases": (None, [u64, u64, P]),
        "orc_lut_index": (u64, [u64, u64, u64, u64, u64]),
        "orc_lut_phasor_field": (None, [P, u64, u64, u64, i64, i64, P]),
        "orc_dft2_brute": (None, [P, i64, i64, i32, P]),
        "orc_fft2": (None, [P, i64, i64, i32]),
        "orc_nmse": (dbl, [P, P, u64]),
        "orc_nmse_direct": (dbl, [P, P, u64]),
        "orc_nmse_pair": (None, [P, P, i64, i64, P]),
        "orc_binarise": (i32, [dbl]),
        "orc_quant8": (i32, [dbl, dbl]),
        "orc_reconstruct": (None, [P, i32, i64, i64, i32, P]),
        "orc_ospr": (None, [P, i64, i64, i32, P, u64, u64, P, P, P, P]),
        "orc_gs": (None, [P, i64, i64, i32, P, P, P, P, P, P]),
        "orc_ospr_mode": (None, [P, i64, i64, i32, P, u64, u64, i32, P, P, P, P]),
        "orc_num_threads": (i32, []),
        "orc_set_threads": (None, [i32]),
        "orc_splitmix64_at": (u64, [u64, u64]),
        "orc_prng_phases": (None, [u64, u64, u64, P]),
        "orc_codes8_phases": (None, [u64, u64, P]),
        "orc_mseq_bits": (None, [C.c_uint32, u64, P]),
        "orc_mseq_codes": (i32, [C.c_uint32, u64, u64, P]),
        "orc_mseq_window": (C.c_uint32, [u64]),
        "orc_mseq_phases": (i32, [u64, u64, u64, P]),
        "orc_conv3x3": (None, [P, i32, i32, i32, P, P, i32, P]),
        "orc_cnn_nparams": (i32, [i32]),
        "orc_bf16": (dbl, [dbl]),
        "orc_cnn_forward": (None, [P, i32, P, i32, i32, i32, P, P, P]),
        "orc_cnn_loss": (dbl, [P, P, P, u64]),
        "orc_cnn_backward": (dbl, [P, i32, P, P, i32, i32, i32, P]),
        "orc_adam": (None, [P, P, P, P, i32, i32, dbl, dbl, dbl, dbl]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (scheduling only; results do not change)."""
    _load().orc_set_threads(n)


def _p(a):
    return None if a is None else a.ctypes.data


def _c128(a) -> np.ndarray:
    """complex array -> contiguous interleaved float64 pairs."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


def _f32(t) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(t, dtype=np.float32))


# ----------------------------------------------------------------------------
# LUT (Section 4 pool, Section 5 cyclic access)
# ----------------------------------------------------------------------------
def splitmix64(seed: int, n: int) -> np.ndarray:
    lib = _load()
    st = np.array([seed], dtype=np.uint64)
    return np.array([lib.orc_splitmix64_next(st.ctypes.data) for _ in range(n)], dtype=np.uint64)


def lut_phases(n_lut: int, seed: int) -> np.ndarray:
    out = np.zeros(max(n_lut, 1), dtype=np.float64)
    _load().orc_lut_phases(n_lut, seed, out.ctypes.data)
    return out[:n_lut]


# ----------------------------------------------------------------------------
# Other phase sources (Section 4: PRNG + trigonometry; Section 7: M-sequence +
# sine/cosine tables; an 8-bit-code table).  Each gives the phases of pool
# positions start .. start+n-1.
# ----------------------------------------------------------------------------
def splitmix64_at(seed: int, i: int) -> int:
    return int(_load().orc_splitmix64_at(seed, i))


def prng_phases(seed: int, start: int, n: int) -> np.ndarray:
    out = np.zeros(max(n, 1))
    _load().orc_prng_phases(seed, start, n, out.ctypes.data)
    return out[:n]


def codes8_phases(n: int, seed: int) -> np.ndarray:
    out = np.zeros(max(n, 1))
    _load().orc_codes8_phases(n, seed, out.ctypes.data)
    return out[:n]


def mseq_bits(window: int, nbits: int) -> np.ndarray:
    out = np.zeros(max(nbits, 1), dtype=np.uint8)
    _load().orc_mseq_bits(window, nbits, out.ctypes.data)
    return out[:nbits]


def mseq_codes(window: int, start: int, n: int) -> np.ndarray:
    out = np.zeros(max(n, 1), dtype=np.uint8)
    assert _load().orc_mseq_codes(window, start, n, out.ctypes.data) == 0
    return out[:n]


def mseq_window(seed: int) -> int:
    return int(_load().orc_mseq_window(seed))


def mseq_phases(seed: int, start: int, n: int) -> np.ndarray:
    out = np.zeros(max(n, 1))
    assert _load().orc_mseq_phases(seed, start, n, out.ctypes.data) == 0
    return out[:n]


def lut_index(cursor: int, k: int, npix: int, p: int, n_lut: int) -> int:
    return int(_load().orc_lut_index(cursor, k, npix, p, n_lut))


def lut_phasor_field(phi: np.ndarray, n_lut: int, cursor: int, k: int, nx: int, ny: int) -> np.ndarray:
    out = np.zeros(2 * nx * ny, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64) if n_lut else np.zeros(1)
    _load().orc_lut_phasor_field(_p(phi), n_lut, cursor, k, nx, ny, out.ctypes.data)
    return out.view(np.complex128).reshape(ny, nx)


# ----------------------------------------------------------------------------
# Eq. (1)-(2)
# ----------------------------------------------------------------------------
def dft2_brute(f, sign: int) -> np.ndarray:
    f = np.asarray(f)
    ny, nx = f.shape
    a = _c128(f)
    out = np.zeros_like(a)
    _load().orc_dft2_brute(a.ctypes.data, nx, ny, sign, out.ctypes.data)
    return out.view(np.complex128).reshape(ny, nx)


def fft2(f, sign: int) -> np.ndarray:
    f = np.asarray(f)
    ny, nx = f.shape
    a = _c128(f).copy()
    _load().orc_fft2(a.ctypes.data, nx, ny, sign)
    return a.view(np.complex128).reshape(ny, nx)


# ----------------------------------------------------------------------------
# Metric and quantisers
# ----------------------------------------------------------------------------
def nmse(i, w) -> float:
    i = np.ascontiguousarray(i, dtype=np.float64).ravel()
    w = np.ascontiguousarray(w, dtype=np.float64).ravel()
    return float(_load().orc_nmse(i.ctypes.data, w.ctypes.data, i.size))


def nmse_direct(i, w) -> float:
    i = np.ascontiguousarray(i, dtype=np.float64).ravel()
    w = np.ascontiguousarray(w, dtype=np.float64).ravel()
    return float(_load().orc_nmse_direct(i.ctypes.data, w.ctypes.data, i.size))


def nmse_pair(ibar, target) -> np.ndarray:
    t = _f32(target)
    ny, nx = t.shape
    i = np.ascontiguousarray(ibar, dtype=np.float64)
    out = np.zeros(2)
    _load().orc_nmse_pair(i.ctypes.data, t.ctypes.data, nx, ny, out.ctypes.data)
    return out


def binarise(re: float) -> int:
    return int(_load().orc_binarise(float(re)))


def quant8(re: float, im: float) -> int:
    return int(_load().orc_quant8(float(re), float(im)))


def reconstruct(holo: np.ndarray, levels: int, nx: int, ny: int, n_sf: int) -> np.ndarray:
    if levels == 2:
        h = np.ascontiguousarray(holo, dtype=np.uint32)
    else:
        h = np.ascontiguousarray(holo, dtype=np.uint8)
    out = np.zeros(nx * ny)
    _load().orc_reconstruct(h.ctypes.data, levels, nx, ny, n_sf, out.ctypes.data)
    return out.reshape(ny, nx)


# ----------------------------------------------------------------------------
# OSPR and GS
# ----------------------------------------------------------------------------
def ospr(target, n_sf: int, phi: np.ndarray, n_lut: int, cursor: int = 0,
         want_reh: bool = True, want_ibar: bool = True):
    """Returns dict(bits [n_sf, words] uint32, reH [n_sf, ny, nx] or None,
    ibar [ny, nx] or None, nmse2 [2])."""
    t = _f32(target)
    ny, nx = t.shape
    n = nx * ny
    words = (n + 31) // 32
    bits = np.zeros((n_sf, words), dtype=np.uint32)
    reh = np.zeros((n_sf, ny, nx)) if want_reh else None
    ibar = np.zeros((ny, nx)) if want_ibar else None
    nm = np.zeros(2)
    phi = np.ascontiguousarray(phi, dtype=np.float64) if n_lut else np.zeros(1)
    _load().orc_ospr(t.ctypes.data, nx, ny, n_sf, phi.ctypes.data, n_lut, cursor,
                     bits.ctypes.data, _p(reh), _p(ibar), nm.ctypes.data)
    return {"bits": bits, "reH": reh, "ibar": ibar, "nmse2": nm}


def ospr_mode(target, n_sf: int, phi: np.ndarray, n_lut: int, cursor: int, mode: int, want_hval: bool = True):
    """OSPR variants: mode 1 = two binary sub-frames (Re, Im) per field,
    mode 2 = eight phase levels.  Returns dict(holo: bits [n_sf, words]
    uint32 or codes [n_sf, ny, nx] uint8, hval: decided values (mode 1:
    [n_sf, ny, nx] float; mode 2: H complex [n_sf, ny, nx]), ibar, nmse2)."""
    t = _f32(target)
    ny, nx = t.shape
    n = nx * ny
    if mode == 1:
        holo = np.zeros((n_sf, (n + 31) // 32), dtype=np.uint32)
        hval = np.zeros((n_sf, ny, nx)) if want_hval else None
    else:
        holo = np.zeros((n_sf, ny, nx), dtype=np.uint8)
        hval = np.zeros((n_sf, ny, nx), dtype=np.complex128) if want_hval else None
    ibar = np.zeros((ny, nx))
    nm = np.zeros(2)
    phi = np.ascontiguousarray(phi, dtype=np.float64) if n_lut else np.zeros(1)
    _load().orc_ospr_mode(t.ctypes.data, nx, ny, n_sf, phi.ctypes.data, n_lut, cursor, mode, holo.ctypes.data,
                          _p(hval), ibar.ctypes.data, nm.ctypes.data)
    return {"holo": holo, "hval": hval, "ibar": ibar, "nmse2": nm}


def gs(target, n_iter: int, init_phasor):
    """Returns dict(nmse [n_iter], err [n_iter], field [ny, nx] complex (R'_n),
    codes [ny, nx] uint8, nmse_final2 [2])."""
    t = _f32(target)
    ny, nx = t.shape
    init = _c128(init_phasor).copy()
    nm = np.zeros(n_iter)
    er = np.zeros(n_iter)
    fld = np.zeros(2 * nx * ny)
    codes = np.zeros((ny, nx), dtype=np.uint8)
    fin = np.zeros(2)
    _load().orc_gs(t.ctypes.data, nx, ny, n_iter, init.ctypes.data, nm.ctypes.data, er.ctypes.data,
                   fld.ctypes.data, codes.ctypes.data, fin.ctypes.data)
    return {"nmse": nm, "err": er, "field": fld.view(np.complex128).reshape(ny, nx),
            "codes": codes, "nmse_final2": fin}


def unpack_bits(bits: np.ndarray, n: int) -> np.ndarray:
    """uint32 words (LSB-first, raster order) -> uint8 bit array of length n."""
    b = np.unpackbits(np.ascontiguousarray(bits, dtype=np.uint32).view(np.uint8), axis=-1,
                      bitorder="little")
    return b[..., :n]


# ----------------------------------------------------------------------------
# Learned GS seed (small CNN; not part of the paper's method)
# ----------------------------------------------------------------------------
def conv3x3(x, w, b=None):
    """x [cin, ny, nx], w [cout, cin, 3, 3] -> [cout, ny, nx] (circular)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    cin, ny, nx = x.shape
    cout = w.shape[0]
    out = np.zeros((cout, ny, nx))
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    _load().orc_conv3x3(x.ctypes.data, cin, ny, nx, w.ctypes.data, _p(bb), cout, out.ctypes.data)
    return out


def cnn_nparams(C: int) -> int:
    return int(_load().orc_cnn_nparams(C))


def bf16(v: float) -> float:
    return float(_load().orc_bf16(float(v)))


def cnn_forward(params, C, target, bf16_store=False):
    """Returns (acts [4, C, ny, nx], out2 [2, ny, nx], phasor complex [ny, nx]).
    bf16_store: hidden activations rounded to BF16 where stored."""
    pr = np.ascontiguousarray(params, dtype=np.float64)
    t = _f32(target)
    ny, nx = t.shape
    acts = np.zeros((4, C, ny, nx))
    out2 = np.zeros((2, ny, nx))
    ph = np.zeros(2 * ny * nx)
    _load().orc_cnn_forward(pr.ctypes.data, C, t.ctypes.data, ny, nx, int(bool(bf16_store)), acts.ctypes.data,
                            out2.ctypes.data, ph.ctypes.data)
    return acts, out2, ph.view(np.complex128).reshape(ny, nx)


def cnn_loss(phasor, label, target) -> float:
    p = _c128(phasor)
    q = _c128(label)
    t = _f32(target)
    return float(_load().orc_cnn_loss(p.ctypes.data, q.ctypes.data, t.ctypes.data, t.size))


def cnn_backward(params, C, target, label, bf16_store=False):
    """Returns (loss, grad [nparams]).  bf16_store: hidden activations and
    hidden-layer gradients rounded to BF16 where stored."""
    pr = np.ascontiguousarray(params, dtype=np.float64)
    t = _f32(target)
    ny, nx = t.shape
    q = _c128(label)
    g = np.zeros(pr.size)
    loss = _load().orc_cnn_backward(pr.ctypes.data, C, t.ctypes.data, q.ctypes.data, ny, nx,
                                    int(bool(bf16_store)), g.ctypes.data)
    return float(loss), g


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().orc_adam(params.ctypes.data, grad.ctypes.data, m.ctypes.data, v.ctypes.data, params.size, t, lr, b1,
                     b2, eps)
