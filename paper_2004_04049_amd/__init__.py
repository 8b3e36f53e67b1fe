"""Python binding of libholo.so, the MI355X (gfx950) hot path for LUT phase
randomisation in OSPR / Gerchberg-Saxton hologram generation (Christopher &
Wilkinson, arXiv:2004.04049).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  Function names follow
the C ABI in include/holo.h (holo_<name>).  There is no fallback: if the
library is missing, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libholo.so")

HOLO_OK, HOLO_EINVAL, HOLO_EUNSUPPORTED, HOLO_ENOMEM, HOLO_EDEVICE = 0, -1, -2, -3, -4
FP32, BF16, FP16 = 0, 1, 2
SRC_TABLE, SRC_CODES8, SRC_PRNG, SRC_MSEQ = 0, 1, 2, 3
F_NMSE_DEVICE, F_OSPR_PAIRS, F_OSPR_LEVELS8 = 1, 2, 4
LUT_FLAT, LUT_NOT_PRIME, LUT_LE_NSF, LUT_LE_MAXDIM, LUT_DIVIDES_FRAME, LUT_LT_FULL = 1, 2, 4, 8, 16, 32

_lib = None

# name -> (restype, argtypes)
_P, _U64, _I64, _I32, _U32 = C.c_void_p, C.c_uint64, C.c_int64, C.c_int32, C.c_uint32
SIGNATURES = {
    "holo_last_error": (C.c_char_p, []),
    "holo_version": (_I32, []),
    "holo_lut_build": (_I32, [_U64, _U64, C.POINTER(_P)]),
    "holo_lut_from_phases": (_I32, [_P, _U64, C.POINTER(_P)]),
    "holo_lut_build_codes": (_I32, [_U64, _U64, C.POINTER(_P)]),
    "holo_lut_prng": (_I32, [_U64, C.POINTER(_P)]),
    "holo_lut_mseq": (_I32, [_U64, C.POINTER(_P)]),
    "holo_lut_kind": (_I32, [_P]),
    "holo_lut_phases": (_I32, [_P, _P, _U64]),
    "holo_lut_size": (_U64, [_P]),
    "holo_lut_free": (None, [_P]),
    "holo_lut_check": (_U32, [_U64, _I64, _I64, _I32]),
    "holo_ospr_generate": (_I32, [_P, _I64, _I64, _I32, _P, C.POINTER(_U64), _P, _P, _P, _I32, _U32, _P]),
    "holo_gs_iterate": (_I32, [_P, _I64, _I64, _I32, _P, C.POINTER(_U64), _P, _P, _P, _P, _P, _P, _P, _I32,
                               _U32, _P]),
    "holo_gs_iterate_noalloc": (_I32, [_P, _I64, _I64, _I32, _P, C.POINTER(_U64), _P, _P, _P, _P, _P, _P, _P,
                                       _I32, _U32, _P]),
    "holo_gs_iterate_batched": (_I32, [_P, _I32, _I64, _I64, _I32, _P, C.POINTER(_U64), _P, _P, _P, _U32, _P]),
    "holo_reconstruct_nmse": (_I32, [_P, _I32, _I64, _I64, _I32, _P, _P, _P, _U32, _P]),
    "holo_fft2": (_I32, [_P, _P, _I64, _I64, _I32, _I32, _P]),
    "holo_phase_mask": (_I32, [_P, _U64, _I64, _I64, _I32, _P, _P]),
    "holo_shutdown": (None, []),
    "holo_prof_enable": (_I32, [_I32]),
    "holo_prof_read": (_I32, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(_I64)]),
    "holo_prof_reset": (None, []),
    "holo_autotune_ospr": (_I32, [_P, _I64, _I64, _I32, _P, _P, _I32, _P, _P]),
    "holo_autotune_gs": (_I32, [_P, _I64, _I64, _P, _I32, _P, _P]),
    "holo_plan_set": (_I32, [_I32, _I64, _I64, _I32, _P]),
    "holo_plan_get": (_I32, [_I32, _I64, _I64, _I32, _P]),
    "holo_plan_save": (_I32, [C.c_char_p]),
    "holo_plan_load": (_I32, [C.c_char_p]),
    "holo_set_graphs": (_I32, [_I32]),
    "holo_ospr_generate_batched": (_I32, [_P, _I32, _P, C.POINTER(_U64), _P, _I32, _U32, _P]),
    "holo_cnn_nparams": (_I32, []),
    "holo_cnn_create": (_I32, [_U64, C.POINTER(_P)]),
    "holo_cnn_get_params": (_I32, [_P, _P, _I32]),
    "holo_cnn_set_params": (_I32, [_P, _P, _I32]),
    "holo_cnn_infer": (_I32, [_P, _P, _I64, _I64, _P, _P]),
    "holo_cnn_loss_grad": (_I32, [_P, _P, _P, _I64, _I64, _P, _P, _P]),
    "holo_cnn_train_step": (_I32, [_P, _P, _P, _I32, _I64, _I64, C.c_float, _P, _P]),
    "holo_cnn_save": (_I32, [_P, C.c_char_p]),
    "holo_cnn_load": (_I32, [C.c_char_p, C.POINTER(_P)]),
    "holo_cnn_free": (None, [_P]),
}


class HoloFrame(C.Structure):
    """holo_frame: one frame of a batched OSPR call (device pointers)."""
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("n_sf", C.c_int32), ("target", C.c_void_p),
                ("holo_bits", C.c_void_p), ("recon", C.c_void_p)]


class HoloGsFrame(C.Structure):
    """holo_gs_frame: one frame of a batched GS call (device pointers)."""
    _fields_ = [("target", C.c_void_p), ("init_phasor", C.c_void_p), ("field", C.c_void_p), ("codes", C.c_void_p),
                ("recon", C.c_void_p)]


class HoloError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"holo status {status}: {msg}")
        self.status = status


def lib():
    """Loads libholo.so (built by paper_2004_04049_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2004_04049_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != HOLO_OK:
        raise HoloError(status, lib().holo_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Lut:
    """Phase-pool handle.  Lut(n, seed) / Lut(n, phases=...): FP32 phasor table
    (holo_lut_build / holo_lut_from_phases); Lut.codes(n, seed): 8-bit codes;
    Lut.prng(seed): counter-based SplitMix64 + sine/cosine; Lut.mseq(seed):
    M-sequence codes."""

    def __init__(self, n_lut: int, seed: int = 1, phases=None, _kind=SRC_TABLE):
        h = C.c_void_p()
        if _kind == SRC_CODES8:
            _check(lib().holo_lut_build_codes(n_lut, seed, C.byref(h)))
        elif _kind == SRC_PRNG:
            _check(lib().holo_lut_prng(seed, C.byref(h)))
        elif _kind == SRC_MSEQ:
            _check(lib().holo_lut_mseq(seed, C.byref(h)))
        elif phases is not None:
            import numpy as np
            ph = np.ascontiguousarray(phases, dtype=np.float64)
            _check(lib().holo_lut_from_phases(ph.ctypes.data_as(C.c_void_p), len(ph), C.byref(h)))
        else:
            _check(lib().holo_lut_build(n_lut, seed, C.byref(h)))
        self._h = h

    @classmethod
    def codes(cls, n_lut: int, seed: int = 1):
        return cls(n_lut, seed, _kind=SRC_CODES8)

    @classmethod
    def prng(cls, seed: int = 1):
        return cls(0, seed, _kind=SRC_PRNG)

    @classmethod
    def mseq(cls, seed: int = 1):
        return cls(0, seed, _kind=SRC_MSEQ)

    @property
    def handle(self):
        return self._h

    @property
    def kind(self) -> int:
        return int(lib().holo_lut_kind(self._h))

    @property
    def size(self) -> int:
        """Pool length (PRNG: 2**64 - 1, unbounded; MSEQ: 2**31 - 1)."""
        return int(lib().holo_lut_size(self._h))

    def __len__(self):
        if self.kind == SRC_PRNG:
            raise TypeError("a counter-based PRNG pool is unbounded (Lut.size gives 2**64 - 1)")
        return self.size

    def phases(self):
        """FP64 phases of a table source (TABLE, CODES8); raises for PRNG and MSEQ."""
        import numpy as np
        n = self.size if self.kind in (SRC_TABLE, SRC_CODES8) else 0
        out = np.zeros(max(n, 1), dtype=np.float64)
        _check(lib().holo_lut_phases(self._h, out.ctypes.data_as(C.c_void_p), n))
        return out[:n]

    def close(self):
        if self._h:
            lib().holo_lut_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lut_build(n_lut: int, seed: int = 1) -> Lut:
    return Lut(n_lut, seed)


def lut_check(n_lut: int, nx: int, ny: int, n_sf: int) -> int:
    return int(lib().holo_lut_check(n_lut, nx, ny, n_sf))


def _nmse_buf(n, device_out):
    import numpy as np
    if device_out is not None:
        return device_out, C.c_void_p(device_out.data_ptr()), F_NMSE_DEVICE
    a = np.zeros(n)
    return a, a.ctypes.data_as(C.c_void_p), 0


OSPR_MODES = {"binary": 0, "pairs": F_OSPR_PAIRS, "levels8": F_OSPR_LEVELS8}


def _holo_buf(mode, n_sf, nx, ny, buf, device):
    """Output of one frame: packed bits int32 [n_sf, nx*ny/32], or uint8 codes
    [n_sf, ny, nx] for the eight-level variant."""
    if mode == "levels8":
        shape, dt = (n_sf, ny, nx), torch.uint8
    else:
        shape, dt = (n_sf, nx * ny // 32), torch.int32
    if buf is None:
        buf = torch.empty(shape, dtype=dt, device=device)
    _dev(buf, dt, shape, "bits")
    return buf


def ospr_generate(target, n_sf: int, lut: Lut, cursor: int, bits=None, recon=None, want_nmse=True,
                  nmse_out=None, stream=None, precision: int = FP32, mode: str = "binary"):
    """holo_ospr_generate.  Returns (bits, nmse2 or None, new_cursor).
    target: cuda float32 [ny, nx]; bits: cuda int32 [n_sf, nx*ny/32] (uint8
    [n_sf, ny, nx] codes for mode "levels8"; allocated if None); recon: cuda
    float32 [ny, nx] or None; nmse_out: cuda float64 [2] to keep the NMSE on
    the device (no synchronisation).  mode: "binary" (the paper's frame),
    "pairs" (sub-frames 2j, 2j+1 from Re and Im of one field) or "levels8"."""
    ny, nx = target.shape
    _dev(target, torch.float32, None, "target")
    bits = _holo_buf(mode, n_sf, nx, ny, bits, target.device)
    if recon is not None:
        _dev(recon, torch.float32, (ny, nx), "recon")
    nm, nm_p, flags = (None, None, 0)
    if want_nmse or nmse_out is not None:
        nm, nm_p, flags = _nmse_buf(2, nmse_out)
    flags |= OSPR_MODES[mode]
    cur = C.c_uint64(cursor)
    _check(lib().holo_ospr_generate(_ptr(target), nx, ny, n_sf, lut.handle, C.byref(cur), _ptr(bits),
                                    _ptr(recon), nm_p, precision, flags, _stream(stream)))
    return bits, nm, int(cur.value)


def gs_iterate(target, n_iter: int, lut: Lut | None, cursor: int, init_phasor=None, field=None, codes=None,
               want_nmse=True, want_err=False, want_final=True, recon=None, stream=None):
    """holo_gs_iterate.  Returns dict(nmse, err, nmse_final2, field, codes,
    cursor).  Tensors: target float32 [ny, nx]; init_phasor/field complex64
    [ny, nx]; codes uint8 [ny, nx]."""
    import numpy as np
    ny, nx = target.shape
    _dev(target, torch.float32, None, "target")
    if init_phasor is not None:
        _dev(init_phasor, torch.complex64, (ny, nx), "init_phasor")
    if field is None:
        field = torch.empty((ny, nx), dtype=torch.complex64, device=target.device)
    _dev(field, torch.complex64, (ny, nx), "field")
    if codes is None and (want_final or recon is not None):
        codes = torch.empty((ny, nx), dtype=torch.uint8, device=target.device)
    if codes is not None:
        _dev(codes, torch.uint8, (ny, nx), "codes")
    nm = np.zeros(n_iter) if want_nmse else None
    er = np.zeros(n_iter) if want_err else None
    fin = np.zeros(2) if want_final else None
    cur = C.c_uint64(cursor)
    _check(lib().holo_gs_iterate(
        _ptr(target), nx, ny, n_iter, lut.handle if lut is not None else None, C.byref(cur), _ptr(init_phasor),
        _ptr(field), _ptr(codes),
        nm.ctypes.data_as(C.c_void_p) if nm is not None else None,
        er.ctypes.data_as(C.c_void_p) if er is not None else None,
        fin.ctypes.data_as(C.c_void_p) if fin is not None else None,
        _ptr(recon), FP32, 0, _stream(stream)))
    return {"nmse": nm, "err": er, "nmse_final2": fin, "field": field, "codes": codes, "cursor": int(cur.value)}


def gs_iterate_batched(targets, n_iter: int, lut: Lut | None, cursor: int, init_phasors=None, fields=None,
                       codes=None, recons=None, want_nmse=True, want_err=False, want_final=False, stream=None):
    """holo_gs_iterate_batched: frames of one size.  targets: list of cuda
    float32 [ny, nx]; init_phasors/fields: lists of complex64 [ny, nx] or
    None entries; codes: list of uint8 [ny, nx] (allocated when want_final or
    recons ask for them); recons: list of float32 [ny, nx] or None entries.
    Returns dict(nmse [n, n_iter], err [n, n_iter], nmse_final2 [n, 2],
    fields, codes, cursor)."""
    import numpy as np
    n = len(targets)
    ny, nx = targets[0].shape
    pick = lambda xs, i: xs[i] if xs is not None else None
    fields = [pick(fields, i) if pick(fields, i) is not None else
              torch.empty((ny, nx), dtype=torch.complex64, device=targets[0].device) for i in range(n)]
    need_codes = want_final or (recons is not None and any(r is not None for r in recons))
    if codes is None and need_codes:
        codes = [torch.empty((ny, nx), dtype=torch.uint8, device=targets[0].device) for _ in range(n)]
    arr = (HoloGsFrame * n)()
    for i in range(n):
        t = targets[i]
        _dev(t, torch.float32, (ny, nx), "target")
        ip, c, r = pick(init_phasors, i), pick(codes, i), pick(recons, i)
        if ip is not None:
            _dev(ip, torch.complex64, (ny, nx), "init_phasor")
        _dev(fields[i], torch.complex64, (ny, nx), "field")
        if c is not None:
            _dev(c, torch.uint8, (ny, nx), "codes")
        if r is not None:
            _dev(r, torch.float32, (ny, nx), "recon")
        arr[i] = HoloGsFrame(t.data_ptr(), ip.data_ptr() if ip is not None else None, fields[i].data_ptr(),
                             c.data_ptr() if c is not None else None, r.data_ptr() if r is not None else None)
    nm = np.zeros((n, n_iter)) if want_nmse else None
    er = np.zeros((n, n_iter)) if want_err else None
    fin = np.zeros((n, 2)) if want_final else None
    cur = C.c_uint64(cursor)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
    _check(lib().holo_gs_iterate_batched(C.cast(arr, C.c_void_p), n, nx, ny, n_iter,
                                         lut.handle if lut is not None else None, C.byref(cur), ptr(nm), ptr(er),
                                         ptr(fin), 0, _stream(stream)))
    return {"nmse": nm, "err": er, "nmse_final2": fin, "fields": fields, "codes": codes, "cursor": int(cur.value)}


def gs_iterate_noalloc(target, n_iter: int, lut: Lut | None, cursor: int, init_phasor=None, field=None,
                       codes=None, nmse=None, err=None, final2=None, recon=None, stream=None):
    """holo_gs_iterate_noalloc: gs_iterate on the library's fixed scratch (no
    device allocation inside the call).  Every output is a caller tensor:
    field/init_phasor complex64 [ny, nx], codes uint8 [ny, nx], recon float32
    [ny, nx]; nmse/err float64 [n_iter] and final2 float64 [2] on the device.
    Returns the new cursor."""
    ny, nx = target.shape
    _dev(target, torch.float32, None, "target")
    for t, dt, shape, name in ((init_phasor, torch.complex64, (ny, nx), "init_phasor"),
                               (field, torch.complex64, (ny, nx), "field"), (codes, torch.uint8, (ny, nx), "codes"),
                               (recon, torch.float32, (ny, nx), "recon"), (nmse, torch.float64, (n_iter,), "nmse"),
                               (err, torch.float64, (n_iter,), "err"), (final2, torch.float64, (2,), "final2")):
        if t is not None:
            _dev(t, dt, shape, name)
    cur = C.c_uint64(cursor)
    _check(lib().holo_gs_iterate_noalloc(
        _ptr(target), nx, ny, n_iter, lut.handle if lut is not None else None, C.byref(cur), _ptr(init_phasor),
        _ptr(field), _ptr(codes), _ptr(nmse), _ptr(err), _ptr(final2), _ptr(recon), FP32, F_NMSE_DEVICE,
        _stream(stream)))
    return int(cur.value)


def reconstruct_nmse(holo, levels: int, nx: int, ny: int, n_sf: int, target, recon=None, stream=None):
    """holo_reconstruct_nmse.  holo: int32 [n_sf, nx*ny/32] bits (levels 2) or
    uint8 [n_sf, ny, nx] codes (levels 8).  Returns the NMSE pair."""
    import numpy as np
    _dev(target, torch.float32, (ny, nx), "target")
    if levels == 2:
        _dev(holo, torch.int32, (n_sf, nx * ny // 32), "holo")
    else:
        _dev(holo, torch.uint8, None, "holo")
        if holo.numel() != n_sf * nx * ny:
            raise ValueError("codes must hold n_sf*ny*nx bytes")
    if recon is not None:
        _dev(recon, torch.float32, (ny, nx), "recon")
    nm = np.zeros(2)
    _check(lib().holo_reconstruct_nmse(_ptr(holo), levels, nx, ny, n_sf, _ptr(target), _ptr(recon),
                                       nm.ctypes.data_as(C.c_void_p), 0, _stream(stream)))
    return nm


def fft2(x, sign: int, out=None, stream=None, precision: int = FP32):
    """holo_fft2: unitary Eq. (1) (sign -1) or Eq. (2) (sign +1) of a complex64 [ny, nx] tensor."""
    _dev(x, torch.complex64, None, "x")
    ny, nx = x.shape
    if out is None:
        out = torch.empty_like(x)
    _dev(out, torch.complex64, (ny, nx), "out")
    _check(lib().holo_fft2(_ptr(x), _ptr(out), nx, ny, sign, precision, _stream(stream)))
    return out


def phase_mask(lut: Lut, cursor: int, nx: int, ny: int, n_sf: int = 1, stream=None):
    """holo_phase_mask: complex64 [n_sf, ny, nx] phasors of pool positions
    cursor + k*nx*ny + y*nx + x, as the generation kernels draw them."""
    out = torch.empty((n_sf, ny, nx), dtype=torch.complex64, device="cuda")
    _check(lib().holo_phase_mask(lut.handle, cursor, nx, ny, n_sf, _ptr(out), _stream(stream)))
    return out


def unpack_bits(bits: torch.Tensor, n: int):
    """int32 words (LSB-first raster order) -> numpy uint8 bits [..., n] (host)."""
    import numpy as np
    a = bits.detach().cpu().numpy().view(np.uint8)
    return np.unpackbits(a, axis=-1, bitorder="little")[..., :n]


def prof_enable(on: bool = True):
    """Start/stop per-launch HIP-event timing inside the library."""
    _check(lib().holo_prof_enable(1 if on else 0))


def prof_read(kernel: str):
    """(total_ms, launches) recorded for `kernel` since the last reset."""
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().holo_prof_read(kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def prof_reset():
    lib().holo_prof_reset()


PLAN_OSPR, PLAN_GS = 0, 1
PLAN_INTS = 7
DEFAULT_PLAN = [0, 0, 0, 0, -1, 0, 0]


def autotune_ospr(target, n_sf: int, lut: Lut, reps: int = 5, stream=None):
    """holo_autotune_ospr: returns the chosen plan [cols, rows, ksplit, recon_cols, pad, chunk, pts]."""
    import numpy as np
    ny, nx = target.shape
    _dev(target, torch.float32, None, "target")
    scratch = torch.empty((n_sf, nx * ny // 32), dtype=torch.int32, device=target.device)
    out = np.zeros(PLAN_INTS, dtype=np.int32)
    _check(lib().holo_autotune_ospr(_ptr(target), nx, ny, n_sf, lut.handle, _ptr(scratch), reps,
                                    out.ctypes.data_as(C.c_void_p), _stream(stream)))
    return out.tolist()


def autotune_gs(target, lut: Lut, reps: int = 5, stream=None):
    """holo_autotune_gs: returns the chosen plan [cols, rows, ksplit, recon_cols, pad, chunk, pts]."""
    import numpy as np
    ny, nx = target.shape
    _dev(target, torch.float32, None, "target")
    out = np.zeros(PLAN_INTS, dtype=np.int32)
    _check(lib().holo_autotune_gs(_ptr(target), nx, ny, lut.handle, reps, out.ctypes.data_as(C.c_void_p),
                                  _stream(stream)))
    return out.tolist()


def plan_set(kind: int, nx: int, ny: int, n_sf: int, cfg):
    """cfg: [cols, rows, ksplit, recon_cols, pad, chunk, pts] (a 6-int plan
    gets pts = 0); DEFAULT_PLAN selects the built-in heuristics."""
    import numpy as np
    a = np.ascontiguousarray(list(cfg) + [0] * (PLAN_INTS - len(cfg)) if len(cfg) == PLAN_INTS - 1 else cfg,
                             dtype=np.int32)
    if a.size != PLAN_INTS:
        raise ValueError("a plan is 7 ints: cols, rows, ksplit, recon_cols, pad, chunk, pts")
    _check(lib().holo_plan_set(kind, nx, ny, n_sf, a.ctypes.data_as(C.c_void_p)))


def plan_get(kind: int, nx: int, ny: int, n_sf: int):
    import numpy as np
    a = np.zeros(PLAN_INTS, dtype=np.int32)
    _check(lib().holo_plan_get(kind, nx, ny, n_sf, a.ctypes.data_as(C.c_void_p)))
    return a.tolist()


def plan_save(path: str):
    _check(lib().holo_plan_save(path.encode()))


def plan_load(path: str):
    _check(lib().holo_plan_load(path.encode()))


def set_graphs(on: bool):
    _check(lib().holo_set_graphs(1 if on else 0))


def ospr_generate_batched(targets, n_sfs, lut: Lut, cursor: int, bits=None, recons=None, nmse_out=None,
                          stream=None, precision: int = FP32, mode: str = "binary"):
    """holo_ospr_generate_batched.  targets: list of cuda float32 [ny, nx];
    n_sfs: list of sub-frame counts; bits: list of int32 [n_sf, nx*ny/32]
    (uint8 [n_sf, ny, nx] for mode "levels8"; allocated if None).  Returns
    (bits list, nmse [n, 2] or None, cursor).  nmse_out: cuda float64 [n, 2]
    keeps the NMSE on the device.  mode as for ospr_generate."""
    import numpy as np
    n = len(targets)
    if bits is None:
        bits = [None] * n
    bits = [_holo_buf(mode, k, t.shape[1], t.shape[0], b, t.device) for t, k, b in zip(targets, n_sfs, bits)]
    arr = (HoloFrame * n)()
    for i, (t, k, b) in enumerate(zip(targets, n_sfs, bits)):
        _dev(t, torch.float32, None, "target")
        ny, nx = t.shape
        r = recons[i] if recons is not None else None
        if r is not None:
            _dev(r, torch.float32, (ny, nx), "recon")
        arr[i] = HoloFrame(nx, ny, k, t.data_ptr(), b.data_ptr(), r.data_ptr() if r is not None else None)
    if nmse_out is not None:
        _dev(nmse_out, torch.float64, (n, 2), "nmse_out")
        nm, nm_p, flags = nmse_out, C.c_void_p(nmse_out.data_ptr()), F_NMSE_DEVICE
    else:
        nm = np.zeros((n, 2))
        nm_p, flags = nm.ctypes.data_as(C.c_void_p), 0
    flags |= OSPR_MODES[mode]
    cur = C.c_uint64(cursor)
    _check(lib().holo_ospr_generate_batched(C.cast(arr, C.c_void_p), n, lut.handle, C.byref(cur), nm_p,
                                            precision, flags, _stream(stream)))
    return bits, nm, int(cur.value)


class Cnn:
    """Learned GS seed network (holo_cnn_*)."""

    def __init__(self, seed: int = 1, path: str | None = None):
        h = C.c_void_p()
        if path is not None:
            _check(lib().holo_cnn_load(path.encode(), C.byref(h)))
        else:
            _check(lib().holo_cnn_create(seed, C.byref(h)))
        self._h = h

    @staticmethod
    def nparams() -> int:
        return int(lib().holo_cnn_nparams())

    def params(self):
        import numpy as np
        out = np.zeros(self.nparams(), dtype=np.float32)
        _check(lib().holo_cnn_get_params(self._h, out.ctypes.data_as(C.c_void_p), out.size))
        return out

    def set_params(self, p):
        import numpy as np
        a = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().holo_cnn_set_params(self._h, a.ctypes.data_as(C.c_void_p), a.size))

    def infer(self, target, out=None, stream=None):
        """target cuda float32 [ny, nx] -> cuda complex64 phasor [ny, nx]."""
        _dev(target, torch.float32, None, "target")
        ny, nx = target.shape
        if out is None:
            out = torch.empty((ny, nx), dtype=torch.complex64, device=target.device)
        _dev(out, torch.complex64, (ny, nx), "out")
        _check(lib().holo_cnn_infer(self._h, _ptr(target), nx, ny, _ptr(out), _stream(stream)))
        return out

    def loss_grad(self, target, label, stream=None):
        """(loss, grad [nparams] float32) for one image; label cuda complex64."""
        import numpy as np
        _dev(target, torch.float32, None, "target")
        ny, nx = target.shape
        _dev(label, torch.complex64, (ny, nx), "label")
        loss = C.c_double()
        g = np.zeros(self.nparams(), dtype=np.float32)
        _check(lib().holo_cnn_loss_grad(self._h, _ptr(target), _ptr(label), nx, ny, C.byref(loss),
                                        g.ctypes.data_as(C.c_void_p), _stream(stream)))
        return loss.value, g

    def train_step(self, target, label, lr: float, want_loss: bool = True, stream=None):
        """One Adam step on a batch.  target: cuda float32 [ny, nx] or
        [batch, ny, nx]; label: complex64 of the same shape.  Returns the mean
        loss (or None)."""
        if target.dim() == 2:
            target = target.unsqueeze(0)
            label = label.unsqueeze(0)
        _dev(target, torch.float32, None, "target")
        b, ny, nx = target.shape
        _dev(label, torch.complex64, (b, ny, nx), "label")
        loss = C.c_double()
        _check(lib().holo_cnn_train_step(self._h, _ptr(target), _ptr(label), b, nx, ny, lr,
                                         C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def save(self, path: str):
        _check(lib().holo_cnn_save(self._h, path.encode()))

    def close(self):
        if self._h:
            lib().holo_cnn_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
