"""FP64 CPU oracle for random-boundary RTM -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  The product library never calls it: it is an independent,
plain C implementation written from the paper (arXiv 2204.03380, Eqs. (1)-(3)
and (6), Algorithms 1 to 3 with the snapshot decimation of Eq. (7)), used to prove the GPU path right.

Array conventions: padded fields are numpy arrays of shape (NZ, NX) in 2-D or
(NZ, NY, NX) in 3-D; positions are (x, y, z) in interior grid units; traces
are (nrec, nt + 1).
"""
import ctypes
import os

import numpy as np

from .build import LIB
from .build import build as build_library

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_library()
        lib = ctypes.CDLL(LIB)
        c_long, c_int, c_double, c_u64 = ctypes.c_long, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        P = ctypes.c_void_p
        lib.orc_splitmix64.argtypes = [c_u64, c_u64]
        lib.orc_splitmix64.restype = c_u64
        lib.orc_rbc_pad.argtypes = [c_int, c_long, c_long, c_long, c_int, P, c_u64, ctypes.c_float, P]
        lib.orc_pad_adjoint.argtypes = [c_int, c_long, c_long, c_long, c_int, P, c_u64, ctypes.c_float, P, P]
        lib.orc_rbc_pad_ex.argtypes = [c_int, c_long, c_long, c_long, c_int, P, c_u64, ctypes.c_float, ctypes.c_uint,
                                       c_double, P]
        lib.orc_pad_adjoint_ex.argtypes = [c_int, c_long, c_long, c_long, c_int, P, c_u64, ctypes.c_float,
                                           ctypes.c_uint, c_double, P, P]
        lib.orc_taper.argtypes = [c_int, c_double, P]
        lib.orc_laplacian.argtypes = [c_int, c_long, c_long, c_long, c_double, P, P]
        lib.orc_model_shot.argtypes = [c_int, c_long, c_long, c_long, c_int, c_double, P, c_double, c_int,
                                       P, P, c_int, P, P, P, P, P]
        lib.orc_rtm_shot.argtypes = [c_int, c_long, c_long, c_long, c_int, c_double, P, c_double, c_int,
                                     P, P, c_int, P, P, c_int, c_double, P, P, P, P, P, c_int, P, P]
        lib.orc_rtm_storage_shot.argtypes = [c_int, c_long, c_long, c_long, c_int, c_double, P, c_double, c_int,
                                             P, P, c_int, P, P, c_int, c_int, c_double, P, P, P]
        lib.orc_rtm_shot_panels.argtypes = [c_int, c_long, c_long, c_long, c_int, c_double, P, c_double, c_int,
                                            P, P, c_int, P, P, c_int, c_double, P, P, P, P, P]
        lib.orc_rtm_shot_panels.restype = c_int
        lib.orc_set_threads.argtypes = [c_int]
        lib.orc_set_threads.restype = c_int
        lib.orc_fp_env.argtypes = []
        lib.orc_fp_env.restype = c_int
        for f in ("orc_rbc_pad", "orc_pad_adjoint", "orc_laplacian", "orc_model_shot", "orc_rtm_shot",
                  "orc_rtm_storage_shot", "orc_rbc_pad_ex", "orc_pad_adjoint_ex", "orc_taper"):
            getattr(lib, f).restype = c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _dims(shape, nb):
    """Interior (ndim, nx, ny, nz) from a padded shape."""
    if len(shape) == 2:
        NZ, NX = shape
        return 2, NX - 2 * nb, 1, NZ - 2 * nb
    NZ, NY, NX = shape
    return 3, NX - 2 * nb, NY - 2 * nb, NZ - 2 * nb


def splitmix64(seed: int, k: int) -> int:
    return int(_load().orc_splitmix64(seed, k))


RBC_TAPER = 1
RBC_FREE_SURFACE = 2


def _rbc_flags(free_surface, taper):
    flags = (RBC_FREE_SURFACE if free_surface else 0) | (RBC_TAPER if taper is not None else 0)
    return flags, float(taper) if taper is not None else 0.0


def rbc_pad(v_int, nb: int, seed: int, v_cap: float = 0.0, free_surface: bool = False, taper=None):
    """Padded FP32 velocity with random boundaries (bit-exact definition).
    taper: None, or the weight alpha in [0, 1] of Eq. (4)'s linear taper
    against Eq. (5)'s Gaussian one; free_surface: zero velocity above the
    interior."""
    v_int = np.ascontiguousarray(v_int, dtype=np.float32)
    if v_int.ndim == 2:
        nz, nx = v_int.shape
        ny, ndim, shape = 1, 2, (nz + 2 * nb, nx + 2 * nb)
    else:
        nz, ny, nx = v_int.shape
        ndim, shape = 3, (nz + 2 * nb, ny + 2 * nb, nx + 2 * nb)
    out = np.empty(shape, dtype=np.float32)
    flags, alpha = _rbc_flags(free_surface, taper)
    _check(_load().orc_rbc_pad_ex(ndim, nx, ny, nz, nb, _ptr(v_int), seed, v_cap, flags, alpha, _ptr(out)),
           "orc_rbc_pad_ex")
    return out


def pad_adjoint(v_int, nb: int, seed: int, v_cap: float, grad_pad, free_surface: bool = False, taper=None):
    v_int = np.ascontiguousarray(v_int, dtype=np.float32)
    grad_pad = np.ascontiguousarray(grad_pad, dtype=np.float64)
    if v_int.ndim == 2:
        nz, nx = v_int.shape
        ny, ndim = 1, 2
    else:
        nz, ny, nx = v_int.shape
        ndim = 3
    out = np.empty(v_int.shape, dtype=np.float64)
    flags, alpha = _rbc_flags(free_surface, taper)
    _check(_load().orc_pad_adjoint_ex(ndim, nx, ny, nz, nb, _ptr(v_int), seed, v_cap, flags, alpha, _ptr(grad_pad),
                                      _ptr(out)), "orc_pad_adjoint_ex")
    return out


def taper(nb: int, alpha: float):
    """c_i, i = 1 .. nb, of the band taper (FP32)."""
    out = np.empty(nb, dtype=np.float32)
    _check(_load().orc_taper(nb, float(alpha), _ptr(out)), "orc_taper")
    return out


def laplacian(p, h: float):
    """L_h p on a grid with zero values outside it (8th-order, 9-point)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    if p.ndim == 2:
        ndim, (NZ, NX), NY = 2, p.shape, 1
    else:
        ndim, (NZ, NY, NX) = 3, p.shape
    out = np.empty_like(p)
    _check(_load().orc_laplacian(ndim, NX, NY, NZ, h, _ptr(p), _ptr(out)), "orc_laplacian")
    return out


def _geom(src, rec):
    src = np.ascontiguousarray(np.asarray(src, dtype=np.float64).reshape(3))
    rec = np.ascontiguousarray(np.asarray(rec, dtype=np.float64).reshape(-1, 3))
    return src, rec


def model_shot(v_pad, h, nb, dt, wavelet, src, rec, m=None, want_last=False):
    """Forward modeling; returns traces (nrec, nt+1) [, p_last, p_prev]."""
    v_pad = np.ascontiguousarray(v_pad, dtype=np.float32)
    ndim, nx, ny, nz = _dims(v_pad.shape, nb)
    w = np.ascontiguousarray(wavelet, dtype=np.float64)
    nt = w.shape[0]
    src, rec = _geom(src, rec)
    nrec = rec.shape[0]
    traces = np.zeros((nrec, nt + 1), dtype=np.float64)
    mm = None if m is None else np.ascontiguousarray(m, dtype=np.float64)
    p_last = np.empty(v_pad.shape, np.float64) if want_last else None
    p_prev = np.empty(v_pad.shape, np.float64) if want_last else None
    rc = _load().orc_model_shot(ndim, nx, ny, nz, nb, h, _ptr(v_pad), dt, nt, _ptr(w), _ptr(src), nrec,
                                _ptr(rec), _ptr(mm), _ptr(traces), _ptr(p_last), _ptr(p_prev))
    _check(rc, "orc_model_shot")
    return (traces, p_last, p_prev) if want_last else traces


def rtm_shot(v_pad, h, nb, dt, wavelet, src, rec, g, reinject=True, eps_rel=1e-6, want_grad=False,
             want_wadj=False, snap_k=-1):
    """RTM with reconstruction; returns a dict with num, den, image (interior)
    and optionally grad (padded dJ/dv), w_adj (nt,), snap_p, snap_mu (padded)."""
    v_pad = np.ascontiguousarray(v_pad, dtype=np.float32)
    ndim, nx, ny, nz = _dims(v_pad.shape, nb)
    w = np.ascontiguousarray(wavelet, dtype=np.float64)
    nt = w.shape[0]
    src, rec = _geom(src, rec)
    nrec = rec.shape[0]
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (nrec, nt + 1)
    ishape = (nz, nx) if ndim == 2 else (nz, ny, nx)
    out = {k: np.empty(ishape, np.float64) for k in ("num", "den", "image")}
    grad = np.empty(v_pad.shape, np.float64) if want_grad else None
    wadj = np.empty(nt, np.float64) if want_wadj else None
    sp = np.zeros(v_pad.shape, np.float64) if snap_k >= 0 else None
    sm = np.zeros(v_pad.shape, np.float64) if snap_k >= 0 else None
    rc = _load().orc_rtm_shot(ndim, nx, ny, nz, nb, h, _ptr(v_pad), dt, nt, _ptr(w), _ptr(src), nrec,
                              _ptr(rec), _ptr(g), int(bool(reinject)), eps_rel, _ptr(out["num"]),
                              _ptr(out["den"]), _ptr(out["image"]), _ptr(grad), _ptr(wadj), snap_k,
                              _ptr(sp), _ptr(sm))
    _check(rc, "orc_rtm_shot")
    if want_grad:
        out["grad"] = grad
    if want_wadj:
        out["w_adj"] = wadj
    if snap_k >= 0:
        out["snap_p"], out["snap_mu"] = sp, sm
    return out


def rtm_shot_from_panels(v_pad, h, nb, dt, wavelet, src, rec, g, p_last, p_prev, reinject=True, eps_rel=1e-6):
    """rtm_shot whose reverse pass starts from given final panels p^nt,
    p^(nt-1) (as model_shot(..., want_last=True) returns them) instead of
    recomputing the forward pass; returns num, den, image."""
    v_pad = np.ascontiguousarray(v_pad, dtype=np.float32)
    ndim, nx, ny, nz = _dims(v_pad.shape, nb)
    w = np.ascontiguousarray(wavelet, dtype=np.float64)
    nt = w.shape[0]
    src, rec = _geom(src, rec)
    nrec = rec.shape[0]
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (nrec, nt + 1)
    pl = np.ascontiguousarray(p_last, dtype=np.float64)
    pp = np.ascontiguousarray(p_prev, dtype=np.float64)
    assert pl.shape == v_pad.shape and pp.shape == v_pad.shape
    ishape = (nz, nx) if ndim == 2 else (nz, ny, nx)
    out = {k: np.empty(ishape, np.float64) for k in ("num", "den", "image")}
    rc = _load().orc_rtm_shot_panels(ndim, nx, ny, nz, nb, h, _ptr(v_pad), dt, nt, _ptr(w), _ptr(src), nrec,
                                     _ptr(rec), _ptr(g), int(bool(reinject)), eps_rel, _ptr(out["num"]),
                                     _ptr(out["den"]), _ptr(out["image"]), _ptr(pl), _ptr(pp))
    _check(rc, "orc_rtm_shot_panels")
    return out


def nyquist_stride(dt, f_max, f_min=0.0):
    """Steps between stored panels: the Nyquist interval of Eq. (7),
    1 / (2 (f_max - f_min)), in whole time steps (at least 1)."""
    dtn = 1.0 / (2.0 * (f_max - f_min))
    return max(1, int(np.floor(dtn / dt + 1e-9)))


def rtm_storage_shot(v_pad, h, nb, dt, wavelet, src, rec, g, stride, phase=0, eps_rel=1e-3):
    """RTM with source-wavefield storage every `stride` steps (Algorithm 2
    with the decimation of Eq. (7)); returns num, den, image (interior)."""
    v_pad = np.ascontiguousarray(v_pad, dtype=np.float32)
    ndim, nx, ny, nz = _dims(v_pad.shape, nb)
    w = np.ascontiguousarray(wavelet, dtype=np.float64)
    nt = w.shape[0]
    src, rec = _geom(src, rec)
    nrec = rec.shape[0]
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (nrec, nt + 1)
    ishape = (nz, nx) if ndim == 2 else (nz, ny, nx)
    out = {k: np.empty(ishape, np.float64) for k in ("num", "den", "image")}
    rc = _load().orc_rtm_storage_shot(ndim, nx, ny, nz, nb, h, _ptr(v_pad), dt, nt, _ptr(w), _ptr(src), nrec,
                                      _ptr(rec), _ptr(g), int(stride), int(phase), eps_rel, _ptr(out["num"]),
                                      _ptr(out["den"]), _ptr(out["image"]))
    _check(rc, "orc_rtm_storage_shot")
    return out


def set_threads(n: int = 0) -> int:
    """Threads the oracle's parallel loops use from now on (n >= 1; 0 only
    queries); returns the count in effect."""
    return int(_load().orc_set_threads(int(n)))


def fp_env() -> dict:
    """Denormal handling of the oracle's floating point: flush-to-zero and
    denormals-are-zero flags of the calling thread."""
    v = int(_load().orc_fp_env())
    return {"ftz": bool(v & 1), "daz": bool(v & 2)}
