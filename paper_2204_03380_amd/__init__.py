"""Random-boundary RTM on MI355X: Python binding of librtm.

Every function here marshals arguments for the C ABI of include/rtm.h and
calls it; all computation runs in the library's HIP kernels.  PyTorch only
provides device memory and the current stream.  Arrays are torch tensors on
the GPU (float32, contiguous); positions are host arrays of (x, y, z) in
interior grid units.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import (RTM_F_ACCUMULATE, RTM_F_CHECK_FINITE, RTM_F_GRAPH, RTM_F_PERSISTENT, RTM_F_NO_REINJECT, RTM_F_SKIP_CHECK, RTM_OP_MODEL,
                   RTM_OP_RBC_PAD, RTM_OP_RTM, RTM_OP_STORAGE, RTM_OP_VJP, RTM_TUNE_EXACT, RtmError)

__all__ = [
    "Grid", "RtmError", "rtm_workspace_bytes", "rtm_set_tuning", "rtm_get_tuning", "rtm_set_tuning3d", "rtm_get_tuning3d", "rtm_set_tile_order3d", "rtm_get_tile_order3d", "rtm_timing_enable", "rtm_timing_read", "rtm_rbc_pad", "rtm_pad_adjoint",
    "rtm_model_shot", "rtm_rtm_shot", "rtm_model_shot_vjp", "RTM_F_SKIP_CHECK", "RTM_F_NO_REINJECT",
    "rtm_nyquist_stride", "rtm_storage_count", "rtm_storage_shot", "RTM_OP_STORAGE",
    "RTM_OP_MODEL", "RTM_OP_RTM", "RTM_OP_VJP", "RTM_OP_RBC_PAD", "RTM_F_ACCUMULATE", "RTM_F_GRAPH", "RTM_F_CHECK_FINITE", "RTM_TUNE_EXACT", "RTM_F_PERSISTENT",
    "BatchShot", "BatchPlan", "rtm_window_extract", "rtm_window_accumulate", "rtm_l2_misfit",
    "rtm_set_tuning2d", "rtm_get_tuning2d", "rtm_set_steps_per_launch", "rtm_get_steps_per_launch",
    "tuning_snapshot", "tuning_restore", "rtm_stream_copy", "rtm_rtm_shot_noalloc",
    "rtm_set_persist_wait", "rtm_get_persist_wait",
]


@dataclass(frozen=True)
class Grid:
    """Interior extents, spacing (m) and random-boundary width (cells)."""
    ndim: int
    nx: int
    ny: int
    nz: int
    h: float
    nb: int

    @staticmethod
    def for_model(v_int, h: float, nb: int) -> "Grid":
        shape = tuple(v_int.shape)
        if len(shape) == 2:
            return Grid(2, shape[1], 1, shape[0], float(h), int(nb))
        return Grid(3, shape[2], shape[1], shape[0], float(h), int(nb))

    @property
    def padded_shape(self):
        nb = self.nb
        if self.ndim == 2:
            return (self.nz + 2 * nb, self.nx + 2 * nb)
        return (self.nz + 2 * nb, self.ny + 2 * nb, self.nx + 2 * nb)

    @property
    def interior_shape(self):
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    def c(self) -> _lib.RtmGrid:
        return _lib.RtmGrid(self.ndim, self.nb, self.nx, self.ny if self.ndim == 3 else 1, self.nz, self.h)


def _dev(t: torch.Tensor, name: str, shape=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _pos(a, name) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, 3))
    if a.shape[0] < 1:
        raise ValueError(f"{name} is empty")
    return a


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def rtm_workspace_bytes(grid: Grid, op: int, nrec: int = 0, nt: int = 0) -> int:
    out = ctypes.c_size_t(0)
    g = grid.c()
    _lib.check(_lib.load().rtm_workspace_bytes(ctypes.byref(g), op, nrec, nt, ctypes.byref(out)))
    return int(out.value)


def _workspace(grid: Grid, op: int, nrec: int, nt: int, device) -> torch.Tensor:
    n = rtm_workspace_bytes(grid, op, nrec, nt)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def rtm_set_tuning(op: int, vec: int, zseg: int) -> None:
    _lib.check(_lib.load().rtm_set_tuning(op, vec, zseg))


def rtm_set_tuning3d(op: int, vec: int, ty: int, zseg: int) -> None:
    _lib.check(_lib.load().rtm_set_tuning3d(op, vec, ty, zseg))


def rtm_get_tuning3d(op: int):
    """(vec, ty, zseg) currently used for `op` on 3-D grids."""
    v, y, z = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _lib.check(_lib.load().rtm_get_tuning3d(op, ctypes.byref(v), ctypes.byref(y), ctypes.byref(z)))
    return int(v.value), int(y.value), int(z.value)


def rtm_set_tile_order3d(op: int, z_inner: int) -> None:
    """3-D tile numbering: 0 y tiles innermost (default), 1 z bands innermost."""
    _lib.check(_lib.load().rtm_set_tile_order3d(op, int(z_inner)))


def rtm_get_tile_order3d(op: int) -> int:
    z = ctypes.c_int()
    _lib.check(_lib.load().rtm_get_tile_order3d(op, ctypes.byref(z)))
    return z.value


def rtm_set_tuning2d(op: int, vec: int, tx: int, zseg: int) -> None:
    _lib.check(_lib.load().rtm_set_tuning2d(op, vec, tx, zseg))


def rtm_get_tuning2d(op: int):
    """(vec, tx, zseg) currently used for `op` on 2-D grids."""
    v, x, z = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _lib.check(_lib.load().rtm_get_tuning2d(op, ctypes.byref(v), ctypes.byref(x), ctypes.byref(z)))
    return int(v.value), int(x.value), int(z.value)


def rtm_set_steps_per_launch(op: int, steps: int) -> None:
    """Time steps per 2-D launch, 1, 2 or 3: RTM_OP_MODEL for every forward
    pass, RTM_OP_RTM for the imaging reverse pass.  Results are the same bits
    whatever the setting; jobs too small to fill the GPU take fewer."""
    _lib.check(_lib.load().rtm_set_steps_per_launch(op, steps))


def rtm_get_steps_per_launch(op: int) -> int:
    """The configured time steps per 2-D launch of `op`."""
    v = ctypes.c_int(0)
    _lib.check(_lib.load().rtm_get_steps_per_launch(op, ctypes.byref(v)))
    return int(v.value)


def rtm_get_tuning(op: int):
    """(vec, zseg) currently used for `op`."""
    v, z = ctypes.c_int(0), ctypes.c_int(0)
    _lib.check(_lib.load().rtm_get_tuning(op, ctypes.byref(v), ctypes.byref(z)))
    return int(v.value), int(z.value)


def tuning_snapshot() -> dict:
    """The process-wide launch settings (2-D and 3-D shapes, the 3-D tile
    order, 2-D steps per launch, the no-narrowing flag), for tuning_restore."""
    snap = {"exact": rtm_get_tuning(RTM_TUNE_EXACT)[0]}
    for op in (RTM_OP_MODEL, RTM_OP_RTM):
        snap[("2d", op)] = rtm_get_tuning2d(op)
        snap[("steps", op)] = rtm_get_steps_per_launch(op)
        snap[("3d", op)] = rtm_get_tuning3d(op)
        snap[("order3d", op)] = rtm_get_tile_order3d(op)
    return snap


def tuning_restore(snap: dict) -> None:
    """Sets the launch settings recorded by tuning_snapshot."""
    rtm_set_tuning(RTM_TUNE_EXACT, int(snap["exact"]), 0)
    for op in (RTM_OP_MODEL, RTM_OP_RTM):
        rtm_set_tuning2d(op, *snap[("2d", op)])
        rtm_set_steps_per_launch(op, snap[("steps", op)])
        rtm_set_tuning3d(op, *snap[("3d", op)])
        rtm_set_tile_order3d(op, snap[("order3d", op)])


def rtm_set_persist_wait(ms: float) -> None:
    """Bounded wait (milliseconds) of RTM_F_PERSISTENT passes."""
    _lib.check(_lib.load().rtm_set_persist_wait(float(ms)))


def rtm_get_persist_wait() -> float:
    v = ctypes.c_double(0.0)
    _lib.check(_lib.load().rtm_get_persist_wait(ctypes.byref(v)))
    return float(v.value)


LOOP_KINDS = ("model_forward", "rtm_forward", "reverse_image", "reverse_grad")


def rtm_timing_enable(on: bool = True) -> None:
    _lib.check(_lib.load().rtm_timing_enable(1 if on else 0))


def rtm_timing_read() -> dict:
    """{kind: (milliseconds, launches)} of the loops recorded since the last
    read (see rtm_timing_enable)."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _lib.check(_lib.load().rtm_timing_read(ms, n))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(LOOP_KINDS)}


def _rbc_opts(seed, v_cap, free_surface, taper):
    flags = (_lib.RTM_RBC_FREE_SURFACE if free_surface else 0) | (_lib.RTM_RBC_TAPER if taper is not None else 0)
    return _lib.RtmRbcOpts(int(seed), float(v_cap), flags, float(taper) if taper is not None else 0.0)


def rtm_rbc_pad(grid: Grid, v_int: torch.Tensor, seed: int, v_cap: float = 0.0,
                out: torch.Tensor = None, free_surface: bool = False, taper=None) -> torch.Tensor:
    """Padded FP32 velocity with the seeded random boundary (see rtm.h);
    taper: None or the weight in [0, 1] of the linear profile against the
    Gaussian one (Eqs. (4)-(5)); free_surface: zero velocity above the
    interior."""
    _dev(v_int, "v_int", grid.interior_shape)
    if out is None:
        v_pad = torch.empty(grid.padded_shape, dtype=torch.float32, device=v_int.device)
    else:
        _dev(out, "out", grid.padded_shape)
        v_pad = out
    ws = _workspace(grid, RTM_OP_RBC_PAD, 0, 0, v_int.device)
    g = grid.c()
    o = _rbc_opts(seed, v_cap, free_surface, taper)
    _lib.check(_lib.load().rtm_rbc_pad_ex(ctypes.byref(g), v_int.data_ptr(), ctypes.byref(o), v_pad.data_ptr(),
                                          ws.data_ptr(), ws.numel(), _stream(v_int.device)))
    return v_pad


def rtm_pad_adjoint(grid: Grid, v_int: torch.Tensor, seed: int, v_cap: float,
                    grad_v_pad: torch.Tensor, free_surface: bool = False, taper=None) -> torch.Tensor:
    _dev(v_int, "v_int", grid.interior_shape)
    _dev(grad_v_pad, "grad_v_pad", grid.padded_shape)
    out = torch.empty(grid.interior_shape, dtype=torch.float32, device=v_int.device)
    ws = _workspace(grid, RTM_OP_RBC_PAD, 0, 0, v_int.device)
    g = grid.c()
    o = _rbc_opts(seed, v_cap, free_surface, taper)
    _lib.check(_lib.load().rtm_pad_adjoint_ex(ctypes.byref(g), v_int.data_ptr(), ctypes.byref(o),
                                              grad_v_pad.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                              _stream(v_int.device)))
    return out


def rtm_model_shot(grid: Grid, v_pad: torch.Tensor, dt: float, wavelet: torch.Tensor, src, rec,
                   want_last: bool = False, flags: int = 0):
    """Traces [nrec, nt + 1] of one shot; with want_last also the final two
    padded states (p^nt, p^(nt-1))."""
    dev = v_pad.device
    _dev(v_pad, "v_pad", grid.padded_shape)
    nt = int(wavelet.numel())
    _dev(wavelet, "wavelet", (nt,))
    src = _pos(src, "src")[0].copy()
    rec = _pos(rec, "rec")
    nrec = rec.shape[0]
    traces = torch.empty((nrec, nt + 1), dtype=torch.float32, device=dev)
    p_last = torch.empty(grid.padded_shape, dtype=torch.float32, device=dev) if want_last else None
    p_prev = torch.empty(grid.padded_shape, dtype=torch.float32, device=dev) if want_last else None
    ws = _workspace(grid, RTM_OP_MODEL, nrec, nt, dev)
    g = grid.c()
    _lib.check(_lib.load().rtm_model_shot(
        ctypes.byref(g), v_pad.data_ptr(), float(dt), nt, wavelet.data_ptr(), _fp(src), nrec, _fp(rec),
        traces.data_ptr(), p_last.data_ptr() if want_last else None, p_prev.data_ptr() if want_last else None,
        int(flags), ws.data_ptr(), ws.numel(), _stream(dev)))
    return (traces, p_last, p_prev) if want_last else traces


def rtm_rtm_shot(grid: Grid, v_pad: torch.Tensor, dt: float, wavelet: torch.Tensor, src, rec,
                 traces: torch.Tensor, eps_rel: float = 1e-3, want_numden: bool = False, snap_k: int = -1,
                 flags: int = 0) -> dict:
    """Image of one shot (interior); optionally num, den and the probe
    snapshots snap_p, snap_mu at step snap_k."""
    dev = v_pad.device
    _dev(v_pad, "v_pad", grid.padded_shape)
    nt = int(wavelet.numel())
    _dev(wavelet, "wavelet", (nt,))
    src = _pos(src, "src")[0].copy()
    rec = _pos(rec, "rec")
    nrec = rec.shape[0]
    _dev(traces, "traces", (nrec, nt + 1))
    out = {"image": torch.empty(grid.interior_shape, dtype=torch.float32, device=dev)}
    if want_numden:
        out["num"] = torch.empty(grid.interior_shape, dtype=torch.float32, device=dev)
        out["den"] = torch.empty(grid.interior_shape, dtype=torch.float32, device=dev)
    probe = None
    if snap_k >= 0:
        out["snap_p"] = torch.zeros(grid.padded_shape, dtype=torch.float32, device=dev)
        out["snap_mu"] = torch.zeros(grid.padded_shape, dtype=torch.float32, device=dev)
        probe = _lib.RtmProbe(snap_k, out["snap_p"].data_ptr(), out["snap_mu"].data_ptr())
    ws = _workspace(grid, RTM_OP_RTM, nrec, nt, dev)
    g = grid.c()
    _lib.check(_lib.load().rtm_rtm_shot(
        ctypes.byref(g), v_pad.data_ptr(), float(dt), nt, wavelet.data_ptr(), _fp(src), nrec, _fp(rec),
        traces.data_ptr(), float(eps_rel), out["image"].data_ptr(),
        out["num"].data_ptr() if want_numden else None, out["den"].data_ptr() if want_numden else None,
        ctypes.byref(probe) if probe is not None else None, int(flags), ws.data_ptr(), ws.numel(), _stream(dev)))
    return out


def rtm_rtm_shot_noalloc(grid: Grid, v_pad: torch.Tensor, dt: float, wavelet: torch.Tensor, src, rec,
                         traces: torch.Tensor, image: torch.Tensor, eps_rel: float = 1e-3, num: torch.Tensor = None,
                         den: torch.Tensor = None, flags: int = 0) -> torch.Tensor:
    """rtm_rtm_shot into caller-provided outputs, with the library's fixed
    scratch array instead of a workspace: allocates no device memory (the
    outputs are given).  Returns image."""
    dev = v_pad.device
    _dev(v_pad, "v_pad", grid.padded_shape)
    nt = int(wavelet.numel())
    _dev(wavelet, "wavelet", (nt,))
    src = _pos(src, "src")[0].copy()
    rec = _pos(rec, "rec")
    nrec = rec.shape[0]
    _dev(traces, "traces", (nrec, nt + 1))
    _dev(image, "image", grid.interior_shape)
    for t, name in ((num, "num"), (den, "den")):
        if t is not None:
            _dev(t, name, grid.interior_shape)
    g = grid.c()
    _lib.check(_lib.load().rtm_rtm_shot_noalloc(
        ctypes.byref(g), v_pad.data_ptr(), float(dt), nt, wavelet.data_ptr(), _fp(src), nrec, _fp(rec),
        traces.data_ptr(), float(eps_rel), image.data_ptr(), num.data_ptr() if num is not None else None,
        den.data_ptr() if den is not None else None, int(flags), _stream(dev)))
    return image


def rtm_nyquist_stride(dt: float, f_max: float, f_min: float = 0.0) -> int:
    """Snapshot step of the stored source wavefield, Eq. (7), in time steps."""
    out = ctypes.c_int32()
    _lib.check(_lib.load().rtm_nyquist_stride(float(dt), float(f_max), float(f_min), ctypes.byref(out)))
    return out.value


def rtm_storage_count(nt: int, stride: int, phase: int = 0) -> int:
    """Number of levels k in [0, nt) with k = phase (mod stride)."""
    out = ctypes.c_int64()
    _lib.check(_lib.load().rtm_storage_count(int(nt), int(stride), int(phase), ctypes.byref(out)))
    return out.value


def rtm_storage_shot(grid: Grid, v_pad: torch.Tensor, dt: float, wavelet: torch.Tensor, src, rec,
                     traces: torch.Tensor, stride: int, phase: int = 0, eps_rel: float = 1e-3,
                     want_numden: bool = False, snapshots: torch.Tensor = None, flags: int = 0) -> dict:
    """Image of one shot with the source wavefield stored every `stride`
    steps in device memory (Algorithm 2 with Eq. (7)).  Returns image
    (interior), the snapshots [count, *interior] and optionally num, den.
    A preallocated `snapshots` tensor of at least that size may be passed."""
    dev = v_pad.device
    _dev(v_pad, "v_pad", grid.padded_shape)
    nt = int(wavelet.numel())
    _dev(wavelet, "wavelet", (nt,))
    src = _pos(src, "src")[0].copy()
    rec = _pos(rec, "rec")
    nrec = rec.shape[0]
    _dev(traces, "traces", (nrec, nt + 1))
    count = rtm_storage_count(nt, stride, phase)
    if snapshots is None:
        snapshots = torch.empty((count,) + tuple(grid.interior_shape), dtype=torch.float32, device=dev)
    _dev(snapshots, "snapshots")
    out = {"image": torch.empty(grid.interior_shape, dtype=torch.float32, device=dev), "snapshots": snapshots}
    if want_numden:
        out["num"] = torch.empty(grid.interior_shape, dtype=torch.float32, device=dev)
        out["den"] = torch.empty(grid.interior_shape, dtype=torch.float32, device=dev)
    ws = _workspace(grid, RTM_OP_STORAGE, nrec, nt, dev)
    g = grid.c()
    _lib.check(_lib.load().rtm_storage_shot(
        ctypes.byref(g), v_pad.data_ptr(), float(dt), nt, wavelet.data_ptr(), _fp(src), nrec, _fp(rec),
        traces.data_ptr(), int(stride), int(phase), float(eps_rel), out["image"].data_ptr(),
        out["num"].data_ptr() if want_numden else None, out["den"].data_ptr() if want_numden else None,
        snapshots.data_ptr(), snapshots.numel() * 4, int(flags), ws.data_ptr(), ws.numel(), _stream(dev)))
    return out


def rtm_model_shot_vjp(grid: Grid, v_pad: torch.Tensor, dt: float, wavelet: torch.Tensor, src, rec,
                       grad_traces: torch.Tensor, want_wavelet_grad: bool = False, flags: int = 0):
    """dJ/dv_pad (padded) for upstream dJ/dtraces; optionally dJ/dwavelet."""
    dev = v_pad.device
    _dev(v_pad, "v_pad", grid.padded_shape)
    nt = int(wavelet.numel())
    _dev(wavelet, "wavelet", (nt,))
    src = _pos(src, "src")[0].copy()
    rec = _pos(rec, "rec")
    nrec = rec.shape[0]
    _dev(grad_traces, "grad_traces", (nrec, nt + 1))
    gv = torch.empty(grid.padded_shape, dtype=torch.float32, device=dev)
    gw = torch.empty((nt,), dtype=torch.float32, device=dev) if want_wavelet_grad else None
    ws = _workspace(grid, RTM_OP_VJP, nrec, nt, dev)
    g = grid.c()
    _lib.check(_lib.load().rtm_model_shot_vjp(
        ctypes.byref(g), v_pad.data_ptr(), float(dt), nt, wavelet.data_ptr(), _fp(src), nrec, _fp(rec),
        grad_traces.data_ptr(), gv.data_ptr(), gw.data_ptr() if want_wavelet_grad else None, int(flags),
        ws.data_ptr(), ws.numel(), _stream(dev)))
    return (gv, gw) if want_wavelet_grad else gv


def rtm_window_extract(global_model: torch.Tensor, x0: int, width: int) -> torch.Tensor:
    """Columns [x0, x0 + width) of a [nz][nx] device array, as a new tensor."""
    _dev(global_model, "global_model")
    nz, nxg = global_model.shape
    out = torch.empty((nz, width), dtype=torch.float32, device=global_model.device)
    _lib.check(_lib.load().rtm_window_extract(nz, nxg, int(x0), int(width), global_model.data_ptr(), out.data_ptr(),
                                              _stream(global_model.device)))
    return out


def rtm_window_accumulate(global_model: torch.Tensor, x0: int, window: torch.Tensor) -> None:
    """global_model[:, x0:x0 + w] += window, in the library's kernel."""
    _dev(global_model, "global_model")
    nz, nxg = global_model.shape
    _dev(window, "window", (nz, window.shape[1]))
    _lib.check(_lib.load().rtm_window_accumulate(nz, nxg, int(x0), int(window.shape[1]), window.data_ptr(),
                                                 global_model.data_ptr(), _stream(global_model.device)))


def rtm_l2_misfit(d: torch.Tensor, d_obs: torch.Tensor, want_residual: bool = True):
    """(J, residual): J = 0.5 sum (d - d_obs)^2 as a float64 device scalar,
    residual = d - d_obs (or None)."""
    _dev(d, "d")
    _dev(d_obs, "d_obs", tuple(d.shape))
    nb = ctypes.c_size_t(0)
    _lib.check(_lib.load().rtm_misfit_ws_bytes(ctypes.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=d.device)
    J = torch.empty((), dtype=torch.float64, device=d.device)
    r = torch.empty_like(d) if want_residual else None
    _lib.check(_lib.load().rtm_l2_misfit(d.numel(), d.data_ptr(), d_obs.data_ptr(), r.data_ptr() if r is not None
                                         else None, J.data_ptr(), ws.data_ptr(), ws.numel(), _stream(d.device)))
    return J, r


def rtm_stream_copy(src: torch.Tensor, dst: torch.Tensor, blocks_per_cu: int = 8) -> None:
    """dst <- src with the library's streaming copy kernel (the bandwidth
    reference of the measurements); both contiguous device tensors of the
    same byte size, a multiple of 16."""
    for t, name in ((src, "src"), (dst, "dst")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous CUDA (HIP) tensor")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _lib.check(_lib.load().rtm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, int(blocks_per_cu),
                                           _stream(src.device)))


@dataclass
class BatchShot:
    """One shot of a batch (see rtm_shot_desc_t): its grid, padded model,
    wavelet, positions and the device buffers the operation reads or writes."""
    grid: Grid
    v_pad: torch.Tensor
    wavelet: torch.Tensor
    src: object
    rec: object
    traces_in: torch.Tensor = None
    traces_out: torch.Tensor = None
    image: torch.Tensor = None
    grad_v_pad: torch.Tensor = None


class BatchPlan:
    """rtm_batch_plan / rtm_batch_run / rtm_batch_free over torch tensors.
    The plan keeps references to every tensor it was given.  The workspace
    is `ws` if given, else one of its own (`ws_bytes`), or none yet with
    `defer_workspace=True` (for plans that will share one workspace sized
    for the largest of them: `bind_workspace` before `run`)."""

    def __init__(self, op: int, shots, dt: float, nt: int, eps_rel: float = 1e-3, flags: int = 0,
                 ws: torch.Tensor = None, defer_workspace: bool = False):
        self._shots = list(shots)
        n = len(self._shots)
        descs = (_lib.RtmShotDesc * n)()
        self._recs = []
        dev = None
        for i, s in enumerate(self._shots):
            _dev(s.v_pad, "v_pad", s.grid.padded_shape)
            _dev(s.wavelet, "wavelet", (nt,))
            rec = _pos(s.rec, "rec")
            self._recs.append(rec)
            nrec = rec.shape[0]
            d = descs[i]
            d.grid = s.grid.c()
            d.v_pad = s.v_pad.data_ptr()
            d.wavelet = s.wavelet.data_ptr()
            src = _pos(s.src, "src")[0]
            for k in range(3):
                d.src[k] = float(src[k])
            d.nrec = nrec
            d.rec = rec.ctypes.data
            if s.traces_in is not None:
                d.traces_in = _dev(s.traces_in, "traces_in", (nrec, nt + 1))
            if s.traces_out is not None:
                d.traces_out = _dev(s.traces_out, "traces_out", (nrec, nt + 1))
            if s.image is not None:
                d.image = _dev(s.image, "image", s.grid.interior_shape)
            if s.grad_v_pad is not None:
                d.grad_v_pad = _dev(s.grad_v_pad, "grad_v_pad", s.grid.padded_shape)
            dev = s.v_pad.device
        self.device = dev
        self.flags = flags
        shared_ws = ws
        plan = ctypes.c_void_p()
        ws = ctypes.c_size_t(0)
        _lib.check(_lib.load().rtm_batch_plan(op, n, descs, float(dt), int(nt), float(eps_rel), int(flags),
                                              ctypes.byref(plan), ctypes.byref(ws)))
        self._plan = plan
        self.ws_bytes = int(ws.value)
        self.ws = None
        if shared_ws is not None or not defer_workspace:
            self.bind_workspace(shared_ws)

    def bind_workspace(self, ws: torch.Tensor = None) -> None:
        """Use `ws` (uint8, at least ws_bytes) as workspace, else allocate one."""
        if ws is not None:
            if ws.dtype != torch.uint8 or ws.numel() < self.ws_bytes or not ws.is_cuda:
                raise ValueError(f"workspace must be a CUDA uint8 tensor of >= {self.ws_bytes} bytes")
            self.ws = ws
        else:
            self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)

    def tensors(self):
        """Every device tensor the plan's runs read or write: the workspace,
        then each shot's buffers."""
        out = [self.ws]
        for s in self._shots:
            out += [t for t in (s.v_pad, s.wavelet, s.traces_in, s.traces_out, s.image, s.grad_v_pad)
                    if t is not None]
        return out

    def run(self, stream: "torch.cuda.Stream" = None) -> None:
        """Runs the plan on `stream` (default: the current stream).

        On a stream other than the current one, both orders of torch's
        stream-ordered memory reuse are covered: the stream first waits for
        the current one (the workspace and inputs were allocated and written
        there, and memory torch hands out on it may still be read by work
        queued on it), and every tensor the run touches is marked as used on
        `stream` (record_stream), so that freeing one on the current stream
        afterwards does not let torch hand its memory out again before the
        run has finished with it."""
        if self.ws is None:
            raise RuntimeError("BatchPlan.run: no workspace bound (defer_workspace=True needs bind_workspace first)")
        cur = torch.cuda.current_stream(self.device)
        side = stream is not None and stream.cuda_stream != cur.cuda_stream
        if side:
            stream.wait_stream(cur)
        st = stream.cuda_stream if stream is not None else cur.cuda_stream
        _lib.check(_lib.load().rtm_batch_run(self._plan, self.ws.data_ptr(), self.ws.numel(), st))
        if side:
            for t in self.tensors():
                t.record_stream(stream)

    def free(self) -> None:
        if getattr(self, "_plan", None) is not None and self._plan.value:
            _lib.load().rtm_batch_free(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
