"""Launch-shape autotuner for the 2-D propagation kernels.

For a given batch (grid, model, shots), times short runs of the forward
and the fused reverse kernels for each candidate shape (floats per lane
`vec`, strips per workgroup `tx` in 2-D or rows per workgroup `ty` in 3-D,
rows or planes per tile `zseg`) with the library's event timing, keeps the
fastest shape per kernel and installs it.  Results do
not depend on the shape (the kernels compute every cell the same way), so
tuning only changes speed.  Choices can be cached in a JSON file keyed by
the batch signature.
"""
from __future__ import annotations

import json
import os
from typing import Iterable, Sequence

import torch

from . import (RTM_F_SKIP_CHECK, RTM_OP_MODEL, RTM_OP_RTM, RTM_TUNE_EXACT, BatchPlan, BatchShot, Grid,
               rtm_set_tuning, rtm_set_tuning2d, rtm_set_tuning3d, rtm_timing_enable, rtm_timing_read)

DEFAULT_SHAPES = tuple((v, x, z) for v in (1, 2, 4) for x in (1, 4) for z in (9, 18, 36, 72, 108))
DEFAULT_SHAPES_3D = tuple((v, y, z) for v in (1, 2, 4) for y in (4, 8) for z in (18, 36))


def signature(grid: Grid, nshots: int) -> str:
    return f"{grid.ndim}d:{grid.nx}x{grid.ny}x{grid.nz}:nb{grid.nb}:shots{nshots}"


def _install(shape, op, ndim):
    """2-D: (vec, zseg) keeps the strips per workgroup, (vec, tx, zseg)
    sets them; 3-D: (vec, ty, zseg)."""
    if ndim == 3:
        rtm_set_tuning3d(op, *shape)
    elif len(shape) == 3:
        rtm_set_tuning2d(op, *shape)
    else:
        rtm_set_tuning(op, *shape)


def _time_shape(shape, grid, v_pad, wavelet, srcs, rec, dt, nt_probe, reps, ws):
    _install(shape, RTM_OP_MODEL, grid.ndim)
    _install(shape, RTM_OP_RTM, grid.ndim)
    dev = v_pad.device
    w = wavelet[:nt_probe].contiguous()
    nrec = len(rec)
    traces = [torch.zeros((nrec, nt_probe + 1), dtype=torch.float32, device=dev) for _ in srcs]
    image = torch.zeros(grid.interior_shape, dtype=torch.float32, device=dev)
    mp = BatchPlan(RTM_OP_MODEL, [BatchShot(grid, v_pad, w, s, rec, traces_out=t) for s, t in zip(srcs, traces)],
                   dt, nt_probe, flags=RTM_F_SKIP_CHECK, ws=ws)
    rp = BatchPlan(RTM_OP_RTM, [BatchShot(grid, v_pad, w, s, rec, traces_in=t, image=image)
                                for s, t in zip(srcs, traces)], dt, nt_probe, flags=RTM_F_SKIP_CHECK, ws=ws)
    mp.run()
    rp.run()  # warm
    torch.cuda.synchronize()
    rtm_timing_read()
    rtm_timing_enable(True)
    for _ in range(reps):
        mp.run()
        rp.run()
    torch.cuda.synchronize()
    rtm_timing_enable(False)
    t = rtm_timing_read()
    fwd = t["model_forward"][0] * 1e3 / max(t["model_forward"][1], 1)
    rev = t["reverse_image"][0] * 1e3 / max(t["reverse_image"][1], 1)
    ws_needed = max(mp.ws_bytes, rp.ws_bytes)
    mp.free()
    rp.free()
    return fwd, rev, ws_needed


def tune_batch(grid: Grid, v_pad: torch.Tensor, wavelet: torch.Tensor, srcs: Sequence, rec, dt: float,
               nt_probe: int = 120, reps: int = 2, shapes: Iterable = None,
               cache_path: str | None = None, verbose: bool = False) -> dict:
    """Picks and installs the fastest forward and reverse shapes for a batch
    of shots on one grid.  Shapes are (vec, tx, zseg) or (vec, zseg) in 2-D
    and (vec, ty, zseg) in 3-D.  Returns {"forward": (*shape, us), "reverse": (*shape, us),
    "table": {...}}."""
    if shapes is None:
        shapes = DEFAULT_SHAPES_3D if grid.ndim == 3 else DEFAULT_SHAPES
    key = signature(grid, len(srcs))
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            res = cache[key]
            _install(tuple(res["forward"][:-1]), RTM_OP_MODEL, grid.ndim)
            _install(tuple(res["reverse"][:-1]), RTM_OP_RTM, grid.ndim)
            return res
    table = {}
    best_f = best_r = None
    rtm_set_tuning(RTM_TUNE_EXACT, 1, 0)   # time each shape as given
    for shape in shapes:
        fwd, rev, _ = _time_shape(shape, grid, v_pad, wavelet, srcs, rec, dt, nt_probe, reps, None)
        table["x".join(str(v) for v in shape)] = (fwd, rev)
        if verbose:
            print(f"  shape {shape}: forward {fwd:9.2f} us  reverse {rev:9.2f} us", flush=True)
        if best_f is None or fwd < best_f[-1]:
            best_f = (*shape, fwd)
        if best_r is None or rev < best_r[-1]:
            best_r = (*shape, rev)
    rtm_set_tuning(RTM_TUNE_EXACT, 0, 0)
    _install(tuple(best_f[:-1]), RTM_OP_MODEL, grid.ndim)
    _install(tuple(best_r[:-1]), RTM_OP_RTM, grid.ndim)
    res = {"forward": best_f, "reverse": best_r, "table": table}
    if cache_path:
        cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        cache[key] = res
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return res
