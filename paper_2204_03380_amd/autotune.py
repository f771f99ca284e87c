"""Launch-shape autotuner for the propagation kernels.

For a given batch (grid, model, shots), times short runs of the forward and
the fused reverse passes for each candidate launch configuration with the
library's event timing, keeps the fastest per pass and installs it.  A 2-D
candidate is (steps per launch, floats per lane `vec`, strips per workgroup
`tx`, rows per tile `zseg`); a 3-D one is (vec, rows per workgroup `ty`,
planes per tile `zseg`, tile order: 0 y tiles innermost, 1 z bands
innermost).  Candidates are compared by device time per time
step, so configurations that advance one, two or three steps per launch
compete on equal terms.  Results do not depend on the configuration (every
cell is computed by the same arithmetic), so tuning only changes speed.
Choices can be cached in a JSON file keyed by the batch signature.
"""
from __future__ import annotations

import json
import os
from typing import Iterable, Sequence

import torch

from . import (RTM_F_SKIP_CHECK, RTM_OP_MODEL, RTM_OP_RTM, RTM_TUNE_EXACT, BatchPlan, BatchShot, Grid,
               rtm_get_tuning, rtm_set_steps_per_launch, rtm_set_tile_order3d, rtm_set_tuning, rtm_set_tuning2d,
               rtm_set_tuning3d, rtm_timing_enable, rtm_timing_read)

# (steps, vec, tx, zseg): the multi-step kernels take one strip per workgroup
DEFAULT_SHAPES = (tuple((3, v, 1, z) for v in (1, 2, 4) for z in (54, 108, 216)) +
                  tuple((2, v, 1, z) for v in (2, 4) for z in (36, 108)) +
                  tuple((1, v, x, z) for v in (1, 2, 4) for x in (1, 4) for z in (18, 36)))
DEFAULT_SHAPES_3D = tuple((v, y, z, o) for v, y, z in ((1, 4, 18), (1, 8, 18), (2, 8, 18), (1, 4, 36), (2, 8, 36),
                                                      (4, 8, 18), (1, 16, 18), (2, 16, 36))
                          for o in (0, 1))


def signature(grid: Grid, nshots: int) -> str:
    return f"{grid.ndim}d:{grid.nx}x{grid.ny}x{grid.nz}:nb{grid.nb}:shots{nshots}"


def install(shape, op, ndim):
    """Sets the launch configuration of `op`'s kernels: 2-D (steps, vec,
    tx, zseg); 3-D (vec, ty, zseg) or (vec, ty, zseg, z_inner tile order)."""
    if ndim == 3:
        rtm_set_tuning3d(op, *shape[:3])
        if len(shape) > 3:
            rtm_set_tile_order3d(op, shape[3])
    else:
        steps, vec, tx, zseg = shape
        rtm_set_tuning2d(op, vec, tx, zseg)
        rtm_set_steps_per_launch(op, steps)


def reverse_capable(shape, ndim) -> bool:
    """The fused 3-D reverse kernel takes 16-row workgroups at vec 1 only
    (a lane's registers are capped at 128 there)."""
    return not (ndim == 3 and shape[1] == 16 and shape[0] != 1)


def _time_shape(shape, grid, v_pad, wavelet, srcs, rec, dt, nt_probe, reps):
    """(forward, reverse) us per step; reverse is inf for a shape only the
    forward kernels take (the reverse then runs at vec 1, untimed)."""
    rev_ok = reverse_capable(shape, grid.ndim)
    install(shape, RTM_OP_MODEL, grid.ndim)
    install(shape if rev_ok else (1, *shape[1:]), RTM_OP_RTM, grid.ndim)
    dev = v_pad.device
    w = wavelet[:nt_probe].contiguous()
    nrec = len(rec)
    traces = [torch.zeros((nrec, nt_probe + 1), dtype=torch.float32, device=dev) for _ in srcs]
    image = torch.zeros(grid.interior_shape, dtype=torch.float32, device=dev)
    mp = BatchPlan(RTM_OP_MODEL, [BatchShot(grid, v_pad, w, s, rec, traces_out=t) for s, t in zip(srcs, traces)],
                   dt, nt_probe, flags=RTM_F_SKIP_CHECK)
    rp = BatchPlan(RTM_OP_RTM, [BatchShot(grid, v_pad, w, s, rec, traces_in=t, image=image)
                                for s, t in zip(srcs, traces)], dt, nt_probe, flags=RTM_F_SKIP_CHECK)
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
    steps = reps * nt_probe
    fwd = t["model_forward"][0] * 1e3 / steps   # us per time step
    rev = t["reverse_image"][0] * 1e3 / steps if rev_ok else float("inf")
    mp.free()
    rp.free()
    return fwd, rev


def tune_batch(grid: Grid, v_pad: torch.Tensor, wavelet: torch.Tensor, srcs: Sequence, rec, dt: float,
               nt_probe: int = 120, reps: int = 2, shapes: Iterable = None,
               cache_path: str | None = None, verbose: bool = False) -> dict:
    """Picks and installs the fastest forward and reverse configurations for
    a batch of shots on one grid (see the module docstring for the shape
    tuples), each timed exactly as given (no narrowing).  nt_probe should be
    a multiple of 6 so that every steps-per-launch setting divides it.
    Returns {"forward": (*shape, us per step), "reverse": (*shape, us per
    step), "table": {shape: (forward us, reverse us)}}.  The no-narrowing
    setting is left as it was."""
    if shapes is None:
        shapes = DEFAULT_SHAPES_3D if grid.ndim == 3 else DEFAULT_SHAPES
    key = signature(grid, len(srcs))
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            res = cache[key]
            install(tuple(res["forward"][:-1]), RTM_OP_MODEL, grid.ndim)
            install(tuple(res["reverse"][:-1]), RTM_OP_RTM, grid.ndim)
            return res
    table = {}
    best_f = best_r = None
    exact = rtm_get_tuning(RTM_TUNE_EXACT)[0]
    rtm_set_tuning(RTM_TUNE_EXACT, 1, 0)   # time each configuration as given
    try:
        for shape in shapes:
            fwd, rev = _time_shape(shape, grid, v_pad, wavelet, srcs, rec, dt, nt_probe, reps)
            table["x".join(str(v) for v in shape)] = (fwd, rev)
            if verbose:
                print(f"  {shape}: forward {fwd:9.3f} us/step  reverse {rev:9.3f} us/step", flush=True)
            if best_f is None or fwd < best_f[-1]:
                best_f = (*shape, fwd)
            if best_r is None or rev < best_r[-1]:
                best_r = (*shape, rev)
    finally:
        rtm_set_tuning(RTM_TUNE_EXACT, exact, 0)
    install(tuple(best_f[:-1]), RTM_OP_MODEL, grid.ndim)
    install(tuple(best_r[:-1]), RTM_OP_RTM, grid.ndim)
    res = {"forward": best_f, "reverse": best_r, "table": table}
    if cache_path:
        cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        cache[key] = res
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return res
