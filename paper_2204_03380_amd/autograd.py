"""Differentiable modeling on top of librtm.

ModelShot makes one shot of modeling (random-boundary padding followed by
Eq. (1) propagation and receiver sampling) a torch.autograd.Function of the
interior velocity.  Its backward is the library's hand-written adjoint:
the receiver wavefield driven by the upstream trace gradient, correlated
with the source wavefield reconstructed backwards from its last two panels
(no wavefield storage), then mapped through the padding adjoint.

WindowedModeling does the same for many shots of uneven aperture that see
windows of one wide 2-D model, in one batched launch per time step, and
accumulates their gradients back into the wide model.  L2Misfit is the
receiver subtraction and 0.5 ||d - d_obs||^2 in the library's kernels.

The random factors and the velocity cap are held fixed under
differentiation, so v_cap must be given explicitly (> 0).
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import (RTM_OP_MODEL, RTM_OP_VJP, BatchPlan, BatchShot, Grid, rtm_l2_misfit, rtm_model_shot,
               rtm_model_shot_vjp, rtm_pad_adjoint, rtm_rbc_pad, rtm_window_accumulate, rtm_window_extract)


class ModelShot(torch.autograd.Function):
    """traces = model_shot(rbc_pad(v_int)); differentiable in v_int (and in
    the wavelet)."""

    @staticmethod
    def forward(ctx, v_int, grid: Grid, seed: int, v_cap: float, dt: float, wavelet, src, rec):
        if not v_cap > 0:
            raise ValueError("v_cap must be > 0: the cap is a constant of the differentiated map")
        v_int_c = v_int.detach().contiguous()
        v_pad = rtm_rbc_pad(grid, v_int_c, seed, v_cap)
        w = wavelet.detach().contiguous()
        traces = rtm_model_shot(grid, v_pad, dt, w, src, rec)
        ctx.save_for_backward(v_int_c, v_pad, w)
        ctx.cfg = (grid, seed, v_cap, dt, src, rec)
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        v_int, v_pad, w = ctx.saved_tensors
        grid, seed, v_cap, dt, src, rec = ctx.cfg
        want_w = ctx.needs_input_grad[5]
        res = rtm_model_shot_vjp(grid, v_pad, dt, w, src, rec, grad_traces.contiguous(), want_wavelet_grad=want_w)
        gv_pad, gw = (res if want_w else (res, None))
        gv = rtm_pad_adjoint(grid, v_int, seed, v_cap, gv_pad) if ctx.needs_input_grad[0] else None
        return gv, None, None, None, None, gw, None, None


def model_shot(v_int, grid: Grid, seed: int, v_cap: float, dt: float, wavelet, src, rec):
    return ModelShot.apply(v_int, grid, seed, v_cap, dt, wavelet, src, rec)


class L2Misfit(torch.autograd.Function):
    """J = 0.5 ||d - d_obs||^2 (float64 scalar) with dJ/dd = d - d_obs."""

    @staticmethod
    def forward(ctx, d, d_obs):
        J, r = rtm_l2_misfit(d.detach().contiguous(), d_obs.detach().contiguous())
        ctx.save_for_backward(r)
        return J

    @staticmethod
    def backward(ctx, gJ):
        (r,) = ctx.saved_tensors
        g = r if bool(gJ == 1) else r * gJ.to(r.dtype)
        return g, None


class WindowedModeling(torch.autograd.Function):
    """Traces of shots that each see columns [x0, x0 + w) of one wide 2-D
    model (uneven apertures), all shots propagated by one batched launch per
    time step.  Returns one trace tensor per shot."""

    @staticmethod
    def forward(ctx, v_global, windows: Sequence, seeds: Sequence, v_cap: float, h: float, nb: int, dt: float,
                wavelet, srcs: Sequence, recs: Sequence):
        if not v_cap > 0:
            raise ValueError("v_cap must be > 0: the cap is a constant of the differentiated map")
        vg = v_global.detach().contiguous()
        nt = int(wavelet.numel())
        w = wavelet.detach().contiguous()
        shots, v_wins, v_pads, grids, outs = [], [], [], [], []
        for (x0, width), seed, src, rec in zip(windows, seeds, srcs, recs):
            v_win = rtm_window_extract(vg, int(x0), int(width))
            grid = Grid.for_model(v_win, h, nb)
            v_pad = rtm_rbc_pad(grid, v_win, int(seed), v_cap)
            tr = torch.empty((len(rec), nt + 1), dtype=torch.float32, device=vg.device)
            shots.append(BatchShot(grid, v_pad, w, src, rec, traces_out=tr))
            v_wins.append(v_win)
            v_pads.append(v_pad)
            grids.append(grid)
            outs.append(tr)
        BatchPlan(RTM_OP_MODEL, shots, dt, nt).run()
        ctx.save_for_backward(vg, w, *v_wins, *v_pads)
        ctx.cfg = (list(windows), list(seeds), v_cap, dt, list(srcs), list(recs), grids, len(outs))
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        windows, seeds, v_cap, dt, srcs, recs, grids, n = ctx.cfg
        saved = ctx.saved_tensors
        vg, w = saved[0], saved[1]
        v_wins, v_pads = saved[2:2 + n], saved[2 + n:2 + 2 * n]
        nt = int(w.numel())
        shots, gpads = [], []
        for i in range(n):
            g = grads[i]
            if g is None:
                g = torch.zeros((len(recs[i]), nt + 1), dtype=torch.float32, device=vg.device)
            gp = torch.empty(grids[i].padded_shape, dtype=torch.float32, device=vg.device)
            shots.append(BatchShot(grids[i], v_pads[i], w, srcs[i], recs[i], traces_in=g.contiguous(), grad_v_pad=gp))
            gpads.append(gp)
        BatchPlan(RTM_OP_VJP, shots, dt, nt).run()
        grad = torch.zeros_like(vg)
        for i in range(n):
            gi = rtm_pad_adjoint(grids[i], v_wins[i], int(seeds[i]), v_cap, gpads[i])
            rtm_window_accumulate(grad, int(windows[i][0]), gi)
        return (grad,) + (None,) * 9


def windowed_misfit(v_global, windows, seeds, v_cap, h, nb, dt, wavelet, srcs, recs, d_obs):
    """Sum over shots of 0.5 ||d_s - d_obs_s||^2 (differentiable in v_global)."""
    traces = WindowedModeling.apply(v_global, windows, seeds, v_cap, h, nb, dt, wavelet, srcs, recs)
    J = None
    for d, do in zip(traces, d_obs):
        j = L2Misfit.apply(d, do)
        J = j if J is None else J + j
    return J
