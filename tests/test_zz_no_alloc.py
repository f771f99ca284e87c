"""The allocation-free RTM entry point (rtm_rtm_shot_noalloc, scratch in a
fixed device array of the library) against rtm_rtm_shot with a workspace:
the same kernels on the same inputs, so num, den and the image must agree
bit for bit.  Two calls in a row, the second on a smaller grid (the array
then holds the first call's larger state, which the second must not see),
then a shot too large for the array, refused before any work."""
import numpy as np
import pytest
import torch

import paper_2204_03380_amd as rtm
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _shot(s):
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vp = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    w = _t(s.wavelet)
    d = rtm.rtm_model_shot(g, vp, s.dt, w, s.src[0], s.rec)
    return g, vp, w, d


def test_noalloc_equals_workspace_entry_point_twice_then_refuses():
    for s in (synth.config_c1(), synth.config_small2d()):  # the second call is the smaller shot
        g, vp, w, d = _shot(s)
        ref = rtm.rtm_rtm_shot(g, vp, s.dt, w, s.src[0], s.rec, d, eps_rel=1e-3, want_numden=True)
        out = {k: torch.full(g.interior_shape, float("nan"), device=DEV) for k in ("image", "num", "den")}
        rtm.rtm_rtm_shot_noalloc(g, vp, s.dt, w, s.src[0], s.rec, d, out["image"], eps_rel=1e-3, num=out["num"],
                                 den=out["den"])
        torch.cuda.synchronize()
        for k in ("image", "num", "den"):
            assert torch.equal(out[k], ref[k]), f"{s.name}: {k}"
        print(f"{s.name}: image, num, den equal to rtm_rtm_shot's")
    big = synth.config_c2(nshot=1, nt=5000)
    gb = rtm.Grid.for_model(big.v_int, big.h, big.nb)
    assert rtm.rtm_workspace_bytes(gb, rtm.RTM_OP_RTM, big.rec.shape[0], big.nt) > (64 << 20)
    vp = torch.ones(gb.padded_shape, device=DEV)
    w = torch.zeros(big.nt, device=DEV)
    d = torch.zeros((big.rec.shape[0], big.nt + 1), device=DEV)
    im = torch.empty(gb.interior_shape, device=DEV)
    with pytest.raises(rtm.RtmError) as e:
        rtm.rtm_rtm_shot_noalloc(gb, vp, big.dt, w, big.src[0], big.rec, d, im)
    assert e.value.status == -4 and "scratch" in str(e.value)
