"""GPU parity of the band options (taper of Eqs. (4)-(5), free-surface
top) against the FP64 oracle: padded velocities bit for bit, the padding
adjoint, modeling, RTM and the velocity gradient within rel-L2 1e-4, and
exact time reversal through the reconstruction probe."""
import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
DEV = "cuda:0"
OPTS = [(None, True), (1.0, False), (0.0, True), (0.5, True)]


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("alpha,fs", OPTS)
def test_band_padding_bit_exact(alpha, fs):
    for v, nb, cap in ((synth.config_small2d().v_int, 12, 0.0), (synth.random_model((20, 18, 16), 3, 1500, 3000), 7,
                                                                 2400.0)):
        g = rtm.Grid.for_model(v, 10.0, nb)
        vg = rtm.rtm_rbc_pad(g, _t(v), 99, cap, free_surface=fs, taper=alpha)
        vo = oracle.rbc_pad(v, nb, 99, cap, free_surface=fs, taper=alpha)
        assert np.array_equal(_n(vg), vo), (alpha, fs, v.ndim)


@pytest.mark.parametrize("alpha,fs", OPTS)
def test_band_pad_adjoint(alpha, fs):
    v = synth.random_model((33, 47), 2, 1500, 2500)
    for nb, cap in ((6, 0.0), (6, 2300.0)):
        g = rtm.Grid.for_model(v, 10.0, nb)
        gp = np.random.default_rng(1).standard_normal(g.padded_shape).astype(np.float32)
        gi = rtm.rtm_pad_adjoint(g, _t(v), 31, cap, _t(gp), free_surface=fs, taper=alpha)
        ref = oracle.pad_adjoint(v, nb, 31, cap, gp.astype(np.float64), free_surface=fs, taper=alpha)
        assert rel_l2(_n(gi), ref) < 1e-6


@pytest.mark.parametrize("alpha,fs", [(0.5, True), (1.0, False)])
def test_model_rtm_vjp_with_band_options(alpha, fs):
    s = synth.config_small2d()
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0, free_surface=fs, taper=alpha)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0, free_surface=fs, taper=alpha)
    w = s.wavelet
    print(f"band alpha {alpha} free surface {fs}", flush=True)
    tr = rtm.rtm_model_shot(g, vg, s.dt, _t(w), s.src[0], s.rec)
    tr_o = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec)
    errs = {"traces": rel_l2(_n(tr), tr_o)}
    d = tr_o.astype(np.float32)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d), eps_rel=1e-3, want_numden=True)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, d.astype(np.float64),
                          eps_rel=1e-3)
    errs.update({k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")})
    gt = np.random.default_rng(4).standard_normal(d.shape).astype(np.float32)
    gv = rtm.rtm_model_shot_vjp(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(gt))
    gref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, gt.astype(np.float64),
                           want_grad=True)["grad"]
    gvn = _n(gv)
    errs["grad"] = rel_l2(gvn, gref)
    print(errs)
    assert all(e < TOL for e in errs.values()), errs
    assert np.all(np.isfinite(gvn))
    if fs:
        assert not np.any(gvn[:s.nb])


def test_time_reversal_with_free_surface_and_taper():
    s = synth.config_c1(nt=600)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0, free_surface=True, taper=0.5)
    w = _t(s.wavelet)
    d = rtm.rtm_model_shot(g, vg, s.dt, w, s.src[0], s.rec)
    for k in (150, 450):
        _, pk, _ = rtm.rtm_model_shot(g, vg, s.dt, w[:k].contiguous(), s.src[0], s.rec, want_last=True)
        out = rtm.rtm_rtm_shot(g, vg, s.dt, w, s.src[0], s.rec, d, snap_k=k)
        e = rel_l2(_n(out["snap_p"]), _n(pk))
        assert e < 1e-4, (k, e)
        assert not np.any(_n(out["snap_p"])[:s.nb])
