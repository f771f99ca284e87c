"""GPU parity of the 3-D path against the FP64 oracle (rel-L2 <= 1e-4),
bit-exact invariance to the 3-D launch shape, and the full 612^2 x 356
padded grid of the layered-salt workload at reduced nt."""
import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
DEV = "cuda:0"


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _small3d(shape=(22, 26, 30), nb=6, nt=150, seed=7):
    """(nz, ny, nx) smooth random model, off-grid source and receivers."""
    v = synth.random_model(shape, seed, 1600, 2800, sigma=2.0)
    nz, ny, nx = shape
    src = np.array([nx * 0.5 + 0.25, ny * 0.4 + 0.5, 3.5])
    xs, ys = np.meshgrid(np.linspace(0.5, nx - 1.5, 7), np.linspace(1.0, ny - 2.0, 5), indexing="xy")
    rec = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, 2.25)], 1).astype(np.float32)
    return v, nb, src, rec, 10.0, 1e-3, nt


def _setup(v, nb, seed=3):
    g = rtm.Grid.for_model(v, 10.0, nb)
    vg = rtm.rtm_rbc_pad(g, _t(v), seed, 0.0)
    vo = oracle.rbc_pad(v, nb, seed, 0.0)
    return g, vg, vo


@pytest.fixture(autouse=True)
def _default_tuning():
    rtm.rtm_set_tuning3d(rtm.RTM_OP_MODEL, 2, 8, 36)
    rtm.rtm_set_tuning3d(rtm.RTM_OP_RTM, 1, 8, 36)
    yield


@pytest.mark.parametrize("shape", [(22, 26, 30), (19, 13, 71)])
def test_model_rtm_vjp_parity_3d(shape):
    v, nb, src, rec, h, dt, nt = _small3d(shape)
    g, vg, vo = _setup(v, nb)
    assert np.array_equal(_n(vg), vo)
    w = synth.ricker(25.0, dt, nt)
    tr, pl, pp = rtm.rtm_model_shot(g, vg, dt, _t(w), src, rec, want_last=True)
    tr_o, pl_o, pp_o = oracle.model_shot(vo, h, nb, dt, w.astype(np.float64), src, rec, want_last=True)
    e = (rel_l2(_n(tr), tr_o), rel_l2(_n(pl), pl_o), rel_l2(_n(pp), pp_o))
    print("3-D model", shape, e)
    assert max(e) < TOL
    d_obs = tr_o.astype(np.float32)
    out = rtm.rtm_rtm_shot(g, vg, dt, _t(w), src, rec, _t(d_obs), eps_rel=1e-3, want_numden=True)
    ref = oracle.rtm_shot(vo, h, nb, dt, w.astype(np.float64), src, rec, d_obs.astype(np.float64), eps_rel=1e-3)
    e = {k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")}
    print("3-D rtm", shape, e)
    assert max(e.values()) < TOL
    gt = np.random.default_rng(1).standard_normal(d_obs.shape).astype(np.float32)
    gv, gw = rtm.rtm_model_shot_vjp(g, vg, dt, _t(w), src, rec, _t(gt), want_wavelet_grad=True)
    ref = oracle.rtm_shot(vo, h, nb, dt, w.astype(np.float64), src, rec, gt.astype(np.float64), want_grad=True,
                          want_wadj=True)
    e = (rel_l2(_n(gv), ref["grad"]), rel_l2(_n(gw), ref["w_adj"]))
    print("3-D vjp", shape, e)
    assert max(e) < TOL


def test_time_reversal_3d():
    v, nb, src, rec, h, dt, nt = _small3d(nt=200)
    g, vg, vo = _setup(v, nb)
    w = synth.ricker(25.0, dt, nt)
    d = rtm.rtm_model_shot(g, vg, dt, _t(w), src, rec)
    for k in (60, 150):
        out = rtm.rtm_rtm_shot(g, vg, dt, _t(w), src, rec, d, snap_k=k)
        _, p_k, _ = rtm.rtm_model_shot(g, vg, dt, _t(w[:k]), src, rec, want_last=True)
        e = rel_l2(_n(out["snap_p"]), _n(p_k))
        print(f"3-D reversal k={k}: {e:.2e}")
        assert e < TOL


def test_launch_shape_invariance_3d():
    v, nb, src, rec, h, dt, nt = _small3d((20, 21, 75), nt=90)
    g, vg, vo = _setup(v, nb)
    w = _t(synth.ricker(25.0, dt, nt))
    d = rtm.rtm_model_shot(g, vg, dt, w, src, rec)
    outs = []
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    try:
        # (forward shape, reverse shape[, tile order]); 16-row workgroups at vec 1 and 2
        for fs, rs, *order in (((1, 4, 9),) * 2, ((2, 8, 18),) * 2, ((4, 8, 36),) * 2, ((2, 4, 27),) * 2,
                               ((1, 8, 9),) * 2, ((1, 16, 9),) * 2, ((2, 16, 18), (1, 16, 27)),
                               ((1, 4, 9), (1, 4, 9), 1), ((2, 8, 18), (1, 8, 27), 1)):
            rtm.rtm_set_tuning3d(rtm.RTM_OP_MODEL, *fs)
            rtm.rtm_set_tuning3d(rtm.RTM_OP_RTM, *rs)
            for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
                rtm.rtm_set_tile_order3d(op, order[0] if order else 0)
            tr = _n(rtm.rtm_model_shot(g, vg, dt, w, src, rec))
            im = _n(rtm.rtm_rtm_shot(g, vg, dt, w, src, rec, d)["image"])
            outs.append((tr, im))
    finally:
        rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 0, 0)
    for tr, im in outs[1:]:
        assert np.array_equal(tr, outs[0][0]) and np.array_equal(im, outs[0][1])



def test_sixteen_row_workgroups_vjp_and_storage():
    """The gradient kernel and the storage receiver pass with 16-row
    workgroups (forward update at vec 2, reverse at vec 1) and with the
    z-innermost tile order give the same bits as with 8-row ones, on a grid
    whose 33 padded rows leave a one-row y tile."""
    v, nb, src, rec, h, dt, nt = _small3d((20, 21, 75), nt=90)
    g, vg, vo = _setup(v, nb)
    w = _t(synth.ricker(25.0, dt, nt))
    d = rtm.rtm_model_shot(g, vg, dt, w, src, rec)
    gt = _t(np.random.default_rng(2).standard_normal(tuple(d.shape)).astype(np.float32))
    outs = []
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    try:
        for fs, rs, order in (((2, 8, 18), (1, 8, 18), 0), ((2, 16, 18), (1, 16, 18), 0), ((1, 16, 27), (1, 16, 9), 0),
                              ((2, 8, 18), (1, 4, 9), 1)):
            rtm.rtm_set_tuning3d(rtm.RTM_OP_MODEL, *fs)
            rtm.rtm_set_tuning3d(rtm.RTM_OP_RTM, *rs)
            for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
                rtm.rtm_set_tile_order3d(op, order)
            gv, gw = rtm.rtm_model_shot_vjp(g, vg, dt, w, src, rec, gt, want_wavelet_grad=True)
            st = rtm.rtm_storage_shot(g, vg, dt, w, src, rec, d, 4, 1, want_numden=True)
            outs.append([_n(gv), _n(gw), _n(st["num"]), _n(st["den"]), _n(st["snapshots"])])
    finally:
        rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 0, 0)
    assert np.any(outs[0][0]) and np.any(outs[0][2])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)

@pytest.mark.timeout(600)
def test_layered_salt_full_grid_reduced_nt():
    """The 512 x 512 x 256 layered-salt workload at its full padded size
    (612 x 612 x 356), 10 steps of a unit-scale random
    wavelet (so that the short run is not dominated by near-zero values):
    traces and image against the oracle."""
    s = synth.config_c3(nt=10)
    g, vg, vo = _setup(s.v_int, s.nb, s.seed)
    nt = 10
    w = np.random.default_rng(0).standard_normal(nt).astype(np.float32)
    src = s.src[0]
    # a sample of the receiver grid near the source keeps the oracle's
    # trace array small; the GPU runs the same geometry
    rec = s.rec[(np.abs(s.rec[:, 0] - src[0]) <= 40) & (np.abs(s.rec[:, 1] - src[1]) <= 40)]
    tr = _n(rtm.rtm_model_shot(g, vg, s.dt, _t(w), src, rec))
    tr_o = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), src, rec)
    e_tr = rel_l2(tr, tr_o)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), src, rec, _t(tr_o), eps_rel=1e-3, want_numden=True)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), src, rec, tr_o.astype(np.float32).astype(np.float64),
                          eps_rel=1e-3)
    e = {k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")}
    print(f"layered salt full grid: traces {e_tr:.2e} {e}")
    assert e_tr < TOL and max(e.values()) < TOL
