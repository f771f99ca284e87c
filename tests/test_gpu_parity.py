"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: relative L2 <= 1e-4 on wavefields, traces, images and gradients;
random-boundary velocities bit-exact.  Inputs are seeded and shared: the
oracle never sees a value produced by the GPU path.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
EPS = 1e-3   # image stabiliser: a water level of 0.1 % of the peak illumination
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


def _case(name):
    if name == "small2d":
        return synth.config_small2d()
    if name == "c1":
        return synth.config_c1()
    if name == "ragged2d":
        s = synth.config_small2d(nx=131, nz=37, nb=9, nt=180, seed=9)
        return s
    raise KeyError(name)


def _setup(s):
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    v_pad_gpu = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    v_pad_orc = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    return g, v_pad_gpu, v_pad_orc


@pytest.fixture(autouse=True)
def _default_tuning():
    steps = {op: rtm.rtm_get_steps_per_launch(op) for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM)}
    rtm.rtm_set_tuning2d(rtm.RTM_OP_MODEL, 1, 1, 18)
    rtm.rtm_set_tuning2d(rtm.RTM_OP_RTM, 1, 1, 18)
    yield
    for op, n in steps.items():  # the library's steps per launch, whatever a test set
        rtm.rtm_set_steps_per_launch(op, n)


# ---------------------------------------------------------------------------

def test_rbc_pad_bit_exact():
    for s in (synth.config_c1(), synth.config_small2d()):
        g, vg, vo = _setup(s)
        assert np.array_equal(_n(vg), vo)
    v3 = synth.random_model((20, 18, 16), 3, 1500, 3000)
    g3 = rtm.Grid.for_model(v3, 10.0, 7)
    for cap in (0.0, 2400.0):
        vg = rtm.rtm_rbc_pad(g3, _t(v3), 123456789, cap)
        assert np.array_equal(_n(vg), oracle.rbc_pad(v3, 7, 123456789, cap))


def test_pad_adjoint_parity():
    v = synth.random_model((33, 47), 2, 1500, 2500)
    for nb, cap in ((6, 0.0), (6, 2300.0), (0, 0.0)):
        g = rtm.Grid.for_model(v, 10.0, nb)
        gp = np.random.default_rng(1).standard_normal(g.padded_shape).astype(np.float32)
        gi = rtm.rtm_pad_adjoint(g, _t(v), 31, cap, _t(gp))
        ref = oracle.pad_adjoint(v, nb, 31, cap, gp.astype(np.float64))
        assert rel_l2(_n(gi), ref) < 1e-6


@pytest.mark.parametrize("name", ["small2d", "ragged2d", "c1"])
def test_model_shot_parity(name):
    s = _case(name)
    g, vg, vo = _setup(s)
    w = s.wavelet
    tr, pl, pp = rtm.rtm_model_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, want_last=True)
    tr_o, pl_o, pp_o = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, want_last=True)
    e_tr, e_pl, e_pp = rel_l2(_n(tr), tr_o), rel_l2(_n(pl), pl_o), rel_l2(_n(pp), pp_o)
    print(f"{name}: traces {e_tr:.2e} p_last {e_pl:.2e} p_prev {e_pp:.2e}")
    assert e_tr < TOL and e_pl < TOL and e_pp < TOL


@pytest.mark.parametrize("name", ["small2d", "ragged2d", "c1"])
def test_rtm_shot_parity(name):
    s = _case(name)
    g, vg, vo = _setup(s)
    w = s.wavelet
    d_obs = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec).astype(np.float32)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d_obs), eps_rel=EPS, want_numden=True)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, d_obs.astype(np.float64),
                          eps_rel=EPS)
    errs = {k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")}
    print(name, errs)
    assert all(e < TOL for e in errs.values()), errs


def test_image_conditioning_small_eps():
    """With a tiny stabiliser the normalised image divides by illumination
    1e6 below its peak, where FP32 wavefields carry relative errors of
    ~1e-3: the image error then grows like ~1e-9 / eps while the Eq. (3)
    integrals stay at ~1e-6.  This pins that the growth is the ratio's
    conditioning, not a drift of num or den."""
    s = synth.config_c1()
    g, vg, vo = _setup(s)
    w = s.wavelet
    d_obs = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec).astype(np.float32)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d_obs), eps_rel=1e-6, want_numden=True)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, d_obs.astype(np.float64),
                          eps_rel=1e-6)
    assert rel_l2(_n(out["num"]), ref["num"]) < TOL and rel_l2(_n(out["den"]), ref["den"]) < TOL
    assert rel_l2(_n(out["image"]), ref["image"]) < 5e-3


def test_time_reversal_and_probe():
    """The reconstructed source wavefield equals the forward one (Sec. on
    wavefield reconstruction), and the receiver wavefield matches the oracle."""
    s = synth.config_c1()
    g, vg, vo = _setup(s)
    w = s.wavelet
    d_obs = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec).astype(np.float32)
    for k in (150, 400, 700):
        out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d_obs), snap_k=k)
        _, p_k, _ = rtm.rtm_model_shot(g, vg, s.dt, _t(w[:k]), s.src[0], s.rec, want_last=True)
        ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, d_obs.astype(np.float64),
                              snap_k=k)
        e_rev = rel_l2(_n(out["snap_p"]), _n(p_k))
        e_p = rel_l2(_n(out["snap_p"]), ref["snap_p"])
        e_mu = rel_l2(_n(out["snap_mu"]), ref["snap_mu"])
        print(f"k={k}: reversal {e_rev:.2e} p vs oracle {e_p:.2e} mu vs oracle {e_mu:.2e}")
        assert e_rev < TOL and e_p < TOL and e_mu < TOL


def test_vjp_parity():
    s = synth.config_small2d(nt=260)
    g, vg, vo = _setup(s)
    w = s.wavelet
    rng = np.random.default_rng(3)
    gt = rng.standard_normal((s.rec.shape[0], s.nt + 1)).astype(np.float32)
    gv, gw = rtm.rtm_model_shot_vjp(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(gt), want_wavelet_grad=True)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, gt.astype(np.float64),
                          want_grad=True, want_wadj=True)
    e_g, e_w = rel_l2(_n(gv), ref["grad"]), rel_l2(_n(gw), ref["w_adj"])
    print(f"grad {e_g:.2e} wavelet grad {e_w:.2e}")
    assert e_g < TOL and e_w < TOL


def test_dot_product_gpu():
    s = synth.config_small2d(nt=200)
    g, vg, _ = _setup(s)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(s.nt).astype(np.float32)
    gt = rng.standard_normal((s.rec.shape[0], s.nt + 1)).astype(np.float32)
    d = _n(rtm.rtm_model_shot(g, vg, s.dt, _t(w), s.src[0], s.rec))
    _, gw = rtm.rtm_model_shot_vjp(g, vg, s.dt, _t(np.zeros_like(w)), s.src[0], s.rec, _t(gt), want_wavelet_grad=True)
    lhs = float(np.sum(gt.astype(np.float64) * d))
    rhs = float(np.dot(w.astype(np.float64), _n(gw)))
    assert abs(lhs - rhs) <= TOL * abs(lhs), (lhs, rhs)


def test_tuning_invariance():
    """Results do not depend on the launch shape: bit-identical."""
    s = synth.config_small2d(nx=150, nz=41, nb=10, nt=150)
    g, vg, vo = _setup(s)
    w = _t(s.wavelet)
    d_obs = _t(oracle.model_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), s.src[0], s.rec))
    outs = []
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    # vec floats per lane, tx strips per workgroup (inner strip ends passed
    # through LDS), zseg rows per tile
    for vec, tx, zseg in ((1, 1, 18), (2, 2, 9), (4, 4, 27), (1, 4, 9), (4, 1, 63), (1, 2, 18), (2, 4, 36)):
        rtm.rtm_set_tuning2d(rtm.RTM_OP_MODEL, vec, tx, zseg)
        rtm.rtm_set_tuning2d(rtm.RTM_OP_RTM, vec, tx, zseg)
        tr = _n(rtm.rtm_model_shot(g, vg, s.dt, w, s.src[0], s.rec))
        im = _n(rtm.rtm_rtm_shot(g, vg, s.dt, w, s.src[0], s.rec, d_obs)["image"])
        outs.append((tr, im))
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 0, 0)
    for tr, im in outs[1:]:
        assert np.array_equal(tr, outs[0][0]) and np.array_equal(im, outs[0][1])


@pytest.mark.parametrize("nt", [150, 151, 152])
def test_two_step_launches_bit_identical(nt):
    """Two and three time steps per launch (overlapping strips, first step
    on a 4- or 8-cell margin) give the same bits as one step per launch, for
    modeling (traces and final panels), RTM (num, den, image) and the
    gradient (its forward pass takes the multi-step launches), for every
    nt mod 2 and mod 3 and several strip widths; off-grid source and
    receivers near strip joins."""
    s = synth.config_small2d(nx=150, nz=41, nb=10, nt=nt)
    g, vg, vo = _setup(s)
    w = _t(s.wavelet)
    d_obs = _t(oracle.model_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), s.src[0], s.rec))
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    outs = []
    try:
        for steps, vec, zseg in ((1, 1, 18), (2, 1, 9), (2, 2, 18), (2, 4, 36), (2, 1, 27), (2, 4, 9), (2, 4, 108),
                                 (3, 1, 9), (3, 2, 18), (3, 4, 36), (3, 1, 27), (3, 4, 9), (3, 4, 108), (3, 2, 9)):
            for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
                rtm.rtm_set_tuning2d(op, vec, 1, zseg)
                rtm.rtm_set_steps_per_launch(op, steps)
            tr, pl, pp = rtm.rtm_model_shot(g, vg, s.dt, w, s.src[0], s.rec, want_last=True)
            out = rtm.rtm_rtm_shot(g, vg, s.dt, w, s.src[0], s.rec, d_obs, want_numden=True)
            gv, gw = rtm.rtm_model_shot_vjp(g, vg, s.dt, w, s.src[0], s.rec, d_obs, want_wavelet_grad=True)
            outs.append([_n(tr), _n(pl), _n(pp), _n(out["num"]), _n(out["den"]), _n(out["image"]), _n(gv), _n(gw)])
    finally:
        rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 0, 0)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), s.src[0], s.rec,
                          _n(d_obs).astype(np.float64), eps_rel=1e-3)
    assert rel_l2(outs[0][5], ref["image"]) < TOL
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_edge_cases():
    # No random boundary, tiny grid, one receiver on the last interior cell, nt = 1.
    v = np.full((5, 7), 2000.0, np.float32)
    for nb, nt in ((0, 1), (0, 30), (3, 25)):
        g = rtm.Grid.for_model(v, 10.0, nb)
        vg = rtm.rtm_rbc_pad(g, _t(v), 1, 0.0)
        vo = oracle.rbc_pad(v, nb, 1, 0.0)
        # Unit-scale random wavelet: a Ricker that has barely started would
        # leave every value near zero and the comparison ill-conditioned.
        w = np.random.default_rng(nt).standard_normal(nt).astype(np.float32)
        src = np.array([[3.0, 0, 2.0]])
        rec = np.array([[6.0, 0, 4.0]])
        tr = _n(rtm.rtm_model_shot(g, vg, 1e-3, _t(w), src[0], rec))
        tr_o = oracle.model_shot(vo, 10.0, nb, 1e-3, w.astype(np.float64), src[0], rec)
        assert rel_l2(tr, tr_o) < TOL or np.abs(tr_o).max() == 0.0
        if nt >= 2:
            out = rtm.rtm_rtm_shot(g, vg, 1e-3, _t(w), src[0], rec, _t(tr_o), want_numden=True)
            ref = oracle.rtm_shot(vo, 10.0, nb, 1e-3, w.astype(np.float64), src[0], rec, tr_o.astype(np.float32).astype(np.float64))
            assert rel_l2(_n(out["num"]), ref["num"]) < TOL


def test_error_codes_on_device():
    s = synth.config_small2d()
    g, vg, _ = _setup(s)
    w = _t(s.wavelet)
    with pytest.raises(rtm.RtmError) as e:
        rtm.rtm_model_shot(g, vg, 0.05, w, s.src[0], s.rec)  # Courant far above the limit
    assert e.value.status == -2
    bad = vg.clone()
    bad[5, 5] = float("nan")
    with pytest.raises(rtm.RtmError) as e:
        rtm.rtm_model_shot(g, bad, s.dt, w, s.src[0], s.rec)
    assert e.value.status == -6
    bad[5, 5] = -1.0
    with pytest.raises(rtm.RtmError) as e:
        rtm.rtm_model_shot(g, bad, s.dt, w, s.src[0], s.rec)
    assert e.value.status == -6


def test_folded_grid_full_size_reduced_nt():
    """The 2301 x 751 folded-layer grid at full size (the benchmark's shot
    shape), with a half-cell source, for 400 steps: traces and image."""
    s = synth.config_c2(nshot=2, nt=400)
    g, vg, vo = _setup(s)
    src = s.src[1]  # x = 24.5: half-cell
    w = s.wavelet
    tr = _n(rtm.rtm_model_shot(g, vg, s.dt, _t(w), src, s.rec))
    tr_o = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), src, s.rec)
    assert rel_l2(tr, tr_o) < TOL
    d_obs = tr_o.astype(np.float32)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), src, s.rec, _t(d_obs), eps_rel=EPS)
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), src, s.rec, d_obs.astype(np.float64),
                          eps_rel=EPS)
    e = rel_l2(_n(out["image"]), ref["image"])
    print(f"folded grid: traces {rel_l2(tr, tr_o):.2e} image {e:.2e}")
    assert e < TOL


def test_check_finite_flag():
    """RTM_F_CHECK_FINITE reports non-finite outputs (here forced by a NaN
    wavelet sample and an infinite trace sample) as RTM_ENUMERIC; the same
    inputs without the flag return normally, and finite runs pass the check."""
    s = synth.config_small2d(nt=80)
    g, vg, vo = _setup(s)
    w = s.wavelet.copy()
    tr = rtm.rtm_model_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, flags=rtm.RTM_F_CHECK_FINITE)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, tr, flags=rtm.RTM_F_CHECK_FINITE)
    assert np.isfinite(_n(out["image"])).all()
    wbad = w.copy()
    wbad[10] = np.nan
    rtm.rtm_model_shot(g, vg, s.dt, _t(wbad), s.src[0], s.rec)   # no check: returns
    with pytest.raises(rtm.RtmError):
        rtm.rtm_model_shot(g, vg, s.dt, _t(wbad), s.src[0], s.rec, flags=rtm.RTM_F_CHECK_FINITE)
    tbad = _n(tr).copy()
    tbad[3, 40] = np.inf
    with pytest.raises(rtm.RtmError):
        rtm.rtm_rtm_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(tbad), flags=rtm.RTM_F_CHECK_FINITE)
    with pytest.raises(rtm.RtmError):
        rtm.rtm_model_shot_vjp(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(tbad), flags=rtm.RTM_F_CHECK_FINITE)


@pytest.mark.parametrize("vec,zseg", [(1, 9), (2, 18), (2, 108)])
def test_three_step_modeling_receiver_rows(vec, zseg):
    """Three-step modeling keeps the middle level only on the rows holding
    receiver nodes, per shot: two shots on one grid with receivers on rows
    that fall in different row tiles (off-grid depths spanning two rows,
    the top and the last interior row, a single receiver) record the same
    bits in one three-step batch as one-step single-shot calls."""
    s = synth.config_small2d(nx=150, nz=41, nb=10, nt=121)
    g, vg, vo = _setup(s)
    w = _t(s.wavelet)
    rec_a = np.array([[x, 0.0, z] for x, z in ((3.0, 0.0), (40.5, 13.75), (77.25, 22.5), (148.0, 40.0),
                                               (100.0, 5.5), (120.75, 31.0))], np.float64)
    rec_b = np.array([[61.5, 0.0, 9.25]], np.float64)
    srcs = (s.src[0], np.array([99.5, 0.0, 20.25]))
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    try:
        rtm.rtm_set_tuning2d(rtm.RTM_OP_MODEL, 1, 1, 18)
        rtm.rtm_set_steps_per_launch(rtm.RTM_OP_MODEL, 1)
        ref = [_n(rtm.rtm_model_shot(g, vg, s.dt, w, src, rec)) for src, rec in zip(srcs, (rec_a, rec_b))]
        rtm.rtm_set_tuning2d(rtm.RTM_OP_MODEL, vec, 1, zseg)
        rtm.rtm_set_steps_per_launch(rtm.RTM_OP_MODEL, 3)
        outs = [torch.empty((rec.shape[0], s.nt + 1), device=DEV) for rec in (rec_a, rec_b)]
        plan = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vg, w, src, rec, traces_out=o)
                                                for src, rec, o in zip(srcs, (rec_a, rec_b), outs)], s.dt, s.nt)
        plan.run()
        got = [_n(o) for o in outs]
    finally:
        rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 0, 0)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    tr_o = oracle.model_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), srcs[0], rec_a)
    assert rel_l2(got[0], tr_o) < TOL


def test_folded_grid_bench_launch_shape():
    """The benchmark's launch configuration (three steps per launch, two
    floats per lane, 108-row tiles, one tile list for several shots) on the
    full 2301 x 751 folded-layer grid for 300 steps: a three-shot batch of
    modeling and RTM.  The half-cell shot's GPU traces against the oracle's;
    its GPU image, migrated from the oracle's traces, against the oracle's
    image of the same traces; every shot against one-step single-shot calls
    on the same inputs, bit for bit."""
    s = synth.config_c2(nshot=3, nt=300)
    g, vg, vo = _setup(s)
    w = _t(s.wavelet)
    w64 = s.wavelet.astype(np.float64)
    srcs = [s.src[i] for i in range(3)]
    tr_o = oracle.model_shot(vo, s.h, s.nb, s.dt, w64, srcs[1], s.rec)
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
        rtm.rtm_set_tuning2d(op, 2, 1, 108)
        rtm.rtm_set_steps_per_launch(op, 3)
    traces = [torch.empty((s.rec.shape[0], s.nt + 1), device=DEV) for _ in srcs]
    plan = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vg, w, x, s.rec, traces_out=t)
                                            for x, t in zip(srcs, traces)], s.dt, s.nt)
    plan.run()
    got_tr = [_n(t) for t in traces]
    d_in = [traces[0], _t(tr_o), traces[2]]  # the half-cell shot migrates the oracle's data
    imgs = [torch.empty(g.interior_shape, device=DEV) for _ in srcs]
    plan = rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, vg, w, x, s.rec, traces_in=t, image=im)
                                          for x, t, im in zip(srcs, d_in, imgs)], s.dt, s.nt, eps_rel=EPS)
    plan.run()
    got_im = [_n(im) for im in imgs]
    for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
        rtm.rtm_set_tuning2d(op, 1, 1, 18)
        rtm.rtm_set_steps_per_launch(op, 1)
    for x, tr, d, im in zip(srcs, got_tr, d_in, got_im):
        ref_tr = rtm.rtm_model_shot(g, vg, s.dt, w, x, s.rec)
        ref_im = rtm.rtm_rtm_shot(g, vg, s.dt, w, x, s.rec, d, eps_rel=EPS)["image"]
        assert np.array_equal(tr, _n(ref_tr)) and np.array_equal(im, _n(ref_im))
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w64, srcs[1], s.rec, tr_o, eps_rel=EPS)
    e_tr, e_im = rel_l2(got_tr[1], tr_o), rel_l2(got_im[1], ref["image"])
    print(f"bench launch shape: traces {e_tr:.2e} image {e_im:.2e}")
    assert e_tr < TOL and e_im < TOL


def test_image_normalisation_interior_max():
    """The water level of Eq. (3)'s ratio uses the maximum of den over the
    interior crop.  On a crafted case where the padded grid's maximum is
    more than 1.5 times the interior's (only the source cell of a 4 x 4
    interior has a velocity; the band corner that takes it collects more
    illumination than the source), the GPU image matches the oracle's."""
    nb, h = 6, 10.0
    v = np.zeros((4, 4), np.float32)
    v[0, 0] = 1500.0
    g = rtm.Grid.for_model(v, h, nb)
    vg = rtm.rtm_rbc_pad(g, _t(v), 3, 0.0)
    vo = oracle.rbc_pad(v, nb, 3, 0.0)
    assert np.array_equal(_n(vg), vo)
    dt = 0.5 * h / (1.3 * 1500.0)
    w = synth.ricker(25.0, dt, 400)
    src, rec = np.array([0.0, 0.0, 0.0]), np.array([[0.0, 0.0, 0.0]])
    d_o = oracle.model_shot(vo, h, nb, dt, w.astype(np.float64), src, rec)
    for eps in (1e-3, 0.5):
        out = rtm.rtm_rtm_shot(g, vg, dt, _t(w), src, rec, _t(d_o), eps_rel=eps, want_numden=True)
        ref = oracle.rtm_shot(vo, h, nb, dt, w.astype(np.float64), src, rec, d_o, eps_rel=eps)
        e = {k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")}
        print(f"interior max, eps {eps}: {e}")
        assert max(e.values()) < TOL


def test_two_layer_long_record_reflector():
    """The two-layer 201 x 201 model recorded for 1.5 s (nt 3000, past the
    interface's two-way time), direct wave removed: GPU traces against the
    oracle's, the GPU image of the oracle's data against the oracle's image,
    and the GPU image's laterally averaged amplitude peaking within two
    cells of the interface at iz = 100."""
    s = synth.config_c1(nt=3000)
    g, vg, vo = _setup(s)
    w, w64 = _t(s.wavelet), s.wavelet.astype(np.float64)
    vh = np.full_like(s.v_int, s.v_int[0, 0])
    cap = float(s.v_int.max())
    vhg = rtm.rtm_rbc_pad(g, _t(vh), s.seed, cap)
    vho = oracle.rbc_pad(vh, s.nb, s.seed, cap)
    d = rtm.rtm_model_shot(g, vg, s.dt, w, s.src[0], s.rec) - rtm.rtm_model_shot(g, vhg, s.dt, w, s.src[0], s.rec)
    d_o = (oracle.model_shot(vo, s.h, s.nb, s.dt, w64, s.src[0], s.rec)
           - oracle.model_shot(vho, s.h, s.nb, s.dt, w64, s.src[0], s.rec))
    e_tr = rel_l2(_n(d), d_o)
    im = _n(rtm.rtm_rtm_shot(g, vg, s.dt, w, s.src[0], s.rec, _t(d_o), eps_rel=EPS)["image"])
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w64, s.src[0], s.rec, d_o, eps_rel=EPS)["image"]
    e_im = rel_l2(im, ref)
    prof = np.abs(im[:, 50:151]).mean(axis=1)
    z = 10 + int(np.argmax(prof[10:]))
    print(f"two-layer long record: reflection data {e_tr:.2e}, image {e_im:.2e}, reflector at iz = {z}")
    assert e_tr < TOL and e_im < TOL
    assert abs(z - 100) <= 2
