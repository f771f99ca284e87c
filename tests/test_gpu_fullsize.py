"""The workloads at the sizes the benchmark and the configurations run, on
the GPU against the FP64 oracle (rel-L2 <= 1e-4) where the oracle can
follow in bounded time:

- the folded-layer survey batch exactly as the benchmark times it (all 240
  shots of the 2301 x 751 grid per launch, three steps per launch, two
  floats per lane, 108-row tiles) at its full 5000 steps;
- the layered-salt 3-D grid at full size (612 x 612 x 356 padded) for 400
  steps, long enough for the wave to cross into the random band;
- the uneven-aperture gradient workload (64 windows, nt 2000), eight
  windows against the oracle's gradients.

The oracle never sees a value produced by the GPU path: each side models its
own data, and where the GPU migrates or differentiates, the oracle's data is
what it is given.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
EPS = 1e-3
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


@pytest.mark.timeout(900)
def test_folded_survey_bench_batch_full_nt(progress):
    """The benchmark's 240-shot batch at its launch shape and full nt 5000.
    Shot 1 (source at a half cell): GPU traces against the oracle's, and the
    GPU image of the oracle's traces against the oracle's image.  Shots 0
    and 239: traces and images equal, bit for bit, one-step single-shot
    calls on the same inputs."""
    nt, B = 5000, 240
    s = synth.config_c2(nshot=B, nt=nt)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    assert np.array_equal(_n(vg), vo)
    w, w64 = _t(s.wavelet), s.wavelet.astype(np.float64)
    srcs = [s.src[i] for i in range(B)]
    progress("oracle: modeling shot 1, nt 5000")
    tr_o = oracle.model_shot(vo, s.h, s.nb, s.dt, w64, srcs[1], s.rec)
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
        rtm.rtm_set_tuning2d(op, 2, 1, 108)
        rtm.rtm_set_steps_per_launch(op, 3)
    progress(f"GPU: {B}-shot modeling and RTM batches")
    traces = [torch.empty((s.rec.shape[0], nt + 1), device=DEV) for _ in srcs]
    plan = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vg, w, x, s.rec, traces_out=t)
                                            for x, t in zip(srcs, traces)], s.dt, nt)
    plan.run()
    plan.free()
    got_tr1 = _n(traces[1])
    traces[1] = _t(tr_o)  # the half-cell shot migrates the oracle's data
    imgs = [torch.empty(g.interior_shape, device=DEV) for _ in srcs]
    plan = rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, vg, w, x, s.rec, traces_in=t, image=im)
                                          for x, t, im in zip(srcs, traces, imgs)], s.dt, nt, eps_rel=EPS)
    plan.run()
    plan.free()
    torch.cuda.synchronize()
    for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
        rtm.rtm_set_tuning2d(op, 1, 1, 18)
        rtm.rtm_set_steps_per_launch(op, 1)
    for i in (0, B - 1):
        progress(f"GPU: one-step single-shot calls, shot {i}")
        ref_tr = rtm.rtm_model_shot(g, vg, s.dt, w, srcs[i], s.rec)
        assert torch.equal(ref_tr, traces[i]), f"shot {i} traces"
        ref_im = rtm.rtm_rtm_shot(g, vg, s.dt, w, srcs[i], s.rec, traces[i], eps_rel=EPS)["image"]
        assert torch.equal(ref_im, imgs[i]), f"shot {i} image"
    progress("oracle: RTM of shot 1, nt 5000")
    ref = oracle.rtm_shot(vo, s.h, s.nb, s.dt, w64, srcs[1], s.rec, tr_o, eps_rel=EPS)
    e_tr, e_im = rel_l2(got_tr1, tr_o), rel_l2(_n(imgs[1]), ref["image"])
    print(f"folded survey batch, nt 5000: traces {e_tr:.2e} image {e_im:.2e}")
    assert e_tr < TOL and e_im < TOL


@pytest.fixture(scope="module")
def salt400(request):
    """The 512 x 512 x 256 layered-salt workload on its full padded grid
    (612 x 612 x 356) with its 12 Hz wavelet for 400 steps (0.4 s: the wave
    from the source two cells below the interior's top crosses about 400 m of
    the 500 m band above it), every receiver of the 256 x 256 surface grid;
    the oracle's padded model and traces (computed once for the two tests)."""
    nt = 400
    s = synth.config_c3(nt=nt)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    tr_o, pl, pp = oracle.model_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), s.src[0], s.rec,
                                     want_last=True)
    return s, vo, tr_o, (pl, pp)


@pytest.mark.timeout(600)
def test_layered_salt_full_grid_nt400_traces(salt400):
    """Random boundary bit for bit and the traces of the 400-step shot."""
    s, vo, tr_o, _ = salt400
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    assert np.array_equal(_n(vg), vo)
    tr = _n(rtm.rtm_model_shot(g, vg, s.dt, _t(s.wavelet), s.src[0], s.rec))
    e_tr = rel_l2(tr, tr_o)
    print(f"layered salt full grid, nt 400: traces {e_tr:.2e}")
    assert e_tr < TOL


@pytest.mark.timeout(600)
def test_layered_salt_full_grid_nt400_image(salt400, progress):
    """The image of the oracle's traces, with num and den, against the
    oracle's RTM of the same traces."""
    s, vo, tr_o, (pl, pp) = salt400
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    out = rtm.rtm_rtm_shot(g, vg, s.dt, _t(s.wavelet), s.src[0], s.rec, _t(tr_o), eps_rel=EPS, want_numden=True)
    got = {k: _n(v) for k, v in out.items()}
    del out, vg
    progress("3-D GPU RTM done; oracle reverse pass, 400 steps of two fields on 133 M cells")
    # the oracle's reverse pass starts from its modeling run's final panels
    # (its full RTM would recompute the same forward pass first)
    ref = oracle.rtm_shot_from_panels(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), s.src[0], s.rec, tr_o,
                                      pl, pp, eps_rel=EPS)
    e = {k: rel_l2(got[k], ref[k]) for k in ("num", "den", "image")}
    print(f"layered salt full grid, nt 400: {e}")
    assert max(e.values()) < TOL


@pytest.mark.timeout(900)
def test_uneven_aperture_gradient_8_windows_vs_oracle():
    """The 64-window uneven-aperture workload at its full size (4000 x 300
    model at 10 m, windows of 401-1201 columns, nt 2000) run as the
    gradient path runs it: one 64-shot modeling batch on the true model and
    one on the current model, the receiver subtraction, one 64-shot gradient
    batch and the padding adjoint.  Eight windows (the narrowest, the widest
    and six seeded others) against the oracle's gradient of
    0.5 ||d - d_obs||^2 for that window, each side from its own data."""
    s = synth.config_c4()
    v_true, v_cur = s.v_int, s.extra["v_cur"]
    windows = [(int(a), int(b)) for a, b in s.extra["windows"]]
    n = len(windows)
    recs = [synth.line_receivers(np.arange(wd, dtype=np.float64), 2.0) for _, wd in windows]
    seeds = [s.seed * 1000 + i for i in range(n)]
    cap = 3500.0
    w, w64 = _t(s.wavelet), s.wavelet.astype(np.float64)
    vt_g, vc_g = _t(v_true), _t(v_cur)
    grids, pads_t, pads_c, wins_c = [], [], [], []
    for (x0, wd), seed in zip(windows, seeds):
        vwt = rtm.rtm_window_extract(vt_g, x0, wd)
        vwc = rtm.rtm_window_extract(vc_g, x0, wd)
        gr = rtm.Grid.for_model(vwc, s.h, s.nb)
        grids.append(gr)
        pads_t.append(rtm.rtm_rbc_pad(gr, vwt, seed, cap))
        pads_c.append(rtm.rtm_rbc_pad(gr, vwc, seed, cap))
        wins_c.append(vwc)
    d_obs = [torch.empty((r.shape[0], s.nt + 1), device=DEV) for r in recs]
    d = [torch.empty((r.shape[0], s.nt + 1), device=DEV) for r in recs]
    for pads, outs in ((pads_t, d_obs), (pads_c, d)):
        rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(gr, vp, w, s.src[i], recs[i], traces_out=o)
                                         for i, (gr, vp, o) in enumerate(zip(grids, pads, outs))],
                      s.dt, s.nt).run()
    res = [rtm.rtm_l2_misfit(a, b)[1] for a, b in zip(d, d_obs)]
    gpads = [torch.empty(gr.padded_shape, device=DEV) for gr in grids]
    rtm.BatchPlan(rtm.RTM_OP_VJP, [rtm.BatchShot(gr, vp, w, s.src[i], recs[i], traces_in=r, grad_v_pad=gp)
                                   for i, (gr, vp, r, gp) in enumerate(zip(grids, pads_c, res, gpads))],
                  s.dt, s.nt).run()
    widths = [wd for _, wd in windows]
    rng = np.random.default_rng(8)
    pick = [int(np.argmin(widths)), int(np.argmax(widths))]
    pick += [int(i) for i in rng.choice([i for i in range(n) if i not in pick], 6, replace=False)]
    errs = []
    for i in pick:
        x0, wd = windows[i]
        gi = _n(rtm.rtm_pad_adjoint(grids[i], wins_c[i], seeds[i], cap, gpads[i]))
        vt = np.ascontiguousarray(v_true[:, x0:x0 + wd])
        vc = np.ascontiguousarray(v_cur[:, x0:x0 + wd])
        vpt = oracle.rbc_pad(vt, s.nb, seeds[i], cap)
        vpc = oracle.rbc_pad(vc, s.nb, seeds[i], cap)
        assert np.array_equal(vpc, _n(pads_c[i]))
        r_o = (oracle.model_shot(vpc, s.h, s.nb, s.dt, w64, s.src[i], recs[i])
               - oracle.model_shot(vpt, s.h, s.nb, s.dt, w64, s.src[i], recs[i]))
        g_pad = oracle.rtm_shot(vpc, s.h, s.nb, s.dt, w64, s.src[i], recs[i], r_o, want_grad=True)["grad"]
        g_o = oracle.pad_adjoint(vc, s.nb, seeds[i], cap, g_pad)
        e_r, e_g = rel_l2(_n(res[i]), r_o), rel_l2(gi, g_o)
        print(f"window {i} (x0 {x0}, width {wd}): residual {e_r:.2e} gradient {e_g:.2e}", flush=True)
        errs.append((e_r, e_g))
    assert max(max(e) for e in errs) < TOL, errs
