"""The launch-configuration autotuner: it times every candidate (steps per
launch, floats per lane, strips per workgroup, rows per tile), installs the
fastest per pass, and the results of a batch do not depend on the
configuration, bit for bit."""
import numpy as np
import pytest
import torch

import paper_2204_03380_amd as rtm
import synth
from paper_2204_03380_amd import autotune

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CANDIDATES = ((3, 2, 1, 54), (3, 1, 1, 108), (2, 2, 1, 36), (1, 1, 4, 18), (1, 4, 1, 36))


def _batch():
    s = synth.config_small2d(nx=300, nz=120, nb=20, nt=120, seed=12)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vp = rtm.rtm_rbc_pad(g, torch.from_numpy(s.v_int).to(DEV), s.seed, 0.0)
    w = torch.from_numpy(s.wavelet).to(DEV)
    srcs = [np.array([x, 0.0, 3.5]) for x in (20.5, 101.0, 177.25, 260.0)]
    return s, g, vp, w, srcs


def _run(s, g, vp, w, srcs):
    tr = [torch.empty((s.rec.shape[0], s.nt + 1), device=DEV) for _ in srcs]
    rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vp, w, x, s.rec, traces_out=t) for x, t in zip(srcs, tr)],
                  s.dt, s.nt).run()
    stack = torch.zeros(g.interior_shape, device=DEV)
    rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, vp, w, x, s.rec, traces_in=t, image=stack)
                                   for x, t in zip(srcs, tr)], s.dt, s.nt, eps_rel=1e-3,
                  flags=rtm.RTM_F_ACCUMULATE).run()
    torch.cuda.synchronize()
    return tr, stack


def test_results_equal_across_candidates():
    s, g, vp, w, srcs = _batch()
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    outs = []
    for shape in CANDIDATES:
        autotune.install(shape, rtm.RTM_OP_MODEL, 2)
        autotune.install(shape, rtm.RTM_OP_RTM, 2)
        outs.append(_run(s, g, vp, w, srcs))
    for (tr, im), shape in zip(outs[1:], CANDIDATES[1:]):
        assert all(torch.equal(a, b) for a, b in zip(tr, outs[0][0])), shape
        assert torch.equal(im, outs[0][1]), shape


def test_tuner_installs_its_fastest_candidate():
    s, g, vp, w, srcs = _batch()
    res = autotune.tune_batch(g, vp, w, srcs, s.rec, s.dt, nt_probe=60, reps=1, shapes=CANDIDATES)
    print("tuner table (us per step, forward / reverse):", res["table"])
    assert len(res["table"]) == len(CANDIDATES)
    assert all(f > 0 and r > 0 for f, r in res["table"].values())
    for op, key in ((rtm.RTM_OP_MODEL, "forward"), (rtm.RTM_OP_RTM, "reverse")):
        best = tuple(res[key][:-1])
        assert best in CANDIDATES
        col = 0 if key == "forward" else 1
        assert res[key][-1] == min(v[col] for v in res["table"].values())
        steps, vec, tx, zseg = best
        assert rtm.rtm_get_tuning2d(op) == (vec, tx, zseg)
        assert rtm.rtm_get_steps_per_launch(op) == steps
    assert rtm.rtm_get_tuning(rtm.RTM_TUNE_EXACT)[0] == 0  # left as found


def test_tuner_3d_with_tile_orders():
    """3-D candidates (vec, rows per workgroup, planes per tile, tile order)
    on a small layered grid: the table covers every candidate, the fastest
    forward and reverse shapes and orders are installed (a forward-only
    candidate has no reverse time), and a shot migrated under the installed
    configuration equals the default one bit for bit."""
    v = synth.layered_salt_3d(44, 37, 30, 5)
    h, nb, dt, nt = 10.0, 8, 1e-3, 60
    g = rtm.Grid.for_model(v, h, nb)
    vp = rtm.rtm_rbc_pad(g, torch.from_numpy(v).to(DEV), 2, 0.0)
    w = torch.from_numpy(synth.ricker(15.0, dt, nt)).to(DEV)
    src = np.array([21.5, 18.0, 2.0])
    xs, ys = np.meshgrid(np.arange(0, 44, 3, dtype=np.float64), np.arange(0, 37, 3, dtype=np.float64), indexing="xy")
    rec = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, 2.0)], 1).astype(np.float32)
    d = rtm.rtm_model_shot(g, vp, dt, w, src, rec)
    ref = rtm.rtm_rtm_shot(g, vp, dt, w, src, rec, d)["image"]
    shapes = ((1, 4, 18, 0), (1, 4, 18, 1), (2, 8, 9, 1), (2, 16, 9, 0))
    res = autotune.tune_batch(g, vp, w, [src], rec, dt, nt_probe=36, reps=1, shapes=shapes)
    print("3-D tuner table (us per step, forward / reverse):", res["table"])
    assert len(res["table"]) == len(shapes)
    assert res["table"]["2x16x9x0"][1] == float("inf")
    for op, key in ((rtm.RTM_OP_MODEL, "forward"), (rtm.RTM_OP_RTM, "reverse")):
        best = tuple(res[key][:-1])
        assert best in shapes
        assert rtm.rtm_get_tuning3d(op) == best[:3] and rtm.rtm_get_tile_order3d(op) == best[3]
    rtm.rtm_set_tuning(rtm.RTM_TUNE_EXACT, 1, 0)
    d2 = rtm.rtm_model_shot(g, vp, dt, w, src, rec)
    im2 = rtm.rtm_rtm_shot(g, vp, dt, w, src, rec, d2)["image"]
    assert torch.equal(d2, d) and torch.equal(im2, ref)
