"""Persistent passes (RTM_F_PERSISTENT): one launch per pass for all time
steps, each shot advancing on its own progress counter.  Results equal the
launch-per-step plans bit for bit (the same one-step arithmetic) for
modeling, migration and the gradient of uneven-aperture shots and of a
single shot; and a bounded wait that is forced to give up (a zero wait
limit, set from the host) ends the run with an error instead of a hang."""
import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _windows(nshot=6, nz=41, nxg=420, nt=200, seed=31):
    """Windows of 60-200 columns of one smooth model, each with its own band."""
    rng = np.random.default_rng(seed)
    big = synth.random_model((nz, nxg), seed, 1600, 3200, sigma=3.0)
    shots = []
    for i in range(nshot):
        w = int(rng.integers(60, 201))
        x0 = int(rng.integers(0, nxg - w))
        v = np.ascontiguousarray(big[:, x0:x0 + w])
        g = rtm.Grid.for_model(v, 10.0, 10)
        vp = rtm.rtm_rbc_pad(g, _t(v), 200 + i, 0.0)
        src = np.array([(w - 1) / 2.0 + 0.25, 0.0, 2.5])
        rec = synth.line_receivers(np.arange(w, dtype=np.float64), 2.0)
        shots.append(dict(v=v, g=g, vp=vp, src=src, rec=rec, seed=200 + i))
    return shots, nt


def _run_all(shots, nt, w, flags):
    """Modeling, RTM (per-shot images) and VJP of every shot as batch plans."""
    dt = 1e-3
    tr = [torch.empty((s["rec"].shape[0], nt + 1), device=DEV) for s in shots]
    rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(s["g"], s["vp"], w, s["src"], s["rec"], traces_out=o)
                                     for s, o in zip(shots, tr)], dt, nt, flags=flags).run()
    im = [torch.empty(s["g"].interior_shape, device=DEV) for s in shots]
    rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(s["g"], s["vp"], w, s["src"], s["rec"], traces_in=d, image=o)
                                   for s, d, o in zip(shots, tr, im)], dt, nt, eps_rel=1e-3, flags=flags).run()
    gv = [torch.empty(s["g"].padded_shape, device=DEV) for s in shots]
    rtm.BatchPlan(rtm.RTM_OP_VJP, [rtm.BatchShot(s["g"], s["vp"], w, s["src"], s["rec"], traces_in=d, grad_v_pad=o)
                                   for s, d, o in zip(shots, tr, gv)], dt, nt, flags=flags).run()
    return tr, im, gv


@pytest.mark.parametrize("vec", [1, 2])
def test_persistent_equals_launch_per_step_uneven_shots(vec):
    shots, nt = _windows()
    w = _t(synth.ricker(20.0, 1e-3, nt))
    for op in (rtm.RTM_OP_MODEL, rtm.RTM_OP_RTM):
        rtm.rtm_set_tuning2d(op, vec, 1, 18)
    ref = _run_all(shots, nt, w, 0)
    got = _run_all(shots, nt, w, rtm.RTM_F_PERSISTENT)
    for kind, a_list, b_list in zip(("traces", "image", "gradient"), got, ref):
        for i, (a, b) in enumerate(zip(a_list, b_list)):
            assert torch.equal(a, b), f"{kind} of shot {i}"
    # and one shot against the oracle
    s = shots[2]
    vo = oracle.rbc_pad(s["v"], 10, s["seed"], 0.0)
    tr_o = oracle.model_shot(vo, 10.0, 10, 1e-3, _n(w).astype(np.float64), s["src"], s["rec"])
    e = float(np.linalg.norm(_n(got[0][2]) - tr_o) / np.linalg.norm(tr_o))
    print(f"persistent vec {vec}: bit-identical to per-step launches; shot 2 traces vs oracle {e:.2e}")
    assert e < 1e-4


def test_persistent_single_shot_two_layer():
    """The 201 x 201 two-layer shot (nt 1000) as a one-shot persistent plan:
    traces and image equal the single-shot entry points'."""
    s = synth.config_c1()
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vp = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    w = _t(s.wavelet)
    d = torch.empty((s.rec.shape[0], s.nt + 1), device=DEV)
    rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(g, vp, w, s.src[0], s.rec, traces_out=d)], s.dt, s.nt,
                  flags=rtm.RTM_F_PERSISTENT).run()
    im = torch.empty(g.interior_shape, device=DEV)
    rtm.BatchPlan(rtm.RTM_OP_RTM, [rtm.BatchShot(g, vp, w, s.src[0], s.rec, traces_in=d, image=im)], s.dt, s.nt,
                  eps_rel=1e-3, flags=rtm.RTM_F_PERSISTENT).run()
    d_ref = rtm.rtm_model_shot(g, vp, s.dt, w, s.src[0], s.rec)
    im_ref = rtm.rtm_rtm_shot(g, vp, s.dt, w, s.src[0], s.rec, d_ref, eps_rel=1e-3)["image"]
    assert torch.equal(d, d_ref) and torch.equal(im, im_ref)


def test_persistent_bounded_wait_gives_up():
    """A zero wait limit makes the first workgroup that finds its shot's
    previous step unfinished give up; every other one stops at its next wait;
    the run returns RTM_EHIP.  The next run with the default limit is
    correct again."""
    shots, nt = _windows(nshot=4, nt=60)
    w = _t(synth.ricker(20.0, 1e-3, nt))
    tr = [torch.empty((s["rec"].shape[0], nt + 1), device=DEV) for s in shots]
    plan = rtm.BatchPlan(rtm.RTM_OP_MODEL, [rtm.BatchShot(s["g"], s["vp"], w, s["src"], s["rec"], traces_out=o)
                                            for s, o in zip(shots, tr)], 1e-3, nt, flags=rtm.RTM_F_PERSISTENT)
    old = rtm.rtm_get_persist_wait()
    try:
        rtm.rtm_set_persist_wait(0.0)
        with pytest.raises(rtm.RtmError) as e:
            plan.run()
        assert e.value.status == -5 and "persistent run stopped" in str(e.value)
    finally:
        rtm.rtm_set_persist_wait(old)
    plan.run()
    ref = [rtm.rtm_model_shot(s["g"], s["vp"], 1e-3, w, s["src"], s["rec"]) for s in shots]
    for a, b in zip(tr, ref):
        assert torch.equal(a, b)
