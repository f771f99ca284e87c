"""GPU parity of migration with a stored source wavefield (Algorithm 2 with
the snapshot decimation of Eq. (7)) against the FP64 oracle: num, den and
image within rel-L2 1e-4, each stored level against the oracle's own modeled
wavefield, 2-D and 3-D, one and two forward steps per launch, ragged grids
and the degenerate decimations (nothing stored, every level stored)."""
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


def _case(name):
    if name == "small2d":
        return synth.config_small2d()
    if name == "ragged2d":
        return synth.config_small2d(nx=131, nz=37, nb=9, nt=180, seed=9)
    if name == "c1":
        return synth.config_c1(nt=600)
    if name == "odd2d":
        return synth.config_small2d(nx=97, nz=53, nb=11, nt=151, seed=13)
    raise KeyError(name)


@pytest.fixture(autouse=True)
def _tuning():
    old = [rtm.rtm_get_steps_per_launch(rtm.RTM_OP_MODEL)]
    rtm.rtm_set_tuning2d(rtm.RTM_OP_MODEL, 1, 1, 18)
    rtm.rtm_set_tuning3d(rtm.RTM_OP_MODEL, 2, 8, 36)
    yield
    rtm.rtm_set_steps_per_launch(rtm.RTM_OP_MODEL, old[0])


def _check_levels(out, vo, s, w, stride, phase, which):
    """Stored levels `which` (indices) against the oracle's p^k."""
    snaps = _n(out["snapshots"])
    nb = s.nb
    nz, nx = s.v_int.shape
    worst = 0.0
    for i in which:
        k = phase + i * stride
        if k == 0:
            assert not np.any(snaps[i])
            continue
        _, pk, _ = oracle.model_shot(vo, s.h, nb, s.dt, w[:k].astype(np.float64), s.src[0], s.rec, want_last=True)
        worst = max(worst, rel_l2(snaps[i], pk[nb:nb + nz, nb:nb + nx]))
    return worst


@pytest.mark.parametrize("name,stride,phase,steps", [
    ("small2d", 1, 0, 2), ("small2d", 10, 0, 1), ("small2d", 10, 0, 2), ("ragged2d", 7, 3, 2),
    ("ragged2d", 4, 1, 1), ("c1", 10, 0, 2), ("odd2d", 3, 2, 2), ("odd2d", 5, 0, 1), ("odd2d", 4, 1, 3)])
def test_storage_shot_parity(name, stride, phase, steps):
    s = _case(name)
    rtm.rtm_set_steps_per_launch(rtm.RTM_OP_MODEL, steps)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    w = s.wavelet
    d_obs = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec).astype(np.float32)
    print(f"case {name} stride {stride} phase {phase} steps {steps}", flush=True)
    out = rtm.rtm_storage_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d_obs), stride, phase, eps_rel=EPS,
                               want_numden=True)
    ref = oracle.rtm_storage_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec,
                                  d_obs.astype(np.float64), stride, phase, eps_rel=EPS)
    errs = {k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")}
    count = rtm.rtm_storage_count(s.nt, stride, phase)
    assert tuple(out["snapshots"].shape) == (count,) + tuple(s.v_int.shape)
    errs["levels"] = _check_levels(out, vo, s, w, stride, phase, sorted({0, count // 2, count - 1}))
    print(name, stride, phase, steps, errs)
    assert all(e < TOL for e in errs.values()), errs


def test_storage_stride1_matches_reconstruction():
    """Every level stored: the image of Algorithm 2 and that of the
    reconstruction path agree (both within the oracle tolerance), and the
    receiver wavefield arithmetic is shared, so num differs only through
    the rounding of the reconstructed p."""
    s = _case("small2d")
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    d_obs = oracle.model_shot(vo, s.h, s.nb, s.dt, s.wavelet.astype(np.float64), s.src[0], s.rec)
    d = _t(d_obs)
    a = rtm.rtm_storage_shot(g, vg, s.dt, _t(s.wavelet), s.src[0], s.rec, d, 1, 0, eps_rel=EPS, want_numden=True)
    b = rtm.rtm_rtm_shot(g, vg, s.dt, _t(s.wavelet), s.src[0], s.rec, d, eps_rel=EPS, want_numden=True)
    for k in ("num", "den", "image"):
        assert rel_l2(_n(a[k]), _n(b[k])) < 2 * TOL


def test_storage_degenerate_decimations():
    """phase >= nt stores nothing (zero sums; the image is then 0 / 0, as in
    the oracle, and not checked); nt = 1; a
    preallocated snapshot buffer is filled in place; a too-small buffer is
    refused."""
    s = synth.config_small2d(nt=40)
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    vg = rtm.rtm_rbc_pad(g, _t(s.v_int), s.seed, 0.0)
    vo = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    w = s.wavelet
    d = oracle.model_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec).astype(np.float32)
    out = rtm.rtm_storage_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d), 50, 45, want_numden=True)
    assert out["snapshots"].shape[0] == 0
    assert not np.any(_n(out["num"])) and not np.any(_n(out["den"]))
    out = rtm.rtm_storage_shot(g, vg, s.dt, _t(w[:1]), s.src[0], s.rec, _t(d[:, :2]), 1, 0, want_numden=True)
    assert out["snapshots"].shape[0] == 1 and not np.any(_n(out["snapshots"]))  # p^0 = 0
    buf = torch.full((5,) + tuple(s.v_int.shape), 7.0, dtype=torch.float32, device=DEV)
    out = rtm.rtm_storage_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d), 10, 0, snapshots=buf, want_numden=True)
    ref = oracle.rtm_storage_shot(vo, s.h, s.nb, s.dt, w.astype(np.float64), s.src[0], s.rec, d.astype(np.float64),
                                  10, 0)
    assert out["snapshots"] is buf and np.all(_n(buf[4]) == 7.0)   # 4 levels stored
    assert rel_l2(_n(out["num"]), ref["num"]) < TOL
    with pytest.raises(rtm.RtmError):
        rtm.rtm_storage_shot(g, vg, s.dt, _t(w), s.src[0], s.rec, _t(d), 10, 0, snapshots=buf[:3])


@pytest.mark.parametrize("shape,stride,phase", [((22, 26, 30), 1, 0), ((19, 13, 71), 6, 2)])
def test_storage_shot_parity_3d(shape, stride, phase):
    v = synth.random_model(shape, 7, 1600, 2800, sigma=2.0)
    nz, ny, nx = shape
    nb, h, dt, nt = 6, 10.0, 1e-3, 150
    src = np.array([nx * 0.5 + 0.25, ny * 0.4 + 0.5, 3.5])
    xs, ys = np.meshgrid(np.linspace(0.5, nx - 1.5, 7), np.linspace(1.0, ny - 2.0, 5), indexing="xy")
    rec = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, 2.25)], 1).astype(np.float32)
    g = rtm.Grid.for_model(v, h, nb)
    vg = rtm.rtm_rbc_pad(g, _t(v), 3, 0.0)
    vo = oracle.rbc_pad(v, nb, 3, 0.0)
    w = synth.ricker(25.0, dt, nt)
    d = oracle.model_shot(vo, h, nb, dt, w.astype(np.float64), src, rec).astype(np.float32)
    print(f"3-D storage {shape} stride {stride} phase {phase}", flush=True)
    out = rtm.rtm_storage_shot(g, vg, dt, _t(w), src, rec, _t(d), stride, phase, eps_rel=EPS, want_numden=True)
    ref = oracle.rtm_storage_shot(vo, h, nb, dt, w.astype(np.float64), src, rec, d.astype(np.float64), stride, phase,
                                  eps_rel=EPS)
    errs = {k: rel_l2(_n(out[k]), ref[k]) for k in ("num", "den", "image")}
    count = rtm.rtm_storage_count(nt, stride, phase)
    i = count // 2
    k = phase + i * stride
    _, pk, _ = oracle.model_shot(vo, h, nb, dt, w[:k].astype(np.float64), src, rec, want_last=True)
    errs["level"] = rel_l2(_n(out["snapshots"][i]), pk[nb:nb + nz, nb:nb + ny, nb:nb + nx])
    print("3-D storage", shape, errs)
    assert all(e < TOL for e in errs.values()), errs
