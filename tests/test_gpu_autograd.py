"""Differentiable modeling: the hand-written adjoint behind
torch.autograd against the FP64 oracle, and the uneven-aperture batched
gradient checked by finite differences on 16 seeded cells."""
import numpy as np
import pytest
import torch

import oracle
import paper_2204_03380_amd as rtm
import synth
from paper_2204_03380_amd.autograd import L2Misfit, ModelShot, WindowedModeling, windowed_misfit

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


def _oracle_grad(v_int, nb, seed, cap, h, dt, w, src, rec, d_obs):
    """Oracle composition: pad, model, residual, reverse gradient, pad adjoint."""
    vp = oracle.rbc_pad(v_int, nb, seed, cap)
    d = oracle.model_shot(vp, h, nb, dt, w.astype(np.float64), src, rec)
    r = d - d_obs.astype(np.float64)
    out = oracle.rtm_shot(vp, h, nb, dt, w.astype(np.float64), src, rec, r, want_grad=True, want_wadj=True)
    return oracle.pad_adjoint(v_int, nb, seed, cap, out["grad"]), out["w_adj"], 0.5 * float(np.sum(r * r))


def test_model_shot_autograd_vs_oracle():
    s = synth.config_small2d(nt=260)
    cap = 3000.0
    g = rtm.Grid.for_model(s.v_int, s.h, s.nb)
    v_true = s.v_int.copy()
    v_true[12:18, :] *= np.float32(1.07)
    d_obs = oracle.model_shot(oracle.rbc_pad(v_true, s.nb, s.seed, cap), s.h, s.nb, s.dt,
                              s.wavelet.astype(np.float64), s.src[0], s.rec).astype(np.float32)
    v = _t(s.v_int).requires_grad_(True)
    w = _t(s.wavelet).requires_grad_(True)
    traces = ModelShot.apply(v, g, s.seed, cap, s.dt, w, s.src[0], s.rec)
    J = L2Misfit.apply(traces, _t(d_obs))
    J.backward()
    gi_o, gw_o, J_o = _oracle_grad(s.v_int, s.nb, s.seed, cap, s.h, s.dt, s.wavelet, s.src[0], s.rec, d_obs)
    e_g, e_w = rel_l2(_n(v.grad), gi_o), rel_l2(_n(w.grad), gw_o)
    print(f"autograd: J {float(J):.6e} vs {J_o:.6e}; grad {e_g:.2e} wavelet grad {e_w:.2e}")
    assert abs(float(J) - J_o) <= 1e-4 * J_o
    assert e_g < TOL and e_w < TOL


def _windows_case(nshot, nz, nxg, wmin, wmax, nt, seed):
    rng = np.random.default_rng(seed)
    v_true = synth.smooth_random_2d(nxg, nz, seed, 5.0, 1500.0, 3500.0)
    from scipy.ndimage import gaussian_filter
    v_cur = gaussian_filter(v_true.astype(np.float64), 20.0, mode="reflect").astype(np.float32)
    widths = rng.integers(wmin, wmax + 1, nshot)
    x0 = np.array([rng.integers(0, nxg - w + 1) for w in widths])
    windows = [(int(a), int(b)) for a, b in zip(x0, widths)]
    srcs = [np.array([(w - 1) // 2, 0.0, 2.0]) for w in widths]
    recs = [synth.line_receivers(np.arange(w, dtype=np.float64), 2.0) for w in widths]
    seeds = [1000 + i for i in range(nshot)]
    return v_true, v_cur, windows, srcs, recs, seeds


def test_windowed_gradient_vs_oracle():
    """Reduced uneven-aperture case (4 shots, 60 x 420 model, nt 300): the
    batched autograd gradient of sum_s 0.5 ||d_s - d_obs_s||^2 equals the sum
    of the oracle's per-shot gradients mapped back into the wide model."""
    h, nb, dt, nt, cap = 10.0, 12, 1e-3, 300, 3500.0
    v_true, v_cur, windows, srcs, recs, seeds = _windows_case(4, 60, 420, 61, 181, nt, 3)
    w = synth.ricker(12.0, dt, nt)
    d_obs, g_ref, J_ref = [], np.zeros(v_cur.shape), 0.0
    for (x0, wd), seed, src, rec in zip(windows, seeds, srcs, recs):
        vt = np.ascontiguousarray(v_true[:, x0:x0 + wd])
        do = oracle.model_shot(oracle.rbc_pad(vt, nb, seed, cap), h, nb, dt, w.astype(np.float64), src,
                               rec).astype(np.float32)
        d_obs.append(do)
        vc = np.ascontiguousarray(v_cur[:, x0:x0 + wd])
        gi, _, J = _oracle_grad(vc, nb, seed, cap, h, dt, w, src, rec, do)
        g_ref[:, x0:x0 + wd] += gi
        J_ref += J
    v = _t(v_cur).requires_grad_(True)
    J = windowed_misfit(v, windows, seeds, cap, h, nb, dt, _t(w), srcs, recs, [_t(d) for d in d_obs])
    J.backward()
    e = rel_l2(_n(v.grad), g_ref)
    print(f"windowed: J {float(J):.6e} vs {J_ref:.6e}; gradient rel-L2 {e:.2e}")
    assert abs(float(J) - J_ref) <= 1e-4 * J_ref
    assert e < TOL


@pytest.mark.timeout(600)
def test_uneven_aperture_gradient_fd_16_cells():
    """The 64-shot uneven-aperture workload (4000 x 300 model at 10 m, windows
    of 401-1201 columns, nt 2000): batched autograd gradient against central
    finite differences of J on 16 seeded cells with large gradient."""
    s = synth.config_c4()
    v_true, v_cur = s.v_int, s.extra["v_cur"]
    windows = [(int(a), int(b)) for a, b in s.extra["windows"]]
    srcs = [s.src[i] for i in range(len(windows))]
    recs = [synth.line_receivers(np.arange(wd, dtype=np.float64), 2.0) for _, wd in windows]
    seeds = [s.seed * 1000 + i for i in range(len(windows))]
    cap = 3500.0
    w = _t(s.wavelet)
    with torch.no_grad():
        d_obs = WindowedModeling.apply(_t(v_true), windows, seeds, cap, s.h, s.nb, s.dt, w, srcs, recs)
    v = _t(v_cur).requires_grad_(True)
    J = windowed_misfit(v, windows, seeds, cap, s.h, s.nb, s.dt, w, srcs, recs, d_obs)
    J.backward()
    grad = _n(v.grad).astype(np.float64)

    def Jof(vm):
        with torch.no_grad():
            return float(windowed_misfit(vm, windows, seeds, cap, s.h, s.nb, s.dt, w, srcs, recs, d_obs))

    rng = np.random.default_rng(16)
    big = np.argwhere(np.abs(grad) >= 0.1 * np.abs(grad).max())
    cells = big[rng.choice(len(big), size=16, replace=False)]
    base = _t(v_cur)
    errs = []
    for (z, x) in cells:
        dv = 1e-3 * float(v_cur[z, x])
        vp = base.clone()
        vm = base.clone()
        vp[z, x] += dv
        vm[z, x] -= dv
        step = float(vp[z, x]) - float(vm[z, x])
        fd = (Jof(vp) - Jof(vm)) / step
        errs.append(abs(fd - grad[z, x]) / abs(grad[z, x]))
    print("FD relative errors on 16 cells:", ["%.1e" % e for e in errs])
    assert max(errs) < 1e-2, errs
