"""Pins of the oracle's band options: the taper of Eqs. (4)-(5) and the
free-surface top.  Each is checked against something outside the oracle's
own formula: properties of the taper, an independent brute force of the band
values with a different depth computation, a dense-matrix leapfrog on a grid
that simply has no band above the surface, time reversal, and finite
differences of the misfit."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import _dense_laplacian_2d, _py_splitmix64


@pytest.mark.parametrize("nb", [1, 2, 7, 50])
def test_taper_properties(nb):
    g = oracle.taper(nb, 1.0)
    h = oracle.taper(nb, 0.0)
    assert g[0] == 1.0 and h[0] == 1.0
    if nb == 1:
        return
    # Eq. (4): linear from 1 to 0, exact steps of 1 / (nb - 1)
    exact = [np.float32(float(Fraction(nb - i, nb - 1))) for i in range(1, nb + 1)]
    assert np.array_equal(g, np.array(exact, np.float32)) and g[-1] == 0.0
    # Eq. (5): h = e^-1 where 120 (i - 1)^2 = (nb - 1)^2 (checked where that i is whole)
    assert np.all(np.diff(h) <= 0) and np.all(np.diff(g) < 0)
    if nb == 50:
        i = 1 + 49 / math.sqrt(120.0)      # not whole: bracket it
        lo, hi = int(math.floor(i)), int(math.ceil(i))
        assert h[hi - 1] < math.exp(-1.0) < h[lo - 1]
    for a in (0.25, 0.5, 0.75):
        c = oracle.taper(nb, a).astype(np.float64)
        assert np.all(c >= h.astype(np.float64) * (1 - 1e-6) - 1e-30)
        assert np.all(c <= g.astype(np.float64) * (1 + 1e-6) + 1e-30)
    with pytest.raises(RuntimeError):
        oracle.taper(nb, 1.5)


def _depth_by_dilation(pshape, nb):
    """Band depth of every padded cell by repeated dilation of the interior
    with the full (8 / 26)-neighbourhood: the layer at which a cell is first
    reached."""
    inner = np.zeros(pshape, bool)
    inner[tuple(slice(nb, n - nb) for n in pshape)] = True
    depth = np.where(inner, 0, -1)
    cur = inner.copy()
    for layer in range(1, nb + 1):
        grown = cur.copy()
        for off in np.ndindex(*([3] * len(pshape))):
            sl_dst, sl_src = [], []
            for o, n in zip(off, pshape):
                o -= 1
                sl_dst.append(slice(max(o, 0), n + min(o, 0)))
                sl_src.append(slice(max(-o, 0), n + min(-o, 0)))
            grown[tuple(sl_dst)] |= cur[tuple(sl_src)]
        depth[grown & ~cur] = layer
        cur = grown
    return depth


@pytest.mark.parametrize("shape,nb,alpha,fs", [((7, 9), 3, 1.0, False), ((7, 9), 4, 0.0, True),
                                               ((5, 4, 6), 3, 0.5, True), ((6, 8), 5, None, True)])
def test_rbc_options_bruteforce(shape, nb, alpha, fs):
    rng = np.random.default_rng(5)
    v = rng.uniform(1500, 3000, shape).astype(np.float32)
    seed, cap = 1234567, np.float32(2950.0)
    vp = oracle.rbc_pad(v, nb, seed, float(cap), free_surface=fs, taper=alpha)
    depth = _depth_by_dilation(vp.shape, nb)
    if alpha is not None:
        tab = []
        for i in range(1, nb + 1):
            gi = Fraction(nb - i, nb - 1)
            hi = math.exp(-120.0 * (i - 1) ** 2 / (nb - 1) ** 2)
            tab.append(np.float32(alpha * float(gi) + (1.0 - alpha) * hi))
    idx = np.indices(vp.shape).reshape(len(shape), -1).T
    for j, c in enumerate(idx):
        inner = [ci - nb for ci in c]
        e = tuple(min(max(ci, 0), n - 1) for ci, n in zip(inner, shape))
        if depth[tuple(c)] == 0:
            assert vp[tuple(c)] == v[e]
            continue
        if fs and inner[0] < 0:
            assert vp[tuple(c)] == 0.0
            continue
        r = _py_splitmix64(seed, j)
        u = np.float32(r >> 40) * np.float32(2.0 ** -24)
        f = np.float32(float(np.float32(0.6)) * float(u) + float(np.float32(0.7)))
        val = np.float32(f * v[e])
        if alpha is not None:
            val = np.float32(tab[depth[tuple(c)] - 1] * val)
        assert vp[tuple(c)] == np.minimum(val, cap), (c, vp[tuple(c)], val)


def test_free_surface_matches_grid_without_top_band():
    """Zero velocity in the top band is a pressure-release surface: the
    oracle's traces and panels equal a dense leapfrog on the grid with the
    top band removed and p = 0 above it (Eq. (1)'s Dirichlet condition one
    row above the surface)."""
    nz, nx, nb, h, dt, nt = 6, 7, 2, 10.0, 1e-3, 11
    v = synth.random_model((nz, nx), 1, 1800, 2600, sigma=1.0)
    vp = oracle.rbc_pad(v, nb, 42, 0.0, free_surface=True, taper=0.5)
    rng = np.random.default_rng(0)
    w = rng.standard_normal(nt)
    src = np.array([2.25, 0.0, 0.5])
    rec = np.array([[0.0, 0, 0.0], [3.5, 0, 1.75], [6.0, 0, 5.0]])
    tr, pl, pp = oracle.model_shot(vp, h, nb, dt, w, src, rec, want_last=True)
    assert not np.any(pl[:nb]) and not np.any(pp[:nb])
    cut = vp[nb:]                       # no band above the surface
    NZc, NX = cut.shape
    A = _dense_laplacian_2d(NZc, NX, h)
    D = (cut.astype(np.float64).ravel() * dt) ** 2

    def op(pos):
        x, z = pos[0] + nb, pos[2]      # z relative to the surface row
        vec = np.zeros(NZc * NX)
        x0, z0 = int(np.floor(x)), int(np.floor(z))
        fx, fz = x - x0, z - z0
        for dz, wz in ((0, 1 - fz), (1, fz)):
            for dx, wx in ((0, 1 - fx), (1, fx)):
                if wz * wx != 0:
                    vec[(z0 + dz) * NX + x0 + dx] += wz * wx
        return vec

    B = op(src) / h ** 2
    R = np.stack([op(r) for r in rec])
    p0, pm = np.zeros(NZc * NX), np.zeros(NZc * NX)
    d = [R @ p0]
    for n in range(nt):
        pn = 2 * p0 - pm + D * (A @ p0 + B * w[n])
        pm, p0 = p0, pn
        d.append(R @ p0)
    d = np.stack(d, axis=1)
    assert np.allclose(tr, d, rtol=1e-12, atol=1e-12 * np.abs(d).max())
    assert np.allclose(pl[nb:].ravel(), p0, rtol=1e-12, atol=1e-12 * np.abs(p0).max())


@pytest.mark.parametrize("alpha,fs", [(1.0, True), (0.0, False), (0.5, True)])
def test_time_reversal_with_band_options(alpha, fs):
    s = synth.config_small2d(nt=260)
    vp = oracle.rbc_pad(s.v_int, s.nb, 17, 0.0, free_surface=fs, taper=alpha)
    w = s.wavelet
    g = np.zeros((s.rec.shape[0], s.nt + 1))
    worst = pmax = 0.0
    for k in (60, 200):
        _, pk, _ = oracle.model_shot(vp, s.h, s.nb, s.dt, w[:k], s.src[0], s.rec, want_last=True)
        out = oracle.rtm_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, g, snap_k=k)
        pmax = max(pmax, np.abs(pk).max())
        worst = max(worst, np.abs(out["snap_p"] - pk).max())
    assert worst <= 1e-10 * pmax


def test_gradient_with_free_surface_vs_finite_differences():
    """Velocity gradient through a tapered free-surface model: central
    differences of the misfit at interior cells, and exactly zero in the
    zero-velocity band (dJ/dv = 2 v dt^2 dJ/dD vanishes there)."""
    s = synth.config_small2d(nt=240)
    nb = s.nb
    vp = oracle.rbc_pad(s.v_int, nb, 29, 0.0, free_surface=True, taper=0.7)
    w = s.wavelet
    vtrue = vp.copy()
    vtrue[nb + 12:nb + 18, nb:-nb] *= np.float32(1.08)
    d_obs = oracle.model_shot(vtrue, s.h, nb, s.dt, w, s.src[0], s.rec)
    d = oracle.model_shot(vp, s.h, nb, s.dt, w, s.src[0], s.rec)
    grad = oracle.rtm_shot(vp, s.h, nb, s.dt, w, s.src[0], s.rec, d - d_obs, want_grad=True)["grad"]
    assert np.all(np.isfinite(grad)) and not np.any(grad[:nb])

    def J(vm):
        r = oracle.model_shot(vm, s.h, nb, s.dt, w, s.src[0], s.rec) - d_obs
        return 0.5 * float(np.sum(r * r))

    rng = np.random.default_rng(12)
    big = np.argwhere(np.abs(grad) >= 1e-2 * np.abs(grad).max())
    for (z, x) in big[rng.choice(len(big), size=8, replace=False)]:
        v0 = float(vp[z, x])
        vpl, vmi = vp.copy(), vp.copy()
        vpl[z, x] = np.float32(v0 * (1 + 1e-5))
        vmi[z, x] = np.float32(v0 * (1 - 1e-5))
        fd = (J(vpl) - J(vmi)) / (float(vpl[z, x]) - float(vmi[z, x]))
        assert abs(fd - grad[z, x]) <= 1e-6 * abs(grad[z, x]) + 1e-9 * np.abs(grad).max(), (z, x)


@pytest.mark.parametrize("alpha,fs", [(0.5, True), (1.0, False)])
def test_pad_adjoint_with_options(alpha, fs):
    """<g, J dv> = <J^T g, dv>, the Jacobian action measured from the FP32
    padding of a unit model (the per-cell factors c f, or 0)."""
    rng = np.random.default_rng(2)
    v = rng.uniform(2000, 2100, (9, 11)).astype(np.float32)
    nb, cap = 5, 1.0e6
    gpad = rng.standard_normal((9 + 2 * nb, 11 + 2 * nb))
    gint = oracle.pad_adjoint(v, nb, 77, cap, gpad, free_surface=fs, taper=alpha)
    dv = rng.uniform(-1, 1, v.shape)
    ones = oracle.rbc_pad(np.ones_like(v), nb, 77, cap, free_surface=fs, taper=alpha).astype(np.float64)
    Jdv = np.empty(ones.shape)
    for z in range(ones.shape[0]):
        for x in range(ones.shape[1]):
            Jdv[z, x] = ones[z, x] * dv[min(max(z - nb, 0), 8), min(max(x - nb, 0), 10)]
    lhs, rhs = float(np.sum(gpad * Jdv)), float(np.sum(gint * dv))
    # the unit-model factors round c f to FP32 once more than the adjoint's
    # double product: agreement to FP32 precision
    assert abs(lhs - rhs) <= 1e-6 * np.abs(gpad * Jdv).sum()
