"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own formulas.

Each test names the passage of the paper (arXiv 2204.03380) or the
mathematical fact it relies on.  None of them needs a GPU.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# P9: random boundary generator
# ---------------------------------------------------------------------------

def test_splitmix64_published_values():
    """SplitMix64 outputs equal the published reference values."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and l[0] != "#"]
    assert rows
    for seed, k, val in rows:
        assert oracle.splitmix64(int(seed), int(k)) == int(val)


def _py_splitmix64(seed, k):
    M = (1 << 64) - 1
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


@pytest.mark.parametrize("shape,nb", [((7, 9), 3), ((5, 4, 6), 2)])
def test_rbc_pad_bruteforce(shape, nb):
    """Tiny grids: every padded value equals min(f * v_edge, v_cap) computed
    independently in Python (exact double arithmetic, one final FP32
    rounding for the fused multiply-add, FP32 product and min)."""
    rng = np.random.default_rng(3)
    v = rng.uniform(1500, 3000, shape).astype(np.float32)
    seed = 987654321
    cap = np.float32(2900.0)
    vp = oracle.rbc_pad(v, nb, seed, float(cap))
    pshape = vp.shape
    idx = np.indices(pshape).reshape(len(pshape), -1).T
    for j, c in enumerate(idx):
        inner = [ci - nb for ci in c]
        e = tuple(min(max(ci, 0), n - 1) for ci, n in zip(inner, shape))
        inside = all(0 <= ci < n for ci, n in zip(inner, shape))
        if inside:
            assert vp[tuple(c)] == v[e]
            continue
        r = _py_splitmix64(seed, j)
        u = np.float32(r >> 40) * np.float32(2.0 ** -24)
        f = np.float32(float(np.float32(0.6)) * float(u) + float(np.float32(0.7)))  # exact, one rounding
        expect = np.minimum(np.float32(f * v[e]), cap)
        assert vp[tuple(c)] == expect, (c, vp[tuple(c)], expect)


def test_rbc_pad_statistics_and_cap():
    """Band factors are uniform on [0.7, 1.3): mean 1, variance 0.03; the
    interior is copied; capping applies; the seed changes the band only;
    v_cap <= 0 means the interior maximum (stability, Sec. on the RBC)."""
    v = np.full((40, 50), 2000.0, dtype=np.float32)
    nb = 30
    vp = oracle.rbc_pad(v, nb, 11, 1.0e9)
    band = np.ones(vp.shape, bool)
    band[nb:-nb, nb:-nb] = False
    f = vp[band].astype(np.float64) / 2000.0
    assert f.min() >= 0.7 - 1e-6 and f.max() < 1.3
    assert abs(f.mean() - 1.0) < 0.01
    assert abs(f.var() - 0.03) < 0.002
    assert np.array_equal(vp[nb:-nb, nb:-nb], v)
    vp2 = oracle.rbc_pad(v, nb, 12, 1.0e9)
    assert np.array_equal(vp2[nb:-nb, nb:-nb], v) and not np.array_equal(vp2[band], vp[band])
    assert np.array_equal(oracle.rbc_pad(v, nb, 11, 1.0e9), vp)  # deterministic
    capped = oracle.rbc_pad(v, nb, 11, 0.0)  # cap = interior max = 2000
    assert capped.max() == 2000.0
    assert np.array_equal(capped, np.minimum(vp, np.float32(2000.0)))


def test_rbc_pad_edge_mapping():
    """A band cell takes its factor times the interior value at its clamped
    coordinates; corners use the corner cell."""
    v = np.arange(1, 13, dtype=np.float32).reshape(3, 4) * 100 + 1000
    nb = 4
    vp = oracle.rbc_pad(v, nb, 5, 1.0e9)
    ratio_ok = 0
    for z in range(vp.shape[0]):
        for x in range(vp.shape[1]):
            e = v[min(max(z - nb, 0), 2), min(max(x - nb, 0), 3)]
            r = vp[z, x] / e
            assert 0.7 - 1e-6 <= r < 1.3 + 1e-6
            ratio_ok += 1
    assert ratio_ok == vp.size


# ---------------------------------------------------------------------------
# P1: stencil consistency (8th order in space, Sec. 3)
# ---------------------------------------------------------------------------

def _poly_field_1d(n, h, power, axis_len=9, ndim=2, axis=1):
    x = (np.arange(n) - n // 2) * h
    f = x ** power
    if ndim == 2:
        shape = [axis_len, axis_len]
        shape[axis] = n
        out = np.empty(shape)
        out[...] = f.reshape([-1 if a == axis else 1 for a in range(2)])
        return out, x
    shape = [axis_len] * 3
    shape[axis] = n
    out = np.empty(shape)
    out[...] = f.reshape([-1 if a == axis else 1 for a in range(3)])
    return out, x


@pytest.mark.parametrize("ndim,axis", [(2, 0), (2, 1), (3, 0), (3, 1), (3, 2)])
def test_stencil_exact_on_polynomials(ndim, axis):
    """L_h x^p is the exact second derivative for p <= 9 away from the edges;
    for p = 10 the error is the textbook truncation term of the 8th-order
    centred difference, -h^8 f^(10) / 3150 = -1152 h^8, at every point."""
    h = 0.7
    n = 31
    c = n // 2
    for p in range(0, 11):
        f, x = _poly_field_1d(n, h, p, ndim=ndim, axis=axis)
        L = oracle.laplacian(f, h)
        sl = [4] * ndim  # a point far from the other axes' edges
        vals = []
        for i in range(c - 6, c + 7):
            sl[axis] = i
            vals.append(L[tuple(sl)])
        vals = np.array(vals)
        xi = x[c - 6:c + 7]
        exact = p * (p - 1) * xi ** (p - 2) if p >= 2 else np.zeros_like(xi)
        if p == 10:
            exact = exact - 1152.0 * h ** 8
        scale = max(1.0, np.abs(exact).max())
        assert np.abs(vals - exact).max() <= 1e-9 * scale, (p, vals - exact)


def test_stencil_nyquist_and_harmonic():
    """The Nyquist mode (-1)^i has symbol -2048/315 / h^2 per axis, and a
    harmonic polynomial of degree <= 9 has zero discrete Laplacian."""
    h = 2.0
    n = 25
    i = np.arange(n)
    f = np.tile(((-1.0) ** i)[None, :], (n, 1))
    L = oracle.laplacian(f, h)
    c = n // 2
    assert abs(L[c, c] / f[c, c] - (-2048.0 / 315.0) / h ** 2) < 1e-12
    # Re (x + i z)^7 is harmonic.
    x = (np.arange(n) - c) * h
    X, Z = np.meshgrid(x, x, indexing="xy")
    P = np.real((X + 1j * Z) ** 7)
    LP = oracle.laplacian(P, h)
    assert np.abs(LP[c - 6:c + 7, c - 6:c + 7]).max() < 1e-9 * np.abs(P).max()
    # 3-D: x^2 - z^2 + 2 y^2 - 2 x^2 ... use x y z (harmonic) and x^2 + y^2 - 2 z^2
    X3, Y3, Z3 = np.meshgrid(x[:15], x[:15], x[:15], indexing="ij")
    Q = (X3 * Y3 * Z3 + X3 ** 2 + Y3 ** 2 - 2 * Z3 ** 2).transpose(2, 1, 0).copy()
    LQ = oracle.laplacian(Q, h)
    assert np.abs(LQ[4:11, 4:11, 4:11]).max() < 1e-9 * np.abs(Q).max()


# ---------------------------------------------------------------------------
# Brute force: the time loop against a dense-matrix implementation
# ---------------------------------------------------------------------------

def _dense_laplacian_2d(NZ, NX, h):
    """Kronecker-sum Laplacian with zero values outside the grid, built from
    the 1-D Toeplitz matrix of the textbook 8th-order weights."""
    from scipy.linalg import toeplitz
    from fractions import Fraction
    # 8th-order centred weights from the Taylor conditions (solve the
    # Vandermonde system exactly in rationals).
    A = [[Fraction(2 * m ** (2 * k)) for m in range(1, 5)] for k in range(1, 5)]
    b = [Fraction(2), Fraction(0), Fraction(0), Fraction(0)]
    # Gaussian elimination in exact arithmetic.
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    for i in range(4):
        piv = M[i][i]
        M[i] = [v / piv for v in M[i]]
        for j in range(4):
            if j != i:
                fac = M[j][i]
                M[j] = [a - fac * c for a, c in zip(M[j], M[i])]
    cm = [float(M[i][4]) for i in range(4)]
    c0 = -2.0 * sum(float(M[i][4]) for i in range(4))

    def one(n):
        col = np.zeros(n)
        col[0] = c0
        for m in range(1, 5):
            if m < n:
                col[m] = cm[m - 1]
        return toeplitz(col)

    Lx, Lz = one(NX), one(NZ)
    return (np.kron(np.eye(NZ), Lx) + np.kron(Lz, np.eye(NX))) / h ** 2


def test_model_shot_matches_dense_bruteforce():
    """On a tiny grid, oracle traces and final panels equal a dense-matrix
    leapfrog p^{n+1} = 2p^n - p^{n-1} + D (A p^n + b^n) with bilinear point
    operators (Eq. (1), Sec. 3, Algorithm 1)."""
    nz, nx, nb, h, dt, nt = 6, 7, 2, 10.0, 1e-3, 9
    v = synth.random_model((nz, nx), 1, 1800, 2600, sigma=1.0)
    vp = oracle.rbc_pad(v, nb, 42, 0.0)
    NZ, NX = vp.shape
    rng = np.random.default_rng(0)
    w = rng.standard_normal(nt)
    src = np.array([2.25, 0.0, 1.5])
    rec = np.array([[0.0, 0, 0.0], [3.5, 0, 2.75], [6.0, 0, 5.0], [1.0, 0, 4.2]])
    tr, pl, pp = oracle.model_shot(vp, h, nb, dt, w, src, rec, want_last=True)

    A = _dense_laplacian_2d(NZ, NX, h)
    D = (vp.astype(np.float64).ravel() * dt) ** 2

    def op(pos):
        x, z = pos[0] + nb, pos[2] + nb
        vec = np.zeros(NZ * NX)
        x0, z0 = int(np.floor(x)), int(np.floor(z))
        fx, fz = x - x0, z - z0
        for dz, wz in ((0, 1 - fz), (1, fz)):
            for dx, wx in ((0, 1 - fx), (1, fx)):
                if wz * wx != 0:
                    vec[(z0 + dz) * NX + x0 + dx] += wz * wx
        return vec

    B = op(src) / h ** 2
    R = np.stack([op(r) for r in rec])
    p0 = np.zeros(NZ * NX)
    pm = np.zeros(NZ * NX)
    d = [R @ p0]
    for n in range(nt):
        pn = 2 * p0 - pm + D * (A @ p0 + B * w[n])
        pm, p0 = p0, pn
        d.append(R @ p0)
    d = np.stack(d, axis=1)
    assert np.allclose(tr, d, rtol=1e-12, atol=1e-12 * np.abs(d).max())
    assert np.allclose(pl.ravel(), p0, rtol=1e-12, atol=1e-12 * np.abs(p0).max())
    assert np.allclose(pp.ravel(), pm, rtol=1e-12, atol=1e-12 * np.abs(p0).max())


# ---------------------------------------------------------------------------
# P3: analytic Green's functions before any boundary arrival
# ---------------------------------------------------------------------------

def _green2d(w_fun, r, v, t):
    """p(r, t) = (1 / 2 pi) int_0^{acosh(v t / r)} w(t - (r / v) cosh s) ds:
    the 2-D solution of p_tt - v^2 lap p = v^2 delta(x) w(t)."""
    if v * t <= r:
        return 0.0
    smax = math.acosh(v * t / r)
    val, _ = integrate.quad(lambda s: w_fun(t - (r / v) * math.cosh(s)), 0.0, smax, limit=200)
    return val / (2 * math.pi)


def _ricker_fun(f, t0):
    def w(t):
        if t < 0:
            return 0.0
        a = (math.pi * f * (t - t0)) ** 2
        return (1 - 2 * a) * math.exp(-a)
    return w


def _green2d_error(h, dt, nt, n_int, f, offgrid):
    v0 = 2000.0
    nb = 10
    v = np.full((n_int, n_int), v0, np.float32)
    vp = oracle.rbc_pad(v, nb, 3, 0.0)
    c = (n_int - 1) // 2
    src = np.array([c + (0.5 if offgrid else 0.0), 0.0, c + (0.25 if offgrid else 0.0)])
    # receivers 120 m .. 360 m from the source (fixed in metres)
    offs_m = [(120.0, 0.0), (0.0, 150.0), (-100.0, 200.0), (250.0, -180.0), (300.0, 0.0)]
    rec = np.array([[src[0] + a / h + (0.3 if offgrid else 0.0), 0.0, src[2] + b / h] for a, b in offs_m])
    w = synth.ricker(f, dt, nt).astype(np.float64)
    tr = oracle.model_shot(vp, h, nb, dt, w, src, rec)
    wf = _ricker_fun(f, 1.5 / f)
    t = np.arange(nt + 1) * dt
    err = num = 0.0
    for r in range(rec.shape[0]):
        dist = math.hypot((rec[r, 0] - src[0]) * h, (rec[r, 2] - src[2]) * h)
        ana = np.array([_green2d(wf, dist, v0, tt) for tt in t])
        err += np.sum((tr[r] - ana) ** 2)
        num += np.sum(ana ** 2)
    return math.sqrt(err / num)


@pytest.mark.parametrize("offgrid,tol", [(False, 1e-2), (True, 8e-2)])
def test_green_2d_and_refinement(offgrid, tol):
    """2-D homogeneous medium (2000 m/s, as in the reconstruction figure of
    the paper): traces match the analytic Green's function convolved with the
    wavelet before any boundary return (the band is 700 m away, t <= 0.3 s),
    and the error falls at least 3x when h and dt are halved at fixed Courant
    number (second order: time stepping on grid, multilinear point operators
    off grid)."""
    f = 15.0
    e1 = _green2d_error(h=10.0, dt=1e-3, nt=300, n_int=141, f=f, offgrid=offgrid)
    e2 = _green2d_error(h=5.0, dt=5e-4, nt=600, n_int=281, f=f, offgrid=offgrid)
    assert e1 < tol, e1
    assert e2 < e1 / 3.0, (e1, e2)


@pytest.mark.parametrize("offgrid,tol", [(False, 1e-2), (True, 8e-2)])
def test_green_3d(offgrid, tol):
    """3-D homogeneous medium: p = w(t - r / v) / (4 pi r) before any boundary
    return (the discrete point source is 1 / h^3)."""
    f, h, dt, nt, v0 = 15.0, 10.0, 1e-3, 260, 2000.0
    n = 71
    nb = 4
    v = np.full((n, n, n), v0, np.float32)
    vp = oracle.rbc_pad(v, nb, 9, 0.0)
    c = (n - 1) // 2
    src = np.array([c, c + (0.5 if offgrid else 0.0), c])
    offs = np.array([[9.0, 0.0, 0.0], [0.0, 8.0, 6.0], [-8.0, 3.0, 7.0], [5.0, -10.0, -4.0]])
    if offgrid:
        offs = offs + np.array([0.25, 0.0, -0.5])
    rec = src[None, :] + offs
    w = synth.ricker(f, dt, nt).astype(np.float64)
    tr = oracle.model_shot(vp, h, nb, dt, w, src, rec)
    t = np.arange(nt + 1) * dt
    wf = _ricker_fun(f, 1.5 / f)
    err = num = 0.0
    for r in range(rec.shape[0]):
        dist = np.linalg.norm(offs[r]) * h
        ana = np.array([wf(tt - dist / v0) for tt in t]) / (4 * math.pi * dist)
        err += np.sum((tr[r] - ana) ** 2)
        num += np.sum(ana ** 2)
    rel = math.sqrt(err / num)
    assert rel < tol, rel


# ---------------------------------------------------------------------------
# P4: time reversal (Sec. on wavefield reconstruction: with random
# boundaries all energy stays inside, so the source wavefield is recovered)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_time_reversal(ndim):
    s = synth.config_small2d(nt=300) if ndim == 2 else None
    if ndim == 2:
        v, h, nb, dt, nt = s.v_int, s.h, s.nb, s.dt, s.nt
        src, rec = s.src[0], s.rec
    else:
        v = synth.random_model((18, 16, 20), 4, 1600, 2800, sigma=2.0)
        h, nb, dt, nt = 10.0, 6, 1e-3, 160
        src = np.array([9.5, 7.25, 3.0])
        rec = np.array([[2.0, 3.0, 2.0], [17.5, 12.0, 2.0]])
    vp = oracle.rbc_pad(v, nb, 17, 0.0)
    w = synth.ricker(20.0, dt, nt)
    g = np.zeros((rec.shape[0], nt + 1))
    pmax = 0.0
    worst = 0.0
    for k in (nt // 5, nt // 2, nt - 2):
        _, pk, _ = oracle.model_shot(vp, h, nb, dt, w[:k], src, rec, want_last=True)
        out = oracle.rtm_shot(vp, h, nb, dt, w, src, rec, g, snap_k=k)
        pmax = max(pmax, np.abs(pk).max())
        worst = max(worst, np.abs(out["snap_p"] - pk).max())
    assert worst <= 1e-10 * pmax, worst / pmax


@pytest.mark.parametrize("ndim", [2, 3])
def test_rtm_from_given_panels_equals_full_rtm(ndim):
    """Starting the reverse pass from the final panels that modeling returns
    gives the migration of the full call bit for bit (both reconstructions
    start from the same p^nt, p^(nt-1))."""
    if ndim == 2:
        s = synth.config_small2d(nt=160)
        v, nb, src, rec = s.v_int, s.nb, s.src[0], s.rec
    else:
        v = synth.random_model((12, 11, 14), 4, 1600, 2600)
        nb, src = 4, np.array([6.5, 5.0, 2.25])
        rec = synth.grid_receivers(np.arange(0, 14, 3), np.arange(0, 11, 3), 2.0)
    vp = oracle.rbc_pad(v, nb, 8, 0.0)
    w = synth.ricker(25.0, 1e-3, 160).astype(np.float64)
    d, pl, pp = oracle.model_shot(vp, 10.0, nb, 1e-3, w, src, rec, want_last=True)
    full = oracle.rtm_shot(vp, 10.0, nb, 1e-3, w, src, rec, d, eps_rel=1e-3)
    part = oracle.rtm_shot_from_panels(vp, 10.0, nb, 1e-3, w, src, rec, d, pl, pp, eps_rel=1e-3)
    for k in ("num", "den", "image"):
        assert np.array_equal(full[k], part[k]), k


def test_reconstruction_without_reinjection_differs_only_early():
    """Eq. (6) as written (zero right-hand side) is exact once the wavelet
    has ended but not while it is still active."""
    s = synth.config_small2d(nt=300)
    vp = oracle.rbc_pad(s.v_int, s.nb, 17, 0.0)
    w = s.wavelet
    g = np.zeros((s.rec.shape[0], s.nt + 1))
    k_late, k_early = 250, 20   # wavelet (20 Hz, t0 = 75 ms) ends near step 150
    _, p_late, _ = oracle.model_shot(vp, s.h, s.nb, s.dt, w[:k_late], s.src[0], s.rec, want_last=True)
    _, p_early, _ = oracle.model_shot(vp, s.h, s.nb, s.dt, w[:k_early + 60], s.src[0], s.rec, want_last=True)
    late = oracle.rtm_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, g, reinject=False, snap_k=k_late)
    early = oracle.rtm_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, g, reinject=False, snap_k=k_early + 60)
    assert np.abs(late["snap_p"] - p_late).max() <= 1e-10 * np.abs(p_late).max()
    assert np.abs(early["snap_p"] - p_early).max() > 1e-3 * np.abs(p_early).max()


# ---------------------------------------------------------------------------
# P5: discrete energy is conserved once the source is off
# ---------------------------------------------------------------------------

def test_energy_invariant():
    """E^{n+1/2} = sum (p^{n+1} - p^n)^2 / D - <p^{n+1}, L_h p^n> is constant
    and positive after the wavelet has ended (closed domain, zero boundary
    values: the energy the random boundary keeps inside)."""
    s = synth.config_small2d(nt=400)
    vp = oracle.rbc_pad(s.v_int, s.nb, 2, 0.0)
    D = (vp.astype(np.float64) * s.dt) ** 2
    w = s.wavelet
    E = []
    for n in (200, 280, 400):
        _, pl, pp = oracle.model_shot(vp, s.h, s.nb, s.dt, w[:n], s.src[0], s.rec, want_last=True)
        E.append(np.sum((pl - pp) ** 2 / D) - np.sum(pl * oracle.laplacian(pp, s.h)))
    E = np.array(E)
    assert E.min() > 0
    assert np.abs(E - E[0]).max() <= 1e-11 * E[0], E


# ---------------------------------------------------------------------------
# P6: dot-product test of the receiver wavefield (Eq. (2)) as the adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_dot_product_adjoint(ndim):
    rng = np.random.default_rng(8)
    if ndim == 2:
        s = synth.config_small2d(nt=150)
        v, h, nb, dt, nt, src, rec = s.v_int, s.h, s.nb, s.dt, s.nt, s.src[0], s.rec
    else:
        v = synth.random_model((12, 11, 13), 6, 1600, 2800, sigma=2.0)
        h, nb, dt, nt = 10.0, 4, 1e-3, 90
        src = np.array([5.5, 4.25, 6.75])
        rec = np.array([[1.0, 2.5, 1.0], [11.25, 9.0, 3.0], [6.0, 6.0, 10.5]])
    vp = oracle.rbc_pad(v, nb, 21, 0.0)
    w = rng.standard_normal(nt)
    g = rng.standard_normal((rec.shape[0], nt + 1))
    d = oracle.model_shot(vp, h, nb, dt, w, src, rec)
    out = oracle.rtm_shot(vp, h, nb, dt, np.zeros(nt), src, rec, g, want_wadj=True)
    lhs = float(np.sum(g * d))
    rhs = float(np.dot(w, out["w_adj"]))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.abs(g).sum() * np.abs(d).max()), (lhs, rhs)


# ---------------------------------------------------------------------------
# P7: the image numerator is the derivative of <g, d> w.r.t. a model
# perturbation: this fixes the p^k <-> mu^(k+1) pairing of Eq. (3)
# ---------------------------------------------------------------------------

def test_image_numerator_identity():
    s = synth.config_small2d(nt=150)
    vp = oracle.rbc_pad(s.v_int, s.nb, 23, 0.0)
    rng = np.random.default_rng(4)
    g = rng.standard_normal((s.rec.shape[0], s.nt + 1))
    w = s.wavelet
    out = oracle.rtm_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, g)
    num = out["num"]
    rng = np.random.default_rng(5)
    big = np.argwhere(np.abs(num) >= 1e-2 * np.abs(num).max())
    cells = big[rng.choice(len(big), size=6, replace=False)]
    eps = 1e-5  # small against |L_h| ~ k^2: the central difference converges quadratically
    for (iz, ix) in cells:
        m = np.zeros(vp.shape)
        m[iz + s.nb, ix + s.nb] = eps
        dp = oracle.model_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, m=m)
        dm = oracle.model_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, m=-m)
        fd = (np.sum(g * dp) - np.sum(g * dm)) / (2 * eps)
        assert abs(fd - num[iz, ix]) <= 1e-6 * abs(num[iz, ix]) + 1e-9 * np.abs(num).max(), (iz, ix, fd, num[iz, ix])


def _dense_den(vp, h, nb, dt, w, src_node):
    """den = sum_{k < nt} (p^k)^2 on the whole padded grid, from a dense-matrix
    leapfrog (Kronecker-sum Laplacian with independently derived weights)
    with an on-grid source."""
    NZ, NX = vp.shape
    A = _dense_laplacian_2d(NZ, NX, h)
    D = (vp.astype(np.float64).ravel() * dt) ** 2
    B = np.zeros(NZ * NX)
    B[(src_node[1] + nb) * NX + src_node[0] + nb] = 1.0 / h ** 2
    p0, pm, den = np.zeros(NZ * NX), np.zeros(NZ * NX), np.zeros(NZ * NX)
    for n in range(len(w)):
        den += p0 * p0
        pm, p0 = p0, 2 * p0 - pm + D * (A @ p0 + B * w[n])
    return den.reshape(NZ, NX)


def test_image_normalisation_takes_the_interior_max():
    """Eq. (3) with the water level: image = num / (den + eps max den), the
    maximum taken over the interior crop (the image's domain), not over the
    padded grid.  Crafted so that the two maxima differ: of a 4 x 4 interior
    only the source cell has a velocity (the other cells never move, a wall),
    so the wave lives in the source cell and the band corner that takes its
    velocity, where a 25 Hz wavelet leaves more illumination than at the
    source.  den over the padded grid comes from a dense-matrix leapfrog."""
    nb, h = 6, 10.0
    v = np.zeros((4, 4), np.float32)
    v[0, 0] = 1500.0
    vp = oracle.rbc_pad(v, nb, 3, 0.0)
    dt = 0.5 * h / (1.3 * 1500.0)
    w = synth.ricker(25.0, dt, 400).astype(np.float64)
    src, rec = np.array([0.0, 0.0, 0.0]), np.array([[0.0, 0.0, 0.0]])
    d = oracle.model_shot(vp, h, nb, dt, w, src, rec)
    den_pad = _dense_den(vp, h, nb, dt, w, (0, 0))
    m_int, m_pad = den_pad[nb:nb + 4, nb:nb + 4].max(), den_pad.max()
    assert m_pad > 1.5 * m_int  # the case tells the two readings apart
    for eps in (0.0, 1e-3, 0.5):
        out = oracle.rtm_shot(vp, h, nb, dt, w, src, rec, d, eps_rel=eps)
        assert np.allclose(out["den"], den_pad[nb:nb + 4, nb:nb + 4], rtol=1e-9, atol=1e-12 * m_int)
        live = out["den"] > 0
        ref = out["num"][live] / (out["den"][live] + eps * m_int)
        assert np.allclose(out["image"][live], ref, rtol=1e-12, atol=0)
        if eps > 0:
            wrong = out["num"][live] / (out["den"][live] + eps * m_pad)
            assert not np.allclose(out["image"][live], wrong, rtol=1e-4, atol=0)
            assert not out["image"][~live].any()  # num = 0 where den = 0


def _reflector_image(s):
    """Image of the two-layer shot with the direct wave removed (the same shot
    recorded on the homogeneous model of the source layer, same band seed,
    subtracted), so that the data hold the interface reflection."""
    w = s.wavelet.astype(np.float64)
    vp = oracle.rbc_pad(s.v_int, s.nb, s.seed, 0.0)
    vh = np.full_like(s.v_int, s.v_int[0, 0])
    vph = oracle.rbc_pad(vh, s.nb, s.seed, float(s.v_int.max()))
    d = oracle.model_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec)
    d -= oracle.model_shot(vph, s.h, s.nb, s.dt, w, s.src[0], s.rec)
    return oracle.rtm_shot(vp, s.h, s.nb, s.dt, w, s.src[0], s.rec, d, eps_rel=1e-3)["image"]


def test_reflector_depth_two_layer():
    """Image physics, not only parity: the 201 x 201 two-layer model
    (1500 m/s above iz = 100, 2500 m/s from it), recorded for 1.5 s (nt
    3000, past the 1.31 s two-way time of the interface), migrated with the
    imaging condition of Eq. (3).  The image amplitude averaged over the
    central half of the line peaks, below the first ten rows, within two
    cells of the interface, well above the profile's typical level."""
    s = synth.config_c1(nt=3000)
    im = _reflector_image(s)
    prof = np.abs(im[:, 50:151]).mean(axis=1)
    z = 10 + int(np.argmax(prof[10:]))
    print(f"reflector at iz = {z}; profile peak {prof[z]:.3g}, median {np.median(prof[10:]):.3g}")
    assert abs(z - 100) <= 2
    assert prof[z] > 5.0 * np.median(prof[10:])


# ---------------------------------------------------------------------------
# P8: velocity gradient against central finite differences
# ---------------------------------------------------------------------------

def test_gradient_vs_finite_differences():
    s = synth.config_small2d(nt=300)
    nb = s.nb
    vp = oracle.rbc_pad(s.v_int, nb, 29, 0.0)
    w = s.wavelet
    vtrue = vp.copy()
    vtrue[nb + 12:nb + 18, :] *= np.float32(1.08)  # a reflector the data sees
    d_obs = oracle.model_shot(vtrue, s.h, nb, s.dt, w, s.src[0], s.rec)
    d = oracle.model_shot(vp, s.h, nb, s.dt, w, s.src[0], s.rec)
    out = oracle.rtm_shot(vp, s.h, nb, s.dt, w, s.src[0], s.rec, d - d_obs, want_grad=True)
    grad = out["grad"]

    def J(vm):
        r = oracle.model_shot(vm, s.h, nb, s.dt, w, s.src[0], s.rec) - d_obs
        return 0.5 * float(np.sum(r * r))

    rng = np.random.default_rng(12)
    big = np.argwhere(np.abs(grad) >= 1e-2 * np.abs(grad).max())
    pick = big[rng.choice(len(big), size=16, replace=False)]
    for (z, x) in pick:
        v0 = float(vp[z, x])
        vpl, vmi = vp.copy(), vp.copy()
        vpl[z, x] = np.float32(v0 * (1 + 1e-5))
        vmi[z, x] = np.float32(v0 * (1 - 1e-5))
        fd = (J(vpl) - J(vmi)) / (float(vpl[z, x]) - float(vmi[z, x]))
        assert abs(fd - grad[z, x]) <= 1e-6 * abs(grad[z, x]) + 1e-9 * np.abs(grad).max(), (z, x, fd, grad[z, x])


def test_pad_adjoint_dot_product():
    """<grad_pad, J dv> = <J^T grad_pad, dv> for the padding Jacobian J,
    where J dv is measured by finite differences of the FP32 padding on a
    model far from the cap (the padding is linear there)."""
    rng = np.random.default_rng(1)
    v = rng.uniform(2000, 2100, (9, 11)).astype(np.float32)
    nb = 5
    cap = 1.0e6
    gpad = rng.standard_normal((9 + 2 * nb, 11 + 2 * nb))
    gint = oracle.pad_adjoint(v, nb, 77, cap, gpad)
    dv = rng.uniform(-1, 1, v.shape)
    # Padding is exactly linear (factor times edge value) up to FP32 rounding:
    # evaluate the Jacobian action in double from the factors the padding used.
    base = oracle.rbc_pad(v, nb, 77, cap).astype(np.float64)
    ones = oracle.rbc_pad(np.ones_like(v) * np.float32(1.0), nb, 77, cap).astype(np.float64)  # factors f_j
    shape = base.shape
    Jdv = np.empty(shape)
    for z in range(shape[0]):
        for x in range(shape[1]):
            e = (min(max(z - nb, 0), 8), min(max(x - nb, 0), 10))
            Jdv[z, x] = ones[z, x] * dv[e]
    lhs = float(np.sum(gpad * Jdv))
    rhs = float(np.sum(gint * dv))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    # With the cap below every band value, all band cells are capped and
    # contribute nothing; interior cells pass their gradient through.
    gint_c = oracle.pad_adjoint(v, nb, 77, 1000.0, gpad)
    assert np.array_equal(gint_c, gpad[nb:-nb, nb:-nb])
