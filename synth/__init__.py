"""Seeded synthetic inputs for random-boundary RTM.

This module only makes inputs: velocity models, wavelets and acquisition
geometry.  It holds none of the method's arithmetic and is the one module
that both the GPU library's callers and the CPU oracle's callers share.

The paper's own models (the 2-D Marmousi benchmark and the 3-D HPC4E
MODEL AF) are not available; the generators below stand in for them with
seeded models of the same extents, spacing, velocity range and structure
(folded layers with faults for the 2-D case, flat layers with a salt body
for the 3-D case).  Nothing here reproduces any item of either dataset.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "ricker", "Survey", "two_layer_2d", "folded_layers_2d", "layered_salt_3d", "smooth_random_2d",
    "config_small2d", "config_c1", "config_c2", "config_c3", "config_c4", "config_c5_models",
    "random_model", "line_receivers", "grid_receivers",
]


def ricker(f_peak: float, dt: float, nt: int, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet w(t) = (1 - 2 a) exp(-a), a = (pi f (t - t0))^2, sampled
    at t = n dt (n = 0..nt-1), FP32.  f_peak is the peak frequency; the
    default delay t0 = 1.5 / f_peak makes w(0) ~ 1e-8, so the wavelet starts
    from rest."""
    if t0 is None:
        t0 = 1.5 / f_peak
    t = np.arange(nt, dtype=np.float64) * dt
    a = (np.pi * f_peak * (t - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def line_receivers(xs, z: float) -> np.ndarray:
    """Receivers at (x, 0, z) for each x: float32 (nrec, 3)."""
    xs = np.asarray(xs, dtype=np.float64)
    r = np.zeros((xs.size, 3), dtype=np.float32)
    r[:, 0] = xs
    r[:, 2] = z
    return r


def grid_receivers(xs, ys, z: float) -> np.ndarray:
    """Receivers on the tensor grid xs x ys at depth z (x fastest)."""
    X, Y = np.meshgrid(np.asarray(xs, np.float64), np.asarray(ys, np.float64), indexing="xy")
    r = np.zeros((X.size, 3), dtype=np.float32)
    r[:, 0] = X.ravel()
    r[:, 1] = Y.ravel()
    r[:, 2] = z
    return r


@dataclass
class Survey:
    """One acquisition: model, grid, time axis and geometry.

    v_int is (nz, nx) or (nz, ny, nx) FP32 in m/s; src is (nshot, 3) and
    rec (nrec, 3) in interior grid units (x, y, z)."""
    name: str
    v_int: np.ndarray
    h: float
    nb: int
    seed: int
    dt: float
    nt: int
    f_peak: float
    src: np.ndarray
    rec: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return self.v_int.ndim

    @property
    def wavelet(self) -> np.ndarray:
        return ricker(self.f_peak, self.dt, self.nt)

    def interior(self):
        """(nx, ny, nz)."""
        if self.v_int.ndim == 2:
            nz, nx = self.v_int.shape
            return nx, 1, nz
        nz, ny, nx = self.v_int.shape
        return nx, ny, nz

    def padded_shape(self):
        nb = self.nb
        if self.v_int.ndim == 2:
            nz, nx = self.v_int.shape
            return (nz + 2 * nb, nx + 2 * nb)
        nz, ny, nx = self.v_int.shape
        return (nz + 2 * nb, ny + 2 * nb, nx + 2 * nb)


# ---------------------------------------------------------------------------
# Velocity models
# ---------------------------------------------------------------------------

def two_layer_2d(nx: int, nz: int, z_if: int, v_top: float, v_bot: float) -> np.ndarray:
    """Two layers: v_top for iz < z_if, v_bot for iz >= z_if."""
    v = np.full((nz, nx), v_top, dtype=np.float32)
    v[z_if:, :] = v_bot
    return v


def folded_layers_2d(nx: int, nz: int, h: float, seed: int, n_layers: int = 20, vmin: float = 1500.0,
                     vmax: float = 5500.0, n_faults: int = 4) -> np.ndarray:
    """Sinusoidally folded layers cut by Gaussian-tapered dipping faults.

    Interfaces z_k(x) = zbar_k + A_k sin(2 pi x / lambda_k + phi_k); layer
    velocities increase monotonically from vmin to vmax, vmax being attained
    by the deepest layer.  Each fault is a dipping plane; on its hanging-wall
    side depths are shifted by a throw that tapers along the fault as a
    Gaussian.  Values are clipped to [vmin, vmax]."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx, dtype=np.float64) * h
    z = np.arange(nz, dtype=np.float64) * h
    zmax = z[-1]
    X, Z = np.meshgrid(x, z, indexing="xy")
    Zs = Z.copy()
    for _ in range(n_faults):
        x0 = rng.uniform(0.15, 0.85) * x[-1]
        dip = np.deg2rad(rng.uniform(50.0, 75.0)) * rng.choice([-1.0, 1.0])
        throw = rng.uniform(0.02, 0.06) * zmax
        zc = rng.uniform(0.3, 0.8) * zmax
        width = rng.uniform(0.25, 0.5) * zmax
        side = (X - x0) - Z / np.tan(dip)
        along = np.exp(-0.5 * ((Z - zc) / width) ** 2)
        Zs = Zs - np.where(side > 0.0, throw * along, 0.0)
    zbar = np.sort(rng.uniform(0.04, 0.96, n_layers)) * zmax
    amp = rng.uniform(0.005, 0.03, n_layers) * zmax
    lam = rng.uniform(0.3, 1.2, n_layers) * x[-1]
    phi = rng.uniform(0.0, 2.0 * np.pi, n_layers)
    vel = np.linspace(vmin, vmax, n_layers + 1)
    layer = np.zeros(X.shape, dtype=np.int64)
    for k in range(n_layers):
        zk = zbar[k] + amp[k] * np.sin(2.0 * np.pi * X / lam[k] + phi[k])
        layer += (Zs >= zk)
    v = vel[layer]
    return np.clip(v, vmin, vmax).astype(np.float32)


def layered_salt_3d(nx: int, ny: int, nz: int, seed: int, n_layers: int = 15, vmin: float = 1500.0,
                    vmax: float = 4500.0, salt: bool = True) -> np.ndarray:
    """Flat layers with velocities rising from vmin to vmax, plus a seeded
    ellipsoidal salt body at vmax.  Shape (nz, ny, nx), FP32."""
    rng = np.random.default_rng(seed)
    bounds = np.sort(rng.uniform(0.03, 0.97, n_layers - 1)) * nz
    vel = np.linspace(vmin, vmax, n_layers)
    iz = np.arange(nz, dtype=np.float64)
    layer = np.searchsorted(bounds, iz, side="right")
    vz = vel[layer].astype(np.float32)
    v = np.empty((nz, ny, nx), dtype=np.float32)
    v[:] = vz[:, None, None]
    if salt:
        cx, cy = rng.uniform(0.35, 0.65, 2) * np.array([nx, ny])
        cz = rng.uniform(0.45, 0.65) * nz
        ax, ay = rng.uniform(0.12, 0.2, 2) * np.array([nx, ny])
        az = rng.uniform(0.1, 0.16) * nz
        for k in range(nz):
            dz = ((k - cz) / az) ** 2
            if dz >= 1.0:
                continue
            yy = ((np.arange(ny) - cy) / ay) ** 2
            xx = ((np.arange(nx) - cx) / ax) ** 2
            inside = (yy[:, None] + xx[None, :] + dz) < 1.0
            v[k][inside] = vmax
    return v


def smooth_random_2d(nx: int, nz: int, seed: int, sigma: float, vmin: float, vmax: float) -> np.ndarray:
    """Gaussian-smoothed white noise scaled affinely onto [vmin, vmax]."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    a = gaussian_filter(rng.standard_normal((nz, nx)), sigma=sigma, mode="reflect")
    a = (a - a.min()) / (a.max() - a.min())
    return (vmin + (vmax - vmin) * a).astype(np.float32)


def random_model(shape, seed: int, vmin: float = 1500.0, vmax: float = 3000.0, sigma: float = 2.0):
    """Smooth random model of any dimension, for small parity cases."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    a = gaussian_filter(rng.standard_normal(shape), sigma=sigma, mode="reflect")
    a = (a - a.min()) / (a.max() - a.min() + 1e-30)
    return (vmin + (vmax - vmin) * a).astype(np.float32)


# ---------------------------------------------------------------------------
# Workload configurations
# ---------------------------------------------------------------------------

def config_c1(nt: int = 1000) -> Survey:
    """2-D two-layer model: 201 x 201 interior at 10 m, 1500 / 2500 m/s with the
    interface at iz = 100, 40-cell random boundary (seed 1), 15 Hz Ricker at
    (100, 2), 201 receivers at z = 2, dt = 0.5 ms, nt = 1000."""
    v = two_layer_2d(201, 201, 100, 1500.0, 2500.0)
    src = np.array([[100.0, 0.0, 2.0]], dtype=np.float32)
    rec = line_receivers(np.arange(201), 2.0)
    return Survey("two_layer_201x201", v, 10.0, 40, 1, 5e-4, nt, 15.0, src, rec)


def config_c2(nshot: int = 240, nt: int = 5000, model_seed: int = 2204) -> Survey:
    """2-D folded-layer model: 2301 x 751 at 4 m, 1500-5500 m/s, 60-cell random
    boundary, 25 Hz Ricker, dt = 0.4 ms, nt = 5000, 240 shots every 38 m
    (9.5 cells: odd shots sit at half-cell positions) at z = 2, 2301
    receivers at z = 2."""
    v = folded_layers_2d(2301, 751, 4.0, model_seed)
    k = np.arange(nshot, dtype=np.float64)
    src = np.zeros((nshot, 3), dtype=np.float32)
    src[:, 0] = 15.0 + 9.5 * k
    src[:, 2] = 2.0
    rec = line_receivers(np.arange(2301), 2.0)
    return Survey("folded_2301x751", v, 4.0, 60, 7, 4e-4, nt, 25.0, src, rec)


def config_c3(nt: int = 4000, model_seed: int = 3303, n=(512, 512, 256)) -> Survey:
    """3-D layered model with a salt body: 512 x 512 x 256 at 10 m,
    1500-4500 m/s, 50-cell random boundary per face, 12 Hz Ricker at
    (256, 256, 2), 256 x 256 receivers at (2i, 2j, 2), dt = 1 ms, nt = 4000."""
    nx, ny, nz = n
    v = layered_salt_3d(nx, ny, nz, model_seed)
    src = np.array([[nx // 2, ny // 2, 2.0]], dtype=np.float32)
    rec = grid_receivers(np.arange(0, nx, 2), np.arange(0, ny, 2), 2.0)
    return Survey(f"layered_salt_{nx}x{ny}x{nz}", v, 10.0, 50, 11, 1e-3, nt, 12.0, src, rec)


def config_c4(nshot: int = 64, nt: int = 2000, seed: int = 4404) -> Survey:
    """Uneven-aperture 2-D shots: a 4000 x 300 model at 10 m from smoothed
    random velocities in [1500, 3500] (sigma 5 cells); the migration model is
    that field smoothed again (sigma 20).  Each shot sees a window of
    401-1201 columns with its source at the window centre and a receiver on
    every column, all at z = 2; 40-cell random boundary, 10 Hz Ricker,
    dt = 1 ms, nt = 2000.  Windows are in extra['windows'] as (x0, width)."""
    from scipy.ndimage import gaussian_filter
    v_true = smooth_random_2d(4000, 300, seed, 5.0, 1500.0, 3500.0)
    v_cur = gaussian_filter(v_true.astype(np.float64), 20.0, mode="reflect").astype(np.float32)
    rng = np.random.default_rng(seed + 1)
    widths = rng.integers(401, 1202, nshot)
    x0 = np.array([rng.integers(0, 4000 - w + 1) for w in widths])
    src = np.zeros((nshot, 3), dtype=np.float32)
    src[:, 0] = (widths - 1) // 2
    src[:, 2] = 2.0
    return Survey("uneven_aperture_4000x300", v_true, 10.0, 40, 5, 1e-3, nt, 10.0, src,
                  np.zeros((0, 3), np.float32),
                  extra={"v_cur": v_cur, "windows": np.stack([x0, widths], axis=1)})


def config_c5_models(n_models: int, seed: int, n: int = 128):
    """Layered + salt 3-D models of n^3 cells for the learned filter."""
    return [layered_salt_3d(n, n, n, seed + i) for i in range(n_models)]


def config_small2d(nx: int = 61, nz: int = 47, nb: int = 12, nt: int = 220, seed: int = 5) -> Survey:
    """Small 2-D smooth random model for fast parity checks, with an off-grid
    source and off-grid receivers."""
    v = random_model((nz, nx), seed, 1500.0, 3000.0, sigma=3.0)
    src = np.array([[nx * 0.43 + 0.3, 0.0, 3.6]], dtype=np.float32)
    rec = line_receivers(np.linspace(0.5, nx - 1.25, 23), 2.25)
    return Survey(f"small2d_{nx}x{nz}", v, 10.0, nb, seed, 1e-3, nt, 20.0, src, rec)
