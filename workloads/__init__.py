"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds none of the method's arithmetic: it only produces velocity models,
acquisition geometry, the source wavelet and the fixed configuration constants.  Both
the GPU library and the CPU oracle consume what it produces; neither is imported here.

The paper's velocity models and data are not available, so seeded stand-ins with the
shapes and value ranges of its workloads are used (2D ocean-bottom-node synthetics:
fixed-spread receivers and sources one cell below the surface, Ricker wavelet,
smoothed-truth starting model, "Posterior sampling using 2D ocean-bottom node synthetic
data"; 3D upscaling study, Table 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def ricker(freq: float, dt: float, nt: int, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(t) = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0,
    sampled at t_n = n dt; default delay t0 = 1.5/f."""
    t0 = 1.5 / freq if t0 is None else t0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * freq * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ------------------------------------------------------------- 2D models

def layered_1d(nz: int, nx: int, seed: int, vmin=1500.0, vmax=4000.0, ninterface=3, zlo=16, zhi=120):
    """1-D layered model: interfaces uniform in [zlo, zhi) cells, top vmin, bottom vmax,
    middle layer velocities sorted uniform draws in (vmin, vmax)."""
    r = rng(seed)
    zs = np.sort(r.integers(zlo, min(zhi, nz), size=ninterface))
    mids = np.sort(r.uniform(vmin, vmax, size=ninterface - 1))
    vel = np.concatenate([[vmin], mids, [vmax]])
    v = np.empty((nz, nx))
    layer = np.searchsorted(zs, np.arange(nz), side="right")
    v[:] = vel[layer][:, None]
    return v


def linear_gradient(nz: int, nx: int, vtop=1500.0, vbot=4000.0):
    """Depth-linear model from vtop (first row) to vbot (last row)."""
    return np.repeat(np.linspace(vtop, vbot, nz)[:, None], nx, axis=1)


def thrust_2d(nz: int, nx: int, seed: int, vmin=2000.0, vmax=6000.0, nlayer=10):
    """Folded-layer thrust stand-in: about nlayer layers increasing vmin -> vmax (+-10 %
    jitter), sinusoidally folded interfaces, one dipping thrust fault with a seeded throw."""
    r = rng(seed)
    base = np.linspace(vmin, vmax, nlayer)
    vel = np.clip(base * (1.0 + r.uniform(-0.1, 0.1, nlayer)), vmin, vmax)
    vel = np.sort(vel)
    z0 = np.sort(r.uniform(0.08, 0.95, nlayer - 1)) * nz
    amp = r.uniform(0.02, 0.08) * nz
    lam = r.uniform(0.4, 1.0) * nx
    ph = r.uniform(0, 2 * math.pi)
    x = np.arange(nx)[None, :]
    z = np.arange(nz)[:, None].astype(np.float64)
    fx0 = r.uniform(0.3, 0.7) * nx
    dip = r.uniform(0.6, 1.5)
    throw = r.uniform(0.05, 0.12) * nz
    hanging = (x - fx0) * dip < (nz - z)  # above/left of a dipping fault plane
    fold = amp * np.sin(2 * math.pi * x / lam + ph)
    zz = z - fold - np.where(hanging, throw, 0.0)
    layer = np.zeros((nz, nx), dtype=np.int64)
    for k in range(nlayer - 1):
        layer += (zz >= z0[k]).astype(np.int64)
    return vel[layer]


def salt_2d(nz: int, nx: int, seed: int, vtop=1500.0, vbot=3500.0, vsalt=4500.0):
    """Salt stand-in: star-shaped polygon (8-12 vertices, radii 15-35 % of the smaller
    dimension) at vsalt in a depth-linear vtop -> vbot background."""
    r = rng(seed)
    v = linear_gradient(nz, nx, vtop, vbot)
    nv = int(r.integers(8, 13))
    m = min(nz, nx)
    ang = np.sort(r.uniform(0, 2 * math.pi, nv))
    rad = r.uniform(0.15, 0.35, nv) * m
    cz = r.uniform(0.35, 0.65) * nz
    cx = r.uniform(0.3, 0.7) * nx
    zz, xx = np.mgrid[0:nz, 0:nx].astype(np.float64)
    th = np.mod(np.arctan2(zz - cz, xx - cx), 2 * math.pi)
    # radius of the polygon boundary along each direction (linear between vertices)
    a_ext = np.concatenate([ang - 2 * math.pi, ang, ang + 2 * math.pi])
    r_ext = np.concatenate([rad, rad, rad])
    rb = np.interp(th, a_ext, r_ext)
    inside = np.hypot(zz - cz, xx - cx) <= rb
    v[inside] = vsalt
    return v


def layered_salt_3d(nz: int, ny: int, nx: int, seed: int, vmin=1500.0, vmax=4500.0, nlayer=5):
    """3D stand-in: nlayer gently dipping layers vmin -> ~0.85 vmax plus a star-shaped salt
    body (per-depth-slice polygon radius shrinking towards its top/bottom) at vmax."""
    r = rng(seed)
    vel = np.sort(r.uniform(vmin, 0.85 * vmax, nlayer))
    vel[0] = vmin
    z0 = np.sort(r.uniform(0.1, 0.9, nlayer - 1)) * nz
    dipx, dipy = r.uniform(-0.1, 0.1, 2)
    z = np.arange(nz)[:, None, None].astype(np.float64)
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    zz = z - dipx * (x - nx / 2) - dipy * (y - ny / 2)
    layer = np.zeros((nz, ny, nx), dtype=np.int64)
    for k in range(nlayer - 1):
        layer += (zz >= z0[k]).astype(np.int64)
    v = vel[layer].astype(np.float64)
    nv = int(r.integers(8, 13))
    ang = np.sort(r.uniform(0, 2 * math.pi, nv))
    rad = r.uniform(0.15, 0.35, nv) * min(nx, ny)
    cz, cy, cx = r.uniform(0.4, 0.7) * nz, r.uniform(0.35, 0.65) * ny, r.uniform(0.35, 0.65) * nx
    hz = r.uniform(0.15, 0.3) * nz
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    th = np.mod(np.arctan2(yy - cy, xx - cx), 2 * math.pi)
    a_ext = np.concatenate([ang - 2 * math.pi, ang, ang + 2 * math.pi])
    rb = np.interp(th, a_ext, np.concatenate([rad, rad, rad]))
    rr = np.hypot(yy - cy, xx - cx)
    for iz in range(nz):
        s = 1.0 - ((iz - cz) / hz) ** 2
        if s > 0:
            v[iz][rr <= rb * math.sqrt(s)] = vmax
    return v


def smooth(v: np.ndarray, sigma_cells: float) -> np.ndarray:
    """Gaussian-smoothed model (starting model = smoothed truth)."""
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(np.asarray(v, dtype=np.float64), sigma_cells, mode="nearest")


# ----------------------------------------------------------- acquisition

def surface_shots_2d(nx: int, nshot: int, z: int = 1) -> np.ndarray:
    """Physical cell indices of nshot sources at row z, x_i = floor((i + 1/2) nx / nshot)."""
    xs = np.floor((np.arange(nshot) + 0.5) * nx / nshot).astype(np.int64)
    return (z * nx + xs).astype(np.int32)


def surface_receivers_2d(nx: int, z: int = 1, every: int = 1) -> np.ndarray:
    xs = np.arange(0, nx, every)
    return (z * nx + xs).astype(np.int32)


def surface_lattice_3d(ny: int, nx: int, n_y: int, n_x: int, z: int = 1) -> np.ndarray:
    """n_y x n_x points on the plane at depth z, centred cell positions."""
    ys = np.floor((np.arange(n_y) + 0.5) * ny / n_y).astype(np.int64)
    xs = np.floor((np.arange(n_x) + 0.5) * nx / n_x).astype(np.int64)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return ((z * ny + yy) * nx + xx).ravel().astype(np.int32)


def receiver_lattice_3d(ny: int, nx: int, every: int = 4, z: int = 1) -> np.ndarray:
    ys = np.arange(0, ny, every)
    xs = np.arange(0, nx, every)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return ((z * ny + yy) * nx + xx).ravel().astype(np.int32)


# -------------------------------------------------------------- configs

@dataclass(frozen=True)
class Config:
    """One workload.  Grid sizes are physical; the sponge of nb cells is added outside."""
    name: str
    ndim: int
    nz: int
    nx: int
    h: float
    nb: int
    dt: float
    nt: int
    rec_every: int
    freq: float
    nshot: int
    vmin: float
    vmax: float
    ny: int = 1
    shots_per_group: int = 1
    groups: int = 1
    nsample: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def v_ref(self) -> float:
        return self.vmax

    @property
    def nt_rec(self) -> int:
        return self.nt // self.rec_every


# 2D single-shot parity workload: 128x128 at 10 m, dt 1 ms, 1000 steps, 20-cell sponge, 8 shots of a 15 Hz
# Ricker, 128 receivers, single-source misfit.
C1 = Config("2d-128x128-8shot-single", 2, 128, 128, 10.0, 20, 1e-3, 1000, 1, 15.0, 8, 1500.0, 4000.0,
            shots_per_group=1, groups=8, nsample=1)
# 2D encoded workload (the benchmark): 400x150 at 20 m, 2 ms x 2000 recorded samples (two 1 ms internal steps per
# sample to respect the stability limit at 6000 m/s), 80 shots encoded into supergathers of
# 8, 16 posterior samples x 10 supergathers.
C2 = Config("2d-400x150-80shot-s8-16x10", 2, 150, 400, 20.0, 20, 1e-3, 4000, 2, 6.0, 80, 2000.0, 6000.0,
            shots_per_group=8, groups=10, nsample=16)
# 2D uneven workload: grids 256x128, 512x200, 800x200 at 10 m, 2000 steps, salt models.
C3_SIZES = ((128, 256), (200, 512), (200, 800))  # (nz, nx)
C3 = Config("2d-uneven-salt-32", 2, 128, 256, 10.0, 20, 1e-3, 2000, 1, 10.0, 16, 1500.0, 4500.0,
            shots_per_group=8, groups=1, nsample=32, extra={"sizes": C3_SIZES, "ckpt_every": 10})
# 3D workload: 200x200x100 at 25 m, dt 2 ms, 1500 steps, 10-cell sponge, 64 shots in 4
# supergathers of 16, 8 posterior samples.
C5 = Config("3d-200x200x100-64shot-s16-8x4", 3, 100, 200, 25.0, 10, 2e-3, 1500, 1, 4.0, 64, 1500.0, 4500.0,
            ny=200, shots_per_group=16, groups=4, nsample=8)
