"""Seeded synthetic inputs for the pressure-Poisson / projection path.

This module only *generates data*: wall-normal face coordinates and seeded
random fields on the staggered grid.  It holds none of the solver's
arithmetic (no divergence, no transforms, no tridiagonal solves), so the
test-only reference implementation and the GPU library can both be fed the
identical bytes it produces.

Grid conventions (shared by every consumer, stated here once):

* x, y periodic with Nx, Ny uniform cells of size dx = Lx/Nx, dy = Ly/Ny.
* z is the wall-normal direction on [0, 1], with Nz cells bounded by the
  faces ``zf[0..Nz]`` (``zf[0] = 0``, ``zf[Nz] = 1``).  Points cluster at the
  walls (Sec. 2.1 of the paper: non-uniform wall-normal grid, uniform
  periodic directions); the clustering law is a tanh map with stretching
  factor ``alpha`` (``alpha = 0`` gives a uniform grid).
* Arrays are C-ordered ``[z][y][x]`` with x fastest.  Cell-centre fields
  (p, phi, u, v) have shape ``(Nz, Ny, Nx)``; z-face fields (w, T) have shape
  ``(Nz + 1, Ny, Nx)`` with the two wall rows stored.
* u sits on x-faces (x = i dx), v on y-faces (y = j dy), w and T on z-faces
  (Fig. 1 of the paper: pressure at the centre, velocities on the faces,
  temperature collocated with the wall-normal velocity).

Random numbers come from numpy's PCG64 generator.  Large fields are drawn
plane by plane from independent child streams of one ``SeedSequence`` so that
generation can run on several host threads and still be reproducible.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
import os

import numpy as np

__all__ = [
    "Config", "CONFIGS", "zfaces", "cell_centres", "random_face_velocity",
    "mode_velocity", "rb_state", "rb_temperature", "face_weights",
]


@dataclass(frozen=True)
class Config:
    """One workload: box, grid and seed."""
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    alpha: float = 3.0
    seed: int = 1000
    extra: dict = field(default_factory=dict, hash=False, compare=False)

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz


# The five workloads.  Shapes of the convection slabs are the paper's own
# Rayleigh-Benard grids (Table 3); the 1024 x 1024 x 512 slab stands in for the
# plane-Couette case.  Seeds are 1000 + index.
CONFIGS = {
    "cube64": Config("cube64", 64, 64, 64, 1.0, 1.0, 3.0, 1000),
    "slab512x512x384": Config("slab512x512x384", 512, 512, 384, 2.0, 2.0, 3.0, 1001),
    "couette1024x1024x512": Config("couette1024x1024x512", 1024, 1024, 512, 4.0, 4.0, 3.0, 1002, {"couette": True}),
    "slab256x256x192": Config("slab256x256x192", 256, 256, 192, 2.0, 2.0, 3.0, 1003),
    "rb768x768x512": Config("rb768x768x512", 768, 768, 512, 1.0, 1.0, 3.0, 1004, {"ra": 1e8, "pr": 1.0}),
    # momentum on the Ra = 1e8 grid of Table 3, temperature refined twice in every direction
    "rb384x384x256": Config("rb384x384x256", 384, 384, 256, 1.0, 1.0, 3.0, 1005, {"ra": 1e8, "pr": 1.0}),
}


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def zfaces(nz: int, alpha: float = 3.0) -> np.ndarray:
    """Wall-normal face coordinates zf[0..nz] on [0, 1], tanh-clustered at both walls."""
    k = np.arange(nz + 1, dtype=np.float64)
    if alpha == 0.0:
        zf = k / nz
    else:
        zf = 0.5 * (1.0 + np.tanh(alpha * (2.0 * k / nz - 1.0)) / np.tanh(alpha))
    zf[0] = 0.0
    zf[nz] = 1.0
    return zf


def cell_centres(zf: np.ndarray) -> np.ndarray:
    """Cell-centre z coordinates (face midpoints)."""
    return 0.5 * (zf[:-1] + zf[1:])


def _normal_planes(seed: int, tag: int, shape, scale: float) -> np.ndarray:
    """N(0, scale^2) samples of ``shape`` (first axis = planes), one child stream per plane."""
    out = np.empty(shape, dtype=np.float64)
    children = np.random.SeedSequence([seed, tag]).spawn(shape[0])

    def fill(k):
        rng = np.random.Generator(np.random.PCG64(children[k]))
        out[k] = rng.standard_normal(shape[1:]) * scale

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fill, range(shape[0])))
    return out


def random_face_velocity(cfg: Config):
    """u, v, w i.i.d. N(0, 1) on every face; wall-face w set to zero (no penetration)."""
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    u = _normal_planes(cfg.seed, 1, (nz, ny, nx), 1.0)
    v = _normal_planes(cfg.seed, 2, (nz, ny, nx), 1.0)
    w = _normal_planes(cfg.seed, 3, (nz + 1, ny, nx), 1.0)
    w[0] = 0.0
    w[nz] = 0.0
    return u, v, w


def _mode_table(seed: int, nmodes: int = 64, kmax: int = 8, kzmax: int = 8):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    kx = np.empty(nmodes, np.int64)
    ky = np.empty(nmodes, np.int64)
    m = 0
    while m < nmodes:
        a, b = rng.integers(-kmax, kmax + 1, size=2)
        if a == 0 and b == 0:
            continue
        kx[m], ky[m] = a, b
        m += 1
    kz = rng.integers(1, kzmax + 1, size=nmodes)
    kk = np.sqrt(kx.astype(np.float64) ** 2 + ky ** 2 + kz ** 2)
    amp = kk ** (-5.0 / 3.0)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    pol = rng.standard_normal((nmodes, 3))
    pol /= np.linalg.norm(pol, axis=1, keepdims=True)
    return kx, ky, kz, amp, theta, pol


def _modal_component(xs, ys, zs, lx, ly, kx, ky, kz, coef, theta):
    """sum_m coef_m cos(2 pi (kx x/Lx + ky y/Ly) + theta_m) sin(pi kz z), as one matrix product.

    cos(a + b) = cos a cos b - sin a sin b, so each plane is
    [Y_c * c(z) | -Y_s * c(z)] @ [X_c ; X_s].
    """
    ax = 2.0 * np.pi * np.outer(kx, xs) / lx                 # (M, Nx)
    by = 2.0 * np.pi * np.outer(ys, ky) / ly + theta          # (Ny, M)
    cz = np.sin(np.pi * np.outer(zs, kz)) * coef              # (Nz', M)
    xmat = np.concatenate([np.cos(ax), np.sin(ax)], axis=0)   # (2M, Nx)
    yc, ys_ = np.cos(by), np.sin(by)
    nzp, ny, nx = cz.shape[0], ys.shape[0], xs.shape[0]
    out = np.empty((nzp, ny, nx), dtype=np.float64)
    chunk = max(1, (1 << 22) // max(1, ny * 2 * len(kx)))

    def do(k0):
        k1 = min(nzp, k0 + chunk)
        c = cz[k0:k1, None, :]                                # (kc, 1, M)
        a = np.concatenate([yc[None] * c, -ys_[None] * c], axis=2)   # (kc, Ny, 2M)
        out[k0:k1] = (a.reshape(-1, a.shape[2]) @ xmat).reshape(k1 - k0, ny, nx)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(do, range(0, nzp, chunk)))
    return out


def mode_velocity(cfg: Config, couette: bool | None = None, noise: float = 1e-2):
    """Velocity built from 64 random Fourier modes with a k^(-5/3) amplitude spectrum.

    Each mode m has integer horizontal wavenumbers (kx, ky) in [-8, 8]^2 minus
    (0, 0), kz in [1, 8], random phase and random unit polarisation; every
    component is evaluated at its own staggered location and vanishes at the
    walls (sin(pi kz z)).  The modal field is scaled to unit RMS over all three
    components, then N(0, noise^2) is added at interior points (wall-face w
    stays zero).  With ``couette`` the base profile u = 2 z - 1 is added (walls
    moving at -1 and +1).
    """
    if couette is None:
        couette = bool(cfg.extra.get("couette", False))
    nx, ny, nz, lx, ly = cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly
    dx, dy = lx / nx, ly / ny
    zf = zfaces(nz, cfg.alpha)
    zc = cell_centres(zf)
    kx, ky, kz, amp, theta, pol = _mode_table(cfg.seed)
    xf = np.arange(nx) * dx
    xc = (np.arange(nx) + 0.5) * dx
    yf = np.arange(ny) * dy
    yc = (np.arange(ny) + 0.5) * dy
    u = _modal_component(xf, yc, zc, lx, ly, kx, ky, kz, amp * pol[:, 0], theta)
    v = _modal_component(xc, yf, zc, lx, ly, kx, ky, kz, amp * pol[:, 1], theta)
    w = _modal_component(xc, yc, zf, lx, ly, kx, ky, kz, amp * pol[:, 2], theta)
    w[0] = 0.0
    w[nz] = 0.0
    ss = float(np.sum(u * u)) + float(np.sum(v * v)) + float(np.sum(w * w))
    rms = np.sqrt(ss / (u.size + v.size + (nz - 1) * nx * ny))
    u /= rms
    v /= rms
    w /= rms
    if noise > 0.0:
        u += _normal_planes(cfg.seed, 11, u.shape, noise)
        v += _normal_planes(cfg.seed, 12, v.shape, noise)
        w[1:nz] += _normal_planes(cfg.seed, 13, (nz - 1, ny, nx), noise)
    if couette:
        u += (2.0 * zc - 1.0)[:, None, None]
    return u, v, w


def rb_state(cfg: Config, tnoise: float = 1e-3, unoise: float = 1e-2):
    """Rayleigh-Benard initial state: linear T plus noise, small random velocity, zero pressure.

    T = 1 - z at the faces plus N(0, tnoise^2) at interior faces (walls exact:
    T = 1 at z = 0, T = 0 at z = 1); u, v, w ~ N(0, unoise^2) at interior
    points with each component's mean removed and wall-face w = 0; p = 0.
    """
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    zf = zfaces(nz, cfg.alpha)
    t = np.empty((nz + 1, ny, nx), dtype=np.float64)
    t[:] = (1.0 - zf)[:, None, None]
    t[1:nz] += _normal_planes(cfg.seed, 21, (nz - 1, ny, nx), tnoise)
    t[0] = 1.0
    t[nz] = 0.0
    u = _normal_planes(cfg.seed, 22, (nz, ny, nx), unoise)
    v = _normal_planes(cfg.seed, 23, (nz, ny, nx), unoise)
    w = np.zeros((nz + 1, ny, nx), dtype=np.float64)
    w[1:nz] = _normal_planes(cfg.seed, 24, (nz - 1, ny, nx), unoise)
    u -= u.mean()
    v -= v.mean()
    w[1:nz] -= w[1:nz].mean()
    p = np.zeros((nz, ny, nx), dtype=np.float64)
    return u, v, w, t, p


def rb_temperature(cfg: Config, zf: np.ndarray, nx: int, ny: int, tnoise: float = 1e-3, seed_tag: int = 25):
    """Temperature on faces ``zf`` of an nx x ny grid: 1 - z plus N(0, tnoise^2) at interior
    faces, walls exact (for a temperature grid finer than the momentum grid of ``cfg``)."""
    nzf = len(zf) - 1
    t = np.empty((nzf + 1, ny, nx), dtype=np.float64)
    t[:] = (1.0 - np.asarray(zf))[:, None, None]
    t[1:nzf] += _normal_planes(cfg.seed, seed_tag, (nzf - 1, ny, nx), tnoise)
    t[0] = 1.0
    t[nzf] = 0.0
    return t


def face_weights(cfg: Config, seed_tag: int = 31):
    """i.i.d. N(0, 1) weights on every free face (u, v everywhere, w on interior faces)."""
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    a = _normal_planes(cfg.seed, seed_tag, (nz, ny, nx), 1.0)
    b = _normal_planes(cfg.seed, seed_tag + 1, (nz, ny, nx), 1.0)
    c = np.zeros((nz + 1, ny, nx), dtype=np.float64)
    c[1:nz] = _normal_planes(cfg.seed, seed_tag + 2, (nz - 1, ny, nx), 1.0)
    return a, b, c


def small(name: str, nx: int, ny: int, nz: int, lx: float = 1.0, ly: float = 1.0,
          alpha: float = 3.0, seed: int = 7) -> Config:
    """A small ad-hoc configuration for tests."""
    return Config(name, nx, ny, nz, lx, ly, alpha, seed)
