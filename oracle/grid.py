"""Grid metrics for the staggered, wall-stretched box (paper Sec. 2.1, Fig. 1).

Notation (z is wall-normal here; the paper calls it x):

* ``dz[k]  = zf[k+1] - zf[k]``               cell heights, k = 0..Nz-1
* ``dzc[k] = (dz[k-1] + dz[k]) / 2``         centre-to-centre distance across
                                            interior face k = 1..Nz-1
                                            (centres are face midpoints)
* ``o[k]   = 1 / dzc[k]`` for interior faces, ``o[0] = o[Nz] = 0``
* modified wavenumbers (Sec. 2.2): the eigenvalues of minus the periodic
  three-point second difference,
  ``lamx[kx] = (4/dx^2) sin^2(pi kx / Nx)``, kx = 0..Nx/2, and likewise lamy
  for ky = 0..Ny-1.  This equals (2/dx^2)(1 - cos(2 pi kx / Nx)) but is
  evaluated through sin^2 so that the smallest eigenvalues keep full relative
  precision.

Parity: pinned by the manufactured-solution, convergence and brute-force tests
(tests/test_oracle_poisson.py).
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64


class Grid:
    def __init__(self, nx: int, ny: int, nz: int, lx: float, ly: float, zf):
        zf = torch.as_tensor(np.asarray(zf, dtype=np.float64))
        assert zf.shape == (nz + 1,)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lx, self.ly = float(lx), float(ly)
        self.dx = self.lx / nx
        self.dy = self.ly / ny
        self.zf = zf
        self.dz = zf[1:] - zf[:-1]
        dzc = torch.zeros(nz + 1, dtype=F64)
        dzc[1:nz] = 0.5 * (self.dz[:-1] + self.dz[1:])
        self.dzc = dzc
        o = torch.zeros(nz + 1, dtype=F64)
        o[1:nz] = 1.0 / dzc[1:nz]
        self.o = o
        self.zc = 0.5 * (zf[:-1] + zf[1:])
        kx = torch.arange(nx // 2 + 1, dtype=F64)
        ky = torch.arange(ny, dtype=F64)
        self.lamx = (4.0 / self.dx ** 2) * torch.sin(math.pi * kx / nx) ** 2
        self.lamy = (4.0 / self.dy ** 2) * torch.sin(math.pi * ky / ny) ** 2
        # Distances from the wall-adjacent centres to the walls, used by the
        # wall-normal second difference of centre fields with Dirichlet walls.
        dzw = torch.zeros(nz + 1, dtype=F64)
        dzw[1:nz] = dzc[1:nz]
        dzw[0] = 0.5 * self.dz[0]
        dzw[nz] = 0.5 * self.dz[nz - 1]
        self.dzw = dzw

    # volume weights (the dx*dy factor is common to all and omitted)
    def vc(self):
        """Cell-centre volume weights, shape (Nz, 1, 1)."""
        return self.dz[:, None, None]

    def vw(self):
        """z-face volume weights (interior faces; walls 0), shape (Nz+1, 1, 1)."""
        return self.dzc[:, None, None]
