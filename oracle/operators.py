"""Discrete operators of the second-order staggered scheme (paper Sec. 2.1, Fig. 1).

Locations: p, phi, f at cell centres (Nz, Ny, Nx); u at x-faces (x = i dx), v at
y-faces (y = j dy), both at z-centres (Nz, Ny, Nx); w, T at z-faces (Nz+1, Ny, Nx)
with the wall rows stored.  x and y are periodic.

* divergence  (D q)_k = (u_{i+1} - u_i)/dx + (v_{j+1} - v_j)/dy + (w_{k+1} - w_k)/dz_k
* gradient    (G phi)_u = (phi_i - phi_{i-1})/dx, (G phi)_v likewise,
              (G phi)_w = (phi_k - phi_{k-1})/dzc_k at interior faces, 0 at the
              two walls (Neumann: the wall-normal velocity is fixed there)
* Laplacian   L = D G (flux form; the operator the direct solve inverts)

Parity: pinned by the closed-form eigenvector, second-order convergence,
summation-by-parts and brute-force tests (tests/test_oracle_poisson.py).
"""
from __future__ import annotations

import math

import torch


def divergence(u, v, w, g):
    return ((torch.roll(u, -1, dims=2) - u) / g.dx
            + (torch.roll(v, -1, dims=1) - v) / g.dy
            + (w[1:] - w[:-1]) / g.dz[:, None, None])


def gradient(phi, g):
    gu = (phi - torch.roll(phi, 1, dims=2)) / g.dx
    gv = (phi - torch.roll(phi, 1, dims=1)) / g.dy
    inner = (phi[1:] - phi[:-1]) / g.dzc[1:g.nz, None, None]
    zero = torch.zeros_like(phi[:1])
    gw = torch.cat([zero, inner, zero], dim=0)
    return gu, gv, gw


def laplacian(phi, g):
    """Flux-form Laplacian L phi = D(G phi)."""
    return divergence(*gradient(phi, g), g)


def dzz_centre_neumann(phi, g):
    """Wall-normal part of L: [o_{k+1}(phi_{k+1}-phi_k) - o_k(phi_k-phi_{k-1})]/dz_k, zero wall flux."""
    flux = torch.cat([torch.zeros_like(phi[:1]),
                      (phi[1:] - phi[:-1]) * g.o[1:g.nz, None, None],
                      torch.zeros_like(phi[:1])], dim=0)
    return (flux[1:] - flux[:-1]) / g.dz[:, None, None]


def dzz_centre_dirichlet(q, g, bot=0.0, top=0.0):
    """Wall-normal second difference of a centre field with wall values ``bot``/``top``.

    The wall sits half a cell below the first centre (and above the last), so the
    wall flux is (q_0 - bot) / (dz_0 / 2).
    """
    inner = (q[1:] - q[:-1]) / g.dzw[1:g.nz, None, None]
    fb = ((q[:1] - bot) / g.dzw[0])
    ft = ((top - q[-1:]) / g.dzw[g.nz])
    flux = torch.cat([fb, inner, ft], dim=0)
    return (flux[1:] - flux[:-1]) / g.dz[:, None, None]


def dzz_face(q, g):
    """Wall-normal second difference of a z-face field at interior faces (walls -> 0).

    [(q_{k+1}-q_k)/dz_k - (q_k-q_{k-1})/dz_{k-1}] / dzc_k for k = 1..Nz-1.
    """
    flux = (q[1:] - q[:-1]) / g.dz[:, None, None]          # at centres, Nz entries
    inner = (flux[1:] - flux[:-1]) / g.dzc[1:g.nz, None, None]
    zero = torch.zeros_like(q[:1])
    return torch.cat([zero, inner, zero], dim=0)


def dxx(q, g):
    return (torch.roll(q, -1, dims=2) - 2.0 * q + torch.roll(q, 1, dims=2)) / (g.dx * g.dx)


def dyy(q, g):
    return (torch.roll(q, -1, dims=1) - 2.0 * q + torch.roll(q, 1, dims=1)) / (g.dy * g.dy)


def weighted_sum(f, g):
    """sum_k dz_k * sum_{j,i} f_{k,j,i}, exactly rounded over planes (math.fsum)."""
    planes = f.sum(dim=(1, 2))
    return math.fsum((g.dz * planes).tolist())


def weighted_mean(f, g):
    """dz-weighted mean of a centre field (the compatibility defect of a Poisson RHS)."""
    return weighted_sum(f, g) / (math.fsum(g.dz.tolist()) * g.nx * g.ny)
