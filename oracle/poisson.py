"""Direct pressure-Poisson solve and projection (paper Sec. 2.1-2.2).

Problem (the plain definition the direct method reaches exactly up to rounding):
find phi at the cell centres with

    L phi = f - mean_dz(f)      and      sum_k dz_k sum_{j,i} phi = 0,

where L = D G is the flux-form staggered Laplacian (periodic x, y; zero normal
flux at the walls), mean_dz is the dz-weighted mean (the left null vector of L
is dz, so the right-hand side is first made compatible) and the gauge is the
dz-weighted zero mean.

Method (Sec. 2.2, the solver's algorithm with the pencil transposes dropped:
one address space holds the whole box):

1. real FFT along x, then complex FFT along y, plane by plane;
2. for each wavenumber pair (kx, ky) one tridiagonal system in z with the
   modified wavenumber lam = lamx[kx] + lamy[ky] (Sec. 2.2: the 2-D transform
   reduces the 3-D problem to independent 1-D problems solved by Thomas);
3. inverse complex FFT along y, inverse real FFT along x.

The per-column system, multiplied by -dz_k so that it is symmetric and an
M-matrix, is

    -o_k P_{k-1} + (o_k + o_{k+1} + lam dz_k) P_k - o_{k+1} P_{k+1} = -dz_k F_k.

It is solved by Gaussian elimination in "excess" form: the amount by which
each pivot exceeds the next off-diagonal is carried explicitly, so no pivot is
formed by cancellation (Grassmann-Taksar-Heyman; the same elimination as
Thomas, algebraically).  The singular column (kx, ky) = (0, 0) is integrated
directly: fluxes are prefix sums of dz_k F_k, the potential is the prefix sum
of dzc_k times the fluxes, and the dz-weighted mean is removed.

Projection (Sec. 2.1, "delta" form; pressure update with the wall-normal
implicit operator): with s = alpha dt and c = alpha dt nu / 2,

    L phi = D u* / s,   u = u* - s G phi,   p <- p + phi - c Dzz phi.

Parity: pinned by tests/test_oracle_poisson.py (closed-form eigenvector,
manufactured solution on the stretched grid, second-order convergence to the
continuous solution, dense brute force on tiny grids, residual and divergence
invariants, projector identities).
"""
from __future__ import annotations

import math

import torch

from . import operators as op

F64 = torch.float64
C128 = torch.complex128


def zsolve_excess(F, lam, g):
    """Solve the dz-scaled column systems for every column at once.

    F: complex (Nz, ...) right-hand sides (Fourier coefficients of f per plane);
    lam: real (...) modified wavenumbers, all > 0.  Returns P with F's shape.
    """
    nz = g.nz
    o = g.o
    dz = g.dz
    pivots = []
    ys = []
    e = lam * dz[0]                           # excess of row 0
    y = -dz[0] * F[0]
    pivots.append(o[1] + e)
    ys.append(y)
    for k in range(1, nz):
        m = o[k] / pivots[k - 1]
        e = lam * dz[k] + m * e
        y = -dz[k] * F[k] + m * y
        pivots.append(o[k + 1] + e)
        ys.append(y)
    out = [None] * nz
    x = ys[nz - 1] / pivots[nz - 1]
    out[nz - 1] = x
    for k in range(nz - 2, -1, -1):
        x = (ys[k] + o[k + 1] * x) / pivots[k]
        out[k] = x
    return torch.stack(out, dim=0)


def _neumaier_prefix(values):
    """Running sums s_k = v_0 + ... + v_k with Neumaier compensation."""
    out = []
    s = 0.0
    c = 0.0
    for v in values:
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
        out.append(s + c)
    return out


def singular_column(F00, g):
    """(kx, ky) = (0, 0) column: compatibility, direct integration, gauge.

    F00: real (Nz,) = plane sums of f.  Returns (Phi00, defect) where defect is
    the dz-weighted mean that was removed from f (per grid point).
    """
    dz = g.dz.tolist()
    dzc = g.dzc.tolist()
    vals = F00.tolist()
    total_dz = math.fsum(dz)
    wsum = math.fsum(d * v for d, v in zip(dz, vals))
    mean_plane = wsum / total_dz               # per plane (sum over NxNy points)
    fixed = [v - mean_plane for v in vals]
    # fluxes at faces: Q_0 = 0, Q_{k+1} = sum_{j<=k} dz_j F_j
    q = [0.0] + _neumaier_prefix([d * v for d, v in zip(dz, fixed)])
    # potential at centres: Phi_0 = 0, Phi_k = Phi_{k-1} + dzc_k Q_k
    phi = [0.0] + _neumaier_prefix([dzc[k] * q[k] for k in range(1, g.nz)])
    shift = math.fsum(d * p for d, p in zip(dz, phi)) / total_dz
    phi = [p - shift for p in phi]
    defect = mean_plane / (g.nx * g.ny)
    return torch.tensor(phi, dtype=F64), defect


def solve(f, g, return_defect=False):
    """phi = L^+ (f - mean_dz f), dz-weighted zero mean."""
    assert f.shape == (g.nz, g.ny, g.nx) and f.dtype == F64
    # Steps 1-2: forward transforms (real along x, complex along y).
    fx = torch.fft.rfft(f, dim=2)
    F = torch.fft.fft(fx, dim=1)
    # Step 3: one tridiagonal solve per wavenumber pair.
    lam = g.lamy[:, None] + g.lamx[None, :]
    lam_safe = lam.clone()
    lam_safe[0, 0] = 1.0                      # placeholder; column replaced below
    P = zsolve_excess(F, lam_safe, g)
    # The plane sums of f are the (0,0) coefficients (pairwise summation).
    plane_sums = f.sum(dim=(1, 2))
    phi00, defect = singular_column(plane_sums, g)
    P = P.clone()
    P[:, 0, 0] = phi00.to(C128)
    # Steps 4-5: inverse transforms.
    px = torch.fft.ifft(P, dim=1)
    phi = torch.fft.irfft(px, n=g.nx, dim=2)
    if return_defect:
        return phi, defect
    return phi


def solve_autograd(f, g):
    """Differentiable version of ``solve`` (same steps, written with torch ops only).

    Used to obtain the adjoint of the solve through torch.autograd.
    """
    nz = g.nz
    # compatibility projection: subtract the dz-weighted mean
    planes = f.sum(dim=(1, 2))
    mean = (g.dz * planes).sum() / (g.dz.sum() * g.nx * g.ny)
    ft = f - mean
    fx = torch.fft.rfft(ft, dim=2)
    F = torch.fft.fft(fx, dim=1)
    lam = g.lamy[:, None] + g.lamx[None, :]
    lam_safe = lam.clone()
    lam_safe[0, 0] = 1.0
    P = zsolve_excess(F, lam_safe, g)
    # singular column by direct integration (same recurrences as singular_column)
    F00 = F[:, 0, 0].real
    flux = torch.cumsum(g.dz * F00, dim=0)                     # Q_1..Q_Nz
    inc = g.dzc[1:nz] * flux[:nz - 1]
    phi00 = torch.cat([torch.zeros(1, dtype=F64), torch.cumsum(inc, dim=0)])
    phi00 = phi00 - (g.dz * phi00).sum() / g.dz.sum()
    mask = torch.zeros_like(P.real)
    mask[:, 0, 0] = 1.0
    P = P * (1 - mask) + phi00[:, None, None].to(C128) * mask
    px = torch.fft.ifft(P, dim=1)
    return torch.fft.irfft(px, n=g.nx, dim=2)


def project(u, v, w, p, g, s=1.0, c=0.0, differentiable=False):
    """Projection and pressure update.  Returns (u, v, w, p, phi) as new tensors."""
    f = op.divergence(u, v, w, g) / s
    phi = solve_autograd(f, g) if differentiable else solve(f, g)
    gu, gv, gw = op.gradient(phi, g)
    un = u - s * gu
    vn = v - s * gv
    wn = w - s * gw
    pn = p + phi - c * op.dzz_centre_neumann(phi, g)
    return un, vn, wn, pn, phi
