"""Pins of the oracle's Poisson solve and projection against what mathematics fixes.

Each test checks the oracle against something other than itself: closed-form
discrete eigenvectors, the continuous solution (second-order convergence),
dense brute-force solves of the defining linear system, banded / extended
precision column solves, and identities of the discrete operators.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import Grid, poisson, operators as op
from paper_1705_01423_amd.synth import zfaces

F64 = torch.float64


def _grid(nx, ny, nz, lx=1.0, ly=1.0, alpha=3.0):
    return Grid(nx, ny, nz, lx, ly, zfaces(nz, alpha))


def _coords(g):
    xc = (torch.arange(g.nx, dtype=F64) + 0.5) * g.dx
    yc = (torch.arange(g.ny, dtype=F64) + 0.5) * g.dy
    return xc, yc, g.zc


def _ccc(g):
    xc, yc, zc = _coords(g)
    return (torch.cos(math.pi * zc)[:, None, None] * torch.cos(2 * math.pi * yc / g.ly)[None, :, None]
            * torch.cos(2 * math.pi * xc / g.lx)[None, None, :])


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("shape", [(16, 12, 10), (64, 64, 64), (24, 48, 16)])
def test_closed_form_eigenvector_uniform(shape):
    """cos(2pi x/Lx) cos(2pi y/Ly) cos(pi z) is an exact eigenvector of the uniform-grid L.

    Periodic three-point second difference: eigenvalue -(4/dx^2) sin^2(pi/N);
    Neumann three-point second difference on cell centres (DCT-II modes):
    eigenvalue -(4/dz^2) sin^2(pi/(2 Nz)).  Written here from trigonometry,
    independently of the oracle's wavenumber tables.
    """
    nx, ny, nz = shape
    lx, ly = 1.3, 0.7
    g = _grid(nx, ny, nz, lx, ly, alpha=0.0)
    phi = _ccc(g)
    dx, dy, dz = lx / nx, ly / ny, 1.0 / nz
    eig = -(4 / dx ** 2 * math.sin(math.pi / nx) ** 2 + 4 / dy ** 2 * math.sin(math.pi / ny) ** 2
            + 4 / dz ** 2 * math.sin(math.pi / (2 * nz)) ** 2)
    f = eig * phi
    # the operator itself has this eigenpair
    assert _rel(op.laplacian(phi, g), f) < 1e-13
    assert _rel(poisson.solve(f, g), phi) < 1e-13


@pytest.mark.parametrize("shape", [(16, 12, 10), (32, 32, 48)])
def test_manufactured_stretched(shape):
    """On the tanh-stretched grid, f = L phi* must give back phi* (zero-mean modes: no gauge shift)."""
    g = _grid(*shape, lx=2.0, ly=1.0, alpha=3.0)
    phi = _ccc(g)
    f = op.laplacian(phi, g)
    assert _rel(poisson.solve(f, g), phi) < 1e-13


@pytest.mark.parametrize("alpha", [0.0, 3.0])
def test_second_order_convergence(alpha):
    """Error against the continuous solution falls by ~4 per grid doubling (second-order scheme)."""
    errs = []
    for n in (16, 32, 64):
        g = _grid(n, n, n, 1.0, 1.0, alpha)
        xc, yc, zc = _coords(g)
        exact = (torch.cos(math.pi * zc)[:, None, None] * torch.cos(2 * math.pi * yc)[None, :, None]
                 * torch.cos(2 * math.pi * xc)[None, None, :])
        f = -math.pi ** 2 * (4 + 4 + 1) * exact
        phi = poisson.solve(f, g)
        errs.append(float((phi - exact).abs().max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.7 < r2 < 4.3, errs


def _dense_laplacian(g):
    n = g.nx * g.ny * g.nz
    cols = []
    for idx in range(n):
        e = torch.zeros(n, dtype=F64)
        e[idx] = 1.0
        cols.append(op.laplacian(e.view(g.nz, g.ny, g.nx), g).reshape(-1))
    return torch.stack(cols, dim=1).numpy()


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 12, 5), (24, 12, 8), (4, 4, 2)])
def test_brute_force_dense(shape):
    """FFT + tridiagonal solve == dense solve of the bordered gauge system [[L, v],[v^T, 0]]."""
    g = _grid(*shape, lx=1.0, ly=1.5, alpha=3.0)
    n = g.nx * g.ny * g.nz
    L = _dense_laplacian(g)
    vol = np.repeat(g.dz.numpy(), g.nx * g.ny)             # dz-weights per cell
    rng = np.random.default_rng(3)
    f = rng.standard_normal(n)
    fc = f - vol @ f / vol.sum()                           # compatible right-hand side
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = L
    A[:n, n] = vol
    A[n, :n] = vol
    sol = np.linalg.solve(A, np.concatenate([fc, [0.0]]))
    assert abs(sol[n]) < 1e-10 * np.abs(sol[:n]).max()    # multiplier ~ 0: system consistent
    phi = poisson.solve(torch.tensor(f).view(g.nz, g.ny, g.nx), g).reshape(-1).numpy()
    assert np.linalg.norm(phi - sol[:n]) / np.linalg.norm(sol[:n]) < 1e-13


def test_residual_and_gauge():
    g = _grid(32, 24, 40, 2.0, 2.0, 3.0)
    torch.manual_seed(1)
    f = torch.randn(g.nz, g.ny, g.nx, dtype=F64) + 0.25
    phi, defect = poisson.solve(f, g, return_defect=True)
    ft = f - defect
    res = ft - op.laplacian(phi, g)
    # evaluating L phi on this stretched grid already rounds at ~eps |L| |phi|
    assert float(res.norm() / ft.norm()) < 1e-12
    assert abs(op.weighted_sum(phi, g)) < 1e-13 * float(phi.abs().sum())
    # defect is the dz-weighted mean: shifting f by a constant shifts it exactly
    _, d2 = poisson.solve(f + 1.5, g, return_defect=True)
    assert abs(d2 - defect - 1.5) < 1e-13
    assert abs(defect - op.weighted_mean(f, g)) < 1e-14


def test_summation_by_parts():
    """D = -Vc^-1 G^T Vf: sum_c dz phi (D q) = -sum_f V q . G phi for w_wall = 0."""
    g = _grid(10, 8, 12, 1.0, 1.0, 3.0)
    torch.manual_seed(2)
    phi = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    u = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    v = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    w = torch.randn(g.nz + 1, g.ny, g.nx, dtype=F64)
    w[0] = 0
    w[-1] = 0
    gu, gv, gw = op.gradient(phi, g)
    lhs = float((g.vc() * phi * op.divergence(u, v, w, g)).sum())
    rhs = -float((g.vc() * u * gu).sum() + (g.vc() * v * gv).sum() + (g.vw() * w * gw).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _curl_fields(g, seed):
    """Exactly divergence-free staggered fields from corner / edge potentials."""
    gen = torch.Generator().manual_seed(seed)
    psi = torch.randn(g.nz, g.ny, g.nx, generator=gen, dtype=F64)      # at (x-face i, y-face j)
    chi = torch.randn(g.nz + 1, g.ny, g.nx, generator=gen, dtype=F64)  # at (x-face i, z-face k)
    chi[0] = 0
    chi[-1] = 0
    u = (torch.roll(psi, -1, 1) - psi) / g.dy + (chi[1:] - chi[:-1]) / g.dz[:, None, None]
    v = -(torch.roll(psi, -1, 2) - psi) / g.dx
    w = -(torch.roll(chi, -1, 2) - chi) / g.dx
    return u, v, w


def test_projector_identities():
    g = _grid(12, 10, 9, 1.0, 1.2, 3.0)
    z = torch.zeros(g.nz, g.ny, g.nx, dtype=F64)
    # exactly solenoidal input is left unchanged
    u, v, w = _curl_fields(g, 5)
    assert float(op.divergence(u, v, w, g).abs().max()) < 1e-11
    pu, pv, pw, _, _ = poisson.project(u, v, w, z, g)
    assert _rel(torch.cat([pu.reshape(-1), pv.reshape(-1), pw.reshape(-1)]),
                torch.cat([u.reshape(-1), v.reshape(-1), w.reshape(-1)])) < 1e-13
    # gradients are removed entirely
    psi = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    gu, gv, gw = op.gradient(psi, g)
    pu, pv, pw, _, _ = poisson.project(gu, gv, gw, z, g)
    scale = float(torch.cat([gu.reshape(-1), gv.reshape(-1), gw.reshape(-1)]).norm())
    assert float(torch.cat([pu.reshape(-1), pv.reshape(-1), pw.reshape(-1)]).norm()) < 1e-13 * scale
    # idempotent, V_f-orthogonal, and divergence-free output
    torch.manual_seed(4)
    u = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    v = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    w = torch.randn(g.nz + 1, g.ny, g.nx, dtype=F64)
    w[0] = 0
    w[-1] = 0
    pu, pv, pw, _, _ = poisson.project(u, v, w, z, g)
    ppu, ppv, ppw, _, _ = poisson.project(pu, pv, pw, z, g)
    assert _rel(ppu, pu) < 1e-13 and _rel(ppv, pv) < 1e-13 and _rel(ppw, pw) < 1e-13
    inner = float((g.vc() * pu * (u - pu)).sum() + (g.vc() * pv * (v - pv)).sum()
                  + (g.vw() * pw * (w - pw)).sum())
    assert abs(inner) < 1e-12 * float((g.vc() * u * u).sum())
    d0 = float(op.divergence(u, v, w, g).abs().max())
    assert float(op.divergence(pu, pv, pw, g).abs().max()) < 1e-13 * d0


def _column_matrix(g, lam):
    nz = g.nz
    o, dz = g.o.numpy(), g.dz.numpy()
    ab = np.zeros((3, nz))
    for k in range(nz):
        ab[1, k] = o[k] + o[k + 1] + lam * dz[k]
        if k + 1 < nz:
            ab[0, k + 1] = -o[k + 1]
            ab[2, k] = -o[k + 1]
    return ab


def test_zsolve_vs_banded():
    """Column solve == scipy banded LU at moderate wavenumbers."""
    g = _grid(8, 8, 64, 1.0, 1.0, 3.0)
    rng = np.random.default_rng(0)
    lam = np.array([[50.0, 400.0], [3000.0, 1.0e5]])
    F = rng.standard_normal((g.nz, 2, 2)) + 1j * rng.standard_normal((g.nz, 2, 2))
    P = poisson.zsolve_excess(torch.tensor(F), torch.tensor(lam, dtype=F64), g).numpy()
    for a in range(2):
        for b in range(2):
            ab = _column_matrix(g, lam[a, b])
            ref = scipy.linalg.solve_banded((1, 1), ab, -g.dz.numpy() * F[:, a, b])
            # LAPACK forms pivots by subtraction: its own error is ~1e-14 here
            assert np.linalg.norm(P[:, a, b] - ref) / np.linalg.norm(ref) < 1e-13


def test_zsolve_low_wavenumber_extended_precision():
    """Smallest wavenumbers on a strongly stretched 512-cell column: agree with a long-double Thomas."""
    nz = 512
    g = _grid(4, 4, nz, 4.0, 4.0, 3.0)
    dx = 4.0 / 1024
    lams = [4 / dx ** 2 * math.sin(math.pi / 1024) ** 2, 2 * 4 / dx ** 2 * math.sin(math.pi / 1024) ** 2, 7.0]
    rng = np.random.default_rng(1)
    for lam in lams:
        F = rng.standard_normal(nz)
        P = poisson.zsolve_excess(torch.tensor(F + 0j), torch.tensor(lam, dtype=F64), g).real.numpy()
        ld = np.longdouble
        zf = np.asarray(zfaces(nz, 3.0), dtype=ld)
        dz = zf[1:] - zf[:-1]
        o = np.zeros(nz + 1, dtype=ld)
        o[1:nz] = 1 / ((dz[:-1] + dz[1:]) / 2)
        diag = o[:-1] + o[1:] + ld(lam) * dz
        rhs = -dz * np.asarray(F, dtype=ld)
        c = np.zeros(nz, dtype=ld)
        d = np.zeros(nz, dtype=ld)
        c[0] = -o[1] / diag[0]
        d[0] = rhs[0] / diag[0]
        for k in range(1, nz):
            den = diag[k] + o[k] * c[k - 1]
            c[k] = -o[k + 1] / den
            d[k] = (rhs[k] + o[k] * d[k - 1]) / den
        x = np.zeros(nz, dtype=ld)
        x[-1] = d[-1]
        for k in range(nz - 2, -1, -1):
            x[k] = d[k] - c[k] * x[k + 1]
        x = x.astype(np.float64)
        assert np.linalg.norm(P - x) / np.linalg.norm(x) < 1e-14
