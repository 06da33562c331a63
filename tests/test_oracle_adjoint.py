"""Pins of the oracle's adjoints (obtained with torch.autograd through the oracle).

The adjoint identities follow from summation by parts: L is self-adjoint in
the dz-weighted inner product, so the Euclidean transpose of the solve is
Vc S Vc^-1, and the projector is Vf-orthogonal, so P^T = Vf P Vf^-1.
"""
import numpy as np
import torch

from oracle import Grid, poisson
from oracle import substep as ss
from paper_1705_01423_amd.synth import zfaces

F64 = torch.float64


def _grid(nx, ny, nz, lx=1.0, ly=1.0, alpha=3.0):
    return Grid(nx, ny, nz, lx, ly, zfaces(nz, alpha))


def test_solve_autograd_matches_solve():
    g = _grid(10, 8, 12)
    f = torch.randn(g.nz, g.ny, g.nx, dtype=F64, generator=torch.Generator().manual_seed(0))
    a = poisson.solve(f, g)
    b = poisson.solve_autograd(f, g)
    assert float((a - b).norm() / a.norm()) < 1e-14


def test_solve_transpose_identity():
    g = _grid(8, 6, 10)
    gen = torch.Generator().manual_seed(1)
    f = torch.randn(g.nz, g.ny, g.nx, dtype=F64, generator=gen, requires_grad=True)
    gphi = torch.randn(g.nz, g.ny, g.nx, dtype=F64, generator=gen)
    phi = poisson.solve_autograd(f, g)
    (gf,) = torch.autograd.grad(phi, f, gphi)
    vc = g.vc()
    ident = vc * poisson.solve(gphi / vc, g)
    assert float((gf - ident).norm() / gf.norm()) < 1e-13


def _flat(*ts):
    return torch.cat([t.reshape(-1) for t in ts])


def test_projection_transpose_dense():
    """Dense Jacobian of the projection on a 4x4x4 grid: P^2 = P and P^T = Vf P Vf^-1."""
    g = _grid(4, 4, 4)
    nc = g.nz * g.ny * g.nx
    nwi = (g.nz - 1) * g.ny * g.nx
    n = 2 * nc + nwi
    z = torch.zeros(g.nz, g.ny, g.nx, dtype=F64)

    def apply(x):
        u = x[:nc].view(g.nz, g.ny, g.nx)
        v = x[nc:2 * nc].view(g.nz, g.ny, g.nx)
        wi = x[2 * nc:].view(g.nz - 1, g.ny, g.nx)
        zero = torch.zeros(1, g.ny, g.nx, dtype=F64)
        w = torch.cat([zero, wi, zero], 0)
        pu, pv, pw, _, _ = poisson.project(u, v, w, z, g, differentiable=True)
        return _flat(pu, pv, pw[1:g.nz])

    P = torch.autograd.functional.jacobian(apply, torch.zeros(n, dtype=F64)).numpy()
    assert np.abs(P @ P - P).max() < 1e-13
    vf = np.concatenate([np.repeat(g.dz.numpy(), g.nx * g.ny)] * 2
                        + [np.repeat(g.dzc[1:g.nz].numpy(), g.nx * g.ny)])
    ident = (vf[:, None] * P) / vf[None, :]
    assert np.abs(P.T - ident).max() < 1e-13
    # forward application agrees with the non-differentiable path
    x = torch.randn(n, dtype=F64, generator=torch.Generator().manual_seed(3))
    assert np.abs(P @ x.numpy() - apply(x).detach().numpy()).max() < 1e-13


def test_substep_vjp_finite_difference():
    """Autograd VJP of one substep agrees with central differences (h = 1e-6) on random directions."""
    g = _grid(8, 8, 8)
    gen = torch.Generator().manual_seed(7)
    u = 1e-1 * torch.randn(g.nz, g.ny, g.nx, dtype=F64, generator=gen)
    v = 1e-1 * torch.randn(g.nz, g.ny, g.nx, dtype=F64, generator=gen)
    w = 1e-1 * torch.randn(g.nz + 1, g.ny, g.nx, dtype=F64, generator=gen)
    w[0] = 0
    w[-1] = 0
    t = (1 - g.zf)[:, None, None].expand(g.nz + 1, g.ny, g.nx).clone()
    t[1:g.nz] += 1e-2 * torch.randn(g.nz - 1, g.ny, g.nx, dtype=F64, generator=gen)
    p = 1e-2 * torch.randn(g.nz, g.ny, g.nx, dtype=F64, generator=gen)
    dt, nu, ka = 2e-2, 1e-2, 1e-2
    ws = [torch.randn_like(a, generator=None) for a in (u, v, w, t, p)]

    def loss(state):
        out, _ = ss.substep(state, g, 1, dt, nu, ka, differentiable=True)
        return sum((a * b).sum() for a, b in zip(out, ws))

    state = [a.clone().requires_grad_(True) for a in (u, v, w, t, p)]
    grads = torch.autograd.grad(loss(state), state)
    for trial in range(3):
        d = [torch.randn(a.shape, dtype=F64, generator=gen) for a in (u, v, w, t, p)]
        for di in (d[2], d[3]):
            di[0] = 0
            di[-1] = 0
        h = 1e-6
        with torch.no_grad():
            lp = loss([a + h * b for a, b in zip((u, v, w, t, p), d)])
            lm = loss([a - h * b for a, b in zip((u, v, w, t, p), d)])
        fd = float((lp - lm) / (2 * h))
        an = float(sum((gr * di).sum() for gr, di in zip(grads, d)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
