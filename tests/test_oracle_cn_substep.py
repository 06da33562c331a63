"""Pins of the oracle's Crank-Nicolson solves, explicit terms, CFL and RK3 substep."""
import math

import numpy as np
import pytest
import torch

from oracle import Grid, cn, operators as op, poisson
from oracle import substep as ss
from paper_1705_01423_amd.synth import zfaces

F64 = torch.float64


def _grid(nx, ny, nz, lx=1.0, ly=1.0, alpha=3.0):
    return Grid(nx, ny, nz, lx, ly, zfaces(nz, alpha))


def _dense(fn, shape):
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = torch.zeros(n, dtype=F64)
        e[i] = 1.0
        cols.append(fn(e.view(shape)).reshape(-1))
    return torch.stack(cols, 1).numpy()


def test_cn_centre_dense():
    """CN solve inverts I - beta Dzz, with Dzz the centre operator with zero wall values."""
    g = _grid(1, 1, 17)
    beta = 3e-4
    M = np.eye(g.nz) - beta * _dense(lambda q: op.dzz_centre_dirichlet(q, g), (g.nz, 1, 1))
    rng = np.random.default_rng(0)
    rhs = rng.standard_normal((g.nz, 3, 2))
    x = cn.solve_centre(torch.tensor(rhs), g, beta).numpy()
    ref = np.linalg.solve(M, rhs.reshape(g.nz, -1)).reshape(rhs.shape)
    assert np.abs(x - ref).max() < 1e-14 * np.abs(ref).max() * 10


def test_cn_face_dense():
    g = _grid(1, 1, 15)
    beta = 2e-4

    def dzz_inner(q):
        full = torch.cat([torch.zeros(1, 1, 1, dtype=F64), q, torch.zeros(1, 1, 1, dtype=F64)], 0)
        return op.dzz_face(full, g)[1:g.nz]

    M = np.eye(g.nz - 1) - beta * _dense(dzz_inner, (g.nz - 1, 1, 1))
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal((g.nz + 1, 2, 2))
    x = cn.solve_face(torch.tensor(rhs), g, beta).numpy()
    ref = np.linalg.solve(M, rhs[1:g.nz].reshape(g.nz - 1, -1)).reshape(g.nz - 1, 2, 2)
    assert np.abs(x[1:g.nz] - ref).max() < 1e-13 * np.abs(ref).max()
    assert np.all(x[0] == 0) and np.all(x[g.nz] == 0)


def test_dzz_linear_profiles():
    """Second differences of linear profiles vanish on the stretched grid (faces and centres)."""
    g = _grid(3, 2, 33)
    t = (1.0 - g.zf)[:, None, None].expand(g.nz + 1, 2, 3)
    assert float(op.dzz_face(t, g).abs().max()) < 1e-9          # O(eps/dz^2)
    zc = g.zc[:, None, None].expand(g.nz, 2, 3)
    d = op.dzz_centre_dirichlet(zc, g, bot=0.0, top=1.0)
    assert float(d.abs().max()) < 1e-9


def test_dzz_centre_convergence():
    """Centre second difference with Dirichlet walls converges to q'' (L2 error)."""
    errs = []
    for n in (32, 64, 128):
        g = _grid(1, 1, n)
        q = torch.sin(math.pi * g.zc)[:, None, None]
        d = op.dzz_centre_dirichlet(q, g)
        ex = -math.pi ** 2 * q
        errs.append(float(torch.sqrt((g.dz[:, None, None] * (d - ex) ** 2).sum())))
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8, errs


def test_rk3_coefficients():
    """Applied explicitly to y' = mu y the three substeps give the cubic Taylor polynomial."""
    for z in (0.3, -0.7, 1.1):
        y, yprev = 1.0, 0.0
        for l in (1, 2, 3):
            f, fprev = z * y, z * yprev
            ynew = y + ss.GAMMA[l - 1] * f + ss.RHO[l - 1] * fprev
            yprev, y = y, ynew
        assert abs(y - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15
    assert abs(sum(ss.alpha_coef(l) for l in (1, 2, 3)) - 1.0) < 1e-15


def test_advection_conserves_energy():
    g = _grid(12, 10, 9, 1.0, 1.2)
    torch.manual_seed(0)
    u = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    v = torch.randn(g.nz, g.ny, g.nx, dtype=F64)
    w = torch.randn(g.nz + 1, g.ny, g.nx, dtype=F64)
    w[0] = 0
    w[-1] = 0
    z = torch.zeros_like(u)
    u, v, w, _, _ = poisson.project(u, v, w, z, g)
    au, av, aw = ss.adv_u(u, v, w, g), ss.adv_v(u, v, w, g), ss.adv_face(w, u, v, w, g)
    e = float((g.vc() * u * au).sum() + (g.vc() * v * av).sum() + (g.vw() * w * aw).sum())
    scale = float((g.vc() * (u * au).abs()).sum())
    assert abs(e) < 1e-13 * scale
    t = torch.randn(g.nz + 1, g.ny, g.nx, dtype=F64)
    t[0] = 0
    t[-1] = 0
    at = ss.adv_face(t, u, v, w, g)
    assert abs(float((g.vw() * t * at).sum())) < 1e-13 * float((g.vw() * (t * at).abs()).sum())


def test_rest_state():
    """Conduction state: velocity stays zero, T unchanged, buoyancy goes into the pressure."""
    g = _grid(8, 6, 10)
    t = (1 - g.zf)[:, None, None].expand(g.nz + 1, g.ny, g.nx).clone()
    z = torch.zeros(g.nz, g.ny, g.nx, dtype=F64)
    zw = torch.zeros(g.nz + 1, g.ny, g.nx, dtype=F64)
    (u, v, w, tn, p), _ = ss.substep((z, z, zw, t, z), g, 1, 1e-3, 1e-4, 1e-4)
    assert float(u.abs().max()) == 0.0 and float(v.abs().max()) == 0.0
    assert float(w.abs().max()) < 1e-15
    assert float((tn - t).abs().max()) < 1e-15
    # hydrostatic: the wall-normal pressure gradient is proportional to T
    gw = (p[1:] - p[:-1]) / g.dzc[1:g.nz, None, None]
    ratio = gw[:, 0, 0] / t[1:g.nz, 0, 0]
    assert torch.allclose(ratio, ratio[0].expand_as(ratio), rtol=1e-12)


def test_cfl_brute_force():
    g = _grid(5, 4, 3)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3, 4, 5))
    v = rng.standard_normal((3, 4, 5))
    w = rng.standard_normal((4, 4, 5))
    dz = g.dz.numpy()
    best = 1e-8
    for k in range(3):
        for j in range(4):
            for i in range(5):
                q = (abs(w[k, j, i] + w[k + 1, j, i]) / dz[k]
                     + abs(v[k, j, i] + v[k, (j + 1) % 4, i]) / g.dy
                     + abs(u[k, j, i] + u[k, j, (i + 1) % 5]) / g.dx)
                best = max(best, 0.5 * q)
    got = ss.cfl(torch.tensor(u), torch.tensor(v), torch.tensor(w), g)
    assert abs(got - best) <= 1e-15 * best
