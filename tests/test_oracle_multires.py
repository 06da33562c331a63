"""Pins of the multiple-resolution temperature grid oracle (paper Sec. 6; reading in
oracle/multires.py).  CPU only."""
import math

import numpy as np
import pytest
import torch

from oracle import Grid, operators as op, poisson
from oracle import multires as mr
from oracle import substep as ss
from paper_1705_01423_amd import synth

F64 = torch.float64


def _grid(nx, ny, nz, lx=1.0, ly=1.0, alpha=3.0):
    return Grid(nx, ny, nz, lx, ly, synth.zfaces(nz, alpha))


def _projected(g, seed=3):
    cfg = synth.small("t", g.nx, g.ny, g.nz, g.lx, g.ly, 3.0, seed)
    u, v, w = (torch.as_tensor(a) for a in synth.mode_velocity(cfg))
    un, vn, wn, _, _ = poisson.project(u, v, w, torch.zeros_like(u), g)
    return un, vn, wn


def test_unit_factors_are_the_identity():
    g = _grid(12, 8, 6)
    u, v, w = _projected(g)
    assert np.array_equal(mr.fine_faces(g.zf.numpy(), 1), g.zf.numpy())
    for a, b in zip(mr.prolong_velocity(u, v, w, g, 1, 1, 1), (u, v, w)):
        assert torch.equal(a, b)
    t = torch.as_tensor(np.random.default_rng(1).standard_normal((7, 8, 12)))
    assert torch.equal(mr.restrict_temperature(t, g, 1, 1, 1), t)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_temperature_substep_is_the_single_grid_one(l):
    """On the momentum grid itself, the temperature substep with the substep's input velocity
    reproduces the temperature output (and its H) of the full single-grid substep."""
    g = _grid(12, 8, 6)
    rng = np.random.default_rng(10 + l)
    u, v, w = _projected(g, seed=4)
    t = torch.as_tensor(rng.standard_normal((7, 8, 12)))
    t[0], t[-1] = 1.0, 0.0
    p = torch.as_tensor(rng.standard_normal((6, 8, 12)))
    hprev = [torch.as_tensor(rng.standard_normal(x.shape)) for x in (u, v, w, t)]
    for h in hprev[2:]:
        h[0] = 0
        h[-1] = 0
    dt, nu, ka = 0.03, 0.02, 0.015
    out, h = ss.substep((u, v, w, t, p), g, l, dt, nu, ka, hprev=hprev)
    tn, ht = mr.t_substep(t, (u, v, w), g, l, dt, ka, hprev[3])
    assert float((tn - out[3]).abs().max()) <= 1e-15 * float(out[3].abs().max())
    assert float((ht - h[3]).abs().max()) <= 1e-15 * float(h[3].abs().max())


@pytest.mark.parametrize("r", [(2, 2, 2), (2, 1, 3), (3, 2, 1), (1, 1, 2)])
def test_prolonged_velocity_is_divergence_free(r):
    g = _grid(12, 8, 6, 1.5, 1.0)
    u, v, w = _projected(g)
    d0 = float(op.divergence(u, v, w, g).abs().max())
    uf, vf, wf = mr.prolong_velocity(u, v, w, g, *r)
    gf = mr.fine_grid(g, *r)
    scale = float(uf.abs().max()) / min(gf.dx, gf.dy, float(gf.dz.min()))
    assert d0 < 1e-13 * scale
    assert float(op.divergence(uf, vf, wf, gf).abs().max()) < 1e-13 * scale
    # wall faces stay closed
    assert float(wf[0].abs().max()) == 0.0 and float(wf[-1].abs().max()) == 0.0


@pytest.mark.parametrize("r", [(2, 2, 2), (3, 1, 2)])
def test_coarse_face_fluxes_are_kept(r):
    """The fine sub-faces of every coarse face carry, on average, the coarse face value."""
    rx, ry, rz = r
    g = _grid(12, 8, 6)
    u, v, w = _projected(g)
    uf, vf, wf = mr.prolong_velocity(u, v, w, g, rx, ry, rz)
    for k in range(g.nz):
        # x-faces i: mean over the ry rz sub-faces with equal areas
        blk = uf[k * rz:(k + 1) * rz, :, ::rx].reshape(rz, g.ny, ry, g.nx).mean(dim=(0, 2))
        assert float((blk - u[k]).abs().max()) < 1e-14 * float(u.abs().max())
        blk = vf[k * rz:(k + 1) * rz, ::ry, :].reshape(rz, g.ny, g.nx, rx).mean(dim=(0, 3))
        assert float((blk - v[k]).abs().max()) < 1e-14 * float(v.abs().max())
    blk = wf[::rz].reshape(g.nz + 1, g.ny, ry, g.nx, rx).mean(dim=(2, 4))
    assert float((blk - w).abs().max()) < 1e-14 * float(w.abs().max())


def _analytic_velocity(lx, ly):
    """A smooth divergence-free field vanishing at the walls z = 0, 1: the curl of
    (A1, A2, 0) with A1 = cos(kx x) cos(ky y) s, A2 = -sin(kx x) cos(ky y) s, s = sin^2(pi z),
    so that u = -dA2/dz, v = dA1/dz, w = dA2/dx - dA1/dy."""
    kx, ky = 2 * math.pi / lx, 2 * math.pi / ly

    def uu(x, y, z):
        return torch.sin(kx * x) * torch.cos(ky * y) * math.pi * torch.sin(2 * math.pi * z)

    def vv(x, y, z):
        return torch.cos(kx * x) * torch.cos(ky * y) * math.pi * torch.sin(2 * math.pi * z)

    def ww(x, y, z):
        s2 = torch.sin(math.pi * z) ** 2
        return (-kx * torch.cos(kx * x) * torch.cos(ky * y) + ky * torch.cos(kx * x) * torch.sin(ky * y)) * s2

    return uu, vv, ww


def _sample_faces(g, fns):
    uu, vv, ww = fns
    xi = torch.arange(g.nx, dtype=F64) * g.dx
    xc = xi + 0.5 * g.dx
    yj = torch.arange(g.ny, dtype=F64) * g.dy
    yc = yj + 0.5 * g.dy
    zc, zf = g.zc, g.zf
    u = uu(xi[None, None, :], yc[None, :, None], zc[:, None, None])
    v = vv(xc[None, None, :], yj[None, :, None], zc[:, None, None])
    w = ww(xc[None, None, :], yc[None, :, None], zf[:, None, None])
    return u, v, w


@pytest.mark.parametrize("alpha", [0.0, 1.5])
@pytest.mark.parametrize("r", [(2, 2, 2), (3, 2, 3)])
def test_prolongation_second_order(alpha, r):
    lx, ly = 1.0, 1.5
    fns = _analytic_velocity(lx, ly)
    errs = []
    for n in (8, 16, 32):
        g = _grid(n, n, n, lx, ly, alpha)
        u, v, w = _sample_faces(g, fns)
        got = mr.prolong_velocity(u, v, w, g, *r)
        exact = _sample_faces(mr.fine_grid(g, *r), fns)
        errs.append(max(float((a - b).abs().max()) for a, b in zip(got, exact)))
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.3 < q < 5.0 for q in rates), (errs, rates)


def test_restriction_keeps_plane_means_and_converges():
    rx, ry, rz = 2, 3, 2
    g = _grid(8, 6, 5)
    tf = torch.as_tensor(np.random.default_rng(2).standard_normal((5 * rz + 1, 6 * ry, 8 * rx)))
    tc = mr.restrict_temperature(tf, g, rx, ry, rz)
    for k in range(g.nz + 1):
        assert abs(float(tc[k].mean()) - float(tf[k * rz].mean())) < 1e-15
    # the column means the momentum equations see: second-order accurate for a smooth T
    errs = []
    for n in (8, 16, 32):
        g = _grid(n, n, n, 1.0, 1.0, 1.5)
        gf = mr.fine_grid(g, rx, ry, rz)

        def temp(gg):
            x = (torch.arange(gg.nx, dtype=F64) + 0.5) * gg.dx
            y = (torch.arange(gg.ny, dtype=F64) + 0.5) * gg.dy
            return (torch.cos(2 * math.pi * x)[None, None, :] * torch.sin(2 * math.pi * y)[None, :, None]
                    * (1 - gg.zf)[:, None, None])
        errs.append(float((mr.restrict_temperature(temp(gf), g, rx, ry, rz) - temp(g)).abs().max()))
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < q < 4.5 for q in rates), (errs, rates)


def _fine_setup(r=(2, 2, 2), n=(8, 6, 4), seed=5):
    g = _grid(*n, 1.0, 1.0)
    gf = mr.fine_grid(g, *r)
    vel0 = mr.prolong_velocity(*_projected(g, seed), g, *r)
    vel1 = mr.prolong_velocity(*_projected(g, seed + 1), g, *r)
    return g, gf, vel0, vel1


def test_uniform_temperature_stays_uniform():
    """Every temperature control volume's transporting fluxes are divergence free."""
    g, gf, vel0, vel1 = _fine_setup()
    t = torch.full((gf.nz + 1, gf.ny, gf.nx), 0.75, dtype=F64)
    tn = mr.temperature_step(t, vel0, vel1, gf, 0.01, 0.003, 3)
    assert float((tn - 0.75).abs().max()) < 1e-14


def test_temperature_step_third_order_in_substep():
    """kappa = 0, velocity varying linearly in time across the step: the stage velocities are
    exact at the stage start times, so the error of the temperature step falls as dt_T^3."""
    g, gf, vel0, vel1 = _fine_setup()
    x = (torch.arange(gf.nx, dtype=F64) + 0.5) * gf.dx
    y = (torch.arange(gf.ny, dtype=F64) + 0.5) * gf.dy
    t0 = (1 - gf.zf)[:, None, None] + 0.1 * (torch.sin(2 * math.pi * x)[None, None, :]
                                           * torch.cos(2 * math.pi * y)[None, :, None]
                                           * torch.sin(math.pi * gf.zf)[:, None, None])
    dt = 0.4 / float(max(a.abs().max() for a in vel0 + vel1)) * gf.dx
    ref = mr.temperature_step(t0, vel0, vel1, gf, dt, 0.0, 64)
    errs = [float((mr.temperature_step(t0, vel0, vel1, gf, dt, 0.0, n) - ref).abs().max()) for n in (2, 4, 8)]
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(6.5 < q < 9.5 for q in rates), (errs, rates)


def test_coupled_step_keeps_the_conduction_state():
    """Rest with the linear conduction profile on the temperature grid: buoyancy is a pure
    wall-normal gradient (taken up by the pressure) and the profile is steady."""
    rx, ry, rz = 2, 2, 2
    g = _grid(8, 6, 5)
    gf = mr.fine_grid(g, rx, ry, rz)
    z = torch.zeros(5, 6, 8, dtype=F64)
    state = (z.clone(), z.clone(), torch.zeros(6, 6, 8, dtype=F64), z.clone())
    tf = (1 - gf.zf)[:, None, None].expand(gf.nz + 1, gf.ny, gf.nx).clone()
    (u, v, w, p), tn = mr.step_mr(state, tf, g, rx, ry, rz, 0.05, 0.01, 0.01, 2)
    assert max(float(a.abs().max()) for a in (u, v, w)) < 1e-13
    assert float((tn - tf).abs().max()) < 1e-14
