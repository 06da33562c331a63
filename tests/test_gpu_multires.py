"""GPU parity of the multiple-resolution temperature grid (Sec. 6) against the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import Grid, operators as op, poisson
from oracle import multires as mr
from paper_1705_01423_amd import synth
from paper_1705_01423_amd.api import MultiRes, Plan
from gpu_util import banner, rel

pytestmark = pytest.mark.gpu
F64 = torch.float64
FACTORS = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (2, 2, 1), (1, 1, 2), (2, 1, 2), (1, 2, 2), (2, 2, 2)]


def _setup(nx, ny, nz, r, nsub=1, lx=1.0, ly=1.0, alpha=3.0, prec="fp64"):
    zf = synth.zfaces(nz, alpha)
    g = Grid(nx, ny, nz, lx, ly, zf)
    plan = Plan(nx, ny, nz, lx, ly, zf, precision=prec)
    return g, plan, MultiRes(plan, *r, nsub=nsub)


def _projected(g, seed):
    cfg = synth.small("t", g.nx, g.ny, g.nz, g.lx, g.ly, 3.0, seed)
    u, v, w = (torch.as_tensor(a) for a in synth.mode_velocity(cfg))
    un, vn, wn, _, _ = poisson.project(u, v, w, torch.zeros_like(u), g)
    return un, vn, wn


def _cuda(xs):
    return [x.clone().to("cuda") for x in xs]


@pytest.mark.parametrize("r", FACTORS)
@pytest.mark.parametrize("shape", [(24, 12, 10), (24, 6, 5)])
def test_prolong_parity(r, shape):
    banner(f"mr prolong {r} {shape}")
    g, plan, m = _setup(*shape, r, lx=1.5)
    vel = _projected(g, 3)
    ref = mr.prolong_velocity(*vel, g, *r)
    got = m.prolong_velocity(*_cuda(vel))
    for name, a, b in zip("uvw", got, ref):
        assert rel(a, b) < 1e-13, name
        assert float((a.cpu() - b).abs().max()) <= 1e-13 * float(b.abs().max()), name
    gf = mr.fine_grid(g, *r)
    div = float(op.divergence(*[a.cpu() for a in got], gf).abs().max())
    scale = float(got[0].abs().max()) / min(gf.dx, gf.dy, float(gf.dz.min()))
    assert div < 1e-13 * scale


@pytest.mark.parametrize("r", [(2, 2, 2), (2, 1, 2), (1, 2, 1)])
def test_restrict_parity(r):
    g, plan, m = _setup(24, 12, 10, r)
    tf = torch.as_tensor(np.random.default_rng(4).standard_normal(m.face_shape))
    ref = mr.restrict_temperature(tf, g, *r)
    got = m.restrict_temperature(tf.to("cuda"))
    assert float((got.cpu() - ref).abs().max()) <= 1e-15 * float(ref.abs().max())


def _temperature(gf, seed):
    rng = np.random.default_rng(seed)
    t = (1 - gf.zf)[:, None, None] + 0.05 * torch.as_tensor(rng.standard_normal((gf.nz + 1, gf.ny, gf.nx)))
    t[0] = 1.0
    t[-1] = 0.0
    return t.contiguous()


@pytest.mark.parametrize("r,nsub", [((2, 2, 2), 2), ((2, 1, 2), 1), ((1, 1, 1), 3)])
def test_temperature_step_parity(r, nsub):
    banner(f"mr temperature step {r} nsub={nsub}")
    g, plan, m = _setup(16, 12, 10, r, nsub=nsub)
    gf = mr.fine_grid(g, *r)
    vel0 = mr.prolong_velocity(*_projected(g, 5), g, *r)
    vel1 = mr.prolong_velocity(*_projected(g, 6), g, *r)
    t = _temperature(gf, 7)
    dt, ka = 0.01, 0.02
    ref = mr.temperature_step(t, vel0, vel1, gf, dt, ka, nsub)
    td = t.clone().to("cuda")
    m.temperature_step(dt, ka, _cuda(vel0), _cuda(vel1), td)
    assert rel(td, ref) < 1e-13
    assert rel(td.cpu() - t, ref - t) < 1e-11      # the change itself


@pytest.mark.parametrize("r,nsub,shape", [((2, 2, 2), 2, (16, 12, 10)), ((2, 1, 2), 1, (24, 6, 5)),
                                          ((1, 1, 1), 1, (12, 8, 6))])
def test_coupled_step_parity(r, nsub, shape):
    banner(f"mr coupled step {r} nsub={nsub} {shape}")
    g, plan, m = _setup(*shape, r, nsub=nsub)
    gf = mr.fine_grid(g, *r)
    u, v, w = _projected(g, 8)
    rng = np.random.default_rng(9)
    p = torch.as_tensor(1e-2 * rng.standard_normal(u.shape))
    t = _temperature(gf, 10)
    dt, nu, ka = 0.02, 0.01, 0.008
    (ru, rv, rw, rp), rt = mr.step_mr((u, v, w, p), t, g, *r, dt, nu, ka, nsub)
    st = _cuda([u, v, w, p, t])
    m.step(nu, ka, *st, dt=dt)
    for name, a, b in zip("uvwp", st[:4], (ru, rv, rw, rp)):
        assert rel(a, b) < 1e-11, name
    assert rel(st[4], rt) < 1e-12
    assert rel(st[4].cpu() - t, rt - t) < 1e-10


def test_coupled_step_conduction_state():
    banner("mr conduction state")
    g, plan, m = _setup(16, 12, 8, (2, 2, 2), nsub=2)
    gf = mr.fine_grid(g, 2, 2, 2)
    z = torch.zeros(plan.centre_shape, dtype=F64, device="cuda")
    u, v, p = z.clone(), z.clone(), z.clone()
    w = torch.zeros(plan.face_shape, dtype=F64, device="cuda")
    tf = (1 - gf.zf)[:, None, None].expand(m.face_shape).contiguous().to("cuda")
    t0 = tf.clone()
    dt, _ = m.step(0.01, 0.01, u, v, w, p, tf, dt=0.05)
    assert max(float(a.abs().max()) for a in (u, v, w)) < 1e-13
    assert float((tf - t0).abs().max()) < 1e-14


def test_bad_factors_and_shapes():
    zf = synth.zfaces(8, 3.0)
    plan = Plan(16, 12, 8, 1.0, 1.0, zf)
    from paper_1705_01423_amd._lib import PsError
    for r in ((3, 1, 1), (1, 0, 1), (2, 2, 4)):
        with pytest.raises(PsError):
            MultiRes(plan, *r)
    with pytest.raises(PsError):
        MultiRes(plan, 2, 2, 2, nsub=0)
