"""GPU parity of the full RK3 step (three substeps, Courant-limited dt) and of the wall-normal
heat-flux statistics against the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import substep as ss
from oracle import timestep as ts
from paper_1705_01423_amd import synth
from gpu_util import banner, grids, rel

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _rb(nx, ny, nz, seed=31, unoise=0.05, lx=1.0, ly=1.0):
    cfg = synth.small("rb", nx, ny, nz, lx, ly, 3.0, seed)
    u, v, w, t, p = synth.rb_state(cfg, tnoise=1e-2, unoise=unoise)
    return [torch.as_tensor(a) for a in (u, v, w, t, p)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_refined", 1e-10)])
@pytest.mark.parametrize("shape", [(16, 12, 10), (96, 24, 20), (4, 2, 2)])
def test_step_parity(shape, prec, tol):
    nx, ny, nz = shape
    banner(f"rk3 step {shape} {prec}")
    g, plan = grids(nx, ny, nz, precision=prec)
    state = _rb(nx, ny, nz)
    dt, nu, ka = 2e-2, 2e-2, 1.5e-2
    ref = ts.rk3_step(state, g, dt, nu, ka)
    dstate = [a.clone().to("cuda") for a in state]
    used, info = plan.step(nu, ka, *dstate, dt=dt)
    assert used == dt
    for name, a, b in zip("uvwTp", dstate, ref):
        assert rel(a, b) < tol, name
    assert info["iterations"] >= 3


def test_step_courant_limited():
    """dt <= 0: the step takes min(dt_max, cfl / Courant number) of the input state."""
    nx, ny, nz = 24, 16, 12
    g, plan = grids(nx, ny, nz)
    state = _rb(nx, ny, nz, unoise=0.3)
    nu, ka = 1e-2, 1e-2
    dt = ts.cfl_dt(state[0], state[1], state[2], g, 1.3)
    ref = ts.rk3_step(state, g, dt, nu, ka)
    dstate = [a.clone().to("cuda") for a in state]
    used, _ = plan.step(nu, ka, *dstate, dt=0.0, cfl=1.3)
    assert abs(used - dt) <= 1e-15 * dt
    for name, a, b in zip("uvwTp", dstate, ref):
        assert rel(a, b) < 1e-12, name
    capped, _ = plan.step(nu, ka, *[a.clone().to("cuda") for a in state], dt=0.0, cfl=1.3, dt_max=1e-4)
    assert capped == 1e-4


def test_step_rk3_amplification():
    """The closed form of the oracle pin: a mode v = eps cos(theta x) carried by uniform u = U."""
    nx, ny, nz, lx = 16, 4, 6, 2.0
    g, plan = grids(nx, ny, nz, lx=lx)
    U, eps, m, dt = 0.7, 1e-3, 3, 0.05
    dx = lx / nx
    theta = 2 * math.pi * m / lx
    xc = (torch.arange(nx, dtype=F64) + 0.5) * dx
    t = (1 - g.zf)[:, None, None].expand(nz + 1, ny, nx).clone()
    u = torch.full((nz, ny, nx), U, dtype=F64)
    v = (eps * torch.cos(theta * xc))[None, None, :].expand(nz, ny, nx).clone()
    w = torch.zeros(nz + 1, ny, nx, dtype=F64)
    p = torch.zeros(nz, ny, nx, dtype=F64)
    d = [a.clone().to("cuda") for a in (u, v, w, t, p)]
    plan.step(0.0, 0.0, *d, dt=dt)
    z = -1j * U * math.sin(theta * dx) / dx * dt
    amp = 1 + z + z * z / 2 + z ** 3 / 6
    expect = eps * (amp * torch.exp(1j * theta * xc.to(torch.complex128))).real
    vn = d[1].cpu()
    assert float((vn - expect[None, None, :]).abs().max()) < 1e-15
    assert float((d[0].cpu() - U).abs().max()) < 1e-15
    assert float(d[2].abs().max()) < 1e-14


@pytest.mark.parametrize("shape", [(16, 12, 10), (96, 24, 33), (384, 6, 5)])
def test_heat_flux_parity(shape):
    nx, ny, nz = shape
    banner(f"heat flux {shape}")
    g, plan = grids(nx, ny, nz)
    _, _, w, t, _ = _rb(nx, ny, nz, unoise=0.2)
    kappa = 7e-3
    rt, rf = ts.heat_flux(w, t, g, kappa)
    mt, f = plan.heat_flux(w.to("cuda"), t.to("cuda"), kappa)
    assert float((mt.cpu() - rt).abs().max()) < 1e-14
    assert rel(f, rf) < 1e-12


def test_step_sequence():
    """Five Courant-limited steps in a row: the time step follows the evolving state."""
    nx, ny, nz = 24, 16, 12
    g, plan = grids(nx, ny, nz)
    state = _rb(nx, ny, nz, unoise=0.3, seed=41)
    nu, ka = 1e-2, 1e-2
    ref = list(state)
    dstate = [a.clone().to("cuda") for a in state]
    for n in range(5):
        dt = ts.cfl_dt(ref[0], ref[1], ref[2], g, 1.2)
        ref = list(ts.rk3_step(ref, g, dt, nu, ka))
        used, _ = plan.step(nu, ka, *dstate, dt=0.0, cfl=1.2)
        assert abs(used - dt) <= 1e-12 * dt, n
    for name, a, b in zip("uvwTp", dstate, ref):
        assert rel(a, b) < 1e-11, name


def test_heat_flux_conduction():
    nx, ny, nz = 32, 24, 40
    g, plan = grids(nx, ny, nz)
    t = (1 - g.zf)[:, None, None].expand(nz + 1, ny, nx).contiguous()
    w = torch.zeros(nz + 1, ny, nx, dtype=F64)
    kappa = 1e-4
    mt, f = plan.heat_flux(w.to("cuda"), t.to("cuda"), kappa)
    assert float((mt.cpu() - (1 - g.zf)).abs().max()) < 1e-15
    assert float((f.cpu() / kappa - 1.0).abs().max()) < 1e-12
