"""GPU parity of projection, CN solves, CFL, adjoints and the RK3 substep against the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import cn, operators as op, poisson
from oracle import substep as ss
from paper_1705_01423_amd import synth
from paper_1705_01423_amd.api import ProjectFn
from gpu_util import banner, grids, rel

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _modes(nx, ny, nz, lx, ly, seed=3):
    cfg = synth.small("t", nx, ny, nz, lx, ly, 3.0, seed)
    return [torch.as_tensor(a) for a in synth.mode_velocity(cfg)]


def _cuda(*ts):
    return [t.clone().to("cuda") for t in ts]


@pytest.mark.parametrize("s,c", [(1.0, 0.0), (0.3, 0.012)])
def test_project_parity(s, c):
    banner(f"project s={s} c={c}")
    g, plan = grids(48, 32, 24, 2.0, 2.0)
    u, v, w = _modes(48, 32, 24, 2.0, 2.0)
    p = torch.as_tensor(np.random.default_rng(1).standard_normal(plan.centre_shape))
    ref = poisson.project(u, v, w, p, g, s, c)
    ud, vd, wd, pd = _cuda(u, v, w, p)
    phi = torch.empty_like(pd)
    plan.project(ud, vd, wd, pd, phi, s, c)
    for a, b in zip((ud, vd, wd, pd, phi), ref):
        assert rel(a, b) < 1e-12
    d0 = float(op.divergence(u, v, w, g).abs().max())
    d1 = float(op.divergence(ud.cpu(), vd.cpu(), wd.cpu(), g).abs().max())
    assert d1 < 1e-12 * d0


@pytest.mark.parametrize("shape", [(48, 32, 24), (24, 6, 10), (96, 24, 40)])
def test_project_fused_divergence(shape):
    """FP64 projections form D u*/s inside the x transform; with the finiteness check the
    divergence is stored first by its own kernel.  Same arithmetic, so bitwise-equal results
    (blocks walk y tiles then z when ny allows, plain row order otherwise)."""
    nx, ny, nz = shape
    banner(f"project fused divergence {shape}")
    g, fused = grids(nx, ny, nz, 2.0, 2.0)
    _, stored = grids(nx, ny, nz, 2.0, 2.0, flags=2)   # PS_FLAG_CHECK_FINITE
    u, v, w = _modes(nx, ny, nz, 2.0, 2.0)
    p = torch.as_tensor(np.random.default_rng(4).standard_normal(fused.centre_shape))
    out = []
    for plan in (fused, stored):
        ud, vd, wd, pd = _cuda(u, v, w, p)
        phi = torch.empty_like(pd)
        plan.project(ud, vd, wd, pd, phi, 0.7, 0.01)
        out.append((ud, vd, wd, pd, phi))
    for a, b in zip(*out):
        assert torch.equal(a, b)
    ref = poisson.project(u, v, w, p, g, 0.7, 0.01)
    for a, b in zip(out[0], ref):
        assert rel(a, b) < 1e-12


def test_project_refined():
    banner("project fp32_refined")
    g, plan = grids(64, 48, 40, 2.0, 2.0, precision="fp32_refined")
    u, v, w = _modes(64, 48, 40, 2.0, 2.0)
    z = torch.zeros(plan.centre_shape, dtype=F64)
    ref = poisson.project(u, v, w, z, g)
    ud, vd, wd = _cuda(u, v, w)
    info = plan.project(ud, vd, wd)
    for a, b in zip((ud, vd, wd), ref):
        assert rel(a, b) < 1e-11, info


@pytest.mark.parametrize("nz", [2, 3, 33, 64, 65, 200, 512, 513, 600])
@pytest.mark.parametrize("kind", [0, 1])
def test_cn_solve(kind, nz):
    """Tiled solve (up to 16 waves of at most 32 rows) and the lane-per-column sweep beyond."""
    banner(f"cn kind={kind} nz={nz}")
    g, plan = grids(24, 16, nz)
    shape = plan.centre_shape if kind == 0 else plan.face_shape
    rhs = torch.as_tensor(np.random.default_rng(2).standard_normal(shape))
    beta = 2.5e-4
    ref = cn.solve_centre(rhs, g, beta) if kind == 0 else cn.solve_face(rhs, g, beta)
    x = rhs.clone().to("cuda")
    plan.cn_solve(kind, beta, x)
    assert rel(x, ref) < 1e-13


def test_cfl():
    g, plan = grids(24, 12, 9)
    rng = np.random.default_rng(4)
    u = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    v = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    w = torch.as_tensor(rng.standard_normal(plan.face_shape))
    ref = ss.cfl(u, v, w, g)
    got = float(plan.cfl(*_cuda(u, v, w)).item())
    assert abs(got - ref) <= 2e-16 * ref


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_refined", 1e-11), ("fp32", 1e-5)])
def test_solve_adjoint_vs_autograd(prec, tol):
    """S^T = Vc S Vc^-1 at every precision: the output scaling Vc must follow the refinement."""
    banner(f"solve adjoint {prec}")
    g, plan = grids(24, 24, 18, 1.5, 1.0, precision=prec)
    rng = np.random.default_rng(5)
    f = torch.as_tensor(rng.standard_normal(plan.centre_shape)).requires_grad_(True)
    gphi = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    (ref,) = torch.autograd.grad(poisson.solve_autograd(f, g), f, gphi)
    got, _ = plan.solve_adjoint(gphi.to("cuda"))
    assert rel(got, ref) < tol


def test_solve_fn_backward_refined():
    """PoissonSolveFn on an FP32-refined plan: forward and backward both to the refined tolerance."""
    from paper_1705_01423_amd.api import PoissonSolveFn
    banner("PoissonSolveFn fp32_refined")
    g, plan = grids(32, 24, 20, 2.0, 1.0, precision="fp32_refined")
    rng = np.random.default_rng(15)
    f = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    gphi = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    fr = f.clone().requires_grad_(True)
    phi_ref = poisson.solve_autograd(fr, g)
    (ref,) = torch.autograd.grad(phi_ref, fr, gphi)
    fd = f.to("cuda").requires_grad_(True)
    phi = PoissonSolveFn.apply(fd, plan)
    assert rel(phi, phi_ref) < 1e-11
    (got,) = torch.autograd.grad(phi, fd, gphi.to("cuda"))
    assert rel(got, ref) < 1e-11


def _project_vjp(g, u, v, w, p, s, c, gu, gv, gw, gp):
    x = [a.clone().requires_grad_(True) for a in (u, v, w)]
    un, vn, wn, pn, _ = poisson.project(x[0], x[1], x[2], p, g, s, c, differentiable=True)
    loss = (un * gu).sum() + (vn * gv).sum() + (wn * gw).sum() + (pn * gp).sum()
    return torch.autograd.grad(loss, x)


@pytest.mark.parametrize("with_p", [False, True])
def test_project_adjoint_vs_autograd(with_p):
    banner(f"project adjoint with_p={with_p}")
    g, plan = grids(24, 16, 20, 2.0, 2.0)
    u, v, w = _modes(24, 16, 20, 2.0, 2.0)
    rng = np.random.default_rng(6)
    p = torch.zeros(plan.centre_shape, dtype=F64)
    gu = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    gv = torch.as_tensor(rng.standard_normal(plan.centre_shape))
    gw = torch.as_tensor(rng.standard_normal(plan.face_shape))
    gw[0] = 0
    gw[-1] = 0
    gp = torch.as_tensor(rng.standard_normal(plan.centre_shape)) if with_p else torch.zeros_like(p)
    s, c = (0.4, 0.02) if with_p else (1.0, 0.0)
    ru, rv, rw = _project_vjp(g, u, v, w, p, s, c, gu, gv, gw, gp)
    du, dv, dw = plan.project_adjoint(*_cuda(gu, gv, gw), gp.to("cuda") if with_p else None, s, c)
    assert rel(du, ru) < 1e-12 and rel(dv, rv) < 1e-12
    assert rel(dw[1:-1], rw[1:-1]) < 1e-12
    assert float(dw[0].abs().max()) == 0.0 and float(dw[-1].abs().max()) == 0.0


@pytest.mark.parametrize("shape", [(48, 32, 24), (24, 6, 10), (96, 24, 40)])
@pytest.mark.parametrize("with_p", [False, True])
def test_project_adjoint_fused_rhs(shape, with_p):
    """FP64 projection adjoints form the solve's right-hand side inside the x transform; with
    the finiteness check it is stored first by its own kernel (the same formula; the two
    compilations may contract it into FMAs differently).  Both match the oracle's VJP, and
    each other to the rounding of the right-hand side amplified by the solve (1e-13)."""
    nx, ny, nz = shape
    banner(f"project adjoint fused rhs {shape} with_p={with_p}")
    g, fused = grids(nx, ny, nz, 2.0, 2.0)
    _, stored = grids(nx, ny, nz, 2.0, 2.0, flags=2)   # PS_FLAG_CHECK_FINITE
    u, v, w = _modes(nx, ny, nz, 2.0, 2.0)
    rng = np.random.default_rng(11)
    gu = torch.as_tensor(rng.standard_normal(fused.centre_shape))
    gv = torch.as_tensor(rng.standard_normal(fused.centre_shape))
    gw = torch.as_tensor(rng.standard_normal(fused.face_shape))
    gw[0] = 0
    gw[-1] = 0
    p = torch.zeros(fused.centre_shape, dtype=F64)
    gp = torch.as_tensor(rng.standard_normal(fused.centre_shape)) if with_p else torch.zeros_like(p)
    s, c = (0.4, 0.02) if with_p else (1.0, 0.0)
    ref = _project_vjp(g, u, v, w, p, s, c, gu, gv, gw, gp)
    outs = [plan.project_adjoint(*_cuda(gu, gv, gw), gp.to("cuda") if with_p else None, s, c)
            for plan in (fused, stored)]
    for a, b in zip(*outs):
        assert rel(a, b) < 1e-13
    du, dv, dw = outs[0]
    assert rel(du, ref[0]) < 1e-12 and rel(dv, ref[1]) < 1e-12
    assert rel(dw[1:-1], ref[2][1:-1]) < 1e-12


def test_project_autograd_finite_difference():
    """ProjectFn backward (hand-written adjoint) vs central differences, h = 1e-6."""
    banner("project FD")
    g, plan = grids(32, 32, 24, 2.0, 2.0)
    u, v, w = _cuda(*_modes(32, 32, 24, 2.0, 2.0))
    rng = np.random.default_rng(7)
    om = [torch.as_tensor(rng.standard_normal(t.shape)).to("cuda") for t in (u, v, w)]
    om[2][0] = 0
    om[2][-1] = 0

    def loss(a, b, c):
        pu, pv, pw = ProjectFn.apply(a, b, c, plan)
        return (pu * om[0]).sum() + (pv * om[1]).sum() + (pw * om[2]).sum()

    xs = [t.clone().requires_grad_(True) for t in (u, v, w)]
    grads = torch.autograd.grad(loss(*xs), xs)
    for trial in range(4):
        d = [torch.as_tensor(rng.standard_normal(t.shape)).to("cuda") for t in (u, v, w)]
        d[2][0] = 0
        d[2][-1] = 0
        h = 1e-6
        with torch.no_grad():
            lp = loss(*[a + h * b for a, b in zip((u, v, w), d)])
            lm = loss(*[a - h * b for a, b in zip((u, v, w), d)])
        fd = float((lp - lm) / (2 * h))
        an = float(sum((gr * di).sum() for gr, di in zip(grads, d)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def _rb(nx, ny, nz, seed=9, unoise=0.05):
    cfg = synth.small("rb", nx, ny, nz, 1.0, 1.0, 3.0, seed)
    u, v, w, t, p = synth.rb_state(cfg, tnoise=1e-2, unoise=unoise)
    p = p + 1e-2 * np.random.default_rng(seed).standard_normal(p.shape)
    return [torch.as_tensor(a) for a in (u, v, w, t, p)]


@pytest.mark.parametrize("l", [1, 2])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_refined", 1e-10)])
def test_substep_parity(l, prec, tol):
    banner(f"substep l={l} {prec}")
    g, plan = grids(16, 12, 10, precision=prec)
    state = _rb(16, 12, 10)
    dt, nu, ka = 3e-2, 2e-2, 1.5e-2
    hprev = None
    if l > 1:
        rng = np.random.default_rng(11)
        hprev = [torch.as_tensor(rng.standard_normal(x.shape)) for x in state[:4]]
        for h in hprev[2:]:
            h[0] = 0
            h[-1] = 0
    ref_state, ref_h = ss.substep(state, g, l, dt, nu, ka, hprev)
    dstate = _cuda(*state)
    hout = [torch.empty_like(x) for x in dstate[:4]]
    plan.substep(l, dt, nu, ka, *dstate, h_prev=_cuda(*hprev) if hprev else None, h_out=hout)
    for name, a, b in zip("uvwTp", dstate, ref_state):
        assert rel(a, b) < tol, name
    for a, b in zip(hout, ref_h):
        assert rel(a, b) < 1e-13


@pytest.mark.parametrize("shape,dt", [((384, 12, 6), 2e-2), ((48, 24, 20), 2e-2), ((96, 6, 9), 2e-2),
                                      ((4, 2, 2), 2e-2), ((8, 3, 3), 2e-2), ((16, 4, 130), 2e-2),
                                      ((8, 4, 257), 2e-2), ((8, 2, 513), 2e-3), ((4, 2, 600), 2e-3)])
def test_substep_shapes(shape, dt):
    """Rows longer than one stencil block (ragged x segments) and ragged y tiles; column heights
    that take each row count per lane of the tiled Crank-Nicolson solve with a ragged last
    chunk (130, 257), and the lane-per-column solve beyond 512 rows (513, 600).  The short
    columns solve in the C q + rhs form, the tall ones (beta Dzz far from zero) add C^-1 rhs.
    The two tallest take a smaller step: at dt = 2e-2 their w reaches the projection's rounding
    floor on these fine wall cells (1e-12 against the oracle, the same with either form)."""
    nx, ny, nz = shape
    banner(f"substep shape {shape} dt={dt}")
    g, plan = grids(nx, ny, nz)
    state = _rb(nx, ny, nz, seed=21)
    nu, ka = 2e-2, 1.5e-2
    ref_state, ref_h = ss.substep(state, g, 1, dt, nu, ka)
    dstate = _cuda(*state)
    hout = [torch.empty_like(x) for x in dstate[:4]]
    plan.substep(1, dt, nu, ka, *dstate, h_out=hout)
    for name, a, b in zip("uvwTp", dstate, ref_state):
        assert rel(a, b) < 1e-12, name
    for a, b in zip(hout, ref_h):
        assert rel(a, b) < 1e-13


@pytest.mark.parametrize("shape", [(12, 12, 8), (384, 6, 5), (4, 2, 3), (16, 4, 130), (8, 2, 257), (4, 2, 513)])
def test_substep_adjoint_shapes(shape):
    nx, ny, nz = shape
    banner(f"substep adjoint shape {shape}")
    g, plan = grids(nx, ny, nz, precision="fp64")
    state = _rb(nx, ny, nz, seed=23, unoise=0.1)
    dt, nu, ka = 2e-2, 1e-2, 8e-3
    rng = np.random.default_rng(24)
    cot = [torch.as_tensor(rng.standard_normal(x.shape)) for x in state]
    for c in (cot[2], cot[3]):
        c[0] = 0
        c[-1] = 0
    xs = [a.clone().requires_grad_(True) for a in state]
    out, _ = ss.substep(xs, g, 1, dt, nu, ka, differentiable=True)
    loss = sum((a * b).sum() for a, b in zip(out, cot))
    ref = torch.autograd.grad(loss, xs)
    got = plan.substep_adjoint(dt, nu, ka, *_cuda(*state), _cuda(*cot))
    for name, a, b in zip("uvwTp", got, ref):
        if name in "wT":
            a, b = a[1:-1], b[1:-1]
        assert rel(a, b) < 1e-11, name


def test_substep_increment_parity():
    """The change of each field over one substep agrees with the oracle's (relative to the change)."""
    g, plan = grids(16, 12, 10)
    state = _rb(16, 12, 10)
    dt, nu, ka = 3e-2, 2e-2, 1.5e-2
    ref_state, _ = ss.substep(state, g, 1, dt, nu, ka)
    dstate = _cuda(*state)
    plan.substep(1, dt, nu, ka, *dstate)
    for a, b, x0 in zip(dstate, ref_state, state):
        if float((b - x0).norm()) > 0:
            assert rel(a.cpu() - x0, b - x0) < 1e-11


def test_substep_adjoint_vs_autograd():
    banner("substep adjoint")
    g, plan = grids(12, 12, 8, precision="fp64")
    state = _rb(12, 12, 8, seed=13, unoise=0.1)
    dt, nu, ka = 2e-2, 1e-2, 8e-3
    rng = np.random.default_rng(14)
    cot = [torch.as_tensor(rng.standard_normal(x.shape)) for x in state]
    for c in (cot[2], cot[3]):
        c[0] = 0
        c[-1] = 0
    xs = [a.clone().requires_grad_(True) for a in state]
    out, _ = ss.substep(xs, g, 1, dt, nu, ka, differentiable=True)
    loss = sum((a * b).sum() for a, b in zip(out, cot))
    ref = torch.autograd.grad(loss, xs)
    got = plan.substep_adjoint(dt, nu, ka, *_cuda(*state), _cuda(*cot))
    for name, a, b in zip("uvwTp", got, ref):
        if name in "wT":
            a, b = a[1:-1], b[1:-1]
        assert rel(a, b) < 1e-11, name
