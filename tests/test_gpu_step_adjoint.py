"""Differentiating whole substeps and whole RK3 steps (Sec. 2.1: three substeps per step).

Substeps 2 and 3 read the previous substep's explicit terms H^{l-1} (their rho term), and
every substep's H feeds the next one, so the adjoint of substep l takes the cotangent of its
own H and returns that of H^{l-1}.  Checked against the oracle's autograd through the same
substeps, and the step adjoint against autograd through the oracle's full step and against
central differences of the library's own step.
"""
import numpy as np
import pytest
import torch

from oracle import substep as ss
from oracle import timestep as ts
from paper_1705_01423_amd.api import StepFn, SubstepFn
from gpu_util import banner, grids, rel

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _rb(plan, seed, unoise=0.1):
    from paper_1705_01423_amd import synth
    cfg = synth.small("rb", plan.nx, plan.ny, plan.nz, 1.0, 1.0, 3.0, seed)
    u, v, w, t, p = synth.rb_state(cfg, tnoise=1e-2, unoise=unoise)
    p = p + 1e-2 * np.random.default_rng(seed).standard_normal(p.shape)
    return [torch.as_tensor(a) for a in (u, v, w, t, p)]


def _cot(shapes, rng, face_idx=(2, 3)):
    out = [torch.as_tensor(rng.standard_normal(s)) for s in shapes]
    for i in face_idx:
        if i < len(out):
            out[i][0] = 0
            out[i][-1] = 0
    return out


def _cuda(xs):
    return [x.clone().to("cuda") for x in xs]


def _interior(name, a, b):
    return (a[1:-1], b[1:-1]) if name in "wT" else (a, b)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_substep_adjoint_with_h(l):
    """VJP of (state, H^{l-1}) -> (state', H^l) for every substep index."""
    banner(f"substep adjoint l={l} with H cotangents")
    g, plan = grids(12, 12, 8, precision="fp64")
    state = _rb(plan, 31 + l)
    dt, nu, ka = 2e-2, 1e-2, 8e-3
    rng = np.random.default_rng(40 + l)
    shapes = [x.shape for x in state]
    hprev = _cot(shapes[:4], rng)
    cot = _cot(shapes, rng)
    cot_h = _cot(shapes[:4], rng)
    xs = [a.clone().requires_grad_(True) for a in state]
    hs = [a.clone().requires_grad_(True) for a in hprev]
    out, h = ss.substep(xs, g, l, dt, nu, ka, hprev=hs if l > 1 else None, differentiable=True)
    loss = sum((a * b).sum() for a, b in zip(out, cot)) + sum((a * b).sum() for a, b in zip(h, cot_h))
    grads = torch.autograd.grad(loss, xs + hs, allow_unused=True)
    ref_in, ref_hp = grads[:5], grads[5:]
    g_in, g_hp = plan.substep_adjoint(dt, nu, ka, *_cuda(state), _cuda(cot), l=l, g_hout=_cuda(cot_h),
                                      want_hprev=True)
    for name, a, b in zip("uvwTp", g_in, ref_in):
        a, b = _interior(name, a, b)
        assert rel(a, b) < 1e-11, name
    for name, a, b in zip("uvwT", g_hp, ref_hp):
        if l == 1:
            assert float(a.abs().max()) == 0.0, name
        else:
            a, b = _interior(name, a, b)
            assert rel(a, b) < 1e-12, name


def test_substep_adjoint_hout_shares_hprev():
    """g_hprev may be the g_hout buffers (the step adjoint hands H cotangents down in place)."""
    banner("substep adjoint in-place H cotangent")
    g, plan = grids(12, 12, 8, precision="fp64")
    state = _cuda(_rb(plan, 51))
    rng = np.random.default_rng(52)
    cot = _cuda(_cot([x.shape for x in state], rng))
    ch = _cuda(_cot([x.shape for x in state[:4]], rng))
    ref_in, ref_hp = plan.substep_adjoint(2e-2, 1e-2, 8e-3, *state, cot, l=2, g_hout=ch, want_hprev=True)
    import ctypes
    from paper_1705_01423_amd.api import _ptr, _stream
    shared = [x.clone() for x in ch]
    g_in = [torch.empty_like(x) for x in state]
    P = ctypes.c_void_p
    go = (P * 5)(*[x.data_ptr() for x in cot])
    gh = (P * 4)(*[x.data_ptr() for x in shared])
    gi = (P * 5)(*[x.data_ptr() for x in g_in])
    assert plan._lib.rk3_substep_adjoint(plan._h, 2, 2e-2, 1e-2, 8e-3, *[_ptr(x, "s") for x in state], go, gh, gi,
                                         gh, _stream(), None) == 0
    for a, b in zip(g_in, ref_in):
        assert torch.equal(a, b)
    for a, b in zip(shared, ref_hp):
        assert torch.equal(a, b)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32_refined", 1e-10)])
def test_step_adjoint_vs_autograd(prec, tol):
    banner(f"step adjoint {prec}")
    g, plan = grids(12, 12, 8, precision=prec)
    state = _rb(plan, 61)
    dt, nu, ka = 2e-2, 1e-2, 8e-3
    rng = np.random.default_rng(62)
    cot = _cot([x.shape for x in state], rng)
    xs = [a.clone().requires_grad_(True) for a in state]
    out = ts.rk3_step(xs, g, dt, nu, ka, differentiable=True)
    loss = sum((a * b).sum() for a, b in zip(out, cot))
    ref = torch.autograd.grad(loss, xs)
    got = plan.step_adjoint(dt, nu, ka, *_cuda(state), _cuda(cot))
    for name, a, b in zip("uvwTp", got, ref):
        a, b = _interior(name, a, b)
        assert rel(a, b) < tol, name


@pytest.mark.parametrize("shape", [(16, 6, 5), (6, 4, 3)])
def test_step_adjoint_shapes(shape):
    banner(f"step adjoint shape {shape}")
    g, plan = grids(*shape, precision="fp64")
    state = _rb(plan, 71)
    dt, nu, ka = 1e-2, 1e-2, 8e-3
    cot = _cot([x.shape for x in state], np.random.default_rng(72))
    xs = [a.clone().requires_grad_(True) for a in state]
    out = ts.rk3_step(xs, g, dt, nu, ka, differentiable=True)
    ref = torch.autograd.grad(sum((a * b).sum() for a, b in zip(out, cot)), xs)
    got = plan.step_adjoint(dt, nu, ka, *_cuda(state), _cuda(cot))
    for name, a, b in zip("uvwTp", got, ref):
        a, b = _interior(name, a, b)
        assert rel(a, b) < 1e-11, name


def _dzz_max(zf):
    """Largest off-diagonal row sum of the wall-normal second difference (centre and face rows)."""
    zf = np.asarray(zf)
    dz = np.diff(zf)
    nz = dz.size
    dzc = 0.5 * (dz[:-1] + dz[1:])
    dzw = np.concatenate([[dz[0] / 2], dzc, [dz[-1] / 2]])
    centre = max(1 / (dzw[k] * dz[k]) + 1 / (dzw[k + 1] * dz[k]) for k in range(nz))
    face = max(1 / (dz[k - 1] * dzc[k - 1]) + 1 / (dz[k] * dzc[k - 1]) for k in range(1, nz))
    return max(centre, face)


def test_step_adjoint_stiff_wall_normal():
    """Wall-normal diffusion stiff enough that every substep's Crank-Nicolson solve takes the
    increment form q + C^-1 rhs (beta max Dzz above 256), so that the forward recomputation's
    substeps seed their output state from the input before the solve."""
    banner("step adjoint stiff wall-normal diffusion")
    g, plan = grids(8, 6, 32, precision="fp64")
    dt, nu, ka = 2e-2, 0.2, 0.16
    dzz = _dzz_max(g.zf)
    alphas = (8 / 15, 2 / 15, 1 / 3)   # gamma_l + rho_l of the three substeps
    assert min(alphas) * dt * min(nu, ka) / 2 * dzz > 256
    state = _rb(plan, 81)
    cot = _cot([x.shape for x in state], np.random.default_rng(82))
    xs = [a.clone().requires_grad_(True) for a in state]
    out = ts.rk3_step(xs, g, dt, nu, ka, differentiable=True)
    ref = torch.autograd.grad(sum((a * b).sum() for a, b in zip(out, cot)), xs)
    got = plan.step_adjoint(dt, nu, ka, *_cuda(state), _cuda(cot))
    for name, a, b in zip("uvwTp", got, ref):
        a, b = _interior(name, a, b)
        print(f"stiff step adjoint {name}: rel {rel(a, b):.3e}", flush=True)
        assert rel(a, b) < 1e-10, name


def test_step_fn_and_substep_fn_finite_difference():
    """StepFn / SubstepFn backward (the hand-written adjoints) against central differences
    of the library's forward step; the map is smooth (quadratic advection), so h = 1e-4
    leaves an O(h^2) truncation far below the tolerance."""
    banner("StepFn / SubstepFn FD")
    g, plan = grids(16, 12, 10, precision="fp64")
    state = _cuda(_rb(plan, 81))
    dt, nu, ka = 2e-2, 1e-2, 8e-3
    rng = np.random.default_rng(82)
    om = _cuda(_cot([x.shape for x in state], rng))
    for fn in (SubstepFn, StepFn):
        def loss(xs):
            out = fn.apply(*xs, plan, dt, nu, ka)
            return sum((a * b).sum() for a, b in zip(out, om))
        xs = [x.clone().requires_grad_(True) for x in state]
        grads = torch.autograd.grad(loss(xs), xs)
        for trial in range(3):
            d = _cuda(_cot([x.shape for x in state], rng))
            h = 1e-4
            with torch.no_grad():
                lp = float(loss([a + h * b for a, b in zip(state, d)]))
                lm = float(loss([a - h * b for a, b in zip(state, d)]))
            fd = (lp - lm) / (2 * h)
            an = float(sum((gr * di).sum() for gr, di in zip(grads, d)))
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fn.__name__, fd, an)
