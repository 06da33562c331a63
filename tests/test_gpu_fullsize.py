"""GPU parity at the full sizes of the five workloads, in the launch configuration the
benchmark uses (same plans, same kernels).

The oracle finishes the 1024^2 x 512 solve and the 512^2 x 384 projection in seconds on
the host, so those are compared element by element.  The adjoints are checked against
central finite differences of the GPU forward map (a property that holds at any size),
the 8^3 sub-case against the oracle's dense Jacobian, and the 768^2 x 512 substep against
the oracle's substep.
"""
import math

import numpy as np
import pytest
import torch

from oracle import Grid, operators as op, poisson
from oracle import substep as ss
from paper_1705_01423_amd import synth
from paper_1705_01423_amd.api import Plan, ProjectFn
from gpu_util import banner, rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
F64 = torch.float64


def _setup(name, precision="fp64"):
    cfg = synth.CONFIGS[name]
    zf = synth.zfaces(cfg.nz, cfg.alpha)
    g = Grid(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf)
    return cfg, zf, g


@pytest.fixture(scope="module")
def couette():
    banner("couette inputs + oracle solve")
    cfg, zf, g = _setup("couette1024x1024x512")
    u, v, w = synth.mode_velocity(cfg)
    f = op.divergence(torch.as_tensor(u), torch.as_tensor(v), torch.as_tensor(w), g)
    del u, v, w
    ref, defect = poisson.solve(f, g, return_defect=True)
    return cfg, zf, g, f, ref, defect


@pytest.mark.timeout(900)
def test_couette_solve_fp64(couette):
    cfg, zf, g, f, ref, defect = couette
    banner("couette fp64 solve")
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    phi, info = plan.solve(f.to("cuda"))
    err = rel(phi, ref)
    print(f"couette fp64 rel-L2 {err:.3e}", flush=True)
    assert err < 1e-12
    assert abs(info["compat_defect"] - defect) < 1e-14
    # gauge: dz-weighted zero mean
    phc = phi.cpu()
    assert abs(op.weighted_sum(phc, g)) < 1e-12 * float(phi.abs().sum())
    # plane by plane (a wall row or a single plane's error would hide in the whole-field norm)
    # and the singular (0, 0) mode alone (the plane means)
    amax = float(ref.abs().max())
    plane_err = (phc - ref).abs().amax(dim=(1, 2))
    print(f"couette fp64 worst plane max-error {float(plane_err.max()):.3e} (max|phi| {amax:.3e})", flush=True)
    assert float(plane_err.max()) < 1e-12 * amax
    # the (0, 0) column (plane means, ~1e-7 here against max|phi| ~ 0.7): its own relative error
    mean_err = (phc - ref).mean(dim=(1, 2)).abs()
    mean_ref = float(ref.mean(dim=(1, 2)).abs().max())
    print(f"couette fp64 (0,0) column max error {float(mean_err.max()):.3e} (max plane mean {mean_ref:.3e})",
          flush=True)
    assert float(mean_err.max()) < 1e-9 * mean_ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,plan_tol,tol", [("fp32_refined", 0.0, 1e-11), ("fp32_refined", 1e-11, 1e-11),
                                               ("fp32_refined", 1e-8, 1e-8), ("fp32", 0.0, 1e-5)])
def test_couette_solve_fp32(couette, prec, plan_tol, tol):
    """The refinement's stop rule meets the requested relative error against the oracle."""
    cfg, zf, g, f, ref, _ = couette
    banner(f"couette {prec} solve tol={plan_tol}")
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision=prec, tol=plan_tol)
    phi, info = plan.solve(f.to("cuda"))
    err = rel(phi, ref)
    print(f"couette {prec} rel-L2 {err:.3e} iterations {info['iterations']}", flush=True)
    assert err < tol


@pytest.mark.timeout(900)
def test_slab512_project():
    banner("slab512 projection")
    cfg, zf, g = _setup("slab512x512x384")
    u, v, w = (torch.as_tensor(a) for a in synth.mode_velocity(cfg))
    z = torch.zeros_like(u)
    ref = poisson.project(u, v, w, z, g)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    ud, vd, wd, pd = (a.to("cuda") for a in (u, v, w, z))
    phi = torch.empty_like(pd)
    plan.project(ud, vd, wd, pd, phi)
    for name, a, b in zip(("u", "v", "w", "p", "phi"), (ud, vd, wd, pd, phi), ref):
        err = rel(a, b)
        print(f"slab512 {name} rel-L2 {err:.3e}", flush=True)
        assert err < 1e-12
    # Discrete divergence after projection: its floor is the rounding of L phi, about
    # eps |L| |phi| (|L| ~ 4/dz_min^2 ~ 7e8 on this grid), so it is compared with the
    # oracle's own post-projection divergence rather than with a fixed fraction.
    d0 = float(op.divergence(u, v, w, g).abs().max())
    d1 = float(op.divergence(ud.cpu(), vd.cpu(), wd.cpu(), g).abs().max())
    dref = float(op.divergence(ref[0], ref[1], ref[2], g).abs().max())
    print(f"slab512 max|div| before {d0:.3e} after {d1:.3e} (oracle {dref:.3e})", flush=True)
    assert d1 < 4.0 * dref + 1e-14 * d0 and d1 < 1e-9 * d0


@pytest.mark.timeout(900)
def test_slab256_project_parity():
    banner("slab256 projection parity")
    cfg, zf, g = _setup("slab256x256x192")
    u, v, w = (torch.as_tensor(a) for a in synth.mode_velocity(cfg))
    ref = poisson.project(u, v, w, torch.zeros_like(u), g)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    ud, vd, wd = (a.to("cuda") for a in (u, v, w))
    phi = torch.empty_like(ud)
    plan.project(ud, vd, wd, None, phi)
    for name, a, b in zip(("u", "v", "w", "phi"), (ud, vd, wd, phi), (ref[0], ref[1], ref[2], ref[4])):
        err = rel(a, b)
        print(f"slab256 {name} rel-L2 {err:.3e}", flush=True)
        assert err < 1e-12


@pytest.mark.timeout(900)
def test_slab256_adjoint_finite_differences():
    """Loss sum(w . u_projected); hand-written adjoint vs central differences, h = 1e-6, 32 directions."""
    banner("slab256 adjoint FD")
    cfg, zf, g = _setup("slab256x256x192")
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    u, v, w = (torch.as_tensor(a).to("cuda") for a in synth.mode_velocity(cfg))
    om = [torch.as_tensor(a).to("cuda") for a in synth.face_weights(cfg)]

    def loss(a, b, c):
        pu, pv, pw = ProjectFn.apply(a, b, c, plan)
        return (pu * om[0]).sum() + (pv * om[1]).sum() + (pw * om[2]).sum()

    xs = [t.clone().requires_grad_(True) for t in (u, v, w)]
    grads = torch.autograd.grad(loss(*xs), xs)
    assert float(grads[2][0].abs().max()) == 0.0 and float(grads[2][-1].abs().max()) == 0.0
    # Scale of a directional derivative along an i.i.d. N(0,1) direction: ||g||_2.  The
    # central difference at h = 1e-6 carries the forward map's rounding times 1/(2h), so
    # errors are measured against max(|an|, ||g||) (a 1e-3 error in g would still show).
    gnorm = float(torch.sqrt(sum((gr * gr).sum() for gr in grads)))
    rng = np.random.default_rng(2024)
    worst = 0.0
    for trial in range(32):
        d = [torch.as_tensor(rng.standard_normal(tuple(t.shape))).to("cuda") for t in (u, v, w)]
        d[2][0] = 0
        d[2][-1] = 0
        h = 1e-6
        with torch.no_grad():
            pp = ProjectFn.apply(*[a + h * b for a, b in zip((u, v, w), d)], plan)
            pm = ProjectFn.apply(*[a - h * b for a, b in zip((u, v, w), d)], plan)
            # the loss is linear in the projected field: difference the fields point by
            # point, then weight and sum (the same central difference, without the
            # cancellation of two large loss values)
            fd = float(sum(((x - y) * o).sum() for x, y, o in zip(pp, pm, om)) / (2 * h))
        an = float(sum((gr * di).sum() for gr, di in zip(grads, d)))
        err = abs(fd - an) / max(abs(an), gnorm)
        worst = max(worst, err)
        assert err <= 1e-6, (trial, fd, an, gnorm)
        if trial < 4:
            # the projection is linear, so the difference quotient is exact for any h:
            # with h = 1 the rounding term is gone and the agreement must be tight
            with torch.no_grad():
                pp = ProjectFn.apply(*[a + b for a, b in zip((u, v, w), d)], plan)
                pm = ProjectFn.apply(*[a - b for a, b in zip((u, v, w), d)], plan)
                fd1 = float(sum(((x - y) * o).sum() for x, y, o in zip(pp, pm, om)) / 2.0)
            assert abs(fd1 - an) <= 1e-9 * max(abs(an), gnorm), (trial, fd1, an)
    print(f"slab256 FD worst relative error {worst:.3e} (scale ||g|| = {gnorm:.3e})", flush=True)


def test_slab256_dense_8cube():
    """8^3 sub-case of the 256^2 x 192 box: the adjoint equals the transpose of the oracle's dense Jacobian."""
    banner("slab256 dense 8^3")
    n = 8
    zf = synth.zfaces(n, 3.0)
    g = Grid(n, n, n, 2.0, 2.0, zf)
    plan = Plan(n, n, n, 2.0, 2.0, zf, precision="fp64")
    nc = n ** 3
    nwi = (n - 1) * n * n
    z = torch.zeros(n, n, n, dtype=F64)

    def apply(x):
        uu = x[:nc].view(n, n, n)
        vv = x[nc:2 * nc].view(n, n, n)
        wi = x[2 * nc:].view(n - 1, n, n)
        zero = torch.zeros(1, n, n, dtype=F64)
        ww = torch.cat([zero, wi, zero], 0)
        pu, pv, pw, _, _ = poisson.project(uu, vv, ww, z, g, differentiable=True)
        return torch.cat([pu.reshape(-1), pv.reshape(-1), pw[1:n].reshape(-1)])

    J = torch.autograd.functional.jacobian(apply, torch.zeros(2 * nc + nwi, dtype=F64))
    rng = np.random.default_rng(5)
    om = torch.as_tensor(rng.standard_normal(2 * nc + nwi))
    ref = J.T @ om
    gw = torch.zeros(n + 1, n, n, dtype=F64)
    gw[1:n] = om[2 * nc:].view(n - 1, n, n)
    gu, gv, gwo = plan.project_adjoint(om[:nc].view(n, n, n).to("cuda"), om[nc:2 * nc].view(n, n, n).to("cuda"),
                                       gw.to("cuda"))
    got = torch.cat([gu.cpu().reshape(-1), gv.cpu().reshape(-1), gwo.cpu()[1:n].reshape(-1)])
    assert rel(got, ref) < 1e-12


@pytest.fixture(scope="module")
def rb768():
    cfg, zf, g = _setup("rb768x768x512")
    ra, pr = cfg.extra["ra"], cfg.extra["pr"]
    nu, ka = math.sqrt(pr / ra), 1.0 / math.sqrt(ra * pr)
    state = [torch.as_tensor(a) for a in synth.rb_state(cfg)]
    dt = 1.3 / ss.cfl(state[0], state[1], state[2], g)
    return cfg, zf, g, state, dt, nu, ka


@pytest.mark.timeout(1200)
def test_rb768_substep_forward(rb768):
    cfg, zf, g, state, dt, nu, ka = rb768
    banner(f"rb768 substep forward dt={dt:.3e}")
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp32_refined")
    dstate = [a.to("cuda") for a in state]
    cfl_gpu = float(plan.cfl(dstate[0], dstate[1], dstate[2]).item())
    assert abs(1.3 / cfl_gpu - dt) <= 1e-15 * dt
    plan.substep(1, dt, nu, ka, *dstate)
    out = [a.cpu() for a in dstate]
    del dstate
    torch.cuda.empty_cache()
    ref, _ = ss.substep(state, g, 1, dt, nu, ka)
    for name, a, b, x0 in zip("uvwTp", out, ref, state):
        err = rel(a, b)
        inc = rel(a - x0, b - x0) if float((b - x0).norm()) > 0 else 0.0
        print(f"rb768 {name} rel-L2 {err:.3e} (increment {inc:.3e})", flush=True)
        assert err < 1e-10 and inc < 1e-9
        # every plane, including the wall rows of w and T, within the same bound in max-norm
        scale = float(b.abs().max())
        plane_err = (a - b).abs().amax(dim=(1, 2))
        assert float(plane_err.max()) < 1e-9 * scale, name
    for name, a in (("w", out[2]), ("T", out[3])):
        assert torch.equal(a[0], state["wT".index(name) + 2][0]) and torch.equal(a[-1], state["wT".index(name) + 2][-1])


@pytest.mark.timeout(900)
def test_rb768_substep_adjoint_fd(rb768):
    """Substep VJP at 768^2 x 512 vs central differences of the FP64 GPU forward, 4 directions."""
    cfg, zf, g, state, dt, nu, ka = rb768
    banner("rb768 substep adjoint FD")
    fwd = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    adj = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp32_refined")
    dstate = [a.to("cuda") for a in state]
    rng = np.random.default_rng(77)
    cot = [torch.as_tensor(rng.standard_normal(tuple(a.shape))).to("cuda") for a in state]
    for c in (cot[2], cot[3]):
        c[0] = 0
        c[-1] = 0
    gin = adj.substep_adjoint(dt, nu, ka, *dstate, cot)
    gnorm = float(torch.sqrt(sum((g_ * g_).sum() for g_ in gin)))   # scale of N(0,1) directional derivatives

    def forward(st):
        s2 = [a.clone() for a in st]
        fwd.substep(1, dt, nu, ka, *s2)
        return s2

    for trial in range(4):
        d = [torch.as_tensor(rng.standard_normal(tuple(a.shape))).to("cuda") for a in state]
        for x in (d[2], d[3]):
            x[0] = 0
            x[-1] = 0
        h = 1e-6
        sp = forward([a + h * b for a, b in zip(dstate, d)])
        sm = forward([a - h * b for a, b in zip(dstate, d)])
        # central difference of sum(cot . out): outputs differenced point by point first
        fd = float(sum(((x - y) * c).sum() for x, y, c in zip(sp, sm, cot))) / (2 * h)
        del sp, sm
        an = float(sum((gi * di).sum() for gi, di in zip(gin, d)))
        err = abs(fd - an) / max(abs(an), gnorm)
        print(f"rb768 FD trial {trial}: fd {fd:.9e} adjoint {an:.9e} rel {err:.2e}", flush=True)
        assert err <= 1e-6


@pytest.mark.timeout(1200)
def test_rb768_step_adjoint_fd(rb768):
    """Whole-step VJP (three substeps, fixed dt) at 768^2 x 512 vs central differences of the
    library's own step, 4 directions."""
    cfg, zf, g, state, dt, nu, ka = rb768
    banner("rb768 step adjoint FD")
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    dstate = [a.to("cuda") for a in state]
    rng = np.random.default_rng(78)
    cot = [torch.as_tensor(rng.standard_normal(tuple(a.shape))).to("cuda") for a in state]
    for c in (cot[2], cot[3]):
        c[0] = 0
        c[-1] = 0
    gin = plan.step_adjoint(dt, nu, ka, *dstate, cot)
    gnorm = float(torch.sqrt(sum((g_ * g_).sum() for g_ in gin)))

    def forward(st):
        s2 = [a.clone() for a in st]
        plan.step(nu, ka, *s2, dt=dt)
        return s2

    for trial in range(4):
        d = [torch.as_tensor(rng.standard_normal(tuple(a.shape))).to("cuda") for a in state]
        for x in (d[2], d[3]):
            x[0] = 0
            x[-1] = 0
        h = 1e-6
        sp = forward([a + h * b for a, b in zip(dstate, d)])
        sm = forward([a - h * b for a, b in zip(dstate, d)])
        fd = float(sum(((x - y) * c).sum() for x, y, c in zip(sp, sm, cot))) / (2 * h)
        del sp, sm
        an = float(sum((gi * di).sum() for gi, di in zip(gin, d)))
        err = abs(fd - an) / max(abs(an), gnorm)
        print(f"rb768 step FD trial {trial}: fd {fd:.9e} adjoint {an:.9e} rel {err:.2e}", flush=True)
        assert err <= 1e-6
    del gin
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_rb384_multires_full_size():
    """The benchmark's multiple-resolution configuration (momentum 384^2 x 256, temperature
    768^2 x 512): the prolonged velocity of a projected state is divergence free on the
    temperature grid, the restriction matches the oracle, and one coupled step keeps the
    temperature's wall rows and stays finite."""
    from oracle import multires as mr
    from paper_1705_01423_amd.api import MultiRes
    banner("rb384 multires full size")
    cfg, zf, g = _setup("rb384x384x256")
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    m = MultiRes(plan, 2, 2, 2, nsub=2)
    u, v, w, _, p = (torch.as_tensor(a).to("cuda") for a in synth.rb_state(cfg, unoise=0.1))
    plan.project(u, v, w)
    uf, vf, wf = m.prolong_velocity(u, v, w)
    gf = mr.fine_grid(g, 2, 2, 2)
    dzf = gf.dz.to("cuda")
    div = ((torch.roll(uf, -1, 2) - uf) / gf.dx + (torch.roll(vf, -1, 1) - vf) / gf.dy
           + (wf[1:] - wf[:-1]) / dzf[:, None, None])
    scale = float(uf.abs().max()) / float(gf.dz.min())
    print(f"rb384 prolonged max|div| {float(div.abs().max()):.3e} (scale {scale:.3e})", flush=True)
    assert float(div.abs().max()) < 1e-12 * scale
    del div, uf, vf, wf
    zff = mr.fine_faces(zf, 2)
    tf = torch.as_tensor(synth.rb_temperature(cfg, zff, m.nxf, m.nyf))
    tc = m.restrict_temperature(tf.to("cuda")).cpu()
    ref = mr.restrict_temperature(tf, g, 2, 2, 2)
    assert float((tc - ref).abs().max()) <= 1e-15
    td = tf.to("cuda")
    dt, _ = m.step(math.sqrt(1e-8), 1e-4, u, v, w, p, td, dt=0.0, cfl=1.3)
    assert dt > 0 and bool(torch.isfinite(td).all())
    assert bool((td[0] == 1.0).all()) and bool((td[-1] == 0.0).all())
