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


def _wall_normal_modes(g):
    """Eigenpairs of the wall-normal second differences (centre fields with zero wall values,
    interior faces), least damped first."""
    def dzz_inner(q):
        full = torch.cat([torch.zeros(1, 1, 1, dtype=F64), q, torch.zeros(1, 1, 1, dtype=F64)], 0)
        return op.dzz_face(full, g)[1:g.nz]

    out = []
    for fn, n in ((lambda q: op.dzz_centre_dirichlet(q, g), g.nz), (dzz_inner, g.nz - 1)):
        lam, vec = np.linalg.eig(_dense(fn, (n, 1, 1)))
        assert np.abs(lam.imag).max() == 0.0 and lam.real.max() < 0
        order = np.argsort(-lam.real)
        out.append((lam.real[order], vec.real[:, order]))
    return out


@pytest.mark.parametrize("l", [1, 2, 3])
def test_substep_crank_nicolson_modes(l):
    """Horizontally uniform u, v and T perturbations along eigenvectors of the wall-normal
    second difference feel neither advection, horizontal diffusion nor a pressure gradient, so
    a substep multiplies each by the trapezoidal (Crank-Nicolson) factor (1 + a/2) / (1 - a/2),
    a = alpha_l dt D lambda (Sec. 2.1: only the wall-normal diffusive term is implicit)."""
    g = _grid(4, 3, 12)
    nu, kappa, dt, eps = 0.02, 0.013, 0.05, 1e-3
    (lc, vc), (lf, vf) = _wall_normal_modes(g)
    shape = (g.nz, g.ny, g.nx)
    u = torch.as_tensor(eps * vc[:, 0])[:, None, None].expand(shape).clone()
    v = torch.as_tensor(eps * vc[:, 2])[:, None, None].expand(shape).clone()
    tmode = torch.zeros(g.nz + 1, dtype=F64)
    tmode[1:g.nz] = torch.as_tensor(eps * vf[:, 1])
    t = (1 - g.zf + tmode)[:, None, None].expand(g.nz + 1, g.ny, g.nx).clone()
    w = torch.zeros(g.nz + 1, g.ny, g.nx, dtype=F64)
    p = torch.zeros(shape, dtype=F64)
    # the previous substep's explicit terms of this state: zero but for the buoyancy on w
    hprev = ss.explicit_terms(u, v, w, t, g, nu, kappa) if l > 1 else None
    (un, vn, wn, tn, _), _ = ss.substep((u, v, w, t, p), g, l, dt, nu, kappa, hprev=hprev)
    alp = ss.GAMMA[l - 1] + ss.RHO[l - 1]

    def factor(diff, lam):
        a = alp * dt * diff * lam
        return (1 + a / 2) / (1 - a / 2)

    def rel(x, y):
        return float((x - y).norm() / y.norm())

    assert rel(un, factor(nu, lc[0]) * u) < 1e-12
    assert rel(vn, factor(nu, lc[2]) * v) < 1e-12
    assert rel(tn - (1 - g.zf)[:, None, None], factor(kappa, lf[1]) * (t - (1 - g.zf)[:, None, None])) < 1e-12
    assert float(wn.abs().max()) < 1e-15


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
    # the floor of Listing 1 for a fluid at rest, and NaN for a broken state
    z = torch.zeros(3, 4, 5, dtype=torch.float64)
    assert ss.cfl(z, z, torch.zeros(4, 4, 5, dtype=torch.float64), g) == 1e-8
    u[1, 2, 3] = float("nan")
    assert math.isnan(ss.cfl(torch.tensor(u), torch.tensor(v), torch.tensor(w), g))


def _fields_and_h(nx, ny, nz, lx, ly, alpha, nu, kappa):
    """Analytic u, v, w, T sampled at their staggered points, and the continuous explicit
    terms H = -div(u q) + diffusivity * (q_xx + q_yy) (+ T on w) at the same points, with
    the derivatives taken by automatic differentiation of the closed forms."""
    g = _grid(nx, ny, nz, lx, ly, alpha)
    kx, ky = 2 * math.pi / lx, 2 * math.pi / ly

    def U(x, y, z):
        return torch.sin(kx * x) * torch.cos(ky * y) * torch.sin(math.pi * z)

    def V(x, y, z):
        return 0.7 * torch.cos(kx * x) * torch.sin(ky * y + 0.3) * torch.sin(math.pi * z)

    def Wf(x, y, z):
        return torch.cos(kx * x + 0.2) * torch.cos(ky * y) * torch.sin(math.pi * z) ** 2

    def Tf(x, y, z):
        return 1.0 - z + 0.1 * torch.cos(kx * x) * torch.sin(ky * y) * torch.sin(math.pi * z)

    def points(xs, ys, zs):
        z, y, x = torch.meshgrid(zs, ys, xs, indexing="ij")
        return [c.clone().requires_grad_(True) for c in (x, y, z)]

    xf = torch.arange(nx, dtype=F64) * g.dx
    xc = xf + 0.5 * g.dx
    yf = torch.arange(ny, dtype=F64) * g.dy
    yc = yf + 0.5 * g.dy

    def h_at(q, diff, xs, ys, zs, buoy):
        x, y, z = points(xs, ys, zs)
        qv = q(x, y, z)
        flux = [U(x, y, z) * qv, V(x, y, z) * qv, Wf(x, y, z) * qv]
        div = sum(torch.autograd.grad(f.sum(), c, create_graph=True)[0] for f, c in zip(flux, (x, y, z)))
        qx, qy = torch.autograd.grad(qv.sum(), (x, y), create_graph=True)
        lap = torch.autograd.grad(qx.sum(), x, retain_graph=True)[0] + torch.autograd.grad(qy.sum(), y)[0]
        h = -div + diff * lap
        if buoy:
            h = h + Tf(x, y, z)
        return qv.detach(), h.detach()

    u, hu = h_at(U, nu, xf, yc, g.zc, False)
    v, hv = h_at(V, nu, xc, yf, g.zc, False)
    w, hw = h_at(Wf, nu, xc, yc, g.zf, True)
    t, ht = h_at(Tf, kappa, xc, yc, g.zf, False)
    return g, (u, v, w, t), (hu, hv, hw, ht)


@pytest.mark.parametrize("alpha", [0.0, 2.0])
def test_explicit_terms_second_order(alpha):
    """The explicit terms converge to the continuous operators at second order (Sec. 2.1:
    second-order central finite differences on the staggered grid), uniform and stretched in
    z: a dropped term, a wrong sign or a misplaced interpolation leaves an O(1) error."""
    nu, kappa = 0.03, 0.02
    errs = []
    for n in (16, 32, 64):
        g, (u, v, w, t), hex_ = _fields_and_h(n, n, n, 1.3, 0.9, alpha, nu, kappa)
        h = ss.explicit_terms(u, v, w, t, g, nu, kappa)
        e = []
        for q, (hd, he) in enumerate(zip(h, hex_)):
            if q >= 2:   # z-face quantities: interior faces only (the wall rows hold no equation)
                hd, he = hd[1:-1], he[1:-1]
            e.append(float((hd - he).abs().max() / he.abs().max()))
        errs.append(e)
    for q in range(4):
        r1 = errs[0][q] / errs[1][q]
        r2 = errs[1][q] / errs[2][q]
        assert errs[2][q] < 2e-2, (q, errs)
        assert r1 > 3.0 and r2 > 3.3, (q, errs)   # ratio 4 for second order
