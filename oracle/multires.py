"""Multiple-resolution temperature grid (paper Sec. 6).  Test infrastructure: plain FP64 torch
on the CPU.

Sec. 6 states the idea only: the temperature lives on a grid of higher resolution than the
momentum, and it is advanced with its own refined time step.  The reading implemented here:

Grids.  The temperature grid refines the momentum grid by integer factors (rx, ry, rz):
Nx' = rx Nx, Ny' = ry Ny, Nz' = rz Nz.  Each momentum cell is split into rx ry rz equal
sub-cells, so the fine wall-normal faces are zf'[rz k + m] = zf[k] + (m / rz) dz[k],
m = 0..rz-1 (every momentum face is a temperature face).  T sits on the fine z-faces and the
fine x-y cell centres, (Nz'+1, Ny', Nx'), wall rows stored (T fixed there).

Velocity on the temperature grid (``prolong_velocity``).  The temperature is advected by a
fine-grid velocity built from the momentum-grid one in three steps, per coarse cell:
  1. every fine face lying on a coarse face takes the coarse face value plus a linear
     variation across the face, with slopes from central differences of the neighbouring
     coarse faces (periodic in x, y; in z the three-point formula on the stretched centres,
     with the no-slip wall value 0 at the wall as the outer point).  The sub-faces are
     placed symmetrically, so each coarse face keeps its flux exactly;
  2. fine faces inside a coarse cell interpolate linearly, along their normal, between the
     two coarse faces that bound the cell;
  3. a local correction makes every sub-cell's divergence equal that of its coarse cell:
     with r the sub-cell divergences of steps 1-2, the interior fine faces receive G psi,
     psi = -(L_loc)^+ r, where L_loc = D G is the Laplacian of the cell's sub-cells with
     no flux through the coarse cell's boundary (so the coarse faces keep their values).
     G psi is the smallest such correction in the volume-weighted norm.
A discretely divergence-free momentum velocity thus gives a discretely divergence-free
temperature-grid velocity; steps 1-2 are exact for linear fields and the correction is of
second order, so the interpolation is second-order accurate.

Buoyancy (``restrict_temperature``).  The momentum equations see the temperature on the
coarse z-faces as the average of the rx ry fine values at the same height in that coarse
column.

Time stepping (``temperature_step``, ``step_mr``).  One momentum step of size dt (the three
RK3 / Crank-Nicolson substeps of Sec. 2.1) runs with the buoyancy of the restricted
temperature at the start of the step.  The temperature is then advanced over the same
interval by nsub full RK3 steps of size dt / nsub on its own grid (the same substep
formulas, Crank-Nicolson for the wall-normal diffusion); the advecting velocity of each
stage is the linear interpolation in time between the temperature-grid velocities at the
start and at the end of the momentum step, taken at the stage's start time
(RK3 stage start times 0, 8/15, 2/3 of a step).

Pins (tests/test_oracle_multires.py): unit factors give the identity (prolongation,
restriction) and the single-grid substep (temperature substep); prolonged velocities of
divergence-free fields are divergence-free to rounding; prolongation and restriction converge
at second order to analytic fields; the restriction keeps plane means; fine advection
conserves the integral of T and keeps a uniform T uniform; the temperature step converges at
third order in its sub-step with a velocity that varies linearly in time.
"""
from __future__ import annotations

import numpy as np
import torch

from .grid import Grid
from . import operators as op
from . import cn
from .substep import GAMMA, RHO, adv_face, substep

F64 = torch.float64
STAGE_START = (0.0, 8.0 / 15.0, 2.0 / 3.0)   # start time of RK3 substep l (fraction of a step)


def fine_faces(zf, rz):
    """Fine wall-normal faces: every coarse cell split into rz equal sub-cells."""
    zf = np.asarray(zf, dtype=np.float64)
    nz = len(zf) - 1
    out = np.empty(nz * rz + 1)
    for k in range(nz):
        dz = zf[k + 1] - zf[k]
        for m in range(rz):
            out[k * rz + m] = zf[k] + (m / rz) * dz
    out[nz * rz] = zf[nz]
    return out


def fine_grid(g, rx, ry, rz):
    return Grid(g.nx * rx, g.ny * ry, g.nz * rz, g.lx, g.ly, fine_faces(g.zf.numpy(), rz))


# ---- velocity prolongation --------------------------------------------------------------
def _zslope(q, g):
    """d q / dz at the coarse centres (three-point formula on the stretched centres, the
    no-slip wall value 0 at z = zf[0] and z = zf[Nz] as the outer points)."""
    zc = g.zc
    zero = torch.zeros_like(q[:1])
    qm = torch.cat([zero, q[:-1]], dim=0)
    qp = torch.cat([q[1:], zero], dim=0)
    zm = torch.cat([g.zf[:1], zc[:-1]])
    zp = torch.cat([zc[1:], g.zf[-1:]])
    hm = (zc - zm)[:, None, None]
    hp = (zp - zc)[:, None, None]
    return (hm * hm * (qp - q) + hp * hp * (q - qm)) / (hm * hp * (hm + hp))


def _offsets(r, h):
    """Offsets of the r sub-cell centres from the coarse centre, for spacing h."""
    return torch.tensor([((b + 0.5) / r - 0.5) * h for b in range(r)], dtype=F64)


def _local_correction_matrix(rx, ry, rz, dxf, dyf, dzf):
    """For one coarse cell: the map from the rx ry rz sub-cell divergences r to the interior
    fine-face corrections G psi, psi = -(D G)^+ r (zero flux on the coarse cell's faces).
    Returns (M, faces) with faces = [('x'|'y'|'z', a, b, m), ...] the interior faces in the
    order of M's rows (sub-cell (a, b, m) indexes x, y, z)."""
    ncell = rx * ry * rz

    def cid(a, b, m):
        return (m * ry + b) * rx + a

    faces = []
    for m in range(rz):
        for b in range(ry):
            for a in range(1, rx):
                faces.append(("x", a, b, m))
    for m in range(rz):
        for b in range(1, ry):
            for a in range(rx):
                faces.append(("y", a, b, m))
    for m in range(1, rz):
        for b in range(ry):
            for a in range(rx):
                faces.append(("z", a, b, m))
    nf = len(faces)
    G = np.zeros((nf, ncell))
    D = np.zeros((ncell, nf))
    for f, (d, a, b, m) in enumerate(faces):
        if d == "x":
            lo, hi, h = cid(a - 1, b, m), cid(a, b, m), dxf
        elif d == "y":
            lo, hi, h = cid(a, b - 1, m), cid(a, b, m), dyf
        else:
            lo, hi, h = cid(a, b, m - 1), cid(a, b, m), dzf
        G[f, hi] += 1.0 / h
        G[f, lo] -= 1.0 / h
        D[lo, f] += 1.0 / h     # outflow of the lower sub-cell
        D[hi, f] -= 1.0 / h     # inflow of the upper one
    L = D @ G
    M = -G @ np.linalg.pinv(L) if ncell > 1 else np.zeros((0, 1))
    return M, faces


def prolong_velocity(u, v, w, g, rx, ry, rz):
    """Coarse face velocity (u, v: (Nz, Ny, Nx); w: (Nz+1, Ny, Nx)) -> temperature-grid face
    velocity (uf, vf: (Nz', Ny', Nx'); wf: (Nz'+1, Ny', Nx'))."""
    nx, ny, nz = g.nx, g.ny, g.nz
    NX, NY, NZ = nx * rx, ny * ry, nz * rz
    dxf, dyf = g.dx / rx, g.dy / ry
    ex, ey = _offsets(rx, g.dx), _offsets(ry, g.dy)
    # 1. fine values on the coarse faces
    syu = (torch.roll(u, -1, 1) - torch.roll(u, 1, 1)) / (2 * g.dy)
    szu = _zslope(u, g)
    sxv = (torch.roll(v, -1, 2) - torch.roll(v, 1, 2)) / (2 * g.dx)
    szv = _zslope(v, g)
    sxw = (torch.roll(w, -1, 2) - torch.roll(w, 1, 2)) / (2 * g.dx)
    syw = (torch.roll(w, -1, 1) - torch.roll(w, 1, 1)) / (2 * g.dy)
    uf = torch.zeros(NZ, NY, NX, dtype=F64)
    vf = torch.zeros(NZ, NY, NX, dtype=F64)
    wf = torch.zeros(NZ + 1, NY, NX, dtype=F64)
    for k in range(nz):
        ez = _offsets(rz, float(g.dz[k]))
        for m in range(rz):
            for b in range(ry):
                uf[k * rz + m, b::ry, ::rx] = u[k] + syu[k] * ey[b] + szu[k] * ez[m]
            for a in range(rx):
                vf[k * rz + m, ::ry, a::rx] = v[k] + sxv[k] * ex[a] + szv[k] * ez[m]
    for k in range(nz + 1):
        for b in range(ry):
            for a in range(rx):
                wf[k * rz, b::ry, a::rx] = w[k] + sxw[k] * ex[a] + syw[k] * ey[b]
    # 2. interior faces: linear along the normal between the cell's two coarse faces
    for a in range(1, rx):
        left = uf[:, :, ::rx]
        right = torch.roll(left, -1, 2)
        uf[:, :, a::rx] = (1 - a / rx) * left + (a / rx) * right
    for b in range(1, ry):
        front = vf[:, ::ry, :]
        back = torch.roll(front, -1, 1)
        vf[:, b::ry, :] = (1 - b / ry) * front + (b / ry) * back
    for m in range(1, rz):
        wf[m:NZ:rz] = (1 - m / rz) * wf[0:NZ:rz] + (m / rz) * wf[rz::rz]
    # 3. local divergence correction, coarse level by coarse level
    gf = fine_grid(g, rx, ry, rz)
    r = op.divergence(uf, vf, wf, gf)
    for k in range(nz):
        M, faces = _local_correction_matrix(rx, ry, rz, dxf, dyf, float(g.dz[k]) / rz)
        if M.shape[0] == 0:
            continue
        rk = r[k * rz:(k + 1) * rz]                     # (rz, NY, NX)
        # sub-cell residuals of every coarse cell, ordered (m, b, a)
        sub = rk.reshape(rz, ny, ry, nx, rx).permute(1, 3, 0, 2, 4).reshape(ny, nx, rz * ry * rx)
        corr = torch.einsum("fc,jic->jif", torch.as_tensor(M), sub)
        for f, (d, a, b, m) in enumerate(faces):
            if d == "x":
                uf[k * rz + m, b::ry, a::rx] += corr[:, :, f]
            elif d == "y":
                vf[k * rz + m, b::ry, a::rx] += corr[:, :, f]
            else:
                wf[k * rz + m, b::ry, a::rx] += corr[:, :, f]
    return uf, vf, wf


# ---- temperature restriction ---------------------------------------------------------------
def restrict_temperature(tf, g, rx, ry, rz):
    """Fine face temperature (Nz'+1, Ny', Nx') -> coarse z-faces (Nz+1, Ny, Nx): mean of the
    rx ry fine values at the coarse face's height within each coarse column."""
    at_faces = tf[::rz]                                  # fine faces rz k, k = 0..Nz
    n = at_faces.shape[0]
    return at_faces.reshape(n, g.ny, ry, g.nx, rx).mean(dim=(2, 4))


# ---- temperature on its own grid -------------------------------------------------------------
def _zero_walls(q):
    q = q.clone()
    q[0] = 0.0
    q[-1] = 0.0
    return q


def t_explicit(t, u, v, w, gf, kappa):
    """Explicit terms of the temperature equation on a grid: -advection + horizontal diffusion."""
    h = -adv_face(t, u, v, w, gf) + kappa * (op.dxx(t, gf) + op.dyy(t, gf))
    return _zero_walls(h)


def t_substep(t, vel, gf, l, dt, kappa, hprev=None):
    """Substep l of the temperature equation with a given velocity (u, v, w) on grid gf."""
    gam, rho = GAMMA[l - 1], RHO[l - 1]
    alp = gam + rho
    h = t_explicit(t, *vel, gf, kappa)
    rt = gam * h + alp * (kappa * op.dzz_face(t, gf))
    if rho != 0.0:
        rt = rt + rho * hprev
    rt = _zero_walls(dt * rt)
    return t + cn.solve_face(rt, gf, alp * dt * kappa / 2.0), h


def temperature_step(t, vel0, vel1, gf, dt, kappa, nsub):
    """Advance T over dt by nsub RK3 steps of dt / nsub; stage velocity interpolated linearly
    in time between vel0 (start of dt) and vel1 (end of dt) at the stage's start time."""
    dts = dt / nsub
    for s in range(nsub):
        h = None
        for l in (1, 2, 3):
            th = (s + STAGE_START[l - 1]) / nsub
            vel = tuple((1.0 - th) * a + th * b for a, b in zip(vel0, vel1))
            t, h = t_substep(t, vel, gf, l, dts, kappa, h)
    return t


def step_mr(state, tf, g, rx, ry, rz, dt, nu, kappa, nsub):
    """One coupled step: state = (u, v, w, p) on the momentum grid, tf on the temperature grid.
    Returns ((u, v, w, p), tf)."""
    u, v, w, p = state
    gf = fine_grid(g, rx, ry, rz)
    tc = restrict_temperature(tf, g, rx, ry, rz)
    vel0 = prolong_velocity(u, v, w, g, rx, ry, rz)
    s = (u, v, w, tc, p)
    h = None
    for l in (1, 2, 3):
        out, h = substep(s, g, l, dt, nu, kappa, hprev=h)
        s = (out[0], out[1], out[2], tc, out[4])       # buoyancy frozen over the step
    vel1 = prolong_velocity(s[0], s[1], s[2], g, rx, ry, rz)
    tf = temperature_step(tf, vel0, vel1, gf, dt, kappa, nsub)
    return (s[0], s[1], s[2], s[4]), tf
