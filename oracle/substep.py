"""Explicit terms, CFL number and one RK3 / Crank-Nicolson substep (paper Sec. 2.1).

Equations (2)-(3) of the paper in free-fall units: nu = sqrt(Pr/Ra),
kappa = 1/sqrt(Ra Pr), Boussinesq buoyancy +T along the wall-normal axis
(temperature sits on the wall-normal velocity points, Fig. 1).  Walls:
no-slip u = v = 0, no penetration w = 0, T fixed (stored in the wall rows of T).

Advection is the conservative (divergence-form), central, second-order
discretisation of Sec. 2.1: every control volume's flux through a face is
(transporting normal velocity) x (transported quantity), both interpolated to
the face by simple averages, except that the horizontal transporting
velocities on the side faces of a z-face control volume are
volume-weighted averages of the two neighbouring centre values,
(dz_{k-1} u_{k-1} + dz_k u_k) / (2 dzc_k).  With these choices the transporting
fluxes of every control volume are exactly divergence free whenever the
pressure-cell divergence is, and advection then conserves discrete kinetic
energy (pinned by tests/test_oracle_cn_substep.py, together with second-order
convergence of the explicit terms to the continuous operators on uniform and
stretched grids).

Time advancement (Sec. 2.1: low-storage RK3 with Crank-Nicolson for the
wall-normal viscous term, pressure in "delta" form), substep l:

    RHS_q = dt [gamma_l H_q + rho_l H_q^{prev} - alpha_l G_q p + alpha_l nu Dzz q]
    (I - alpha_l dt nu / 2 Dzz) dq = RHS_q,   q* = q + dq
    L phi = D u* / (alpha_l dt),  u = u* - alpha_l dt G phi,
    p <- p + phi - (alpha_l dt nu / 2) Dzz phi
    T likewise with kappa and without pressure, using the substep's input
    velocity in its advection (the same stage as the momentum terms).

with gamma = (8/15, 5/12, 3/4), rho = (0, -17/60, -5/12), alpha = gamma + rho.

CFL number (Listing 1 of the paper): the maximum over cells of
0.5 (|w_k + w_{k+1}| / dz_k + |v_j + v_{j+1}| / dy + |u_i + u_{i+1}| / dx).

Which velocity advects the temperature inside a substep: Sec. 2.2 lists the
temperature update after the velocity correction, which could be read as
advecting T with the corrected velocity; Sec. 2.1 states a third-order time
error for the scheme.  Only the substep's input velocity keeps that order (the
corrected one gives about first order in T), so that is the reading taken.
Pinned by tests/test_oracle_timestep.py::test_step_third_order_in_time, with
the other reading planted as a mistake in tests/test_oracle_mutations.py.
"""
from __future__ import annotations

import math

import torch

from . import operators as op
from . import cn
from . import poisson

GAMMA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
RHO = (0.0, -17.0 / 60.0, -5.0 / 12.0)


def alpha_coef(l):
    return GAMMA[l - 1] + RHO[l - 1]


def _xm(q):   # value at i-1
    return torch.roll(q, 1, dims=2)


def _xp(q):   # value at i+1
    return torch.roll(q, -1, dims=2)


def _ym(q):
    return torch.roll(q, 1, dims=1)


def _yp(q):
    return torch.roll(q, -1, dims=1)


def adv_u(u, v, w, g):
    """Advection of u at (x-face i, y-centre j, z-centre k)."""
    fx = (0.5 * (u + _xp(u))) ** 2                          # at centre i (i+1/2)
    ax = (fx - _xm(fx)) / g.dx
    fy = (0.5 * (v + _xm(v))) * (0.5 * (u + _ym(u)))        # at (face i, y-face j)
    ay = (_yp(fy) - fy) / g.dy
    wz = 0.5 * (w + _xm(w))                                 # (Nz+1): at (face i, z-face k)
    ubar = 0.5 * (u[1:] + u[:-1])                           # interior z-faces 1..Nz-1
    fz_in = wz[1:g.nz] * ubar
    zero = torch.zeros_like(u[:1])
    fz = torch.cat([zero, fz_in, zero], dim=0)              # walls: u = 0, w = 0
    az = (fz[1:] - fz[:-1]) / g.dz[:, None, None]
    return ax + ay + az


def adv_v(u, v, w, g):
    """Advection of v at (x-centre i, y-face j, z-centre k)."""
    fy = (0.5 * (v + _yp(v))) ** 2
    ay = (fy - _ym(fy)) / g.dy
    fx = (0.5 * (u + _ym(u))) * (0.5 * (v + _xm(v)))        # at (x-face i, y-face j)
    ax = (_xp(fx) - fx) / g.dx
    wz = 0.5 * (w + _ym(w))
    vbar = 0.5 * (v[1:] + v[:-1])
    fz_in = wz[1:g.nz] * vbar
    zero = torch.zeros_like(v[:1])
    fz = torch.cat([zero, fz_in, zero], dim=0)
    az = (fz[1:] - fz[:-1]) / g.dz[:, None, None]
    return ax + ay + az


def _face_transport(u, v, w, g):
    """Volume-weighted horizontal velocities on the side faces of z-face cells (interior faces)."""
    dzm = g.dz[:-1, None, None]
    dzp = g.dz[1:, None, None]
    den = 2.0 * g.dzc[1:g.nz, None, None]
    uw = (dzm * u[:-1] + dzp * u[1:]) / den                 # (Nz-1): at (x-face i, z-face k)
    vw = (dzm * v[:-1] + dzp * v[1:]) / den
    return uw, vw


def adv_face(q, u, v, w, g):
    """Advection of a z-face quantity q (w or T) at interior faces; wall rows -> 0."""
    nz = g.nz
    uw, vw = _face_transport(u, v, w, g)
    qi = q[1:nz]
    fx = uw * (0.5 * (qi + _xm(qi)))                        # at (x-face i, z-face k)
    ax = (_xp(fx) - fx) / g.dx
    fy = vw * (0.5 * (qi + _ym(qi)))
    ay = (_yp(fy) - fy) / g.dy
    fz = (0.5 * (w[1:] + w[:-1])) * (0.5 * (q[1:] + q[:-1]))   # at centres k (Nz)
    az = (fz[1:] - fz[:-1]) / g.dzc[1:nz, None, None]
    zero = torch.zeros_like(q[:1])
    return torch.cat([zero, ax + ay + az, zero], dim=0)


def explicit_terms(u, v, w, t, g, nu, kappa):
    """H for u, v, w, T: -advection + horizontal diffusion (+ buoyancy on w)."""
    hu = -adv_u(u, v, w, g) + nu * (op.dxx(u, g) + op.dyy(u, g))
    hv = -adv_v(u, v, w, g) + nu * (op.dxx(v, g) + op.dyy(v, g))
    hw = -adv_face(w, u, v, w, g) + nu * (op.dxx(w, g) + op.dyy(w, g)) + t
    ht = -adv_face(t, u, v, w, g) + kappa * (op.dxx(t, g) + op.dyy(t, g))
    hw = _zero_walls(hw, g)
    ht = _zero_walls(ht, g)
    return hu, hv, hw, ht


def _zero_walls(q, g):
    mask = torch.ones(g.nz + 1, 1, 1, dtype=q.dtype)
    mask[0] = 0.0
    mask[g.nz] = 0.0
    return q * mask


def cfl(u, v, w, g):
    """Maximum CFL number (Listing 1 of the paper), for unit time step, at least 1e-8.

    A non-finite velocity gives NaN (the paper does not treat that case; the maximum is
    taken to propagate NaN so that a time step is never derived from a broken state)."""
    q = (torch.abs(w[:-1] + w[1:]) / g.dz[:, None, None]
         + torch.abs(v + _yp(v)) / g.dy
         + torch.abs(u + _xp(u)) / g.dx)
    c = float((0.5 * q).max())
    return c if math.isnan(c) else max(1e-8, c)


def substep(state, g, l, dt, nu, kappa, hprev=None, differentiable=False):
    """One RK3 substep.  state = (u, v, w, T, p).  Returns (new_state, H)."""
    u, v, w, t, p = state
    gam, rho, alp = GAMMA[l - 1], RHO[l - 1], alpha_coef(l)
    hu, hv, hw, ht = explicit_terms(u, v, w, t, g, nu, kappa)
    gu, gv, gw = op.gradient(p, g)

    def comb(h, hp, gp, lapz):
        r = gam * h - alp * gp + alp * lapz
        if rho != 0.0:
            r = r + rho * hp
        return dt * r

    hpu, hpv, hpw, hpt = hprev if hprev is not None else (None,) * 4
    ru = comb(hu, hpu, gu, nu * op.dzz_centre_dirichlet(u, g))
    rv = comb(hv, hpv, gv, nu * op.dzz_centre_dirichlet(v, g))
    rw = _zero_walls(comb(hw, hpw, gw, nu * op.dzz_face(w, g)), g)
    rt = _zero_walls(comb(ht, hpt, torch.zeros_like(t), kappa * op.dzz_face(t, g)), g)
    bnu = alp * dt * nu / 2.0
    bka = alp * dt * kappa / 2.0
    us = u + cn.solve_centre(ru, g, bnu)
    vs = v + cn.solve_centre(rv, g, bnu)
    ws = w + cn.solve_face(rw, g, bnu)
    tn = t + cn.solve_face(rt, g, bka)
    s = alp * dt
    un, vn, wn, pn, _ = poisson.project(us, vs, ws, p, g, s=s, c=bnu,
                                        differentiable=differentiable)
    return (un, vn, wn, tn, pn), (hu, hv, hw, ht)
