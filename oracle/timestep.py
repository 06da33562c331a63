"""A full RK3 time step, the CFL-limited time step and wall-normal statistics (paper Sec. 2.1,
Listing 1; the Nusselt number reported in Sec. 5, Table 3).  Test infrastructure: plain FP64 torch on the CPU.

* One time step is the three substeps l = 1, 2, 3 of the low-storage RK3 scheme with the
  same dt, each substep handing its explicit terms H^l to the next (rho_l H^{l-1}).
* The time step follows the Courant number of Listing 1: dt = cfl_target / cfl(u, v, w),
  capped by dt_max.
* Statistics of a convection state, per wall-normal position (averages over the periodic
  x-y plane): the plane-mean temperature on the z-faces, and the total vertical heat flux
  through each cell-centre plane,
      F_k = < wbar_k Tbar_k > - kappa (<T>_{k+1} - <T>_k) / dz_k,
  with wbar_k, Tbar_k the averages of the two faces bounding cell k (the advective flux
  the temperature equation's z-faces exchange, in the form the discretisation uses).
  With the wall temperatures 1 and 0 and unit height the Nusselt profile is F_k / kappa.
"""
from __future__ import annotations

import math

import torch

from .substep import cfl, substep


def rk3_step(state, g, dt, nu, kappa, differentiable=False):
    """Three substeps with a fixed dt.  state = (u, v, w, T, p); returns the new state.
    differentiable=True runs the Poisson solves through their autograd form (for adjoints)."""
    h = None
    for l in (1, 2, 3):
        state, h = substep(state, g, l, dt, nu, kappa, hprev=h, differentiable=differentiable)
    return state


def cfl_dt(u, v, w, g, cfl_target, dt_max=math.inf):
    """Time step of Courant number cfl_target (Listing 1), at most dt_max."""
    return min(dt_max, cfl_target / cfl(u, v, w, g))


def plane_mean(q):
    """Average over the x-y plane of every z-plane, summed with math.fsum."""
    return torch.tensor([math.fsum(q[k].reshape(-1).tolist()) / q[k].numel() for k in range(q.shape[0])],
                        dtype=torch.float64)


def heat_flux(w, t, g, kappa):
    """(mean T on the nz + 1 faces, total vertical heat flux F on the nz centre planes)."""
    tm = plane_mean(t)
    wbar = 0.5 * (w[:-1] + w[1:])
    tbar = 0.5 * (t[:-1] + t[1:])
    adv = plane_mean(wbar * tbar)
    cond = kappa * (tm[1:] - tm[:-1]) / g.dz
    return tm, adv - cond
