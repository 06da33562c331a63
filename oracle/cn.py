"""Wall-normal Crank-Nicolson solves (paper Sec. 2.1-2.2).

Only the wall-normal viscous/diffusive term is implicit (the horizontal ones
are explicit, Sec. 2.2), so each substep solves, per (x, y) column,

    (I - beta Dzz) dq = rhs,      beta = alpha_l dt nu / 2  (kappa for T),

in "delta" form: dq is the increment, so its wall values are zero
(homogeneous Dirichlet) and the wall values of q enter only through the
explicit Dzz q on the right-hand side.

* centre fields (u, v): Nz unknowns; the wall lies half a cell beyond the
  first and last centres (distance dz/2).
* face fields (w, T): the Nz-1 interior faces are unknown; wall faces fixed.

The matrix is the same for every column, so it is factored once (plain
Thomas LU; it is strictly diagonally dominant) and applied to all columns.

Parity: pinned by a dense solve on random columns and by Dzz of a linear
profile being zero (tests/test_oracle_cn.py).
"""
from __future__ import annotations

import torch

F64 = torch.float64


def centre_matrix(g, beta):
    """(sub, diag, sup) of I - beta Dzz for centre fields, each of length Nz."""
    nz = g.nz
    am = torch.empty(nz, dtype=F64)
    ap = torch.empty(nz, dtype=F64)
    for k in range(nz):
        am[k] = 1.0 / (g.dzw[k] * g.dz[k])
        ap[k] = 1.0 / (g.dzw[k + 1] * g.dz[k])
    diag = 1.0 + beta * (am + ap)
    sub = -beta * am
    sup = -beta * ap
    sub[0] = 0.0
    sup[nz - 1] = 0.0
    return sub, diag, sup


def face_matrix(g, beta):
    """(sub, diag, sup) of I - beta Dzz for the Nz-1 interior faces k = 1..Nz-1."""
    nz = g.nz
    n = nz - 1
    bm = torch.empty(n, dtype=F64)
    bp = torch.empty(n, dtype=F64)
    for r in range(n):
        k = r + 1
        bm[r] = 1.0 / (g.dz[k - 1] * g.dzc[k])
        bp[r] = 1.0 / (g.dz[k] * g.dzc[k])
    diag = 1.0 + beta * (bm + bp)
    sub = -beta * bm
    sup = -beta * bp
    sub[0] = 0.0
    sup[n - 1] = 0.0
    return sub, diag, sup


def thomas(sub, diag, sup, rhs):
    """Plain Thomas algorithm along dim 0 of ``rhs`` (shared coefficients)."""
    n = diag.shape[0]
    cp = [None] * n
    dp = [None] * n
    cp[0] = sup[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for k in range(1, n):
        den = diag[k] - sub[k] * cp[k - 1]
        cp[k] = sup[k] / den
        dp[k] = (rhs[k] - sub[k] * dp[k - 1]) / den
    x = [None] * n
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return torch.stack(x, dim=0)


def solve_centre(rhs, g, beta):
    return thomas(*centre_matrix(g, beta), rhs)


def solve_face(rhs, g, beta):
    """rhs has shape (Nz+1, ...); wall rows of the result are zero."""
    inner = thomas(*face_matrix(g, beta), rhs[1:g.nz])
    zero = torch.zeros_like(rhs[:1])
    return torch.cat([zero, inner, zero], dim=0)
