// One RK3 / Crank-Nicolson substep (paper Sec. 2.1) and its adjoint.
//
// Forward, substep l with coefficients gamma, rho, alpha = gamma + rho:
//   H_q   = -A(q) + nu (Dxx + Dyy) q   (+ T on w; kappa for T)
//   rhs_q = dt [gamma H_q + rho H_q^prev - alpha G_q p + alpha nu Dzz q]
//   (I - alpha dt nu/2 Dzz) dq = rhs_q, q* = q + dq           (k_cn_solve_add)
//   projection of (u*, v*, w*) with s = alpha dt, c = alpha dt nu / 2
//
// Advection A is the conservative central form on the staggered grid: for each
// control volume, (outgoing minus incoming) face fluxes divided by its width,
// each flux = transporting velocity x transported quantity, both simple
// two-point averages, except the horizontal transporting velocities on the
// side faces of z-face volumes, which are volume-weighted:
//   Uw(k) = (dz_{k-1} u_{k-1} + dz_k u_k) / (2 dzc_k).
// Walls: u = v = 0, w = 0, T fixed (its wall rows); no flux through a wall.
#include "ps_internal.h"

namespace ps {

namespace {

struct Ix {
    int nx, ny, nz;
    size_t plane;
    __device__ __forceinline__ size_t at(int k, int j, int i) const {
        return (size_t)k * plane + (size_t)j * nx + i;
    }
};

__device__ __forceinline__ int wrapm(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrapp(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ double sq(double a) { return a * a; }

}  // namespace



// One thread per cell (k, j, i): rhs of u, v at the cell's x/y faces, and of w, T at
// its bottom z-face k (interior faces only; wall rows are zeroed).
__global__ void __launch_bounds__(256) k_explicit(SubstepArgs a, GridDev g) {
    int i, j, k;
    if (!stencil_cell(g, i, j, k)) return;
    const size_t id = ((size_t)k * g.ny + j) * g.nx + i;
    const Ix X{g.nx, g.ny, g.nz, (size_t)g.nx * g.ny};
    const int im = wrapm(i, g.nx), ip = wrapp(i, g.nx);
    const int jm = wrapm(j, g.ny), jp = wrapp(j, g.ny);
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double idx2 = idx * idx, idy2 = idy * idy;
    const int nz = g.nz;
    const double *u = a.u, *v = a.v, *w = a.w, *t = a.t, *p = a.p;

    // ---- u at (x-face i, y-centre j, z-centre k) ----
    {
        const double uc = u[id], uim = u[X.at(k, j, im)], uip = u[X.at(k, j, ip)];
        const double ujm = u[X.at(k, jm, i)], ujp = u[X.at(k, jp, i)];
        const double ax = (sq(0.5 * (uc + uip)) - sq(0.5 * (uim + uc))) * idx;
        const double fyb = 0.5 * (v[X.at(k, j, i)] + v[X.at(k, j, im)]) * (0.5 * (uc + ujm));
        const double fyt = 0.5 * (v[X.at(k, jp, i)] + v[X.at(k, jp, im)]) * (0.5 * (ujp + uc));
        const double ay = (fyt - fyb) * idy;
        double fzb = 0.0, fzt = 0.0, ukm = 0.0, ukp = 0.0;
        if (k > 0) {
            ukm = u[X.at(k - 1, j, i)];
            fzb = 0.5 * (w[X.at(k, j, i)] + w[X.at(k, j, im)]) * (0.5 * (ukm + uc));
        }
        if (k + 1 < nz) {
            ukp = u[X.at(k + 1, j, i)];
            fzt = 0.5 * (w[X.at(k + 1, j, i)] + w[X.at(k + 1, j, im)]) * (0.5 * (uc + ukp));
        }
        const double az = (fzt - fzb) / g.dz[k];
        const double h = -(ax + ay + az) + a.nu * ((uip - 2.0 * uc + uim) * idx2 + (ujp - 2.0 * uc + ujm) * idy2);
        const double fb = (k > 0) ? (uc - ukm) / g.dzw[k] : uc / g.dzw[0];
        const double ft = (k + 1 < nz) ? (ukp - uc) / g.dzw[k + 1] : -uc / g.dzw[nz];
        const double dzz = (ft - fb) / g.dz[k];
        const double gp = (p[id] - p[X.at(k, j, im)]) * idx;
        double r = a.gam * h - a.alp * gp + a.alp * (a.nu * dzz);
        if (a.rho != 0.0) r += a.rho * a.hpu[id];
        a.ru[id] = a.dt * r;
        if (a.hu) a.hu[id] = h;
    }
    // ---- v at (x-centre i, y-face j, z-centre k) ----
    {
        const double vc = v[id], vjm = v[X.at(k, jm, i)], vjp = v[X.at(k, jp, i)];
        const double vim = v[X.at(k, j, im)], vip = v[X.at(k, j, ip)];
        const double ay = (sq(0.5 * (vc + vjp)) - sq(0.5 * (vjm + vc))) * idy;
        const double fxl = 0.5 * (u[X.at(k, j, i)] + u[X.at(k, jm, i)]) * (0.5 * (vc + vim));
        const double fxr = 0.5 * (u[X.at(k, j, ip)] + u[X.at(k, jm, ip)]) * (0.5 * (vip + vc));
        const double ax = (fxr - fxl) * idx;
        double fzb = 0.0, fzt = 0.0, vkm = 0.0, vkp = 0.0;
        if (k > 0) {
            vkm = v[X.at(k - 1, j, i)];
            fzb = 0.5 * (w[X.at(k, j, i)] + w[X.at(k, jm, i)]) * (0.5 * (vkm + vc));
        }
        if (k + 1 < nz) {
            vkp = v[X.at(k + 1, j, i)];
            fzt = 0.5 * (w[X.at(k + 1, j, i)] + w[X.at(k + 1, jm, i)]) * (0.5 * (vc + vkp));
        }
        const double az = (fzt - fzb) / g.dz[k];
        const double h = -(ax + ay + az) + a.nu * ((vip - 2.0 * vc + vim) * idx2 + (vjp - 2.0 * vc + vjm) * idy2);
        const double fb = (k > 0) ? (vc - vkm) / g.dzw[k] : vc / g.dzw[0];
        const double ft = (k + 1 < nz) ? (vkp - vc) / g.dzw[k + 1] : -vc / g.dzw[nz];
        const double dzz = (ft - fb) / g.dz[k];
        const double gp = (p[id] - p[X.at(k, jm, i)]) * idy;
        double r = a.gam * h - a.alp * gp + a.alp * (a.nu * dzz);
        if (a.rho != 0.0) r += a.rho * a.hpv[id];
        a.rv[id] = a.dt * r;
        if (a.hv) a.hv[id] = h;
    }
    // ---- w and T at (x-centre i, y-centre j, z-face k), interior faces ----
    if (k == 0) {
        a.rw[id] = 0.0;
        a.rt[id] = 0.0;
        if (a.hw) a.hw[id] = 0.0;
        if (a.ht) a.ht[id] = 0.0;
    } else {
        const double dzm = g.dz[k - 1], dzp = g.dz[k], den = 1.0 / (2.0 * g.dzc[k]);
        // volume-weighted horizontal transport on the side faces
        const double uwl = (dzm * u[X.at(k - 1, j, i)] + dzp * u[X.at(k, j, i)]) * den;
        const double uwr = (dzm * u[X.at(k - 1, j, ip)] + dzp * u[X.at(k, j, ip)]) * den;
        const double vwb = (dzm * v[X.at(k - 1, j, i)] + dzp * v[X.at(k, j, i)]) * den;
        const double vwt = (dzm * v[X.at(k - 1, jp, i)] + dzp * v[X.at(k, jp, i)]) * den;
        const double wc = w[id], wim = w[X.at(k, j, im)], wip = w[X.at(k, j, ip)];
        const double wjm = w[X.at(k, jm, i)], wjp = w[X.at(k, jp, i)];
        const double wkm = w[X.at(k - 1, j, i)], wkp = w[X.at(k + 1, j, i)];
        const double tc = t[id], tim = t[X.at(k, j, im)], tip = t[X.at(k, j, ip)];
        const double tjm = t[X.at(k, jm, i)], tjp = t[X.at(k, jp, i)];
        const double tkm = t[X.at(k - 1, j, i)], tkp = t[X.at(k + 1, j, i)];
        const double idzc = 1.0 / g.dzc[k];
        const double wtop = 0.5 * (wc + wkp), wbot = 0.5 * (wkm + wc);   // at centres k, k-1
        // w
        {
            const double ax = (uwr * (0.5 * (wc + wip)) - uwl * (0.5 * (wim + wc))) * idx;
            const double ay = (vwt * (0.5 * (wc + wjp)) - vwb * (0.5 * (wjm + wc))) * idy;
            const double az = (sq(wtop) - sq(wbot)) * idzc;
            const double h = -(ax + ay + az) +
                             a.nu * ((wip - 2.0 * wc + wim) * idx2 + (wjp - 2.0 * wc + wjm) * idy2) + tc;
            const double dzz = ((wkp - wc) / dzp - (wc - wkm) / dzm) * idzc;
            const double gp = (p[id] - p[X.at(k - 1, j, i)]) * idzc;
            double r = a.gam * h - a.alp * gp + a.alp * (a.nu * dzz);
            if (a.rho != 0.0) r += a.rho * a.hpw[id];
            a.rw[id] = a.dt * r;
            if (a.hw) a.hw[id] = h;
        }
        // T
        {
            const double ax = (uwr * (0.5 * (tc + tip)) - uwl * (0.5 * (tim + tc))) * idx;
            const double ay = (vwt * (0.5 * (tc + tjp)) - vwb * (0.5 * (tjm + tc))) * idy;
            const double az = (wtop * (0.5 * (tc + tkp)) - wbot * (0.5 * (tkm + tc))) * idzc;
            const double h = -(ax + ay + az) + a.ka * ((tip - 2.0 * tc + tim) * idx2 + (tjp - 2.0 * tc + tjm) * idy2);
            const double dzz = ((tkp - tc) / dzp - (tc - tkm) / dzm) * idzc;
            double r = a.gam * h + a.alp * (a.ka * dzz);
            if (a.rho != 0.0) r += a.rho * a.hpt[id];
            a.rt[id] = a.dt * r;
            if (a.ht) a.ht[id] = h;
        }
    }
    if (k + 1 == nz) {
        const size_t top = id + X.plane;
        a.rw[top] = 0.0;
        a.rt[top] = 0.0;
        if (a.hw) a.hw[top] = 0.0;
        if (a.ht) a.ht[top] = 0.0;
    }
}

// Crank-Nicolson solve with the column-independent LU factors (fac = [l, invd, c]),
// rhs used as scratch, result added to q: q += (I - beta Dzz)^-1 rhs.
__global__ void __launch_bounds__(256)
k_cn_solve_add(GridDev g, int kind, const double* __restrict__ fac, double* __restrict__ rhs, double* __restrict__ q) {
    const size_t plane = (size_t)g.nx * g.ny;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    const int n = kind == 0 ? g.nz : g.nz - 1;
    const size_t off = (kind == 0 ? 0 : plane) + col;
    const double* l = fac;
    const double* invd = fac + n;
    const double* cs = fac + 2 * n;
    double* r = rhs + off;
    double* x = q + off;
    double y = r[0];
    for (int k = 1; k < n; ++k) {
        y = r[(size_t)k * plane] - l[k] * y;
        r[(size_t)k * plane] = y;
    }
    double d = y * invd[n - 1];
    x[(size_t)(n - 1) * plane] += d;
    for (int k = n - 2; k >= 0; --k) {
        d = (r[(size_t)k * plane] - cs[k] * d) * invd[k];
        x[(size_t)k * plane] += d;
    }
}

// out = V (I - beta Dzz)^-1 V^-1 in: the transpose of the CN solve (V = dz for centre
// fields, dzc for interior faces; V (I - beta Dzz) is symmetric).  Face walls -> 0.
__global__ void __launch_bounds__(256)
k_cn_solve_t(GridDev g, int kind, const double* __restrict__ fac, const double* __restrict__ in,
             double* __restrict__ out) {
    const size_t plane = (size_t)g.nx * g.ny;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    const int n = kind == 0 ? g.nz : g.nz - 1;
    const int ko = kind == 0 ? 0 : 1;
    const double* wv = kind == 0 ? g.dz : g.dzc;
    const double* l = fac;
    const double* invd = fac + n;
    const double* cs = fac + 2 * n;
    const double* r = in + (size_t)ko * plane + col;
    double* x = out + (size_t)ko * plane + col;
    double y = r[0] / wv[ko];
    x[0] = y;
    for (int k = 1; k < n; ++k) {
        y = r[(size_t)k * plane] / wv[k + ko] - l[k] * y;
        x[(size_t)k * plane] = y;
    }
    double d = y * invd[n - 1];
    x[(size_t)(n - 1) * plane] = d * wv[n - 1 + ko];
    for (int k = n - 2; k >= 0; --k) {
        d = (x[(size_t)k * plane] - cs[k] * d) * invd[k];
        x[(size_t)k * plane] = d * wv[k + ko];
    }
    if (kind == 1) {
        out[col] = 0.0;
        out[(size_t)g.nz * plane + col] = 0.0;
    }
}



// Vector-Jacobian product of the explicit right-hand sides, gathered per output
// point.  For a control-volume equation sum_faces +-F_f / h with cotangent kappa,
// each face carries Lambda_f = kappa_c / h_c - kappa_{c+1} / h_{c+1}; a flux
// F = U Q sends Lambda U dQ and Lambda Q dU to the points averaged into Q and U.
__global__ void __launch_bounds__(256) k_explicit_adj(SubstepAdjArgs a, GridDev g) {
    int i, j, k;
    if (!stencil_cell(g, i, j, k)) return;
    const size_t id = ((size_t)k * g.ny + j) * g.nx + i;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const Ix X{nx, ny, nz, (size_t)nx * ny};
    const int im = wrapm(i, nx), ip = wrapp(i, nx);
    const int jm = wrapm(j, ny), jp = wrapp(j, ny);
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double idx2 = idx * idx, idy2 = idy * idy;
    const double cadv = -a.dt * a.gam;   // kappa = cadv * lambda (A enters the rhs as -dt gamma A)
    const double *u = a.u, *v = a.v, *w = a.w, *t = a.t;
    auto U = [&](int kk, int jj, int ii) { return u[X.at(kk, jj, ii)]; };
    auto V = [&](int kk, int jj, int ii) { return v[X.at(kk, jj, ii)]; };
    auto Wf = [&](int kk, int jj, int ii) { return w[X.at(kk, jj, ii)]; };
    auto Tf = [&](int kk, int jj, int ii) { return t[X.at(kk, jj, ii)]; };
    auto KU = [&](int kk, int jj, int ii) { return cadv * a.lu[X.at(kk, jj, ii)]; };
    auto KV = [&](int kk, int jj, int ii) { return cadv * a.lv[X.at(kk, jj, ii)]; };
    // kappa of interior z-face equations (zero on the wall rows)
    auto KW = [&](int kk, int jj, int ii) { return (kk >= 1 && kk <= nz - 1) ? cadv * a.lw[X.at(kk, jj, ii)] : 0.0; };
    auto KT = [&](int kk, int jj, int ii) { return (kk >= 1 && kk <= nz - 1) ? cadv * a.lt[X.at(kk, jj, ii)] : 0.0; };
    auto idzc = [&](int kk) { return (kk >= 1 && kk <= nz - 1) ? 1.0 / g.dzc[kk] : 0.0; };
    // volume-weighted transport at (x-face ii or y-face jj, z-face kk)
    auto UW = [&](int kk, int jj, int ii) {
        return (g.dz[kk - 1] * U(kk - 1, jj, ii) + g.dz[kk] * U(kk, jj, ii)) / (2.0 * g.dzc[kk]);
    };
    auto VW = [&](int kk, int jj, int ii) {
        return (g.dz[kk - 1] * V(kk - 1, jj, ii) + g.dz[kk] * V(kk, jj, ii)) / (2.0 * g.dzc[kk]);
    };

    // ================= g_u at (k, j, i) =================
    {
        double s = 0.0;
        // u-eq, x faces at centres i, i-1: F = U^2
        {
            const double L0 = (KU(k, j, i) - KU(k, j, ip)) * idx, U0 = 0.5 * (U(k, j, i) + U(k, j, ip));
            const double L1 = (KU(k, j, im) - KU(k, j, i)) * idx, U1 = 0.5 * (U(k, j, im) + U(k, j, i));
            s += L0 * U0 + L1 * U1;
        }
        // u-eq, y faces j, j+1 (x-face i): Q = avg u
        {
            const double Lj = (KU(k, jm, i) - KU(k, j, i)) * idy;
            const double Lp = (KU(k, j, i) - KU(k, jp, i)) * idy;
            const double Vj = 0.5 * (V(k, j, i) + V(k, j, im));
            const double Vp = 0.5 * (V(k, jp, i) + V(k, jp, im));
            s += 0.5 * (Lj * Vj + Lp * Vp);
        }
        // u-eq, z faces k, k+1 (interior): Q = avg u
        if (k >= 1) {
            const double L = KU(k - 1, j, i) / g.dz[k - 1] - KU(k, j, i) / g.dz[k];
            s += 0.5 * L * 0.5 * (Wf(k, j, i) + Wf(k, j, im));
        }
        if (k + 1 <= nz - 1) {
            const double L = KU(k, j, i) / g.dz[k] - KU(k + 1, j, i) / g.dz[k + 1];
            s += 0.5 * L * 0.5 * (Wf(k + 1, j, i) + Wf(k + 1, j, im));
        }
        // v-eq, x faces at (x-face i, y-faces j and j+1): U = avg of u over y
        {
            const double L0 = (KV(k, j, im) - KV(k, j, i)) * idx, Q0 = 0.5 * (V(k, j, im) + V(k, j, i));
            const double L1 = (KV(k, jp, im) - KV(k, jp, i)) * idx, Q1 = 0.5 * (V(k, jp, im) + V(k, jp, i));
            s += 0.5 * (L0 * Q0 + L1 * Q1);
        }
        // w- and T-eq, x faces at (x-face i, z-faces k and k+1): volume-weighted u
        for (int kf = k; kf <= k + 1; ++kf) {
            if (kf < 1 || kf > nz - 1) continue;
            const double wt = g.dz[k] / (2.0 * g.dzc[kf]);
            const double Lw = (KW(kf, j, im) - KW(kf, j, i)) * idx, Qw = 0.5 * (Wf(kf, j, im) + Wf(kf, j, i));
            const double Lt = (KT(kf, j, im) - KT(kf, j, i)) * idx, Qt = 0.5 * (Tf(kf, j, im) + Tf(kf, j, i));
            s += wt * (Lw * Qw + Lt * Qt);
        }
        // linear terms: horizontal diffusion (symmetric) and Dzz^T = dz Dzz dz^-1
        const double lc = a.lu[id];
        double lin = a.gam * a.nu *
                     ((a.lu[X.at(k, j, ip)] - 2.0 * lc + a.lu[X.at(k, j, im)]) * idx2 +
                      (a.lu[X.at(k, jp, i)] - 2.0 * lc + a.lu[X.at(k, jm, i)]) * idy2);
        {
            const double mc = lc / g.dz[k];
            const double fb = (k > 0) ? (mc - a.lu[X.at(k - 1, j, i)] / g.dz[k - 1]) / g.dzw[k] : mc / g.dzw[0];
            const double ft = (k + 1 < nz) ? (a.lu[X.at(k + 1, j, i)] / g.dz[k + 1] - mc) / g.dzw[k + 1] : -mc / g.dzw[nz];
            lin += a.alp * a.nu * (ft - fb);
        }
        a.gu[id] = a.du[id] + s + a.dt * lin;
    }
    // ================= g_v at (k, j, i) =================
    {
        double s = 0.0;
        {
            const double L0 = (KV(k, j, i) - KV(k, jp, i)) * idy, U0 = 0.5 * (V(k, j, i) + V(k, jp, i));
            const double L1 = (KV(k, jm, i) - KV(k, j, i)) * idy, U1 = 0.5 * (V(k, jm, i) + V(k, j, i));
            s += L0 * U0 + L1 * U1;
        }
        {
            const double Li = (KV(k, j, im) - KV(k, j, i)) * idx;
            const double Lp = (KV(k, j, i) - KV(k, j, ip)) * idx;
            const double Ui = 0.5 * (U(k, j, i) + U(k, jm, i));
            const double Up = 0.5 * (U(k, j, ip) + U(k, jm, ip));
            s += 0.5 * (Li * Ui + Lp * Up);
        }
        if (k >= 1) {
            const double L = KV(k - 1, j, i) / g.dz[k - 1] - KV(k, j, i) / g.dz[k];
            s += 0.5 * L * 0.5 * (Wf(k, j, i) + Wf(k, jm, i));
        }
        if (k + 1 <= nz - 1) {
            const double L = KV(k, j, i) / g.dz[k] - KV(k + 1, j, i) / g.dz[k + 1];
            s += 0.5 * L * 0.5 * (Wf(k + 1, j, i) + Wf(k + 1, jm, i));
        }
        // u-eq, y faces at (x-faces i and i+1, y-face j): V = avg of v over x
        {
            const double L0 = (KU(k, jm, i) - KU(k, j, i)) * idy, Q0 = 0.5 * (U(k, jm, i) + U(k, j, i));
            const double L1 = (KU(k, jm, ip) - KU(k, j, ip)) * idy, Q1 = 0.5 * (U(k, jm, ip) + U(k, j, ip));
            s += 0.5 * (L0 * Q0 + L1 * Q1);
        }
        for (int kf = k; kf <= k + 1; ++kf) {
            if (kf < 1 || kf > nz - 1) continue;
            const double wt = g.dz[k] / (2.0 * g.dzc[kf]);
            const double Lw = (KW(kf, jm, i) - KW(kf, j, i)) * idy, Qw = 0.5 * (Wf(kf, jm, i) + Wf(kf, j, i));
            const double Lt = (KT(kf, jm, i) - KT(kf, j, i)) * idy, Qt = 0.5 * (Tf(kf, jm, i) + Tf(kf, j, i));
            s += wt * (Lw * Qw + Lt * Qt);
        }
        const double lc = a.lv[id];
        double lin = a.gam * a.nu *
                     ((a.lv[X.at(k, j, ip)] - 2.0 * lc + a.lv[X.at(k, j, im)]) * idx2 +
                      (a.lv[X.at(k, jp, i)] - 2.0 * lc + a.lv[X.at(k, jm, i)]) * idy2);
        {
            const double mc = lc / g.dz[k];
            const double fb = (k > 0) ? (mc - a.lv[X.at(k - 1, j, i)] / g.dz[k - 1]) / g.dzw[k] : mc / g.dzw[0];
            const double ft = (k + 1 < nz) ? (a.lv[X.at(k + 1, j, i)] / g.dz[k + 1] - mc) / g.dzw[k + 1] : -mc / g.dzw[nz];
            lin += a.alp * a.nu * (ft - fb);
        }
        a.gv[id] = a.dv[id] + s + a.dt * lin;
    }
    // ================= g_p at (k, j, i):  -dt alpha G^T lambda =================
    {
        double gt = (a.lu[id] - a.lu[X.at(k, j, ip)]) * idx + (a.lv[id] - a.lv[X.at(k, jp, i)]) * idy;
        if (k >= 1) gt += a.lw[id] / g.dzc[k];
        if (k + 1 <= nz - 1) gt -= a.lw[X.at(k + 1, j, i)] / g.dzc[k + 1];
        a.gp[id] = a.dp[id] - a.dt * a.alp * gt;
    }
    // ================= g_w, g_T at z-face k (interior) =================
    if (k == 0) {
        a.gw[id] = 0.0;
        a.gt[id] = 0.0;
    } else {
        double sw = 0.0, st = 0.0;
        // w-eq z faces at centres k and k-1: F = U^2, U = avg w
        {
            const double L0 = KW(k, j, i) * idzc(k) - KW(k + 1, j, i) * idzc(k + 1);
            const double L1 = KW(k - 1, j, i) * idzc(k - 1) - KW(k, j, i) * idzc(k);
            sw += L0 * 0.5 * (Wf(k, j, i) + Wf(k + 1, j, i)) + L1 * 0.5 * (Wf(k - 1, j, i) + Wf(k, j, i));
        }
        // T-eq z faces at centres k and k-1: U = avg w, Q = avg T
        {
            const double L0 = KT(k, j, i) * idzc(k) - KT(k + 1, j, i) * idzc(k + 1);
            const double L1 = KT(k - 1, j, i) * idzc(k - 1) - KT(k, j, i) * idzc(k);
            sw += 0.5 * (L0 * 0.5 * (Tf(k, j, i) + Tf(k + 1, j, i)) + L1 * 0.5 * (Tf(k - 1, j, i) + Tf(k, j, i)));
            st += 0.5 * (L0 * 0.5 * (Wf(k, j, i) + Wf(k + 1, j, i)) + L1 * 0.5 * (Wf(k - 1, j, i) + Wf(k, j, i)));
        }
        // w- and T-eq x faces i, i+1 (transport UW) and y faces j, j+1 (transport VW)
        {
            const double Lw0 = (KW(k, j, im) - KW(k, j, i)) * idx, Lw1 = (KW(k, j, i) - KW(k, j, ip)) * idx;
            const double Lt0 = (KT(k, j, im) - KT(k, j, i)) * idx, Lt1 = (KT(k, j, i) - KT(k, j, ip)) * idx;
            const double U0 = UW(k, j, i), U1 = UW(k, j, ip);
            sw += 0.5 * (Lw0 * U0 + Lw1 * U1);
            st += 0.5 * (Lt0 * U0 + Lt1 * U1);
            const double Mw0 = (KW(k, jm, i) - KW(k, j, i)) * idy, Mw1 = (KW(k, j, i) - KW(k, jp, i)) * idy;
            const double Mt0 = (KT(k, jm, i) - KT(k, j, i)) * idy, Mt1 = (KT(k, j, i) - KT(k, jp, i)) * idy;
            const double V0 = VW(k, j, i), V1 = VW(k, jp, i);
            sw += 0.5 * (Mw0 * V0 + Mw1 * V1);
            st += 0.5 * (Mt0 * V0 + Mt1 * V1);
        }
        // u-eq z faces at (x-faces i, i+1; z-face k): W = avg of w over x, Q = avg of u over z
        {
            const double L0 = KU(k - 1, j, i) / g.dz[k - 1] - KU(k, j, i) / g.dz[k];
            const double L1 = KU(k - 1, j, ip) / g.dz[k - 1] - KU(k, j, ip) / g.dz[k];
            sw += 0.5 * (L0 * 0.5 * (U(k - 1, j, i) + U(k, j, i)) + L1 * 0.5 * (U(k - 1, j, ip) + U(k, j, ip)));
        }
        // v-eq z faces at (y-faces j, j+1; z-face k)
        {
            const double L0 = KV(k - 1, j, i) / g.dz[k - 1] - KV(k, j, i) / g.dz[k];
            const double L1 = KV(k - 1, jp, i) / g.dz[k - 1] - KV(k, jp, i) / g.dz[k];
            sw += 0.5 * (L0 * 0.5 * (V(k - 1, j, i) + V(k, j, i)) + L1 * 0.5 * (V(k - 1, jp, i) + V(k, jp, i)));
        }
        // linear terms
        const double lwc = a.lw[id], ltc = a.lt[id];
        double linw = a.gam * a.nu *
                      ((a.lw[X.at(k, j, ip)] - 2.0 * lwc + a.lw[X.at(k, j, im)]) * idx2 +
                       (a.lw[X.at(k, jp, i)] - 2.0 * lwc + a.lw[X.at(k, jm, i)]) * idy2);
        double lint = a.gam * a.ka *
                      ((a.lt[X.at(k, j, ip)] - 2.0 * ltc + a.lt[X.at(k, j, im)]) * idx2 +
                       (a.lt[X.at(k, jp, i)] - 2.0 * ltc + a.lt[X.at(k, jm, i)]) * idy2);
        {
            // Dzz^T on faces = dzc Dzz dzc^-1 (wall rows of lambda are zero)
            const double mw = lwc * idzc(k), mwm = a.lw[X.at(k - 1, j, i)] * idzc(k - 1),
                         mwp = a.lw[X.at(k + 1, j, i)] * idzc(k + 1);
            const double mt = ltc * idzc(k), mtm = a.lt[X.at(k - 1, j, i)] * idzc(k - 1),
                         mtp = a.lt[X.at(k + 1, j, i)] * idzc(k + 1);
            linw += a.alp * a.nu * ((mwp - mw) / g.dz[k] - (mw - mwm) / g.dz[k - 1]);
            lint += a.alp * a.ka * ((mtp - mt) / g.dz[k] - (mt - mtm) / g.dz[k - 1]);
        }
        a.gw[id] = a.dw[id] + sw + a.dt * linw;
        a.gt[id] = a.dt_[id] + st + a.dt * lint + a.dt * a.gam * lwc;   // buoyancy +T in the w equation
    }
    if (k + 1 == nz) {
        a.gw[id + X.plane] = 0.0;
        a.gt[id + X.plane] = 0.0;
    }
}

hipError_t launch_cn_solve_t(const GridDev& g, int kind, const double* fac, const double* in, double* out,
                             hipStream_t st) {
    hipError_t e;
    if (launch_cn_tiled_t(g, kind, fac, in, out, st, &e)) return e;
    const size_t plane = (size_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_cn_solve_t, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, st, g, kind, fac, in, out);
    return hipGetLastError();
}

hipError_t launch_explicit_adj(const GridDev& g, const SubstepAdjArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_explicit_adj, dim3(stencil_blocks(g)), dim3(kStencilBlock), 0, st, a, g);
    return hipGetLastError();
}

hipError_t launch_explicit(const GridDev& g, const SubstepArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_explicit, dim3(stencil_blocks(g)), dim3(kStencilBlock), 0, st, a, g);
    return hipGetLastError();
}

hipError_t launch_cn_solve_add(const GridDev& g, int kind, const double* fac, double* rhs, double* q,
                               hipStream_t st) {
    hipError_t e;
    if (launch_cn_tiled_add(g, kind, fac, rhs, q, st, &e)) return e;
    const size_t plane = (size_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_cn_solve_add, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, st, g, kind, fac, rhs, q);
    return hipGetLastError();
}

}  // namespace ps
