// Multiple-resolution temperature grid (paper Sec. 6): the temperature lives on a grid that
// refines the momentum grid by integer factors (rx, ry, rz), every momentum cell split into
// rx ry rz equal sub-cells.
//
//   k_mr_prolong    momentum-grid face velocity -> temperature-grid face velocity, one
//                   thread per momentum cell: linear profiles across the coarse faces
//                   (coarse fluxes kept), linear interpolation along the normal inside the
//                   cell, then the local correction G psi, psi = -(L_loc)^+ r, that gives
//                   every sub-cell the divergence of its coarse cell (L_loc: Laplacian of
//                   the cell's sub-cells with closed coarse faces; (L_loc)^+ per coarse
//                   level from the host)
//   k_mr_restrict   temperature -> coarse z-faces: mean over the rx ry fine columns of each
//                   coarse column, at the coarse face's height
//   k_mr_explicit_t explicit terms of the temperature equation on its own grid, with the
//                   advecting velocity interpolated in time between two fine velocity
//                   fields (z-marching over column tiles, as k_explicit)
#include "ps_internal.h"

namespace ps {

// Stores of the prolonged velocity: non-temporal (the fine fields are several times the
// caches and are read again only by the temperature steps; 768^2 x 512: 3.40 -> 3.29 ms).
__device__ __forceinline__ void mr_st(double* p, double v) { __builtin_nontemporal_store(v, p); }

namespace {
__device__ __forceinline__ double sq(double a) { return a * a; }
}  // namespace

// Offsets of the R sub-cell centres from the coarse centre, for a spacing h.
template <int R>
__device__ __forceinline__ double sub_offset(int b, double h) {
    return ((b + 0.5) / R - 0.5) * h;
}

// The fine faces of momentum cell (i, j, k).
template <int RX, int RY, int RZ>
__device__ __forceinline__ void prolong_cell(const double* __restrict__ u, const double* __restrict__ v,
                                             const double* __restrict__ w, double* __restrict__ uf,
                                             double* __restrict__ vf, double* __restrict__ wf, const GridDev& g,
                                             const MrDev& m, int i, int j, int k) {
    constexpr int NS = RX * RY * RZ;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t plane = (size_t)nx * ny;
    const int im = (i == 0) ? nx - 1 : i - 1, ip = (i + 1 == nx) ? 0 : i + 1;
    const int jm = (j == 0) ? ny - 1 : j - 1, jp = (j + 1 == ny) ? 0 : j + 1;
    const bool lo = k > 0, hi = k + 1 < nz;
    const int km = lo ? k - 1 : k, kp = hi ? k + 1 : k;
    auto at = [&](int kk, int jj, int ii) { return (size_t)kk * plane + (size_t)jj * nx + ii; };
    // coarse faces of this cell and the neighbours of each across it (all loads unconditional)
    const double uL = u[at(k, j, i)], uLyp = u[at(k, jp, i)], uLym = u[at(k, jm, i)], uLzm = u[at(km, j, i)],
                 uLzp = u[at(kp, j, i)];
    const double uR = u[at(k, j, ip)], uRyp = u[at(k, jp, ip)], uRym = u[at(k, jm, ip)], uRzm = u[at(km, j, ip)],
                 uRzp = u[at(kp, j, ip)];
    const double vF = v[at(k, j, i)], vFxp = v[at(k, j, ip)], vFxm = v[at(k, j, im)], vFzm = v[at(km, j, i)],
                 vFzp = v[at(kp, j, i)];
    const double vB = v[at(k, jp, i)], vBxp = v[at(k, jp, ip)], vBxm = v[at(k, jp, im)], vBzm = v[at(km, jp, i)],
                 vBzp = v[at(kp, jp, i)];
    const double wD = w[at(k, j, i)], wDxp = w[at(k, j, ip)], wDxm = w[at(k, j, im)], wDyp = w[at(k, jp, i)],
                 wDym = w[at(k, jm, i)];
    const double wU = w[at(k + 1, j, i)], wUxp = w[at(k + 1, j, ip)], wUxm = w[at(k + 1, j, im)],
                 wUyp = w[at(k + 1, jp, i)], wUym = w[at(k + 1, jm, i)];
    anchor(uL); anchor(uLyp); anchor(uLym); anchor(uLzm); anchor(uLzp);
    anchor(uR); anchor(uRyp); anchor(uRym); anchor(uRzm); anchor(uRzp);
    anchor(vF); anchor(vFxp); anchor(vFxm); anchor(vFzm); anchor(vFzp);
    anchor(vB); anchor(vBxp); anchor(vBxm); anchor(vBzm); anchor(vBzp);
    anchor(wD); anchor(wDxp); anchor(wDxm); anchor(wDyp); anchor(wDym);
    anchor(wU); anchor(wUxp); anchor(wUxm); anchor(wUyp); anchor(wUym);
    // wall-normal slopes at the coarse centre: three-point formula, the no-slip wall value 0
    // at the wall as the outer point
    // Every quotient below divides by one of a few spacings: one reciprocal each, then
    // products (an FP64 quotient costs about ten VALU instructions, a product one)
    const double hm = m.zhm[k], hp = m.zhp[k];
    const double izs = 1.0 / (hm * hp * (hm + hp)), ix2 = 0.5 / g.dx, iy2 = 0.5 / g.dy;
    auto zsl = [&](double qm, double qc, double qp) {
        qm = lo ? qm : 0.0;
        qp = hi ? qp : 0.0;
        return (hm * hm * (qp - qc) + hp * hp * (qc - qm)) * izs;
    };
    const double syL = (uLyp - uLym) * iy2, szL = zsl(uLzm, uL, uLzp);
    const double syR = (uRyp - uRym) * iy2, szR = zsl(uRzm, uR, uRzp);
    const double sxF = (vFxp - vFxm) * ix2, szF = zsl(vFzm, vF, vFzp);
    const double sxB = (vBxp - vBxm) * ix2, szB = zsl(vBzm, vB, vBzp);
    const double sxD = (wDxp - wDxm) * ix2, syD = (wDyp - wDym) * iy2;
    const double sxU = (wUxp - wUxm) * ix2, syU = (wUyp - wUym) * iy2;
    const double dzk = g.dz[k];
    double ex[RX], ey[RY], ez[RZ];
#pragma unroll
    for (int a = 0; a < RX; ++a) ex[a] = sub_offset<RX>(a, g.dx);
#pragma unroll
    for (int b = 0; b < RY; ++b) ey[b] = sub_offset<RY>(b, g.dy);
#pragma unroll
    for (int c = 0; c < RZ; ++c) ez[c] = sub_offset<RZ>(c, dzk);
    // fine face values: fu[a][b][c] on the x-faces a = 0..RX of the cell (0, RX: coarse faces)
    double fu[RX + 1][RY][RZ], fv[RX][RY + 1][RZ], fw[RX][RY][RZ + 1];
#pragma unroll
    for (int b = 0; b < RY; ++b)
#pragma unroll
        for (int c = 0; c < RZ; ++c) {
            fu[0][b][c] = uL + syL * ey[b] + szL * ez[c];
            fu[RX][b][c] = uR + syR * ey[b] + szR * ez[c];
#pragma unroll
            for (int a = 1; a < RX; ++a)
                fu[a][b][c] = (1 - (double)a / RX) * fu[0][b][c] + ((double)a / RX) * fu[RX][b][c];
        }
#pragma unroll
    for (int a = 0; a < RX; ++a)
#pragma unroll
        for (int c = 0; c < RZ; ++c) {
            fv[a][0][c] = vF + sxF * ex[a] + szF * ez[c];
            fv[a][RY][c] = vB + sxB * ex[a] + szB * ez[c];
#pragma unroll
            for (int b = 1; b < RY; ++b)
                fv[a][b][c] = (1 - (double)b / RY) * fv[a][0][c] + ((double)b / RY) * fv[a][RY][c];
        }
#pragma unroll
    for (int a = 0; a < RX; ++a)
#pragma unroll
        for (int b = 0; b < RY; ++b) {
            fw[a][b][0] = wD + sxD * ex[a] + syD * ey[b];
            fw[a][b][RZ] = wU + sxU * ex[a] + syU * ey[b];
#pragma unroll
            for (int c = 1; c < RZ; ++c)
                fw[a][b][c] = (1 - (double)c / RZ) * fw[a][b][0] + ((double)c / RZ) * fw[a][b][RZ];
        }
    if constexpr (NS > 1) {
        // sub-cell divergences, then psi = (L_loc)^+ r and the correction -(G psi) on the
        // interior faces; sub-cell (a, b, c) has index (c RY + b) RX + a
        const double ixf = 1.0 / m.dxf, iyf = 1.0 / m.dyf;
        double izf[RZ];
#pragma unroll
        for (int c = 0; c < RZ; ++c) izf[c] = 1.0 / m.dzf[k * RZ + c];
        double r[NS];
#pragma unroll
        for (int c = 0; c < RZ; ++c) {
#pragma unroll
            for (int b = 0; b < RY; ++b)
#pragma unroll
                for (int a = 0; a < RX; ++a)
                    r[(c * RY + b) * RX + a] = ((fu[a + 1][b][c] - fu[a][b][c]) * ixf +
                                                (fv[a][b + 1][c] - fv[a][b][c]) * iyf) +
                                               (fw[a][b][c + 1] - fw[a][b][c]) * izf[c];
        }
        const double* L = m.linv + (size_t)k * NS * NS;   // uniform per block: scalar loads
        double psi[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < NS; ++t) acc += L[s * NS + t] * r[t];
            psi[s] = acc;
        }
#pragma unroll
        for (int c = 0; c < RZ; ++c)
#pragma unroll
            for (int b = 0; b < RY; ++b)
#pragma unroll
                for (int a = 1; a < RX; ++a)
                    fu[a][b][c] -= (psi[(c * RY + b) * RX + a] - psi[(c * RY + b) * RX + a - 1]) * ixf;
#pragma unroll
        for (int c = 0; c < RZ; ++c)
#pragma unroll
            for (int b = 1; b < RY; ++b)
#pragma unroll
                for (int a = 0; a < RX; ++a)
                    fv[a][b][c] -= (psi[(c * RY + b) * RX + a] - psi[(c * RY + b - 1) * RX + a]) * iyf;
#pragma unroll
        for (int c = 1; c < RZ; ++c) {
            // sub-cells of one coarse cell: equal heights, so the face spacing is the height
#pragma unroll
            for (int b = 0; b < RY; ++b)
#pragma unroll
                for (int a = 0; a < RX; ++a)
                    fw[a][b][c] -= (psi[(c * RY + b) * RX + a] - psi[((c - 1) * RY + b) * RX + a]) * izf[c];
        }
    }
    // this cell's faces of the fine grid: its lower x, y and z coarse faces and the interior ones
    const size_t NX = (size_t)nx * RX, NYX = NX * (size_t)(ny * RY);
#pragma unroll
    for (int c = 0; c < RZ; ++c)
#pragma unroll
        for (int b = 0; b < RY; ++b) {
            const size_t row = (size_t)(k * RZ + c) * NYX + (size_t)(j * RY + b) * NX + (size_t)i * RX;
#pragma unroll
            for (int a = 0; a < RX; ++a) {
                mr_st(uf + row + a, fu[a][b][c]);
                mr_st(vf + row + a, fv[a][b][c]);
                mr_st(wf + row + a, fw[a][b][c]);
            }
        }
    if (!hi) {
#pragma unroll
        for (int b = 0; b < RY; ++b) {
            const size_t row = (size_t)(nz * RZ) * NYX + (size_t)(j * RY + b) * NX + (size_t)i * RX;
#pragma unroll
            for (int a = 0; a < RX; ++a) mr_st(wf + row + a, fw[a][b][RZ]);
        }
    }
}

// One block per run of kMrPx consecutive x of one (y, z) row of momentum cells, one thread per
// cell (128-thread runs leave no thread idle at nx = 384 or 768, where 256-thread runs left a
// quarter idle); neighbouring y rows of one z level are numbered to run on one XCD.
constexpr int kMrPx = 128;
template <int RX, int RY, int RZ>
__global__ void __launch_bounds__(kMrPx)
k_mr_prolong(const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
             double* __restrict__ uf, double* __restrict__ vf, double* __restrict__ wf, GridDev g, MrDev m) {
    int r = xcd_remap(blockIdx.x, gridDim.x);
    const int nxs = (g.nx + kMrPx - 1) / kMrPx;
    const int xs = r % nxs;
    r /= nxs;
    const int j = r % g.ny, k = r / g.ny;
    const int i = xs * kMrPx + (int)threadIdx.x;
    if (i >= g.nx) return;
    prolong_cell<RX, RY, RZ>(u, v, w, uf, vf, wf, g, m, i, j, k);
}

// tc[k][j][i] = mean of tf[rz k][ry j + b][rx i + a], k = 0..nz (one thread per coarse face point)
__global__ void __launch_bounds__(256)
k_mr_restrict(const double* __restrict__ tf, double* __restrict__ tc, int nx, int ny, int nz, int rx, int ry,
              int rz) {
    const size_t n = (size_t)nx * ny * (nz + 1);
    const size_t id = (size_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = (int)(id % nx);
    const size_t r = id / nx;
    const int j = (int)(r % ny);
    const int k = (int)(r / ny);
    const size_t NX = (size_t)nx * rx, NY = (size_t)ny * ry;
    const double* base = tf + (size_t)k * rz * NX * NY + (size_t)j * ry * NX + (size_t)i * rx;
    double s = 0.0;
    for (int b = 0; b < ry; ++b)
        for (int a = 0; a < rx; ++a) s += base[(size_t)b * NX + a];
    tc[id] = s / (double)(rx * ry);
}

// ---- explicit terms of the temperature equation on its own grid ------------------------
// z-marching over 64 x 4 column tiles with a three-plane LDS ring of u, v, w, T (the velocity
// staged as (1 - th) vel0 + th vel1), as in k_explicit.  Writes the Crank-Nicolson input
// rt = C T + dt [gamma H + rho Hprev + alpha kappa Dzz T] on interior faces (C = I - bka Dzz~,
// Dzz~ with zero wall values; walls 0, never read by the solve), or the bracket alone when
// cq = 0 (bka is then 0 too), and H (optional).
// (64 x 4 against 32 x 8 and 16 x 16 for the coupled step at 768^2 x 512: 48.9 / 49.4 / 51.5 ms)
constexpr int kMtTX = 64, kMtTY = 4, kMtZSEG = 64;

template <int NF, int TX, int TY>
struct MtRing {
    static constexpr int HX = TX + 2, HY = TY + 2, PL = HX * HY;
    static constexpr int NQ = (PL + TX * TY - 1) / (TX * TY);
    double* s;
    int tx, ty;
    __device__ __forceinline__ static int slot(int kk) { return (kk + 3) % 3; }
    __device__ __forceinline__ double operator()(int k, int f, int dk, int dj, int di) const {
        return s[(slot(k + dk) * NF + f) * PL + (ty + 1 + dj) * HX + (tx + 1 + di)];
    }
};

__global__ void __launch_bounds__(kMtTX * kMtTY) k_mr_explicit_t(MrTArgs a, GridDev g) {
    constexpr int TX = kMtTX, TY = kMtTY, NF = 4;
    using RingT = MtRing<NF, TX, TY>;
    constexpr int NQ = RingT::NQ, PL = RingT::PL, HX = RingT::HX;
    enum { FU, FV, FW, FT };
    __shared__ double lds[3 * NF * PL];
    const int nxt = (g.nx + TX - 1) / TX, nyt = (g.ny + TY - 1) / TY;
    int rb = xcd_remap(blockIdx.x, gridDim.x);
    const int xt = rb % nxt;
    rb /= nxt;
    const int yt = rb % nyt;
    const int zs = rb / nyt;
    const int i0 = xt * TX, j0 = yt * TY, kb = zs * kMtZSEG, ke = min(g.nz, kb + kMtZSEG);
    RingT R{lds, (int)threadIdx.x % TX, (int)threadIdx.x / TX};
    const int i = i0 + R.tx, j = j0 + R.ty;
    const bool valid = i < g.nx && j < g.ny;
    const size_t plane = (size_t)g.nx * g.ny;
    // periodic column offsets of this thread's halo cells (the same for every plane), and which
    // of them each velocity component is read at: u at x offsets 0 and +1 of its own row, v at
    // y offsets 0 and +1 of its own column, w in its own column only (T at every halo cell).
    // The others are not loaded (their ring entries stay zero and are never read), so that the
    // cache lines only the halo touches are fetched for T alone.
    unsigned off[NQ];
    bool need_u[NQ], need_v[NQ], need_w[NQ];
#pragma unroll
    for (int qi = 0; qi < NQ; ++qi) {
        const int q = min((int)threadIdx.x + qi * TX * TY, PL - 1);
        const int hy = q / HX, hx = q - hy * HX;
        int gj = j0 - 1 + hy, gi = i0 - 1 + hx;
        gj = gj < 0 ? gj + g.ny : gj % g.ny;
        gi = gi < 0 ? gi + g.nx : gi % g.nx;
        off[qi] = (unsigned)gj * (unsigned)g.nx + (unsigned)gi;
        const bool in_x = hx >= 1 && hx <= TX, in_y = hy >= 1 && hy <= TY;
        need_u[qi] = in_y && hx >= 1;
        need_v[qi] = in_x && hy >= 1;
        need_w[qi] = in_x && in_y;
    }
    const double th = a.th, th1 = 1.0 - a.th;
    // plane kk of every field into registers, both velocity time levels as loaded; put()
    // blends them in time and zeroes absent planes (uniform flags) into the ring, so that the
    // loads of a stage are not waited for until the next step
    double s0[NQ][3], s1[NQ][3], stt[NQ];
    bool okc = false, okf = false;
    auto fetch = [&](int kk) {
        const int kc = kk < 0 ? 0 : (kk > g.nz - 1 ? g.nz - 1 : kk);
        const int kf = kk < 0 ? 0 : (kk > g.nz ? g.nz : kk);
        okc = kk >= 0 && kk < g.nz;
        okf = kk >= 0 && kk <= g.nz;
        const size_t pc = (size_t)kc * plane, pf = (size_t)kf * plane;
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
            const size_t oc = pc + off[qi], of = pf + off[qi];
            s0[qi][FU] = s1[qi][FU] = s0[qi][FV] = s1[qi][FV] = s0[qi][FW] = s1[qi][FW] = 0.0;
            if (need_u[qi]) {
                s0[qi][FU] = a.u0[oc];
                s1[qi][FU] = a.u1[oc];
            }
            if (need_v[qi]) {
                s0[qi][FV] = a.v0[oc];
                s1[qi][FV] = a.v1[oc];
            }
            if (need_w[qi]) {
                s0[qi][FW] = a.w0[of];
                s1[qi][FW] = a.w1[of];
            }
            stt[qi] = a.t[of];
        }
    };
    auto put = [&](int kk) {
        const int sl = RingT::slot(kk);
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
            const int q = (int)threadIdx.x + qi * TX * TY;
            if (q < PL) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const bool ok = f == FW ? okf : okc;
                    lds[(sl * NF + f) * PL + q] = ok ? th1 * s0[qi][f] + th * s1[qi][f] : 0.0;
                }
                lds[(sl * NF + FT) * PL + q] = okf ? stt[qi] : 0.0;
            }
        }
    };
    // the segment's grid metrics (cell planes kb - 1 .. ke, face planes kb .. ke + 1) in LDS:
    // a global load inside a step would make the wave wait for the next plane's prefetch too
    constexpr int ZT = kMtZSEG + 2;
    __shared__ double m_idz[ZT], m_dz[ZT], m_o[ZT];
    for (int q = threadIdx.x; q < ZT; q += TX * TY) {
        const int kc = min(max(kb - 1 + q, 0), g.nz - 1), kf = min(kb + q, g.nz);
        m_idz[q] = g.idz[kc];
        m_dz[q] = g.dz[kc];
        m_o[q] = g.o[kf];
    }
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double idx2 = idx * idx, idy2 = idy * idy;
    const int nz = g.nz;
    fetch(kb - 1);
    put(kb - 1);
    fetch(kb);
    put(kb);
    fetch(kb + 1);
    for (int k = kb; k < ke; ++k) {
        put(k + 1);
        __syncthreads();
        const size_t id = (size_t)k * plane + (size_t)j * g.nx + i;
        // previous H (substep 1 reads T's first value, one cache line for every lane, in its place
        // and drops it), then the next plane's prefetch, both unconditional (the last step
        // fetches a clamped plane it never stores)
        const double hp = (a.rho != 0.0 ? a.hp : a.t)[a.rho != 0.0 ? (valid ? id : (size_t)k * plane) : 0];
        asm volatile("" ::: "memory");
        fetch(k + 2);
        if (valid) {
            auto L = [&](int f, int dk, int dj, int di) { return R(k, f, dk, dj, di); };
            if (k == 0) {
                a.rt[id] = 0.0;
                if (a.hout) a.hout[id] = 0.0;
            } else {
                const int mq = k - kb;   // tables: cell plane k - 1 at mq, face k at mq
                const double dzm = m_dz[mq], dzp = m_dz[mq + 1], den = 0.5 * m_o[mq];
                const double uwl = (dzm * L(FU, -1, 0, 0) + dzp * L(FU, 0, 0, 0)) * den;
                const double uwr = (dzm * L(FU, -1, 0, 1) + dzp * L(FU, 0, 0, 1)) * den;
                const double vwb = (dzm * L(FV, -1, 0, 0) + dzp * L(FV, 0, 0, 0)) * den;
                const double vwt = (dzm * L(FV, -1, 1, 0) + dzp * L(FV, 0, 1, 0)) * den;
                const double wc = L(FW, 0, 0, 0), wkm = L(FW, -1, 0, 0), wkp = L(FW, 1, 0, 0);
                const double tc = L(FT, 0, 0, 0), tim = L(FT, 0, 0, -1), tip = L(FT, 0, 0, 1);
                const double tjm = L(FT, 0, -1, 0), tjp = L(FT, 0, 1, 0);
                const double tkm = L(FT, -1, 0, 0), tkp = L(FT, 1, 0, 0);
                const double idzc = m_o[mq];
                const double wtop = 0.5 * (wc + wkp), wbot = 0.5 * (wkm + wc);
                const double ax = (uwr * (0.5 * (tc + tip)) - uwl * (0.5 * (tim + tc))) * idx;
                const double ay = (vwt * (0.5 * (tc + tjp)) - vwb * (0.5 * (tjm + tc))) * idy;
                const double az = (wtop * (0.5 * (tc + tkp)) - wbot * (0.5 * (tkm + tc))) * idzc;
                const double h = -(ax + ay + az) + a.ka * ((tip - 2.0 * tc + tim) * idx2 + (tjp - 2.0 * tc + tjm) * idy2);
                const double dzz = ((tkp - tc) * m_idz[mq + 1] - (tc - tkm) * m_idz[mq]) * idzc;
                const double dzh = dzz - (k == 1 ? tkm * m_idz[mq] * idzc : 0.0) -
                                   (k + 1 == nz ? tkp * m_idz[mq + 1] * idzc : 0.0);
                double r = a.gam * h + a.alp * (a.ka * dzz);
                if (a.rho != 0.0) r += a.rho * hp;
                const double rr = a.dt * r - a.bka * dzh;
                __builtin_nontemporal_store(a.cq ? tc + rr : rr, a.rt + id);
                if (a.hout) __builtin_nontemporal_store(h, a.hout + id);
            }
            if (k + 1 == nz) {
                a.rt[id + plane] = 0.0;
                if (a.hout) a.hout[id + plane] = 0.0;
            }
        }
        __syncthreads();
    }
}

// ---- launchers ------------------------------------------------------------------------------
bool mr_factors_supported(int rx, int ry, int rz) {
    return rx >= 1 && rx <= 2 && ry >= 1 && ry <= 2 && rz >= 1 && rz <= 2;
}

hipError_t launch_mr_prolong(const GridDev& g, const MrDev& m, const double* u, const double* v, const double* w,
                             double* uf, double* vf, double* wf, hipStream_t st) {
    const int nxs = (g.nx + kMrPx - 1) / kMrPx;
    const dim3 grid((unsigned)nxs * (unsigned)g.ny * (unsigned)g.nz), block(kMrPx);
#define PS_MR_CASE(X, Y, Z)                                                                          \
    if (m.rx == X && m.ry == Y && m.rz == Z) {                                                       \
        hipLaunchKernelGGL((k_mr_prolong<X, Y, Z>), grid, block, 0, st, u, v, w, uf, vf, wf, g, m); \
        return hipGetLastError();                                                                    \
    }
    PS_MR_CASE(1, 1, 1)
    PS_MR_CASE(2, 1, 1)
    PS_MR_CASE(1, 2, 1)
    PS_MR_CASE(2, 2, 1)
    PS_MR_CASE(1, 1, 2)
    PS_MR_CASE(2, 1, 2)
    PS_MR_CASE(1, 2, 2)
    PS_MR_CASE(2, 2, 2)
#undef PS_MR_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_mr_restrict(const GridDev& g, const MrDev& m, const double* tf, double* tc, hipStream_t st) {
    const size_t n = (size_t)g.nx * g.ny * (g.nz + 1);
    hipLaunchKernelGGL(k_mr_restrict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tf, tc, g.nx, g.ny, g.nz,
                       m.rx, m.ry, m.rz);
    return hipGetLastError();
}

hipError_t launch_mr_explicit_t(const GridDev& gf, const MrTArgs& a, hipStream_t st) {
    const int nblk = ((gf.nx + kMtTX - 1) / kMtTX) * ((gf.ny + kMtTY - 1) / kMtTY) * ((gf.nz + kMtZSEG - 1) / kMtZSEG);
    hipLaunchKernelGGL(k_mr_explicit_t, dim3(nblk), dim3(kMtTX * kMtTY), 0, st, a, gf);
    return hipGetLastError();
}

}  // namespace ps
