// One RK3 / Crank-Nicolson substep (paper Sec. 2.1) and its adjoint.
//
// Forward, substep l with coefficients gamma, rho, alpha = gamma + rho:
//   H_q   = -A(q) + nu (Dxx + Dyy) q   (+ T on w; kappa for T)
//   rhs_q = dt [gamma H_q + rho H_q^prev - alpha G_q p + alpha nu Dzz q]
//   (I - alpha dt nu/2 Dzz) dq = rhs_q, q* = q + dq
// The explicit kernel writes s_q = C q + rhs_q with C = I - alpha dt nu/2 Dzz~ (Dzz~: Dzz
// with zero wall values, the operator of the Crank-Nicolson rows), so that the solve is
// q* = C^-1 s_q: the same q* = q + C^-1 rhs_q, but the solve reads one field and writes
// one instead of reading two (8 B per point and field less).  Its rounding is relative to q,
// not to the increment, so when C is far from the identity (large beta over fine wall
// cells) the kernel writes rhs_q itself and the solve adds (cq = 0).
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

__device__ __forceinline__ double sq(double a) { return a * a; }

// Stores of the explicit kernels' outputs (right-hand sides, H, gradients): each is read
// again only by a later kernel, after far more data than the caches hold has passed.
#ifndef PS_EX_NT_STORE
#define PS_EX_NT_STORE 1
#endif
__device__ __forceinline__ void st_out(double* p, double v) {
    if (PS_EX_NT_STORE)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Buffer accesses of one plane: the base (a field's plane, the same for the whole block) in
// scalar registers and the lane's byte offset in one vector register, so that no per-access
// 64-bit address arithmetic is spent (the plane offsets stay below 2^31 bytes).
using u32x2_t = vec2_t<unsigned int>;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const double* base, size_t plane) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(plane * sizeof(double)), 0x00020000);
}
__device__ __forceinline__ double ld_plane(__amdgpu_buffer_rsrc_t r, unsigned boff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)boff, 0, 0));
}
__device__ __forceinline__ void st_plane(double* base, size_t plane, unsigned boff, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), plane_rsrc(base, plane), (int)boff, 0,
                                          PS_EX_NT_STORE ? 2 : 0);   // 2: the non-temporal hint
}

}  // namespace



// ---------------------------------------------------------------------------
// z-marching stencil blocks.  A block owns a TX x TY tile of (x, y) columns and a
// segment of ZSEG planes; it keeps three consecutive z-planes (k-1, k, k+1) of its
// NF stencil fields in LDS, each as a (TY + 2) x (TX + 2) tile with a one-cell
// periodic halo, and walks up the segment loading one new plane per step.  Every
// field value is read from memory about once (plus the halo and two planes per
// segment), and neighbour reads are LDS reads.
template <int NF, int TX, int TY>
struct Ring {
    static constexpr int HX = TX + 2, HY = TY + 2, PL = HX * HY;
    double* s;   // [3][NF][PL]
    int tx, ty;
    __device__ __forceinline__ static int slot(int kk) { return (kk + 3) % 3; }
    // field f at (k + dk, j + dj, i + di) of this thread's cell
    __device__ __forceinline__ double operator()(int k, int f, int dk, int dj, int di) const {
        return s[(slot(k + dk) * NF + f) * PL + (ty + 1 + dj) * HX + (tx + 1 + di)];
    }
    // Plane kk of every field, staged through registers so that the loads of a later
    // plane are in flight while the current one is computed: fetch() issues the loads
    // (zeros where a field has no such plane: centre fields have planes 0..nz-1, face
    // fields 0..nz), put() stores them into the plane's LDS slot.  Each thread copies the
    // halo cells q = thread + qi * TX * TY; their (periodic) column offsets are the same
    // for every plane and are formed once by columns().
    static constexpr int NQ = (PL + TX * TY - 1) / (TX * TY);
    struct Stage {
        double v[NQ][NF];
    };
    struct Cols {
        unsigned off[NQ];    // j * nx + i of the halo cell (a cell inside the tile for q >= PL)
        unsigned boff[NQ];   // the same in bytes
    };
    __device__ __forceinline__ static Cols columns(const GridDev& g, int i0, int j0) {
        Cols c;
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
            const int q = min((int)threadIdx.x + qi * TX * TY, PL - 1);
            const int hy = q / HX, hx = q - hy * HX;
            int gj = j0 - 1 + hy, gi = i0 - 1 + hx;
            gj = gj < 0 ? gj + g.ny : gj % g.ny;
            gi = gi < 0 ? gi + g.nx : gi % g.nx;
            c.off[qi] = (unsigned)gj * (unsigned)g.nx + (unsigned)gi;
            c.boff[qi] = c.off[qi] * (unsigned)sizeof(double);
        }
        return c;
    }
    // Every load is unconditional (plane index clamped into the field) and absent values
    // are zeroed by a select, so that all of the stage's loads are in flight together.
    __device__ __forceinline__ void fetch(int kk, const double* const (&F)[NF], const bool (&face)[NF],
                                          const GridDev& g, const Cols& cols, Stage& st) const {
        const size_t plane = (size_t)g.nx * g.ny;
        const int kc = kk < 0 ? 0 : (kk > g.nz - 1 ? g.nz - 1 : kk);
        const int kf = kk < 0 ? 0 : (kk > g.nz ? g.nz : kk);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const bool ok = kk >= 0 && (kk < g.nz || (face[f] && kk == g.nz));
            const double* base = F[f] + (size_t)(face[f] ? kf : kc) * plane;
#pragma unroll
            for (int qi = 0; qi < NQ; ++qi) {
                const double v = base[cols.off[qi]];
                st.v[qi][f] = ok ? v : 0.0;
            }
        }
    }
    __device__ __forceinline__ void put(int kk, const Stage& st) {
        const int sl = slot(kk);
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
            const int q = (int)threadIdx.x + qi * TX * TY;
            if (q < PL) {
#pragma unroll
                for (int f = 0; f < NF; ++f) s[(sl * NF + f) * PL + q] = st.v[qi][f];
            }
        }
    }
};

// The same z-marching scheme with a window of its own depth for each field: field f keeps
// Win::ns(f) consecutive planes (1 to 3) in LDS, so that a field whose neighbours are
// needed on fewer planes takes less LDS (and more blocks fit one CU).  Values on the
// thread's own column below the window are carried in registers by the kernel.
template <int TX, int TY, class Win>
struct WinRing {
    static constexpr int NF = Win::NF;
    static constexpr int HX = TX + 2, HY = TY + 2, PL = HX * HY;
    static constexpr int NQ = (PL + TX * TY - 1) / (TX * TY);
    static constexpr int base(int f) { return f == 0 ? 0 : base(f - 1) + Win::ns(f - 1); }
    static constexpr int PLANES = base(NF);
    double* s;        // PLANES planes of PL cells
    int tx, ty;
    __device__ __forceinline__ static int slot(int f, int kk) {
        const int n = Win::ns(f);
        return base(f) + (n == 1 ? 0 : ((kk % n) + n) % n);
    }
    // field f at plane kk, (j + dj, i + di) of this thread's cell
    __device__ __forceinline__ double at(int f, int kk, int dj, int di) const {
        return s[slot(f, kk) * PL + (ty + 1 + dj) * HX + (tx + 1 + di)];
    }
    // raw loaded values and, per field, whether the plane exists (uniform): the zeroing of
    // absent planes waits for put(), so that no value is touched (and waited for) before
    // the next step's stores into the ring
    struct Stage {
        double v[NQ][NF];
        bool ok[NF];
    };
    using Cols = typename Ring<Win::NF, TX, TY>::Cols;
    // plane kk[f] of field f for the fields with want[f] (the others keep their values)
    __device__ __forceinline__ void fetch(const int (&kk)[NF], const bool (&want)[NF], const double* const (&F)[NF],
                                          const bool (&face)[NF], const GridDev& g, const Cols& cols,
                                          Stage& st) const {
        const size_t plane = (size_t)g.nx * g.ny;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (!want[f]) continue;
            const int k = kk[f];
            const int kc = k < 0 ? 0 : (k > g.nz - 1 ? g.nz - 1 : k);
            const int kf = k < 0 ? 0 : (k > g.nz ? g.nz : k);
            st.ok[f] = k >= 0 && (k < g.nz || (face[f] && k == g.nz));
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(F[f] + (size_t)(face[f] ? kf : kc) * plane, plane);
#pragma unroll
            for (int qi = 0; qi < NQ; ++qi) st.v[qi][f] = ld_plane(rs, cols.boff[qi]);
        }
    }
    __device__ __forceinline__ void put(const int (&kk)[NF], const bool (&want)[NF], const Stage& st) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (!want[f]) continue;
            double* d = s + slot(f, kk[f]) * PL;
#pragma unroll
            for (int qi = 0; qi < NQ; ++qi) {
                const int q = (int)threadIdx.x + qi * TX * TY;
                if (q < PL) d[q] = st.ok[f] ? st.v[qi][f] : 0.0;
            }
        }
    }
};

// Column tile of the forward kernel: 32 x 8 (halo 1.33 cells per cell, 40.8 KB of LDS: four
// blocks fit one CU's 160 KB) measured 7.60 -> 6.9-7.1 ms against 64 x 4 at 768^2 x 512; 16 x 16:
// 7.24 ms.  The adjoint's eight-field ring keeps 64 x 4 (32 x 8 measured the same).
#ifndef PS_EX_TX
#define PS_EX_TX 32
#endif
#ifndef PS_EX_TY
#define PS_EX_TY 8
#endif
constexpr int kExTX = PS_EX_TX, kExTY = PS_EX_TY, kExZSEG = 64;

// Block -> (x tile, y tile, z segment), x tile fastest so that neighbouring y tiles
// (which share halo rows) run together on one XCD.
struct ExTile {
    int i0, j0, kb, ke;
};
template <int TX, int TY, int ZSEG>
__device__ __forceinline__ ExTile ex_tile(const GridDev& g) {
    const int nxt = (g.nx + TX - 1) / TX, nyt = (g.ny + TY - 1) / TY;
    int r = xcd_remap(blockIdx.x, gridDim.x);
    const int xt = r % nxt;
    r /= nxt;
    const int yt = r % nyt;
    const int zs = r / nyt;
    ExTile t;
    t.i0 = xt * TX;
    t.j0 = yt * TY;
    t.kb = zs * ZSEG;
    t.ke = min(g.nz, t.kb + ZSEG);
    return t;
}
template <int TX, int TY, int ZSEG>
inline int ex_blocks(const GridDev& g) {
    return ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + ZSEG - 1) / ZSEG);
}

// Crank-Nicolson inputs s_q = C q + rhs_q of u, v at the cell's x/y faces and of w, T at
// its bottom z-face k (interior faces; wall rows are zeroed and never read by the solve).
//
// Windows (step k computes u, v of cell plane k and w, T of its bottom face k): u and v
// are read with neighbours on planes k - 1 (by the face terms) and k, and on their own
// column at k + 1; w with neighbours on faces k and k + 1; T and p with neighbours on
// plane k only.  So u, v keep planes k-1..k+1, w and T faces k..k+1, p plane k: 11 planes
// of LDS instead of 15 (29.9 KB for a 32 x 8 tile: five blocks per CU instead of three).
// The own-column values of w, T, p at k - 1 are the previous step's centre values, carried
// in registers.
struct ExWin {
    static constexpr int NF = 5;   // u, v, w, T, p
    __host__ __device__ static constexpr int ns(int f) { return f < 2 ? 3 : (f < 4 ? 2 : 1); }
};
// Waves per SIMD the register allocation must allow (0: no cap).
#ifndef PS_EX_WPE
#define PS_EX_WPE 0
#endif
#ifndef PS_EX_SPLIT
#define PS_EX_SPLIT 1
#endif
#if PS_EX_SPLIT
#define PS_EX_FENCE() asm volatile("" ::: "memory")
#else
#define PS_EX_FENCE() ((void)0)
#endif
#if PS_EX_WPE > 0
#define PS_EX_ATTR __attribute__((amdgpu_waves_per_eu(PS_EX_WPE)))
#else
#define PS_EX_ATTR
#endif
__global__ void __launch_bounds__(kExTX * kExTY) PS_EX_ATTR k_explicit(SubstepArgs a, GridDev g) {
    constexpr int TX = kExTX, TY = kExTY, NF = ExWin::NF;
    enum { FU, FV, FW, FT, FP };
    using RR = WinRing<TX, TY, ExWin>;
    static_assert(RR::PLANES == 11, "window planes");
    __shared__ double lds[RR::PLANES * RR::PL];
    // the segment's grid metrics: LDS reads, so that no global load inside a step makes the
    // wave wait for the next plane's prefetch (a vector-memory wait counts every load)
    constexpr int ZT = kExZSEG + 1;
    __shared__ double m_idz[ZT], m_dz[ZT], m_idzw[ZT], m_o[ZT];
    const ExTile tile = ex_tile<TX, TY, kExZSEG>(g);
    RR R{lds, (int)threadIdx.x % TX, (int)threadIdx.x / TX};
    for (int q = threadIdx.x; q < ZT; q += TX * TY) {
        const int kc = min(max(tile.kb - 1 + q, 0), g.nz - 1);   // cell planes kb - 1 .. (clamped)
        const int kf = min(tile.kb + q, g.nz);                    // face planes kb ..
        m_idz[q] = g.idz[kc];
        m_dz[q] = g.dz[kc];
        m_idzw[q] = g.idzw[kf];
        m_o[q] = g.o[kf];
    }
    const double idzw_lo = g.idzw[0], idzw_hi = g.idzw[g.nz];
    const typename RR::Cols cols = Ring<NF, TX, TY>::columns(g, tile.i0, tile.j0);
    const int i = tile.i0 + R.tx, j = tile.j0 + R.ty;
    const bool valid = i < g.nx && j < g.ny;
    const double* const F[NF] = {a.u, a.v, a.w, a.t, a.p};
    const bool face[NF] = {false, false, true, true, false};
    const size_t plane = (size_t)g.nx * g.ny;
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double idx2 = idx * idx, idy2 = idy * idy;
    const double qx = 0.25 * idx, qy = 0.25 * idy;                 // flux products of two sums
    const double nux = a.nu * idx2, nuy = a.nu * idy2, kax = a.ka * idx2, kay = a.ka * idy2;
    // RK3 weights times dt: rhs = dt [gamma H + rho H_prev - alpha G p + alpha nu Dzz q]
    const double cg = a.dt * a.gam, cr = a.dt * a.rho, ca = a.dt * a.alp;
    const double can = ca * a.nu, cak = ca * a.ka;
    // centre fields: Dzz already has homogeneous wall rows (the wall value is zero), so the
    // rhs weight and the Crank-Nicolson beta combine
    const double cdn = can - a.bnu;
    const int nz = g.nz;
    const int kb = tile.kb;
    typename RR::Stage st;
    // prologue: u, v at kb - 1 and kb, w and T at kb; then the step's leading planes
    // (u, v, w, T at k + 1 and p at k), which the loop stores at the top of step k
    constexpr bool kUV[NF] = {true, true, false, false, false};
    constexpr bool kUVWT[NF] = {true, true, true, true, false};
    constexpr bool kAll[NF] = {true, true, true, true, true};
    {
        const int p0[NF] = {kb - 1, kb - 1, kb - 1, kb - 1, kb - 1};
        R.fetch(p0, kUV, F, face, g, cols, st);
        R.put(p0, kUV, st);
        const int p1[NF] = {kb, kb, kb, kb, kb};
        R.fetch(p1, kUVWT, F, face, g, cols, st);
        R.put(p1, kUVWT, st);
        const int p2[NF] = {kb + 1, kb + 1, kb + 1, kb + 1, kb};
        R.fetch(p2, kAll, F, face, g, cols, st);
    }
    // own-column values at k - 1 of w (face), T (face) and p (cell); zero below the box
    const size_t own = valid ? (size_t)j * g.nx + i : 0;
    const unsigned own_b = (unsigned)(own * sizeof(double));   // the thread's column in bytes
    double w_km = 0.0, t_km = 0.0, p_km = 0.0;
    if (kb > 0) {
        w_km = a.w[(size_t)(kb - 1) * plane + own];
        t_km = a.t[(size_t)(kb - 1) * plane + own];
        p_km = a.p[(size_t)(kb - 1) * plane + own];
    }
    for (int k = kb; k < tile.ke; ++k) {
        {
            const int pk[NF] = {k + 1, k + 1, k + 1, k + 1, k};
            R.put(pk, kAll, st);
        }
        __syncthreads();
        const size_t kp = (size_t)k * plane;   // this step's plane
        // Previous-substep H of this cell, loaded before the next plane's prefetch (cells
        // outside the box read the plane's first cell).  These loads and the prefetch are
        // unconditional (substep 1 has no H: it reads the first value of u, one cache line for
        // every lane, and drops it; the last step fetches a plane it never stores): a load
        // under a branch would make every wait after the branch's end count conservatively,
        // and so wait for the whole prefetch.  (Reading u at the cell instead cost HBM traffic:
        // substep 1 fetched 74 B per point against 40 B of state.)
        const bool use_hp = a.rho != 0.0;
        const size_t hk = use_hp ? (size_t)k * plane : 0;
        const unsigned hoff = use_hp ? own_b : 0u;
        double hp[4];
        hp[0] = ld_plane(plane_rsrc((use_hp ? a.hpu : a.u) + hk, plane), hoff);
        hp[1] = ld_plane(plane_rsrc((use_hp ? a.hpv : a.u) + hk, plane), hoff);
        hp[2] = ld_plane(plane_rsrc((use_hp ? a.hpw : a.u) + hk, plane), hoff);
        hp[3] = ld_plane(plane_rsrc((use_hp ? a.hpt : a.u) + hk, plane), hoff);
        asm volatile("" ::: "memory");   // issue order: H first, then the prefetch
        {
            const int pn[NF] = {k + 2, k + 2, k + 2, k + 2, k + 1};
            R.fetch(pn, kAll, F, face, g, cols, st);
        }
        // this step's own-column centre values of w, T, p (carried to the next step)
        const double w_kc = R.at(FW, k, 0, 0), t_kc = R.at(FT, k, 0, 0), p_kc = R.at(FP, k, 0, 0);
        if (valid) {
            // neighbours on the window's planes; the own column at k - 1 of w, T, p from registers
            auto L = [&](int f, int dk, int dj, int di) { return R.at(f, k + dk, dj, di); };
            // The two-point averages of every flux product are taken as plain sums, their
            // factor 1/4 folded into the per-direction scale with the inverse spacing; a
            // difference of squared averages is formed as (a - b)(a + b); dt folds into the
            // RK3 weights.  The same discrete operators, fewer FP64 instructions.
            const int mq = k - tile.kb;   // metric tables: cell plane k at mq + 1, face k at mq
            const double idzk = m_idz[mq + 1];
            const bool lo = k > 0, hi = k + 1 < nz;
            // ---- u at (x-face i, y-centre j, z-centre k) ----
            {
                const double uc = L(FU, 0, 0, 0), uim = L(FU, 0, 0, -1), uip = L(FU, 0, 0, 1);
                const double ujm = L(FU, 0, -1, 0), ujp = L(FU, 0, 1, 0);
                const double ukm = L(FU, -1, 0, 0), ukp = L(FU, 1, 0, 0);
                const double ax = (uip - uim) * (uip + uim + 2.0 * uc) * qx;
                const double ay = ((L(FV, 0, 1, 0) + L(FV, 0, 1, -1)) * (ujp + uc) -
                                   (L(FV, 0, 0, 0) + L(FV, 0, 0, -1)) * (uc + ujm)) * qy;
                const double fzb = lo ? (L(FW, 0, 0, 0) + L(FW, 0, 0, -1)) * (ukm + uc) : 0.0;
                const double fzt = hi ? (L(FW, 1, 0, 0) + L(FW, 1, 0, -1)) * (uc + ukp) : 0.0;
                const double az = (fzt - fzb) * (0.25 * idzk);
                const double h = (nux * (uip + uim - 2.0 * uc) + nuy * (ujp + ujm - 2.0 * uc)) - (ax + ay + az);
                const double fb = lo ? (uc - ukm) * m_idzw[mq] : uc * idzw_lo;
                const double ft = hi ? (ukp - uc) * m_idzw[mq + 1] : -uc * idzw_hi;
                const double dzz = (ft - fb) * idzk;
                const double gp = (L(FP, 0, 0, 0) - L(FP, 0, 0, -1)) * idx;
                double r = cg * h - ca * gp + cdn * dzz;
                if (a.rho != 0.0) r += cr * hp[0];
                st_plane(a.ru + kp, plane, own_b, a.cq ? uc + r : r);
                if (a.hu) st_plane(a.hu + kp, plane, own_b, h);
            }
            // (the three blocks run one after the other: their LDS reads are not hoisted
            // together, which keeps the register count, and the occupancy, where the window's
            // LDS size allows)
            PS_EX_FENCE();
            // ---- v at (x-centre i, y-face j, z-centre k) ----
            {
                const double vc = L(FV, 0, 0, 0), vjm = L(FV, 0, -1, 0), vjp = L(FV, 0, 1, 0);
                const double vim = L(FV, 0, 0, -1), vip = L(FV, 0, 0, 1);
                const double vkm = L(FV, -1, 0, 0), vkp = L(FV, 1, 0, 0);
                const double ay = (vjp - vjm) * (vjp + vjm + 2.0 * vc) * qy;
                const double ax = ((L(FU, 0, 0, 1) + L(FU, 0, -1, 1)) * (vip + vc) -
                                   (L(FU, 0, 0, 0) + L(FU, 0, -1, 0)) * (vc + vim)) * qx;
                const double fzb = lo ? (L(FW, 0, 0, 0) + L(FW, 0, -1, 0)) * (vkm + vc) : 0.0;
                const double fzt = hi ? (L(FW, 1, 0, 0) + L(FW, 1, -1, 0)) * (vc + vkp) : 0.0;
                const double az = (fzt - fzb) * (0.25 * idzk);
                const double h = (nux * (vip + vim - 2.0 * vc) + nuy * (vjp + vjm - 2.0 * vc)) - (ax + ay + az);
                const double fb = lo ? (vc - vkm) * m_idzw[mq] : vc * idzw_lo;
                const double ft = hi ? (vkp - vc) * m_idzw[mq + 1] : -vc * idzw_hi;
                const double dzz = (ft - fb) * idzk;
                const double gp = (L(FP, 0, 0, 0) - L(FP, 0, -1, 0)) * idy;
                double r = cg * h - ca * gp + cdn * dzz;
                if (a.rho != 0.0) r += cr * hp[1];
                st_plane(a.rv + kp, plane, own_b, a.cq ? vc + r : r);
                if (a.hv) st_plane(a.hv + kp, plane, own_b, h);
            }
            PS_EX_FENCE();
            // ---- w and T at (x-centre i, y-centre j, z-face k), interior faces ----
            // (rt NULL: the temperature is not advanced, only its buoyancy is used)
            const bool with_t = a.rt != nullptr;
            if (k == 0) {
                st_plane(a.rw + kp, plane, own_b, 0.0);
                if (with_t) st_plane(a.rt + kp, plane, own_b, 0.0);
                if (a.hw) st_plane(a.hw + kp, plane, own_b, 0.0);
                if (a.ht && with_t) st_plane(a.ht + kp, plane, own_b, 0.0);
            } else {
                const double dzm = m_dz[mq], dzp = m_dz[mq + 1], idzc = m_o[mq];   // o = 1/dzc (interior face)
                // volume-weighted horizontal transport on the side faces (times 2 dzc)
                const double uwl = dzm * L(FU, -1, 0, 0) + dzp * L(FU, 0, 0, 0);
                const double uwr = dzm * L(FU, -1, 0, 1) + dzp * L(FU, 0, 0, 1);
                const double vwb = dzm * L(FV, -1, 0, 0) + dzp * L(FV, 0, 0, 0);
                const double vwt = dzm * L(FV, -1, 1, 0) + dzp * L(FV, 0, 1, 0);
                const double sx = qx * idzc, sy = qy * idzc, sz = 0.25 * idzc;
                const double wc = L(FW, 0, 0, 0), wim = L(FW, 0, 0, -1), wip = L(FW, 0, 0, 1);
                const double wjm = L(FW, 0, -1, 0), wjp = L(FW, 0, 1, 0);
                const double wkm = w_km, wkp = L(FW, 1, 0, 0);
                const double tc = L(FT, 0, 0, 0), tim = L(FT, 0, 0, -1), tip = L(FT, 0, 0, 1);
                const double tjm = L(FT, 0, -1, 0), tjp = L(FT, 0, 1, 0);
                const double tkm = t_km, tkp = L(FT, 1, 0, 0);
                const double wtop = wc + wkp, wbot = wkm + wc;   // twice the centre values k, k-1
                // w
                {
                    const double ax = (uwr * (wc + wip) - uwl * (wim + wc)) * sx;
                    const double ay = (vwt * (wc + wjp) - vwb * (wjm + wc)) * sy;
                    const double az = (wkp - wkm) * (wtop + wbot) * sz;
                    const double h = (nux * (wip + wim - 2.0 * wc) + nuy * (wjp + wjm - 2.0 * wc) + tc) - (ax + ay + az);
                    const double dzz = ((wkp - wc) * idzk - (wc - wkm) * m_idz[mq]) * idzc;
                    // the Crank-Nicolson operator has homogeneous wall rows: the wall values'
                    // share of Dzz is left out of its beta term
                    const double dzh = dzz - (k == 1 ? wkm * m_idz[mq] * idzc : 0.0) -
                                       (k + 1 == nz ? wkp * idzk * idzc : 0.0);
                    const double gp = (L(FP, 0, 0, 0) - p_km) * idzc;
                    double r = cg * h - ca * gp + can * dzz - a.bnu * dzh;
                    if (a.rho != 0.0) r += cr * hp[2];
                    st_plane(a.rw + kp, plane, own_b, a.cq ? wc + r : r);
                    if (a.hw) st_plane(a.hw + kp, plane, own_b, h);
                }
                // T
                if (with_t) {
                    const double ax = (uwr * (tc + tip) - uwl * (tim + tc)) * sx;
                    const double ay = (vwt * (tc + tjp) - vwb * (tjm + tc)) * sy;
                    const double az = (wtop * (tc + tkp) - wbot * (tkm + tc)) * sz;
                    const double h = (kax * (tip + tim - 2.0 * tc) + kay * (tjp + tjm - 2.0 * tc)) - (ax + ay + az);
                    const double dzz = ((tkp - tc) * idzk - (tc - tkm) * m_idz[mq]) * idzc;
                    const double dzh = dzz - (k == 1 ? tkm * m_idz[mq] * idzc : 0.0) -
                                       (k + 1 == nz ? tkp * idzk * idzc : 0.0);
                    double r = cg * h + cak * dzz - a.bka * dzh;
                    if (a.rho != 0.0) r += cr * hp[3];
                    st_plane(a.rt + kp, plane, own_b, a.cq ? tc + r : r);
                    if (a.ht) st_plane(a.ht + kp, plane, own_b, h);
                }
            }
            if (k + 1 == nz) {
                st_plane(a.rw + kp + plane, plane, own_b, 0.0);
                if (with_t) st_plane(a.rt + kp + plane, plane, own_b, 0.0);
                if (a.hw) st_plane(a.hw + kp + plane, plane, own_b, 0.0);
                if (a.ht && with_t) st_plane(a.ht + kp + plane, plane, own_b, 0.0);
            }
        }
        w_km = w_kc;
        t_km = t_kc;
        p_km = p_kc;
        __syncthreads();
    }
}

// Vector-Jacobian product of the explicit right-hand sides, gathered per output
// point.  For a control-volume equation sum_faces +-F_f / h with cotangent kappa,
// each face carries Lambda_f = kappa_c / h_c - kappa_{c+1} / h_{c+1}; a flux
// F = U Q sends Lambda U dQ and Lambda Q dU to the points averaged into Q and U.
// The right-hand sides hold H through dt gamma H, and the substep's own H output may carry
// a cotangent gH: everything that acts through H (advection, horizontal diffusion,
// buoyancy) is driven by mu = dt gamma lambda + gH, which the LDS ring holds; the terms
// weighted by alpha (wall-normal diffusion, pressure gradient) act on lambda itself, read
// from memory along the thread's column.  z-marching blocks as in k_explicit, with the
// state and mu in the LDS ring.
#ifndef PS_AD_TX
#define PS_AD_TX 64
#endif
#ifndef PS_AD_TY
#define PS_AD_TY 4
#endif
constexpr int kAdTX = PS_AD_TX, kAdTY = PS_AD_TY, kAdZSEG = 64;
// The next plane is prefetched through registers as in k_explicit (the LDS ring already
// limits the adjoint to two waves per SIMD, so the staged values cost no occupancy):
// 768^2 x 512, 18.6 -> 16.0 ms against loading each plane when needed.
// GHV: a cotangent gH is given (the ring then cannot give lambda back, which is read along
// the thread's column instead); without it lambda = mu / (dt gamma) comes from the ring.
// Grid metrics of planes [k0, k0 + N) in LDS (indices outside clamp into the table; the
// kernels use such entries only in terms that are then discarded).  Reading them from LDS
// keeps global loads out of the steps: a vector-memory wait inside a step would also wait
// for the next plane's prefetch.
template <int N>
struct ZTab {
    double idz_[N], dz_[N], idzw_[N], o_[N];
    __device__ __forceinline__ void fill(const GridDev& g, int k0) {
        for (int q = threadIdx.x; q < N; q += blockDim.x) {
            const int kc = min(max(k0 + q, 0), g.nz - 1), kf = min(max(k0 + q, 0), g.nz);
            idz_[q] = g.idz[kc];
            dz_[q] = g.dz[kc];
            idzw_[q] = g.idzw[kf];
            o_[q] = g.o[kf];
        }
    }
};

template <bool GHV>
__global__ void __launch_bounds__(kAdTX * kAdTY) k_explicit_adj(SubstepAdjArgs a, GridDev g) {
    constexpr int TX = kAdTX, TY = kAdTY, NF = 8;
    using RingT = Ring<NF, TX, TY>;
    constexpr int NQ = RingT::NQ;
    enum { FU, FV, FW, FT, FMU, FMV, FMW, FMT };
    __shared__ double lds[3 * NF * (TX + 2) * (TY + 2)];
    constexpr int ZN = kAdZSEG + 5;   // planes kb - 2 .. ke + 2
    __shared__ ZTab<ZN> zt;
    const ExTile tile = ex_tile<TX, TY, kAdZSEG>(g);
    RingT R{lds, (int)threadIdx.x % TX, (int)threadIdx.x / TX};
    const int zk0 = tile.kb - 2;
    zt.fill(g, zk0);
    auto zq = [&](int kk) { const int q = kk - zk0; return q < 0 ? 0 : (q >= ZN ? ZN - 1 : q); };
    auto m_idz = [&](int kk) { return zt.idz_[zq(kk)]; };
    auto m_dz = [&](int kk) { return zt.dz_[zq(kk)]; };
    auto m_idzw = [&](int kk) { return zt.idzw_[zq(kk)]; };
    auto m_o = [&](int kk) { return zt.o_[zq(kk)]; };
    const double idzw_lo = g.idzw[0], idzw_hi = g.idzw[g.nz];
    const typename RingT::Cols cols = RingT::columns(g, tile.i0, tile.j0);
    const int i = tile.i0 + R.tx, j = tile.j0 + R.ty;
    const bool valid = i < g.nx && j < g.ny;
    const double* const F[NF] = {a.u, a.v, a.w, a.t, a.lu, a.lv, a.lw, a.lt};
    const double* const GH[4] = {a.ghu, a.ghv, a.ghw, a.ght};
    const bool face[NF] = {false, false, true, true, false, false, true, true};
    constexpr bool with_gh = GHV;
    const int nz = g.nz;
    const size_t plane = (size_t)g.nx * g.ny;
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double idx2 = idx * idx, idy2 = idy * idy;
    const double muc = a.dt * a.gam;        // mu = dt gamma lambda + gH
    const double cal = a.dt * a.alp;        // weight of the alpha terms (on lambda)
    // The direct cotangent of q* (q* = C^-1 (C q + rhs), C = I - beta Dzz~) is C^T lambda =
    // lambda - beta Dzz~^T lambda, formed here from lambda instead of being read: with the
    // rhs's alpha-weighted Dzz^T it gives lambda + (dt alpha nu - beta) Dzz^T lambda.
    const double cdn = cal * a.nu - a.bnu, cdk = cal * a.ka - a.bka;
    // plane kk of the state, lambda and gH into registers (zeros outside a field); the loaded
    // values are not touched until put() blends mu = dt gamma lambda + gH into the ring, so
    // that every load of the stage stays in flight together
    double sgh[NQ][4];
    bool sok[NF];   // whether the staged plane exists, per field (uniform)
    // Which halo cells each state field is read at (the stencil below): T and w at x and y
    // offsets -1 and 0 only, u at y offsets -1 and 0, v at x offsets -1 and 0; lambda and gH
    // at the whole cross.  The others are not loaded (their ring entries are never read), so
    // that cache lines only an unread halo side touches are not fetched.
    bool need_lo[NQ], need_u[NQ], need_v[NQ];
#pragma unroll
    for (int qi = 0; qi < NQ; ++qi) {
        const int q = min((int)threadIdx.x + qi * TX * TY, (TX + 2) * (TY + 2) - 1);
        const int hy = q / (TX + 2), hx = q - hy * (TX + 2);
        need_u[qi] = hy <= TY;
        need_v[qi] = hx <= TX;
        need_lo[qi] = hx <= TX && hy <= TY;
    }
    auto fetch = [&](int kk, typename RingT::Stage& st) {
        const int kc = kk < 0 ? 0 : (kk > nz - 1 ? nz - 1 : kk);
        const int kf = kk < 0 ? 0 : (kk > nz ? nz : kk);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            sok[f] = kk >= 0 && (kk < nz || (face[f] && kk == nz));
            const size_t po = (size_t)(face[f] ? kf : kc) * plane;
#pragma unroll
            for (int qi = 0; qi < NQ; ++qi) {
                const bool need = f == FU ? need_u[qi] : (f == FV ? need_v[qi] : (f <= FT ? need_lo[qi] : true));
                double x = 0.0;
                if (need) x = F[f][po + cols.off[qi]];
                st.v[qi][f] = x;
                if (f >= FMU) sgh[qi][f - FMU] = with_gh ? GH[f - FMU][po + cols.off[qi]] : 0.0;
            }
        }
    };
    auto put = [&](int kk, typename RingT::Stage& st) {
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi)
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double v = f >= FMU ? muc * st.v[qi][f] + sgh[qi][f - FMU] : st.v[qi][f];
                st.v[qi][f] = sok[f] ? v : 0.0;
            }
        R.put(kk, st);
    };
    // lambda along this thread's column (planes k - 1, k, k + 1, rotated as the block marches,
    // the plane above fetched one step ahead like the ring) and at the x / y neighbours the
    // pressure-gradient transpose needs; cells outside the box use column (0, 0), missing
    // planes the nearest one (their values are never used)
    const int ic = valid ? i : 0, jc = valid ? j : 0;
    const int ip = (ic + 1 == g.nx) ? 0 : ic + 1, jp = (jc + 1 == g.ny) ? 0 : jc + 1;
    const size_t col = (size_t)jc * g.nx + ic, col_ip = (size_t)jc * g.nx + ip, col_jp = (size_t)jp * g.nx + ic;
    auto lcol = [&](const double* L, int kk, bool facef) {
        const int kc = kk < 0 ? 0 : (kk > (facef ? nz : nz - 1) ? (facef ? nz : nz - 1) : kk);
        return L[(size_t)kc * plane + col];
    };
    auto kcen = [&](int kk) { return (size_t)(kk > nz - 1 ? nz - 1 : kk) * plane; };
    double cu[3] = {0, 0, 0}, cv[3] = {0, 0, 0}, cw[3] = {0, 0, 0}, ct[3] = {0, 0, 0};
    double lu_ip = 0.0, lv_jp = 0.0;
    if constexpr (GHV) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cu[q] = lcol(a.lu, tile.kb - 1 + q, false);
            cv[q] = lcol(a.lv, tile.kb - 1 + q, false);
            cw[q] = lcol(a.lw, tile.kb - 1 + q, true);
            ct[q] = lcol(a.lt, tile.kb - 1 + q, true);
        }
        lu_ip = a.lu[kcen(tile.kb) + col_ip];
        lv_jp = a.lv[kcen(tile.kb) + col_jp];
    }
    const double imuc = 1.0 / muc;
    typename RingT::Stage st;
    fetch(tile.kb - 1, st);
    put(tile.kb - 1, st);
    fetch(tile.kb, st);
    put(tile.kb, st);
    fetch(tile.kb + 1, st);
    for (int k = tile.kb; k < tile.ke; ++k) {
        put(k + 1, st);
        __syncthreads();
        const size_t id = (size_t)k * plane + (size_t)j * g.nx + i;
        // the direct pressure cotangent of this cell, and lambda for the next step, loaded before the
        // next plane's prefetch (cells outside the box read the plane's first cell)
        const size_t idd = valid ? id : (size_t)k * plane;
        const double dpc = a.dp[idd];
        double nu_ = 0.0, nv_ = 0.0, nw_ = 0.0, nt_ = 0.0, nuip = 0.0, nvjp = 0.0;
        if constexpr (GHV) {
            nu_ = lcol(a.lu, k + 2, false);
            nv_ = lcol(a.lv, k + 2, false);
            nw_ = lcol(a.lw, k + 2, true);
            nt_ = lcol(a.lt, k + 2, true);
            nuip = a.lu[kcen(k + 1) + col_ip];
            nvjp = a.lv[kcen(k + 1) + col_jp];
        } else {
            // lambda from the ring (mu / (dt gamma)); planes outside a field read zero there
            cu[0] = R(k, FMU, -1, 0, 0) * imuc;
            cu[1] = R(k, FMU, 0, 0, 0) * imuc;
            cu[2] = R(k, FMU, 1, 0, 0) * imuc;
            cv[0] = R(k, FMV, -1, 0, 0) * imuc;
            cv[1] = R(k, FMV, 0, 0, 0) * imuc;
            cv[2] = R(k, FMV, 1, 0, 0) * imuc;
            cw[0] = R(k, FMW, -1, 0, 0) * imuc;
            cw[1] = R(k, FMW, 0, 0, 0) * imuc;
            cw[2] = R(k, FMW, 1, 0, 0) * imuc;
            ct[0] = R(k, FMT, -1, 0, 0) * imuc;
            ct[1] = R(k, FMT, 0, 0, 0) * imuc;
            ct[2] = R(k, FMT, 1, 0, 0) * imuc;
            lu_ip = R(k, FMU, 0, 0, 1) * imuc;
            lv_jp = R(k, FMV, 0, 1, 0) * imuc;
        }
        const double lum = cu[0], lu0 = cu[1], lup = cu[2];
        const double lvm = cv[0], lv0 = cv[1], lvp = cv[2];
        const double lwm = cw[0], lw0 = cw[1], lwp = cw[2];
        const double ltm = ct[0], lt0 = ct[1], ltp = ct[2];
        // the next plane's prefetch, unconditional and issued after this step's loads (a
        // conditional one would make later waits count conservatively; the last step fetches
        // a clamped plane it never stores)
        asm volatile("" ::: "memory");
        fetch(k + 2, st);
        if (valid) {
            // fields at absolute plane kk (k - 1 <= kk <= k + 1) and horizontal offsets (dj, di)
            auto U = [&](int kk, int dj, int di) { return R(k, FU, kk - k, dj, di); };
            auto V = [&](int kk, int dj, int di) { return R(k, FV, kk - k, dj, di); };
            auto Wf = [&](int kk, int dj, int di) { return R(k, FW, kk - k, dj, di); };
            auto Tf = [&](int kk, int dj, int di) { return R(k, FT, kk - k, dj, di); };
            auto MU = [&](int kk, int dj, int di) { return R(k, FMU, kk - k, dj, di); };
            auto MV = [&](int kk, int dj, int di) { return R(k, FMV, kk - k, dj, di); };
            auto MW = [&](int kk, int dj, int di) { return R(k, FMW, kk - k, dj, di); };
            auto MT = [&](int kk, int dj, int di) { return R(k, FMT, kk - k, dj, di); };
            // kappa = -mu (advection enters H with a minus sign); zero on the wall rows of
            // z-face equations
            auto KU = [&](int kk, int dj, int di) { return -MU(kk, dj, di); };
            auto KV = [&](int kk, int dj, int di) { return -MV(kk, dj, di); };
            auto KW = [&](int kk, int dj, int di) { return (kk >= 1 && kk <= nz - 1) ? -MW(kk, dj, di) : 0.0; };
            auto KT = [&](int kk, int dj, int di) { return (kk >= 1 && kk <= nz - 1) ? -MT(kk, dj, di) : 0.0; };
            auto idzc = [&](int kk) { return m_o(kk); };   // 1/dzc at interior faces, 0 at the walls
            // volume-weighted transport at (x-face or y-face, z-face kk)
            auto UW = [&](int kk, int dj, int di) {
                return (m_dz(kk - 1) * U(kk - 1, dj, di) + m_dz(kk) * U(kk, dj, di)) * (0.5 * m_o(kk));
            };
            auto VW = [&](int kk, int dj, int di) {
                return (m_dz(kk - 1) * V(kk - 1, dj, di) + m_dz(kk) * V(kk, dj, di)) * (0.5 * m_o(kk));
            };
            // transpose of the centre-field Dzz (dz Dzz dz^-1, Dirichlet walls) applied to lambda
            auto dzzt_c = [&](double lm, double l0, double lp) {
                const double mc = l0 * m_idz(k);
                const double fb = (k > 0) ? (mc - lm * m_idz(k - 1)) * m_idzw(k) : mc * idzw_lo;
                const double ft = (k + 1 < nz) ? (lp * m_idz(k + 1) - mc) * m_idzw(k + 1) : -mc * idzw_hi;
                return ft - fb;
            };

            // ================= g_u at (k, j, i) =================
            {
                double s = 0.0;
                // u-eq, x faces at centres i, i-1: F = U^2
                {
                    const double L0 = (KU(k, 0, 0) - KU(k, 0, 1)) * idx, U0 = 0.5 * (U(k, 0, 0) + U(k, 0, 1));
                    const double L1 = (KU(k, 0, -1) - KU(k, 0, 0)) * idx, U1 = 0.5 * (U(k, 0, -1) + U(k, 0, 0));
                    s += L0 * U0 + L1 * U1;
                }
                // u-eq, y faces j, j+1 (x-face i): Q = avg u
                {
                    const double Lj = (KU(k, -1, 0) - KU(k, 0, 0)) * idy;
                    const double Lp = (KU(k, 0, 0) - KU(k, 1, 0)) * idy;
                    const double Vj = 0.5 * (V(k, 0, 0) + V(k, 0, -1));
                    const double Vp = 0.5 * (V(k, 1, 0) + V(k, 1, -1));
                    s += 0.5 * (Lj * Vj + Lp * Vp);
                }
                // u-eq, z faces k, k+1 (interior): Q = avg u
                if (k >= 1) {
                    const double L = KU(k - 1, 0, 0) * m_idz(k - 1) - KU(k, 0, 0) * m_idz(k);
                    s += 0.5 * L * 0.5 * (Wf(k, 0, 0) + Wf(k, 0, -1));
                }
                if (k + 1 <= nz - 1) {
                    const double L = KU(k, 0, 0) * m_idz(k) - KU(k + 1, 0, 0) * m_idz(k + 1);
                    s += 0.5 * L * 0.5 * (Wf(k + 1, 0, 0) + Wf(k + 1, 0, -1));
                }
                // v-eq, x faces at (x-face i, y-faces j and j+1): U = avg of u over y
                {
                    const double L0 = (KV(k, 0, -1) - KV(k, 0, 0)) * idx, Q0 = 0.5 * (V(k, 0, -1) + V(k, 0, 0));
                    const double L1 = (KV(k, 1, -1) - KV(k, 1, 0)) * idx, Q1 = 0.5 * (V(k, 1, -1) + V(k, 1, 0));
                    s += 0.5 * (L0 * Q0 + L1 * Q1);
                }
                // w- and T-eq, x faces at (x-face i, z-faces k and k+1): volume-weighted u
                for (int kf = k; kf <= k + 1; ++kf) {
                    if (kf < 1 || kf > nz - 1) continue;
                    const double wt = m_dz(k) * (0.5 * m_o(kf));
                    const double Lw = (KW(kf, 0, -1) - KW(kf, 0, 0)) * idx, Qw = 0.5 * (Wf(kf, 0, -1) + Wf(kf, 0, 0));
                    const double Lt = (KT(kf, 0, -1) - KT(kf, 0, 0)) * idx, Qt = 0.5 * (Tf(kf, 0, -1) + Tf(kf, 0, 0));
                    s += wt * (Lw * Qw + Lt * Qt);
                }
                // linear terms: horizontal diffusion of mu (symmetric), Dzz^T of lambda
                const double mc = MU(k, 0, 0);
                const double hd = a.nu * ((MU(k, 0, 1) - 2.0 * mc + MU(k, 0, -1)) * idx2 +
                                          (MU(k, 1, 0) - 2.0 * mc + MU(k, -1, 0)) * idy2);
                st_out(a.gu + (id), lu0 + s + hd + cdn * dzzt_c(lum, lu0, lup));
            }
            // ================= g_v at (k, j, i) =================
            {
                double s = 0.0;
                {
                    const double L0 = (KV(k, 0, 0) - KV(k, 1, 0)) * idy, U0 = 0.5 * (V(k, 0, 0) + V(k, 1, 0));
                    const double L1 = (KV(k, -1, 0) - KV(k, 0, 0)) * idy, U1 = 0.5 * (V(k, -1, 0) + V(k, 0, 0));
                    s += L0 * U0 + L1 * U1;
                }
                {
                    const double Li = (KV(k, 0, -1) - KV(k, 0, 0)) * idx;
                    const double Lp = (KV(k, 0, 0) - KV(k, 0, 1)) * idx;
                    const double Ui = 0.5 * (U(k, 0, 0) + U(k, -1, 0));
                    const double Up = 0.5 * (U(k, 0, 1) + U(k, -1, 1));
                    s += 0.5 * (Li * Ui + Lp * Up);
                }
                if (k >= 1) {
                    const double L = KV(k - 1, 0, 0) * m_idz(k - 1) - KV(k, 0, 0) * m_idz(k);
                    s += 0.5 * L * 0.5 * (Wf(k, 0, 0) + Wf(k, -1, 0));
                }
                if (k + 1 <= nz - 1) {
                    const double L = KV(k, 0, 0) * m_idz(k) - KV(k + 1, 0, 0) * m_idz(k + 1);
                    s += 0.5 * L * 0.5 * (Wf(k + 1, 0, 0) + Wf(k + 1, -1, 0));
                }
                // u-eq, y faces at (x-faces i and i+1, y-face j): V = avg of v over x
                {
                    const double L0 = (KU(k, -1, 0) - KU(k, 0, 0)) * idy, Q0 = 0.5 * (U(k, -1, 0) + U(k, 0, 0));
                    const double L1 = (KU(k, -1, 1) - KU(k, 0, 1)) * idy, Q1 = 0.5 * (U(k, -1, 1) + U(k, 0, 1));
                    s += 0.5 * (L0 * Q0 + L1 * Q1);
                }
                for (int kf = k; kf <= k + 1; ++kf) {
                    if (kf < 1 || kf > nz - 1) continue;
                    const double wt = m_dz(k) * (0.5 * m_o(kf));
                    const double Lw = (KW(kf, -1, 0) - KW(kf, 0, 0)) * idy, Qw = 0.5 * (Wf(kf, -1, 0) + Wf(kf, 0, 0));
                    const double Lt = (KT(kf, -1, 0) - KT(kf, 0, 0)) * idy, Qt = 0.5 * (Tf(kf, -1, 0) + Tf(kf, 0, 0));
                    s += wt * (Lw * Qw + Lt * Qt);
                }
                const double mc = MV(k, 0, 0);
                const double hd = a.nu * ((MV(k, 0, 1) - 2.0 * mc + MV(k, 0, -1)) * idx2 +
                                          (MV(k, 1, 0) - 2.0 * mc + MV(k, -1, 0)) * idy2);
                st_out(a.gv + (id), lv0 + s + hd + cdn * dzzt_c(lvm, lv0, lvp));
            }
            // ================= g_p at (k, j, i):  -dt alpha G^T lambda =================
            {
                double gt = (lu0 - lu_ip) * idx + (lv0 - lv_jp) * idy;
                if (k >= 1) gt += lw0 * m_o(k);
                if (k + 1 <= nz - 1) gt -= lwp * m_o(k + 1);
                st_out(a.gp + (id), dpc - cal * gt);
            }
            // ================= g_w, g_T at z-face k (interior) =================
            if (k == 0) {
                st_out(a.gw + (id), 0.0);
                st_out(a.gt + (id), 0.0);
            } else {
                double sw = 0.0, st_ = 0.0;
                // w-eq z faces at centres k and k-1: F = U^2, U = avg w
                {
                    const double L0 = KW(k, 0, 0) * idzc(k) - KW(k + 1, 0, 0) * idzc(k + 1);
                    const double L1 = KW(k - 1, 0, 0) * idzc(k - 1) - KW(k, 0, 0) * idzc(k);
                    sw += L0 * 0.5 * (Wf(k, 0, 0) + Wf(k + 1, 0, 0)) + L1 * 0.5 * (Wf(k - 1, 0, 0) + Wf(k, 0, 0));
                }
                // T-eq z faces at centres k and k-1: U = avg w, Q = avg T
                {
                    const double L0 = KT(k, 0, 0) * idzc(k) - KT(k + 1, 0, 0) * idzc(k + 1);
                    const double L1 = KT(k - 1, 0, 0) * idzc(k - 1) - KT(k, 0, 0) * idzc(k);
                    sw += 0.5 * (L0 * 0.5 * (Tf(k, 0, 0) + Tf(k + 1, 0, 0)) + L1 * 0.5 * (Tf(k - 1, 0, 0) + Tf(k, 0, 0)));
                    st_ += 0.5 * (L0 * 0.5 * (Wf(k, 0, 0) + Wf(k + 1, 0, 0)) + L1 * 0.5 * (Wf(k - 1, 0, 0) + Wf(k, 0, 0)));
                }
                // w- and T-eq x faces i, i+1 (transport UW) and y faces j, j+1 (transport VW)
                {
                    const double Lw0 = (KW(k, 0, -1) - KW(k, 0, 0)) * idx, Lw1 = (KW(k, 0, 0) - KW(k, 0, 1)) * idx;
                    const double Lt0 = (KT(k, 0, -1) - KT(k, 0, 0)) * idx, Lt1 = (KT(k, 0, 0) - KT(k, 0, 1)) * idx;
                    const double U0 = UW(k, 0, 0), U1 = UW(k, 0, 1);
                    sw += 0.5 * (Lw0 * U0 + Lw1 * U1);
                    st_ += 0.5 * (Lt0 * U0 + Lt1 * U1);
                    const double Mw0 = (KW(k, -1, 0) - KW(k, 0, 0)) * idy, Mw1 = (KW(k, 0, 0) - KW(k, 1, 0)) * idy;
                    const double Mt0 = (KT(k, -1, 0) - KT(k, 0, 0)) * idy, Mt1 = (KT(k, 0, 0) - KT(k, 1, 0)) * idy;
                    const double V0 = VW(k, 0, 0), V1 = VW(k, 1, 0);
                    sw += 0.5 * (Mw0 * V0 + Mw1 * V1);
                    st_ += 0.5 * (Mt0 * V0 + Mt1 * V1);
                }
                // u-eq z faces at (x-faces i, i+1; z-face k): W = avg of w over x, Q = avg of u over z
                {
                    const double L0 = KU(k - 1, 0, 0) * m_idz(k - 1) - KU(k, 0, 0) * m_idz(k);
                    const double L1 = KU(k - 1, 0, 1) * m_idz(k - 1) - KU(k, 0, 1) * m_idz(k);
                    sw += 0.5 * (L0 * 0.5 * (U(k - 1, 0, 0) + U(k, 0, 0)) + L1 * 0.5 * (U(k - 1, 0, 1) + U(k, 0, 1)));
                }
                // v-eq z faces at (y-faces j, j+1; z-face k)
                {
                    const double L0 = KV(k - 1, 0, 0) * m_idz(k - 1) - KV(k, 0, 0) * m_idz(k);
                    const double L1 = KV(k - 1, 1, 0) * m_idz(k - 1) - KV(k, 1, 0) * m_idz(k);
                    sw += 0.5 * (L0 * 0.5 * (V(k - 1, 0, 0) + V(k, 0, 0)) + L1 * 0.5 * (V(k - 1, 1, 0) + V(k, 1, 0)));
                }
                // linear terms: horizontal diffusion of mu, Dzz^T (faces: dzc Dzz dzc^-1) of lambda
                // (lambda's wall rows are zero), buoyancy +T in the w equation (through H)
                const double mwc = MW(k, 0, 0), mtc = MT(k, 0, 0);
                const double hdw = a.nu * ((MW(k, 0, 1) - 2.0 * mwc + MW(k, 0, -1)) * idx2 +
                                           (MW(k, 1, 0) - 2.0 * mwc + MW(k, -1, 0)) * idy2);
                const double hdt = a.ka * ((MT(k, 0, 1) - 2.0 * mtc + MT(k, 0, -1)) * idx2 +
                                           (MT(k, 1, 0) - 2.0 * mtc + MT(k, -1, 0)) * idy2);
                const double mw = lw0 * idzc(k), mwm = lwm * idzc(k - 1), mwp = lwp * idzc(k + 1);
                const double mt = lt0 * idzc(k), mtm = ltm * idzc(k - 1), mtp = ltp * idzc(k + 1);
                const double dzw_ = (mwp - mw) * m_idz(k) - (mw - mwm) * m_idz(k - 1);
                const double dzt_ = (mtp - mt) * m_idz(k) - (mt - mtm) * m_idz(k - 1);
                st_out(a.gw + (id), lw0 + sw + hdw + cdn * dzw_);
                st_out(a.gt + (id), lt0 + st_ + hdt + cdk * dzt_ + mwc);
            }
            if (k + 1 == nz) {
                st_out(a.gw + (id + plane), 0.0);
                st_out(a.gt + (id + plane), 0.0);
            }

        }
        if constexpr (GHV) {
            cu[0] = cu[1];
            cu[1] = cu[2];
            cu[2] = nu_;
            cv[0] = cv[1];
            cv[1] = cv[2];
            cv[2] = nv_;
            cw[0] = cw[1];
            cw[1] = cw[2];
            cw[2] = nw_;
            ct[0] = ct[1];
            ct[1] = ct[2];
            ct[2] = nt_;
            lu_ip = nuip;
            lv_jp = nvjp;
        }
        __syncthreads();
    }
}

hipError_t launch_explicit_adj(const GridDev& g, const SubstepAdjArgs& a, hipStream_t st) {
    const dim3 grid(ex_blocks<kAdTX, kAdTY, kAdZSEG>(g)), block(kAdTX * kAdTY);
    if (a.ghu)
        hipLaunchKernelGGL(k_explicit_adj<true>, grid, block, 0, st, a, g);
    else
        hipLaunchKernelGGL(k_explicit_adj<false>, grid, block, 0, st, a, g);
    return hipGetLastError();
}

hipError_t launch_explicit(const GridDev& g, const SubstepArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_explicit, dim3(ex_blocks<kExTX, kExTY, kExZSEG>(g)), dim3(kExTX * kExTY), 0, st, a, g);
    return hipGetLastError();
}

}  // namespace ps
