// Wall-normal solves of the direct Poisson method (paper Sec. 2.2, step 7:
// after the 2-D transform each wavenumber pair (kx, ky) leaves one
// tridiagonal system in z, solved by Thomas elimination).
//
// Per column, with lam = lamx[kx] + lamy[ky] (modified wavenumbers) and the
// system multiplied by -dz_k so that it is a symmetric M-matrix:
//   -o_k P_{k-1} + (o_k + o_{k+1} + lam dz_k) P_k - o_{k+1} P_{k+1} = -dz_k F_k
// Elimination in excess form: e_k = lam dz_k + m_k e_{k-1},
// p_k = o_{k+1} + e_k, m_k = o_k / p_{k-1}; no pivot is formed by
// subtraction, which keeps the smallest wavenumbers accurate on strongly
// stretched grids.
//
// The (0,0) column is singular (Neumann in z, zero horizontal wavenumber):
// its right-hand side is made compatible (dz-weighted mean removed), then it
// is integrated directly - wall-normal fluxes Q_{k+1} = Q_k + dz_k F_k, then
// P_k = P_{k-1} + dzc_k Q_k - and re-gauged to zero dz-weighted mean.
#include "ps_internal.h"

namespace ps {

// One lane per column; the forward sweep keeps y in place and the pivots in
// `piv`, the backward sweep overwrites y with the solution.
template <typename T>
__global__ void __launch_bounds__(256)
k_zsolve_seq(cx<T>* __restrict__ b, T* __restrict__ piv, int nz, int ny, int nkxb, int nxh,
             const double* __restrict__ dz, const double* __restrict__ o, const double* __restrict__ lamx,
             const double* __restrict__ lamy) {
    constexpr int W = TileW<T>::value;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= (size_t)nkxb * ny * W) return;
    const int w = (int)(col % W);
    const size_t kyb = col / W;
    const int ky = (int)(kyb % ny);
    const int kxb = (int)(kyb / ny);
    const int kx = kxb * W + w;
    if (kx >= nxh || (kx == 0 && ky == 0)) return;
    const T lam = (T)(lamx[kx] + lamy[ky]);
    cx<T>* c = b + ((size_t)kxb * ny + ky) * (size_t)nz * W + w;
    T* pv = piv + ((size_t)kxb * ny + ky) * (size_t)nz * W + w;
    T e = lam * (T)dz[0];
    T p = (T)o[1] + e;
    cx<T> y = scal(c[0], -(T)dz[0]);
    c[0] = y;
    pv[0] = p;
    for (int k = 1; k < nz; ++k) {
        const T m = (T)o[k] / p;
        e = lam * (T)dz[k] + m * e;
        p = (T)o[k + 1] + e;
        y = scal(c[(size_t)k * W], -(T)dz[k]) + scal(y, m);
        c[(size_t)k * W] = y;
        pv[(size_t)k * W] = p;
    }
    cx<T> x = {y.x / p, y.y / p};
    c[(size_t)(nz - 1) * W] = x;
    for (int k = nz - 2; k >= 0; --k) {
        const cx<T> yk = c[(size_t)k * W];
        const T ok = (T)o[k + 1];
        const T pk = pv[(size_t)k * W];
        x = {(yk.x + ok * x.x) / pk, (yk.y + ok * x.y) / pk};
        c[(size_t)k * W] = x;
    }
}

// ---------------------------------------------------------------------------
// Tiled z solve: one block per (kx tile, ky); the nz x W tile is read once into
// registers and written once.  Lane (l, c) owns rows [l K, l K + K) of column c.
// The sequential elimination is split into three chunked scans over l:
//  (A) excesses: e_k = s_k + o_k e_{k-1} / (o_k + e_{k-1}) is the Moebius map of
//      the non-negative matrix [[s_k + o_k, s_k o_k], [1, o_k]] (row 0: [[0, s_0],
//      [0, 1]]), so chunk maps compose by 2x2 products of non-negative numbers
//      (still subtraction-free); products are rescaled by powers of two.
//  (B) forward sweep y_k = g_k + m_k y_{k-1}: affine maps, prefix scan.
//  (C) back substitution P_k = rp_k y_k + o_{k+1} rp_k P_{k+1}: affine maps,
//      suffix scan.
// Each scan: sequential composition inside the lane, shuffles across the lanes
// of one wave, and an LDS pass across waves.
template <typename T>
struct Mob {
    T a, b, c, d;   // [[a, b], [c, d]]
};

template <typename T>
__device__ __forceinline__ Mob<T> mob_mul(const Mob<T>& L, const Mob<T>& E) {
    return {L.a * E.a + L.b * E.c, L.a * E.b + L.b * E.d, L.c * E.a + L.d * E.c, L.c * E.b + L.d * E.d};
}

template <typename T>
__device__ __forceinline__ void mob_norm(Mob<T>& m) {
    T mx = fmax(fmax(m.a, m.b), fmax(m.c, m.d));
    if (mx > (T)0) {
        int ex;
        frexp(mx, &ex);
        m.a = ldexp(m.a, -ex);
        m.b = ldexp(m.b, -ex);
        m.c = ldexp(m.c, -ex);
        m.d = ldexp(m.d, -ex);
    }
}

template <typename T>
struct Aff {
    T a;
    cx<T> b;   // x -> a x + b
};

// L after E (L outer)
template <typename T>
__device__ __forceinline__ Aff<T> aff_mul(const Aff<T>& L, const Aff<T>& E) {
    return {L.a * E.a, {L.a * E.b.x + L.b.x, L.a * E.b.y + L.b.y}};
}

template <typename T>
__device__ __forceinline__ Mob<T> shfl_up_mob(const Mob<T>& m, int d) {
    return {__shfl_up(m.a, d, 64), __shfl_up(m.b, d, 64), __shfl_up(m.c, d, 64), __shfl_up(m.d, d, 64)};
}
template <typename T>
__device__ __forceinline__ Aff<T> shfl_up_aff(const Aff<T>& m, int d) {
    return {__shfl_up(m.a, d, 64), {__shfl_up(m.b.x, d, 64), __shfl_up(m.b.y, d, 64)}};
}
template <typename T>
__device__ __forceinline__ Aff<T> shfl_down_aff(const Aff<T>& m, int d) {
    return {__shfl_down(m.a, d, 64), {__shfl_down(m.b.x, d, 64), __shfl_down(m.b.y, d, 64)}};
}

// Rows per lane; blocks of up to 1024 threads, so columns of up to 1024 rows run
// tiled (taller ones use the lane-per-column sweep).
template <typename T>
struct ZRows {
    static constexpr int value = 4;   // 74 VGPRs (FP64), 65 (FP32); 8 rows spill
};
// Columns per block: 4 (half an FP64 tile, a quarter of an FP32 tile), so that
// 512-thread blocks at nz = 512 let three blocks share a CU and overlap one block's
// loads with another's scans.
#ifndef PS_Z_COLS
#define PS_Z_COLS 4
#endif
template <typename T>
struct ZCols {
    static constexpr int value = PS_Z_COLS;
};
#ifdef PS_Z_WAVES_PER_EU
#define PS_Z_ATTR __attribute__((amdgpu_waves_per_eu(PS_Z_WAVES_PER_EU)))
#else
#define PS_Z_ATTR
#endif

template <typename T, int K>
__global__ void __launch_bounds__(1024) PS_Z_ATTR
k_zsolve_scan(cx<T>* __restrict__ b, int nz, int ny, int nxh, const double* __restrict__ dz,
              const double* __restrict__ o, const double* __restrict__ lamx, const double* __restrict__ lamy) {
    constexpr int W = TileW<T>::value;
    constexpr int WZ = ZCols<T>::value;   // columns of this block (a sub-tile of the W-wide tile)
    constexpr int NSUB = W / WZ;
    constexpr int LPW = 64 / WZ;          // lanes of one column inside a wave
    __shared__ T xs[16 * WZ * 4];         // per-wave totals
    const int tid = threadIdx.x;
    const int c = tid % WZ;
    const int l = tid / WZ;
    const int wave = tid >> 6;
    const int nwave = blockDim.x >> 6;
    const int lw = l % LPW;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int csub = bid % NSUB;
    const int tile_id = bid / NSUB;
    const int ky = tile_id % ny;
    const int kxb = tile_id / ny;
    const int kx = kxb * W + csub * WZ + c;
    const bool store = kx < nxh && !(kx == 0 && ky == 0);
    const T lam = store ? (T)(lamx[kx] + lamy[ky]) : (T)1;
    cx<T>* tile = b + (size_t)tile_id * nz * W + csub * WZ + c;
    const int k0 = l * K;

    cx<T> v[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        v[i] = (k < nz) ? tile[(size_t)k * W] : cx<T>{(T)0, (T)0};
    }

    // ---- (A) excesses -------------------------------------------------------
    Mob<T> acc = {(T)1, (T)0, (T)0, (T)1};
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        if (k < nz) {
            const T s = lam * (T)dz[k];
            Mob<T> m;
            if (k == 0) {
                m = {(T)0, s, (T)0, (T)1};
            } else {
                const T ok = (T)o[k];
                m = {s + ok, s * ok, (T)1, ok};
            }
            acc = mob_mul(m, acc);
            // entries grow by at most a factor ~ (o + s + 1) per row: rescale every 4 rows
            if ((i & 3) == 3) mob_norm(acc);
        }
    }
    mob_norm(acc);
    Mob<T> inc = acc;
#pragma unroll
    for (int d = 1; d < LPW; d <<= 1) {
        Mob<T> oth = shfl_up_mob(inc, d * WZ);
        if (lw >= d) {
            inc = mob_mul(inc, oth);
            mob_norm(inc);
        }
    }
    if (lw == LPW - 1) {
        T* q = xs + (wave * WZ + c) * 4;
        q[0] = inc.a;
        q[1] = inc.b;
        q[2] = inc.c;
        q[3] = inc.d;
    }
    Mob<T> ex = shfl_up_mob(inc, WZ);
    if (lw == 0) ex = {(T)1, (T)0, (T)0, (T)1};
    __syncthreads();
    Mob<T> pw = {(T)1, (T)0, (T)0, (T)1};
    for (int w2 = 0; w2 < wave; ++w2) {
        const T* q = xs + (w2 * WZ + c) * 4;
        pw = mob_mul(Mob<T>{q[0], q[1], q[2], q[3]}, pw);
        mob_norm(pw);
    }
    ex = mob_mul(ex, pw);
    T eprev = (ex.d != (T)0) ? ex.b / ex.d : (T)0;   // e_{k0-1}
    __syncthreads();

    // ---- pivots and multipliers ----------------------------------------------
    T mk[K], rp[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        mk[i] = (T)0;
        rp[i] = (T)0;
        if (k < nz) {
            const T s = lam * (T)dz[k];
            T e;
            if (k == 0) {
                e = s;
            } else {
                const T ok = (T)o[k];
                const T mm = (i == 0) ? ok / (ok + eprev) : ok * rp[i - 1];
                mk[i] = mm;
                e = s + mm * eprev;
            }
            rp[i] = (T)1 / ((T)o[k + 1] + e);
            eprev = e;
        }
    }

    // ---- (B) forward sweep ------------------------------------------------------
    Aff<T> fa = {(T)1, {(T)0, (T)0}};
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        if (k < nz) {
            const T g = -(T)dz[k];
            v[i] = {g * v[i].x, g * v[i].y};   // g_k = -dz_k F_k
            fa = {mk[i] * fa.a, {mk[i] * fa.b.x + v[i].x, mk[i] * fa.b.y + v[i].y}};
        }
    }
    Aff<T> finc = fa;
#pragma unroll
    for (int d = 1; d < LPW; d <<= 1) {
        Aff<T> oth = shfl_up_aff(finc, d * WZ);
        if (lw >= d) finc = aff_mul(finc, oth);
    }
    if (lw == LPW - 1) {
        T* q = xs + (wave * WZ + c) * 4;
        q[0] = finc.a;
        q[1] = finc.b.x;
        q[2] = finc.b.y;
    }
    Aff<T> fex = shfl_up_aff(finc, WZ);
    if (lw == 0) fex = {(T)1, {(T)0, (T)0}};
    __syncthreads();
    Aff<T> fpw = {(T)1, {(T)0, (T)0}};
    for (int w2 = 0; w2 < wave; ++w2) {
        const T* q = xs + (w2 * WZ + c) * 4;
        fpw = aff_mul(Aff<T>{q[0], {q[1], q[2]}}, fpw);
    }
    fex = aff_mul(fex, fpw);
    cx<T> y = fex.b;   // y_{k0-1} (y_{-1} = 0)
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        if (k < nz) {
            y = {v[i].x + mk[i] * y.x, v[i].y + mk[i] * y.y};
            v[i] = y;
        }
    }
    __syncthreads();

    // ---- (C) back substitution -------------------------------------------------
    Aff<T> ba = {(T)1, {(T)0, (T)0}};
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        const int k = k0 + i;
        if (k < nz) {
            const T ak = (T)o[k + 1] * rp[i];
            ba = {ak * ba.a, {ak * ba.b.x + rp[i] * v[i].x, ak * ba.b.y + rp[i] * v[i].y}};
        }
    }
    Aff<T> binc = ba;
#pragma unroll
    for (int d = 1; d < LPW; d <<= 1) {
        Aff<T> oth = shfl_down_aff(binc, d * WZ);
        if (lw + d < LPW) binc = aff_mul(binc, oth);
    }
    if (lw == 0) {
        T* q = xs + (wave * WZ + c) * 4;
        q[0] = binc.a;
        q[1] = binc.b.x;
        q[2] = binc.b.y;
    }
    Aff<T> bex = shfl_down_aff(binc, WZ);
    if (lw == LPW - 1) bex = {(T)1, {(T)0, (T)0}};
    __syncthreads();
    Aff<T> bpw = {(T)1, {(T)0, (T)0}};
    for (int w2 = nwave - 1; w2 > wave; --w2) {
        const T* q = xs + (w2 * WZ + c) * 4;
        bpw = aff_mul(Aff<T>{q[0], {q[1], q[2]}}, bpw);
    }
    bex = aff_mul(bex, bpw);
    cx<T> x = bex.b;   // solution just above this chunk (zero above the top wall)
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        const int k = k0 + i;
        if (k < nz) {
            const T ak = (T)o[k + 1] * rp[i];
            x = {rp[i] * v[i].x + ak * x.x, rp[i] * v[i].y + ak * x.y};
            v[i] = x;
        }
    }
    if (store) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int k = k0 + i;
            if (k < nz) tile[(size_t)k * W] = v[i];
        }
    }
}

// inclusive scan over the 64 lanes of one wave
__device__ __forceinline__ double wave_scan_incl(double v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The singular (0,0) column, always in FP64.  One wave; lane l owns rows
// [l K, l K + K).  Column (kx, ky, w) = (0, 0, 0) of buffer b.
template <typename T>
__global__ void __launch_bounds__(64)
k_zsolve00(cx<T>* __restrict__ b, int nz, int nxny, const double* __restrict__ dz,
           const double* __restrict__ dzc, double* __restrict__ defect) {
    constexpr int W = TileW<T>::value;
    constexpr int KMAX = 32;   // nz <= 2048
    const int lane = threadIdx.x;
    const int K = (nz + 63) / 64;
    const int k0 = lane * K;
    double fv[KMAX];
    double s_dzf = 0.0, s_dz = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        fv[i] = 0.0;
        if (i < K && k < nz) {
            fv[i] = (double)b[(size_t)k * W].x;
            s_dzf += dz[k] * fv[i];
            s_dz += dz[k];
        }
    }
    const double tot_dz = wave_sum(s_dz);
    const double mean_plane = wave_sum(s_dzf) / tot_dz;
    // fluxes: Q_{k+1} = sum_{j <= k} dz_j (F_j - mean)
    double loc = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        if (i < K && k < nz) loc += dz[k] * (fv[i] - mean_plane);
    }
    double qexcl = wave_scan_incl(loc) - loc;   // Q at face k0
    // potential increments: P_k = P_{k-1} + dzc_k Q_k for k >= 1, P_0 = 0
    double q = qexcl;
    double inc[KMAX];
    double locp = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        inc[i] = 0.0;
        if (i < K && k < nz) {
            inc[i] = (k >= 1) ? dzc[k] * q : 0.0;
            locp += inc[i];
            q += dz[k] * (fv[i] - mean_plane);
        }
    }
    double pexcl = wave_scan_incl(locp) - locp;
    double pv = pexcl;
    double s_dzp = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        if (i < K && k < nz) {
            pv += inc[i];
            fv[i] = pv;
            s_dzp += dz[k] * pv;
        }
    }
    const double shift = wave_sum(s_dzp) / tot_dz;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        if (i < K && k < nz) b[(size_t)k * W] = cx<T>{(T)(fv[i] - shift), (T)0};
    }
    if (lane == 0 && defect) defect[0] = mean_plane / (double)nxny;
}

template <typename T>
hipError_t launch_zsolve(const GridDev& g, const SpecDev<T>& s, hipStream_t st) {
    constexpr int W = TileW<T>::value;
    constexpr int WZ = ZCols<T>::value;
    constexpr int LPW = 64 / WZ;
    auto lanes = [&](int K) {
        int lc = (g.nz + K - 1) / K;
        return (lc + LPW - 1) / LPW * LPW;
    };
    const int nblk = s.nkxb * g.ny * (W / WZ);
    const int nxh = g.nx / 2 + 1;
    constexpr int K = ZRows<T>::value;
    if (WZ * lanes(K) <= 1024) {
        hipLaunchKernelGGL((k_zsolve_scan<T, K>), dim3(nblk), dim3(WZ * lanes(K)), 0, st, s.b, g.nz, g.ny, nxh, g.dz,
                           g.o, g.lamx, g.lamy);
        return hipGetLastError();
    }
    // taller columns: one lane per column, pivots kept in the scratch buffer
    const size_t ncol = (size_t)s.nkxb * g.ny * W;
    const int nblk_seq = (int)((ncol + 255) / 256);
    hipLaunchKernelGGL((k_zsolve_seq<T>), dim3(nblk_seq), dim3(256), 0, st, s.b, s.piv, g.nz, g.ny, s.nkxb,
                       g.nx / 2 + 1, g.dz, g.o, g.lamx, g.lamy);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zsolve00(const GridDev& g, const SpecDev<T>& s, double* defect, hipStream_t st) {
    hipLaunchKernelGGL((k_zsolve00<T>), dim3(1), dim3(64), 0, st, s.b, g.nz, g.nx * g.ny, g.dz, g.dzc, defect);
    return hipGetLastError();
}

template hipError_t launch_zsolve<double>(const GridDev&, const SpecDev<double>&, hipStream_t);
template hipError_t launch_zsolve<float>(const GridDev&, const SpecDev<float>&, hipStream_t);
template hipError_t launch_zsolve00<double>(const GridDev&, const SpecDev<double>&, double*, hipStream_t);
template hipError_t launch_zsolve00<float>(const GridDev&, const SpecDev<float>&, double*, hipStream_t);

}  // namespace ps
