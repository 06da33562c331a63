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
#include <algorithm>

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
// Pivot excesses at the lane-chunk boundaries of the tiled solve: entry
// [tile][l][w] is e_{lK-1} of column (tile, w) (0 for l = 0), formed by the
// sequential excess recurrence in FP64.  They depend only on the grid and
// lam = lamx + lamy, so a plan forms them once.  One lane per column.
template <typename T, int K>
__global__ void __launch_bounds__(256)
k_zexcess(T* __restrict__ etab, int nz, int ny, int nkxb, int nxh, const double* __restrict__ dz,
          const double* __restrict__ o, const double* __restrict__ lamx, const double* __restrict__ lamy) {
    constexpr int W = TileW<T>::value;
    const int nchunk = (nz + K - 1) / K;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= (size_t)nkxb * ny * W) return;
    const int w = (int)(col % W);
    const size_t tile = col / W;
    const int ky = (int)(tile % ny);
    const int kx = (int)(tile / ny) * W + w;
    // padding columns (kx > nx/2) are never stored; any finite excess serves them
    const double lam = kx < nxh ? lamx[kx] + lamy[ky] : 1.0;
    T* out = etab + tile * (size_t)nchunk * W + w;
    out[0] = (T)0;
    double e = lam * dz[0];
    for (int k = 1; k < nz; ++k) {
        if (k % K == 0) out[(size_t)(k / K) * W] = (T)e;
        const double m = o[k] / (o[k] + e);
        e = lam * dz[k] + m * e;
    }
}

// ---------------------------------------------------------------------------
// Tiled z solve: one block per (kx tile, ky); the nz x W tile is read once into
// registers and written once.  Lane (l, c) owns rows [l K, l K + K) of column c.
//  (A) pivots: from the excess entering the chunk (per-plan table), the lane forms
//      its own excesses e_k = s_k + m_k e_{k-1} and pivots p_k = o_{k+1} + e_k.
//  (B) forward sweep y_k = g_k + m_k y_{k-1}: affine maps, prefix scan.
//  (C) back substitution P_k = rp_k y_k + o_{k+1} rp_k P_{k+1}: affine maps,
//      suffix scan.
// Each scan: sequential composition inside the lane, shuffles across the lanes
// of one wave, and an LDS pass across waves.
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
__device__ __forceinline__ Aff<T> shfl_up_aff(const Aff<T>& m, int d) {
    return {__shfl_up(m.a, d, 64), {__shfl_up(m.b.x, d, 64), __shfl_up(m.b.y, d, 64)}};
}
template <typename T>
__device__ __forceinline__ Aff<T> shfl_down_aff(const Aff<T>& m, int d) {
    return {__shfl_down(m.a, d, 64), {__shfl_down(m.b.x, d, 64), __shfl_down(m.b.y, d, 64)}};
}

// Rows per lane (K) and columns per block (WZ), per precision.  A block holds
// WZ columns of nz rows in WZ * ceil(nz / K) lanes (rounded up to whole per-wave
// lane groups), at most 1024 threads: tall columns run in narrower blocks (WZ/2,
// WZ/4), and only columns too tall for those use the lane-per-column sweep (never
// with the default shapes, which tile every nz <= 2048).
// FP64: 16 rows per lane (with non-temporal tile accesses, 1024^2 x 512 z stage 1.45 ->
// 1.41 ms against 8 rows; 4 rows 1.64 ms).
#ifndef PS_Z_ROWS64
#define PS_Z_ROWS64 16
#endif
#ifndef PS_Z_ROWS32
#define PS_Z_ROWS32 16
#endif
#ifndef PS_Z_COLS64
#define PS_Z_COLS64 8
#endif
#ifndef PS_Z_COLS32
#define PS_Z_COLS32 16
#endif
template <typename T>
struct ZRows {
    static constexpr int value = sizeof(T) == 8 ? PS_Z_ROWS64 : PS_Z_ROWS32;
};
template <typename T>
struct ZCols {
    static constexpr int value = sizeof(T) == 8 ? PS_Z_COLS64 : PS_Z_COLS32;
};

// 1/x for the positive, normal pivots of the excess elimination: the hardware
// reciprocal refined by Newton steps (two in FP64, one in FP32; within an ulp of the
// quotient) in place of the full IEEE division, which sits on the dependent chain of
// the pivots.
__device__ __forceinline__ double pivot_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float pivot_rcp(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Barrier of the scans: __syncthreads, or (RAW) an LDS-only barrier (this wave's LDS
// accesses complete, then s_barrier) that leaves outstanding global->LDS copies in flight.
template <bool RAW>
__device__ __forceinline__ void zbar() {
    if constexpr (RAW) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt and expcnt left at their maxima
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    } else {
        __syncthreads();
    }
}

// Grid metrics of one lane's rows k0 .. k0 + K - 1 (dz_k, and o_k .. o_{k0+K}), as
// the solve reads them: dz(i) = dz_{k0+i}, oc(i) = o_{k0+i}.
// ZCoef holds them in registers, loaded once with clamped indices (so the loads need no
// guard and are all in flight before the tile's own loads: the pivots then depend on
// nothing but these and the chunk's entry excess).  ZCoefLds reads them from LDS where
// they are used (only for existing rows).
template <typename T, int K>
struct ZCoef {
    T dzr[K];
    T ocr[K + 1];
    __device__ __forceinline__ void load(int k0, int nz, const double* __restrict__ dzp,
                                         const double* __restrict__ op) {
#pragma unroll
        for (int i = 0; i < K; ++i) dzr[i] = (T)dzp[min(k0 + i, nz - 1)];
#pragma unroll
        for (int i = 0; i <= K; ++i) ocr[i] = (T)op[min(k0 + i, nz)];
    }
    __device__ __forceinline__ T dz(int i) const { return dzr[i]; }
    __device__ __forceinline__ T oc(int i) const { return ocr[i]; }
};
template <typename T>
struct ZCoefLds {
    const double* dzp;
    const double* op;
    int k0;
    __device__ __forceinline__ T dz(int i) const { return (T)dzp[k0 + i]; }
    __device__ __forceinline__ T oc(int i) const { return (T)op[k0 + i]; }
};

// Pivots, forward sweep and back substitution of one block's columns: lane (l, c) holds
// rows [k0, k0 + K) of column c in v (the right-hand side in, the solution out) and the
// excess eprev = e_{k0-1} entering its chunk.  FULL: every lane's K rows exist
// (nz a multiple of K, and of K times the lanes of a column in one wave), so no row
// needs a guard.
template <typename T, int K, int WZ, bool RAW, bool FULL, int NWMAX, typename CF>
__device__ __forceinline__ void zscan_solve(cx<T> (&v)[K], T eprev, T lam, int k0, int nz, int c, int wave,
                                            int nwave, int lw, T* xs, const CF& cf) {
    constexpr int LPW = 64 / WZ;
    auto row = [&](int i) { return FULL || k0 + i < nz; };
    // ---- pivots: rp_k = 1 / p_k; the chunk's first multiplier m0 = o_k0 / p_{k0-1} --------
    // Only rp and the scaled right-hand side stay in registers; the multipliers
    // m_k = o_k rp_{k-1} and the back-substitution coefficients o_{k+1} rp_k are re-formed
    // where they are used.
    T rp[K];
    T m0 = (T)0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        rp[i] = (T)0;
        if (row(i)) {
            const T s = lam * cf.dz(i);
            const T ok = cf.oc(i);
            T mm;
            if (i == 0) {
                // the chunk's first multiplier o_k0 / p_{k0-1}: zero at the bottom wall
                // (o_0 = 0), where the absent pivot is replaced by 1 (e_{-1} = 0 from the
                // table, so e_0 = s_0 exactly); a select rather than a branch, so the
                // table's load is not sunk behind the tile's
                mm = ok * pivot_rcp(k == 0 ? (T)1 : ok + eprev);
                m0 = mm;
            } else {
                mm = ok * rp[i - 1];
            }
            const T e = s + mm * eprev;
            rp[i] = pivot_rcp(cf.oc(i + 1) + e);
            eprev = e;
        }
    }
    // the pivot chain above needs none of the tile's values: keep the first use of the
    // tile (which waits for its loads) after it
    __builtin_amdgcn_sched_barrier(0);
    auto mult = [&](int i) -> T { return i == 0 ? m0 : cf.oc(i) * rp[i - 1]; };

    // ---- (B) forward sweep ------------------------------------------------------
    Aff<T> fa = {(T)1, {(T)0, (T)0}};
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (row(i)) {
            const T g = -cf.dz(i);
            v[i] = {g * v[i].x, g * v[i].y};   // g_k = -dz_k F_k
            const T m = mult(i);
            fa = {m * fa.a, {m * fa.b.x + v[i].x, m * fa.b.y + v[i].y}};
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
    zbar<RAW>();
    // totals of the waves below, composed in order (all of them read at once)
    Aff<T> fpw = {(T)1, {(T)0, (T)0}};
#pragma unroll
    for (int w2 = 0; w2 < NWMAX - 1; ++w2) {
        if (w2 < wave) {
            const T* q = xs + (w2 * WZ + c) * 4;
            fpw = aff_mul(Aff<T>{q[0], {q[1], q[2]}}, fpw);
        }
    }
    fex = aff_mul(fex, fpw);
    cx<T> y = fex.b;   // y_{k0-1} (y_{-1} = 0)
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (row(i)) {
            const T m = mult(i);
            y = {v[i].x + m * y.x, v[i].y + m * y.y};
            v[i] = y;
        }
    }
    zbar<RAW>();

    // ---- (C) back substitution -------------------------------------------------
    Aff<T> ba = {(T)1, {(T)0, (T)0}};
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        if (row(i)) {
            const T ak = cf.oc(i + 1) * rp[i];
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
    zbar<RAW>();
    Aff<T> bpw = {(T)1, {(T)0, (T)0}};
#pragma unroll
    for (int w2 = NWMAX - 1; w2 > 0; --w2) {
        if (w2 < nwave && w2 > wave) {
            const T* q = xs + (w2 * WZ + c) * 4;
            bpw = aff_mul(Aff<T>{q[0], {q[1], q[2]}}, bpw);
        }
    }
    bex = aff_mul(bex, bpw);
    cx<T> x = bex.b;   // solution just above this chunk (zero above the top wall)
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        if (row(i)) {
            const T ak = cf.oc(i + 1) * rp[i];
            x = {rp[i] * v[i].x + ak * x.x, rp[i] * v[i].y + ak * x.y};
            v[i] = x;
        }
    }
}

#ifdef PS_Z_WAVES_PER_EU
#define PS_Z_ATTR __attribute__((amdgpu_waves_per_eu(PS_Z_WAVES_PER_EU)))
#else
#define PS_Z_ATTR
#endif
template <typename T, int K, int WZ, int MAXT, bool FULL>
__global__ void __launch_bounds__(MAXT) PS_Z_ATTR
k_zsolve_scan(const cx<T>* b, cx<T>* bo, const T* __restrict__ etab, int nz, int ny, int nxh,
              const double* __restrict__ dz, const double* __restrict__ o, const double* __restrict__ lamx,
              const double* __restrict__ lamy) {
    constexpr int W = TileW<T>::value;
    static_assert(W % WZ == 0, "columns per block must divide the tile width");   // WZ: a sub-tile
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
    const bool real_col = kx < nxh;
    // Out of place (bo != b), padding columns kx > nx/2 are stored too (a finite dummy
    // solution), so that the output buffer holds no stale values; the (0,0) column is
    // always written by its own kernel.
    const bool store = (real_col || bo != b) && !(kx == 0 && ky == 0);
    const size_t toff = (size_t)tile_id * nz * W + csub * WZ + c;
    const cx<T>* tile = b + toff;
    cx<T>* otile = bo + toff;
    const int k0 = l * K;
    const int nchunk = (nz + K - 1) / K;

    // Everything the pivots need is requested first (metrics, wavenumbers, the excess
    // entering the chunk e_{k0-1}), then the tile: the pivot chain runs while the tile's
    // loads are still in flight.
    ZCoef<T, K> cf;
    cf.load(k0, nz, dz, o);
    const double lsum = lamx[min(kx, nxh - 1)] + lamy[ky];
    const T elo = etab[((size_t)tile_id * nchunk + (FULL ? l : min(l, nchunk - 1))) * W + csub * WZ + c];
    cx<T> v[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = k0 + i;
        if (FULL)
            v[i] = ld_stream<PS_NT_Z>(tile + (size_t)k * W);
        else
            v[i] = (k < nz) ? ld_stream<PS_NT_Z>(tile + (size_t)k * W) : cx<T>{(T)0, (T)0};
    }
    // every load above is issued before any arithmetic is scheduled
    __builtin_amdgcn_sched_barrier(0);
    const T lam = (real_col && !(kx == 0 && ky == 0)) ? (T)lsum : (T)1;
    const T eprev = (FULL || l < nchunk) ? elo : (T)0;

    zscan_solve<T, K, WZ, false, FULL, MAXT / 64>(v, eprev, lam, k0, nz, c, wave, nwave, lw, xs, cf);
    if (store) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int k = k0 + i;
            if (FULL || k < nz) st_stream<PS_NT_Z>(otile + (size_t)k * W, v[i]);
        }
    }
}

// Streamed z solve: a fixed grid of full-tile blocks walks the tiles; while a block
// solves tile t from registers, the next tile (nz x W contiguous values) streams into
// the other half of a double LDS buffer by global->LDS copies (1 KB per wave
// instruction), so every CU keeps a tile of loads in flight through the solve.  The
// scans' barriers are LDS-only so that they do not wait for those copies.
// Measured at 1024^2 x 512: FP32 z solve 1.36 -> 1.03 ms against the register-tile kernel
// of that time; in FP64 the solve work of the streaming blocks is the limit (1.92 ms
// register-tile kernel against 1.98 ms with a double buffer and 2.14 ms with one buffer and
// two blocks per CU).  Since the register-tile kernel reads and writes non-temporally with 16
// rows per lane it is faster in both precisions (FP32 0.82 ms against 1.03 ms streamed), so
// the streamed kernel is off by default (kept, and selectable, for measurement).
#ifndef PS_Z_PIPE32
#define PS_Z_PIPE32 0
#endif
#ifndef PS_Z_PIPE64
#define PS_Z_PIPE64 0
#endif
// tiles held in LDS per block: 2 (double buffer, one block per CU at nz = 512) or 1
// (refilled once the tile is in registers, two blocks per CU)
#ifndef PS_Z_PIPE_NBUF64
#define PS_Z_PIPE_NBUF64 1
#endif
#ifndef PS_Z_PIPE_NBUF32
#define PS_Z_PIPE_NBUF32 2
#endif
typedef __attribute__((address_space(3))) unsigned char lds_u8;
constexpr int kZPipeMaxNz = 512;

template <typename T, int K, int MAXT, int NBUF>
__global__ void __launch_bounds__(MAXT)
k_zsolve_pipe(const cx<T>* b, cx<T>* bo, const T* __restrict__ etab, int nz, int ny, int nxh, int ntiles,
              const double* __restrict__ dz, const double* __restrict__ o, const double* __restrict__ lamx,
              const double* __restrict__ lamy) {
    constexpr int W = TileW<T>::value, WZ = W, LPW = 64 / WZ;
    extern __shared__ __align__(16) unsigned char zsm[];
    __shared__ T xs[16 * WZ * 4];
    // grid metrics in LDS (nz <= kZPipeMaxNz): the solve then issues no global loads of its
    // own, which would have to wait behind the copies of the next tile
    __shared__ double zdz[kZPipeMaxNz], zo[kZPipeMaxNz + 1];
    cx<T>* buf = reinterpret_cast<cx<T>*>(zsm);   // [NBUF][nz * W]
    for (int q = threadIdx.x; q <= nz; q += blockDim.x) {
        zo[q] = o[q];
        if (q < nz) zdz[q] = dz[q];
    }
    const int tid = threadIdx.x;
    const int c = tid % WZ, l = tid / WZ, lane = tid & 63, lw = l % LPW;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwave = blockDim.x >> 6;
    const int k0 = l * K, nchunk = (nz + K - 1) / K;
    const size_t telems = (size_t)nz * W;
    const int nkb = (int)(telems * sizeof(cx<T>) / 1024);   // 1 KB copies per tile (nz * W * sizeof % 1024 == 0)
    auto copy_tile = [&](int t, int sel) {
        const unsigned char* src = reinterpret_cast<const unsigned char*>(b + (size_t)t * telems);
        lds_u8* dst = (lds_u8*)(reinterpret_cast<unsigned char*>(buf + sel * telems));   // LDS address
        for (int q = wave; q < nkb; q += nwave)
            __builtin_amdgcn_global_load_lds(src + (size_t)q * 1024 + lane * 16, dst + q * 1024, 16, 0, 0);
    };
    int t = blockIdx.x;
    if (t < ntiles) copy_tile(t, 0);
    for (int it = 0; t < ntiles; ++it, t += gridDim.x) {
        const int sel = NBUF == 2 ? (it & 1) : 0;
        __builtin_amdgcn_s_waitcnt(0);   // this wave's copies (and stores) are done
        __syncthreads();                 // ... and every other wave's
        const int ky = t % ny, kxb = t / ny, kx = kxb * W + c;
        const bool real_col = kx < nxh && !(kx == 0 && ky == 0);
        // out of place, padding columns are stored too (a finite dummy solution)
        const bool store = real_col || (bo != b && !(kx == 0 && ky == 0));
        const T lam = real_col ? (T)(lamx[kx] + lamy[ky]) : (T)1;
        T eprev = (T)0;
        if (l < nchunk) eprev = etab[((size_t)t * nchunk + l) * W + c];
        cx<T> v[K];
        const cx<T>* cur = buf + sel * telems;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int k = k0 + i;
            v[i] = (k < nz) ? cur[(size_t)k * W + c] : cx<T>{(T)0, (T)0};
        }
        // this tile's global loads complete before the copies are issued (the counter
        // that tracks them is in order)
        asm volatile("" ::"v"(lam), "v"(eprev));
        // one buffer: every wave has its values in registers before the buffer is refilled
        if (NBUF == 1) __syncthreads();
        // the next tile streams into the (other) buffer while this one is solved
        if (t + (int)gridDim.x < ntiles) copy_tile(t + gridDim.x, NBUF == 2 ? sel ^ 1 : 0);
        zscan_solve<T, K, WZ, true, false, MAXT / 64>(v, eprev, lam, k0, nz, c, wave, nwave, lw, xs,
                                                      ZCoefLds<T>{zdz, zo, k0});
        if (store) {
            cx<T>* tile = bo + (size_t)t * telems + c;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int k = k0 + i;
                if (k < nz) st_stream<PS_NT_ZPIPE_STORE>(tile + (size_t)k * W, v[i]);
            }
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

// FP64 plane sums from the x transform's row sums: one block per plane, a fixed
// summation order (the same result on every run).
__global__ void __launch_bounds__(256) k_rows_to_planes(const double* __restrict__ rowsum, int ny,
                                                    double* __restrict__ psum) {
    __shared__ double red[4];
    const int z = blockIdx.x;
    double v = 0.0;
    for (int y = threadIdx.x; y < ny; y += 256) v += rowsum[(size_t)z * ny + y];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) psum[z] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The singular (0,0) column, always in FP64.  One wave; lane l owns rows
// [l K, l K + K).  Column (kx, ky, w) = (0, 0, 0) of buffer b.  With psum (FP32
// spectra) the plane sums come from there in FP64 and the result goes to col00 in FP64,
// the spectrum's own entry being set to zero.
template <typename T>
__global__ void __launch_bounds__(64)
k_zsolve00(const cx<T>* b, cx<T>* bo, int nz, int nxny, const double* __restrict__ dz,
           const double* __restrict__ dzc, double* __restrict__ defect, const double* __restrict__ psum,
           double* __restrict__ col00) {
    constexpr int W = TileW<T>::value;
    constexpr int KMAX = 32;   // nz <= 2048
    const int lane = threadIdx.x;
    const int K = (nz + 63) / 64;
    const int k0 = lane * K;
    double fv[KMAX], dzv[KMAX], dzcv[KMAX];
    double s_dzf = 0.0, s_dz = 0.0;
    // all of the lane's loads first (clamped rows, anchored so that they stay together),
    // then the sums over its existing rows
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int kc = min(k0 + i, nz - 1);
        fv[i] = psum ? psum[kc] : (double)b[(size_t)kc * W].x;
        dzv[i] = dz[kc];
        dzcv[i] = dzc[kc];
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        anchor(fv[i]);
        anchor(dzv[i]);
        anchor(dzcv[i]);
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        if (i < K && k < nz) {
            s_dzf += dzv[i] * fv[i];
            s_dz += dzv[i];
        } else {
            fv[i] = 0.0;
        }
    }
    const double tot_dz = wave_sum(s_dz);
    const double mean_plane = wave_sum(s_dzf) / tot_dz;
    // fluxes: Q_{k+1} = sum_{j <= k} dz_j (F_j - mean)
    double loc = 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        if (i < K && k < nz) loc += dzv[i] * (fv[i] - mean_plane);
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
            inc[i] = (k >= 1) ? dzcv[i] * q : 0.0;
            locp += inc[i];
            q += dzv[i] * (fv[i] - mean_plane);
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
            s_dzp += dzv[i] * pv;
        }
    }
    const double shift = wave_sum(s_dzp) / tot_dz;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = k0 + i;
        if (i < K && k < nz) {
            if (col00) {
                col00[k] = fv[i] - shift;
                bo[(size_t)k * W] = cx<T>{(T)0, (T)0};
            } else {
                bo[(size_t)k * W] = cx<T>{(T)(fv[i] - shift), (T)0};
            }
        }
    }
    if (lane == 0 && defect) defect[0] = mean_plane / (double)nxny;
}

// Lanes of one column (a whole number of per-wave lane groups) and whether a block of
// WZ columns fits in 1024 threads.
template <int K, int WZ>
int zscan_threads(int nz) {
    constexpr int LPW = 64 / WZ;
    const int lc = (nz + K - 1) / K;
    return WZ * ((lc + LPW - 1) / LPW * LPW);
}

template <typename T, int K, int WZ>
hipError_t zscan_launch(const GridDev& g, const SpecDev<T>& s, hipStream_t st) {
    constexpr int W = TileW<T>::value;
    const int threads = zscan_threads<K, WZ>(g.nz);
    const int nblk = s.nkxb * g.ny * (W / WZ);
    const int nxh = g.nx / 2 + 1;
    constexpr int LPW = 64 / WZ;
    // every lane holds K existing rows: no row guards
    const bool full = g.nz % K == 0 && (g.nz / K) % LPW == 0;
#define PS_ZSCAN(MAXT, FULL)                                                                               \
    hipLaunchKernelGGL((k_zsolve_scan<T, K, WZ, MAXT, FULL>), dim3(nblk), dim3(threads), 0, st, s.b,          \
                       s.bz ? s.bz : s.b, s.etab, g.nz, g.ny, nxh, g.dz, g.o, g.lamx, g.lamy)
#define PS_ZSCAN2(MAXT)           \
    if (full)                     \
        PS_ZSCAN(MAXT, true);     \
    else                          \
        PS_ZSCAN(MAXT, false)
    if (threads <= 256)
        PS_ZSCAN2(256);
    else if (threads <= 512)
        PS_ZSCAN2(512);
    else
        PS_ZSCAN2(1024);
#undef PS_ZSCAN2
#undef PS_ZSCAN
    return hipGetLastError();
}

// Tiled solve with the widest block (ZCols, ZCols/2, ZCols/4 columns) that holds whole
// columns in 1024 threads: 0 when none does.
template <typename T>
int zscan_cols(const GridDev& g) {
    constexpr int K = ZRows<T>::value, C = ZCols<T>::value;
    if (zscan_threads<K, C>(g.nz) <= 1024) return C;
    if constexpr (C >= 2) {
        if (zscan_threads<K, C / 2>(g.nz) <= 1024) return C / 2;
    }
    if constexpr (C >= 4) {
        if (zscan_threads<K, C / 4>(g.nz) <= 1024) return C / 4;
    }
    return 0;
}

// Streamed variant: full tiles, whole KB copies, two tiles in LDS (<= 128 KB), <= 1024 threads.
template <typename T>
static bool zpipe_applies(const GridDev& g) {
    constexpr int W = TileW<T>::value, K = ZRows<T>::value;
    const size_t tbytes = (size_t)g.nz * W * sizeof(cx<T>);
    constexpr bool enabled = sizeof(T) == 4 ? PS_Z_PIPE32 : PS_Z_PIPE64;
    constexpr int NBUF = sizeof(T) == 4 ? PS_Z_PIPE_NBUF32 : PS_Z_PIPE_NBUF64;
    return enabled && g.nz <= kZPipeMaxNz && tbytes % 1024 == 0 && NBUF * tbytes <= 131072 &&
           zscan_threads<K, W>(g.nz) <= 1024;
}

template <typename T>
static hipError_t zpipe_launch(const GridDev& g, const SpecDev<T>& s, hipStream_t st, bool* launched) {
    constexpr int W = TileW<T>::value, K = ZRows<T>::value;
    *launched = false;
    const size_t tbytes = (size_t)g.nz * W * sizeof(cx<T>);
    const int threads = zscan_threads<K, W>(g.nz);
    constexpr int NBUF = sizeof(T) == 4 ? PS_Z_PIPE_NBUF32 : PS_Z_PIPE_NBUF64;
    if (!zpipe_applies<T>(g) || !s.etab) return hipSuccess;
    const int ncu = s.ncu > 0 ? s.ncu : 256;
    const int ntiles = s.nkxb * g.ny;
    const int nblk = std::min(ntiles, ncu * (NBUF == 1 ? 2 : 1));
    const int nxh = g.nx / 2 + 1;
#define PS_ZPIPE(MAXT)                                                                                           \
    hipLaunchKernelGGL((k_zsolve_pipe<T, K, MAXT, NBUF>), dim3(nblk), dim3(threads), NBUF * tbytes, st, s.b,       \
                       s.bz ? s.bz : s.b, s.etab, g.nz, g.ny, nxh, ntiles, g.dz, g.o, g.lamx, g.lamy)
    if (threads <= 256)
        PS_ZPIPE(256);
    else if (threads <= 512)
        PS_ZPIPE(512);
    else
        PS_ZPIPE(1024);
#undef PS_ZPIPE
    *launched = true;
    return hipGetLastError();
}

// Out of place (reading b, writing another buffer) measured faster than in place:
// 1024^2 x 512 FP64 solve 8.43 -> 8.27 ms, FP32-refined solve 21.37 -> 20.82 ms.  Through
// the register-tile and the streamed kernels (not the lane-per-column fallback).
#ifndef PS_Z_OOP
#define PS_Z_OOP 1
#endif
template <typename T>
bool zsolve_out_of_place(const GridDev& g) {
    return PS_Z_OOP && zscan_cols<T>(g) > 0;
}

template <typename T>
hipError_t launch_zsolve(const GridDev& g, const SpecDev<T>& s, hipStream_t st) {
    constexpr int W = TileW<T>::value;
    constexpr int K = ZRows<T>::value, C = ZCols<T>::value;
    const int wz = zscan_cols<T>(g);
    if (wz > 0 && !s.etab) return hipErrorInvalidValue;
    if (s.bz && !zsolve_out_of_place<T>(g)) return hipErrorInvalidValue;
    {
        bool launched = false;
        const hipError_t e = zpipe_launch<T>(g, s, st, &launched);
        if (launched || e != hipSuccess) return e;
    }
    if (wz == C) return zscan_launch<T, K, C>(g, s, st);
    if constexpr (C >= 2) {
        if (wz == C / 2) return zscan_launch<T, K, C / 2>(g, s, st);
    }
    if constexpr (C >= 4) {
        if (wz == C / 4) return zscan_launch<T, K, C / 4>(g, s, st);
    }
    // taller columns: one lane per column, pivots kept in the scratch buffer
    const size_t ncol = (size_t)s.nkxb * g.ny * W;
    const int nblk_seq = (int)((ncol + 255) / 256);
    hipLaunchKernelGGL((k_zsolve_seq<T>), dim3(nblk_seq), dim3(256), 0, st, s.b, s.piv, g.nz, g.ny, s.nkxb,
                       g.nx / 2 + 1, g.dz, g.o, g.lamx, g.lamy);
    return hipGetLastError();
}

template <typename T>
bool zsolve_tiled(const GridDev& g) {
    return zscan_cols<T>(g) > 0;
}

template <typename T>
size_t zexcess_elems(const GridDev& g, int nkxb) {
    constexpr int K = ZRows<T>::value;
    if (!zsolve_tiled<T>(g)) return 0;
    return (size_t)nkxb * g.ny * ((g.nz + K - 1) / K) * TileW<T>::value;
}

template <typename T>
hipError_t launch_zexcess(const GridDev& g, int nkxb, T* etab, hipStream_t st) {
    constexpr int K = ZRows<T>::value;
    const size_t ncol = (size_t)nkxb * g.ny * TileW<T>::value;
    const int nblk = (int)((ncol + 255) / 256);
    hipLaunchKernelGGL((k_zexcess<T, K>), dim3(nblk), dim3(256), 0, st, etab, g.nz, g.ny, nkxb, g.nx / 2 + 1, g.dz,
                       g.o, g.lamx, g.lamy);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zsolve00(const GridDev& g, const SpecDev<T>& s, double* defect, hipStream_t st) {
    if (s.rowsum) {
        hipLaunchKernelGGL(k_rows_to_planes, dim3(g.nz), dim3(256), 0, st, s.rowsum, g.ny, s.psum);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_zsolve00<T>), dim3(1), dim3(64), 0, st, s.b, s.bz ? s.bz : s.b, g.nz, g.nx * g.ny, g.dz,
                       g.dzc, defect, s.rowsum ? s.psum : nullptr, s.rowsum ? s.col00 : nullptr);
    return hipGetLastError();
}

template hipError_t launch_zsolve<double>(const GridDev&, const SpecDev<double>&, hipStream_t);
template hipError_t launch_zsolve<float>(const GridDev&, const SpecDev<float>&, hipStream_t);
template bool zsolve_tiled<double>(const GridDev&);
template bool zsolve_out_of_place<double>(const GridDev&);
template bool zsolve_out_of_place<float>(const GridDev&);
template bool zsolve_tiled<float>(const GridDev&);
template size_t zexcess_elems<double>(const GridDev&, int);
template size_t zexcess_elems<float>(const GridDev&, int);
template hipError_t launch_zexcess<double>(const GridDev&, int, double*, hipStream_t);
template hipError_t launch_zexcess<float>(const GridDev&, int, float*, hipStream_t);
template hipError_t launch_zsolve00<double>(const GridDev&, const SpecDev<double>&, double*, hipStream_t);
template hipError_t launch_zsolve00<float>(const GridDev&, const SpecDev<float>&, double*, hipStream_t);

}  // namespace ps
