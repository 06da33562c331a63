// FFT stages of the direct Poisson solve (paper Sec. 2.2, steps 3, 5, 9, 11:
// real transform along the first periodic direction, complex transform along
// the second, and their inverses).
//
// Layouts (kx = kxb * W + w, kx in [0, nx/2]; columns above nx/2 are padding):
//   physical field  [nz][ny][nx]          FP64
//   buffer a        [nz][nkxb][ny][W]     after the x transform
//   buffer b        [nkxb][ny][nz][W]     after the y transform (z-solve layout)
//
// x transform: a real row of length nx is packed into nx/2 complex values
// z_n = f_{2n} + i f_{2n+1}, transformed with the register/LDS engine, and
// unpacked with X_k = (Z_k + Z*_{M-k})/2 - i e^{-2 pi i k/nx} (Z_k - Z*_{M-k})/2.
// The inverse runs the same steps backwards.  One block transforms R rows.
//
// y transform: a block owns WY columns of one (z, kxb) tile; element e of
// column c lives at LDS[e][c].
#include "ps_internal.h"
#include "reduce.h"

namespace ps {

// Elements per thread (the largest radix schedule fitting this many registers):
// x transforms hold whole rows in LDS, so fewer elements per thread (one row per
// wave) means less LDS per wave and more waves per CU.  Powers of two take 8 either
// way; lengths with a factor 3 take 12 (radices 12, 4, 4, 2 for 384 instead of six
// radix-2 passes after a radix 6: 768^2 x 512 x inverse 1.01 -> 0.88 ms).
#ifndef PS_X_EMAX64
#define PS_X_EMAX64 12
#endif
#ifndef PS_X_EMAX32
#define PS_X_EMAX32 8
#endif
#ifndef PS_Y_EMAX
#define PS_Y_EMAX 16
#endif
#ifndef PS_X_EMAX64_INV
#define PS_X_EMAX64_INV PS_X_EMAX64
#endif
#ifndef PS_X_EMAX32_INV
#define PS_X_EMAX32_INV PS_X_EMAX32
#endif
template <typename T, bool INV = false>
struct XEmax {
    static constexpr int value =
        sizeof(T) == 8 ? (INV ? PS_X_EMAX64_INV : PS_X_EMAX64) : (INV ? PS_X_EMAX32_INV : PS_X_EMAX32);
};
constexpr int kYEmax = PS_Y_EMAX;

// Launch shapes (tunable at build time; results do not depend on them).
// FP64 forward transforms: 256 threads (several rows per block, so that the divergence
// loader's y-neighbour rows are mostly rows the block's other waves load): 768^2 x 512
// projection 10.49 -> 10.10 ms against 64 threads, the 1024^2 solve unchanged.
#ifndef PS_X_THREADS
#define PS_X_THREADS 256
#endif
// FP32 forward transforms (the refinement's residual loader reads five rows of the
// iterate per output row): four rows per block let the y neighbours come from the rows
// the block's other waves load (1024^2 x 512 residual transform 3.09 -> 2.78 ms).
#ifndef PS_X_THREADS32
#define PS_X_THREADS32 256
#endif
// the inverse x transform reads strided tiles: two rows per block make each read 256 B
#ifndef PS_X_THREADS_INV
#define PS_X_THREADS_INV 128
#endif
#ifndef PS_X_LDS
#define PS_X_LDS 72000
#endif
// up to 1024 threads: FP32 tiles (16 columns) then run whole per block; FP64 tiles are
// limited to 8 columns (512 threads) by the LDS budget either way
#ifndef PS_Y_THREADS
#define PS_Y_THREADS 1024
#endif
#ifndef PS_Y_LDS
#define PS_Y_LDS 140000
#endif
#ifndef PS_Y_ZFAST
#define PS_Y_ZFAST 1
#endif

// Rows of one block: LDS row = lds_len(M) slots (odd for M >= 16, so that rows
// start in different banks).
template <typename T, int M, bool INV = false>
struct XShape {
    static constexpr int EM = XEmax<T, INV>::value;
    using Sh = FftShape<M, EM>;
    static constexpr int NT = Sh::NT;
    static constexpr int LROW = lds_len(M);
    static constexpr int TH = INV ? PS_X_THREADS_INV : (sizeof(T) == 4 ? PS_X_THREADS32 : PS_X_THREADS);
    static constexpr int R0 = TH / NT > 0 ? TH / NT : 1;
    static constexpr int RL0 = PS_X_LDS / (LROW * (int)sizeof(cx<T>));
    static constexpr int RL = RL0 > 0 ? RL0 : 1;
    static constexpr int R = R0 < RL ? R0 : RL;
    static constexpr int THREADS = R * NT;
    static constexpr size_t LDS = (size_t)R * LROW * sizeof(cx<T>);
};

// FP64 inverse y transforms of columns of 512 or 1024: 32 elements per thread and the LDS
// exchange in two halves (real, then imaginary parts), so that a whole tile takes half the
// LDS (70 KB) and two blocks share a CU: one block's arithmetic then runs under the other's
// loads.  (A single block per CU alternates the two; its arithmetic was exposed.)
#ifndef PS_Y_SPLIT_INV
#define PS_Y_SPLIT_INV 1
#endif

// Columns of one block (a power of two dividing the tile width).
template <typename T, int N, int S = -1>
struct YShape {
    static constexpr bool SPLIT = S > 0 && PS_Y_SPLIT_INV && sizeof(T) == 8 && (N == 512 || N == 1024) &&
                                  choose_e(N, 32) == 32;
    static constexpr int EMAX = SPLIT ? 32 : kYEmax;
    using Sh = FftShape<N, EMAX>;
    static constexpr int NT = Sh::NT;
    static constexpr int W = TileW<T>::value;
    static constexpr int EB = SPLIT ? (int)sizeof(T) : (int)sizeof(cx<T>);   // bytes of one LDS slot
    static constexpr int A = SPLIT ? W : PS_Y_LDS / (lds_len(N) * EB);
    static constexpr int B = SPLIT ? W : PS_Y_THREADS / NT;
    static constexpr int WY0 = (W < A ? W : A) < B ? (W < A ? W : A) : B;
    static constexpr int WY = WY0 >= 16 ? 16 : (WY0 >= 8 ? 8 : (WY0 >= 4 ? 4 : (WY0 >= 2 ? 2 : 1)));
    static constexpr int THREADS = WY * NT;
    static constexpr size_t LDS = (size_t)lds_len(N) * WY * EB;
};

// ---------------------------------------------------------------------------
// What the x transform's loader reads (XL_* below):
//  XL_PLAIN: the field f (optionally scaled per plane).
//  XL_RESID: the refinement residual (f - mu) - L x of the flux-form Laplacian, with
//            L x read from the FP64 iterate x around each point.
//  XL_DIV:   the divergence D u* / s of a face velocity (u at x-faces, v at y-faces,
//            w at z-faces with nz + 1 planes), so that the projection never stores f.
//  XL_ADJ:   the right-hand side of the projection adjoint's solve, D (g / V) of the
//            velocity cotangents plus the pressure cotangent's terms (the arithmetic of
//            k_adj_rhs), so that the adjoint never stores it either.
enum { XL_PLAIN = 0, XL_RESID = 1, XL_DIV = 2, XL_ADJ = 3 };
struct ResidIn {
    const double* x;      // current iterate (whole box; the f pointer is offset to the launch's first plane)
    const double* mu;     // mu[0] * mu_scale = weighted mean of f
    double mu_scale;
    int z0;               // first plane of this launch (for the z neighbours)
    // XL_DIV: velocity components offset to the launch's first plane, and 1/s
    // (XL_ADJ: the cotangents g_u, g_v, g_w, and g_p or NULL, with 1/s and c)
    const double* u;
    const double* v;
    const double* w;
    double div_scale;
    const double* gp;
    double adj_c;
};

// Minimum waves per SIMD of the x transforms (register caps; 1: none).
#ifndef PS_XF_WPE
#define PS_XF_WPE 1
#endif
#ifndef PS_XR_WPE
#define PS_XR_WPE 1
#endif
#ifndef PS_XI_WPE
#define PS_XI_WPE 1
#endif
// FP64 sum of x over the NT consecutive threads of each row (NT a power of two); every
// thread of the row receives it.  red: THREADS / 64 doubles of LDS (NT > 64 only).  The
// whole block calls this (it synchronises when rows span several waves).
template <int NT>
__device__ __forceinline__ double row_sum(double x, int tid, double* red) {
    static_assert((NT & (NT - 1)) == 0, "threads per row: a power of two");
    if constexpr (NT <= 64) {
#pragma unroll
        for (int o = NT / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        return x;
    } else {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = x;
        __syncthreads();
        const int w0 = (tid / NT) * (NT / 64);
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) sum += red[w0 + i];
        return sum;
    }
}

template <typename T, int M, int LM>
__global__ void __launch_bounds__((XShape<T, M>::THREADS), (LM == XL_RESID ? PS_XR_WPE : PS_XF_WPE))
k_xfwd(const double* __restrict__ f, cx<T>* __restrict__ out, int nrows, int ny, int nkxb,
       const cx<T>* __restrict__ tw, const cx<T>* __restrict__ ptw, const double* __restrict__ scale_z,
       const double* __restrict__ dz, double* __restrict__ partial, ResidIn rin, GridDev g,
       double* __restrict__ rowsum) {
    using X = XShape<T, M>;
    constexpr int NT = X::NT, R = X::R, LROW = X::LROW;
    constexpr int W = TileW<T>::value;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
    const int tid = threadIdx.x;
    const int rl = tid / NT;
    const int t = tid - rl * NT;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring rows on one XCD
    int row0 = blk * R;
    if constexpr (LM != XL_PLAIN) {
        // The residual and divergence stencils read rows at y +- 1 and z +- 1.  Blocks walk
        // tiles of kYT row groups in y, then z, then the next tile, so that the rows a block
        // needs were loaded a few blocks earlier on the same XCD (L2 hits, not refetches).
        constexpr int kYT = 8;
        const int nzb = nrows / ny, nyb = ny / R;
        if (ny % R == 0 && nyb % kYT == 0 && nzb * nyb == (int)gridDim.x) {
            const int yi = blk % kYT, tz = blk / kYT;
            const int zz = tz % nzb, yt = tz / nzb;
            row0 = zz * ny + (yt * kYT + yi) * R;
        }
    }
    const int row_u = row0 + rl;
    const bool valid = row_u < nrows;
    // Rows past the end (a partial last block) read the last row and contribute zeros:
    // every load is unconditional, so a thread's loads are all in flight together
    // (a load under a branch would be waited for before the next one is issued).
    const int row = valid ? row_u : nrows - 1;
    const double* frow = f + (size_t)row * (2 * M);
    const double zs = scale_z ? scale_z[row / ny] : 1.0;
    cx<T>* lrow = smem + rl * LROW;
    double acc0 = 0.0, acc1 = 0.0;
    double accs = 0.0;   // residual mode: the row's sum of r (FP64), for the (0,0) column
    // residual mode: row (z, y) of the whole box and its neighbours
    const int zl = row / ny;
    const int zg = rin.z0 + zl;
    const int yr = row - zl * ny;
    const size_t plane = (size_t)ny * (2 * M);
    constexpr bool RESID = LM == XL_RESID;
    const double* xrow = RESID ? rin.x + (size_t)zg * plane + (size_t)yr * (2 * M) : nullptr;
    const double* xjm = RESID ? rin.x + (size_t)zg * plane + (size_t)(yr == 0 ? ny - 1 : yr - 1) * (2 * M) : nullptr;
    const double* xjp = RESID ? rin.x + (size_t)zg * plane + (size_t)(yr + 1 == ny ? 0 : yr + 1) * (2 * M) : nullptr;
    const double mu = RESID ? rin.mu[0] * rin.mu_scale : 0.0;
    // Residual loader: the stencil of the next element (in the order the transform asks for
    // them) is requested before this element's values are used, so that two elements'
    // loads are in flight at a time; each element's value is formed before the next call
    // (an empty asm reads it), which keeps one element's stencil per register set.
    struct RawR {
        double2 f, c, a, b, qu, qd;
        double xl, xr;
    };
    const bool up = zg + 1 < g.nz, dn = zg > 0;
    // a missing neighbour's coefficient is zero (its difference is zero too), so the sums
    // are those of the present terms alone
    const double ou = RESID && up ? g.o[zg + 1] : 0.0, od = RESID && dn ? g.o[zg] : 0.0;
    const double iz = RESID ? g.idz[zg] : 0.0;
    auto rload = [&](int e, RawR& r) {
        const int n = 2 * M;
        r.f = ld_stream2<PS_NT_XF>(frow + 2 * e);
        r.c = *reinterpret_cast<const double2*>(xrow + 2 * e);
        // periodic x neighbours and the z neighbours (the row itself stands in for a missing
        // one; its term is dropped), addressed by index arithmetic so that every load is
        // unconditional
        const int il = 2 * e - 1 + (int)(e == 0) * n;
        const int ir = 2 * e + 2 - (int)(2 * e + 2 == n) * n;
        r.xl = xrow[il];
        r.xr = xrow[ir];
        r.a = *reinterpret_cast<const double2*>(xjm + 2 * e);
        r.b = *reinterpret_cast<const double2*>(xjp + 2 * e);
        r.qu = *reinterpret_cast<const double2*>(xrow + (size_t)up * plane + 2 * e);
        r.qd = *reinterpret_cast<const double2*>(xrow - (size_t)dn * plane + 2 * e);
    };
    using ShX = FftShape<M, X::EM>;
    constexpr int R0 = ShX::P.r[0];
    auto elem_of = [&](int q) { return t + (q / R0) * NT + (q % R0) * (M / R0); };
    RawR rcur, rnxt;
    int rcall = 0;   // residual loader calls so far (a compile-time count once unrolled)
    auto ld = [&](int e) -> cx<T> {
        double2 v = {0.0, 0.0};
        if constexpr (LM == XL_PLAIN) v = ld_stream2<PS_NT_XF>(frow + 2 * e);
        if constexpr (RESID) {
            if (rcall == 0) rload(e, rcur);
            if (rcall + 1 < ShX::E) rload(elem_of(rcall + 1), rnxt);
            v = rcur.f;
            const double2 c = rcur.c, a = rcur.a, b = rcur.b, qu = rcur.qu, qd = rcur.qd;
            const double xl = rcur.xl, xr = rcur.xr;
            const double idx2 = 1.0 / (g.dx * g.dx), idy2 = 1.0 / (g.dy * g.dy);
            double lz0 = 0.0, lz1 = 0.0;
            lz0 += (qu.x - c.x) * ou;
            lz1 += (qu.y - c.y) * ou;
            lz0 -= (c.x - qd.x) * od;
            lz1 -= (c.y - qd.y) * od;
            const double l0 = ((c.y - c.x) - (c.x - xl)) * idx2 + ((b.x - c.x) - (c.x - a.x)) * idy2 + lz0 * iz;
            const double l1 = ((xr - c.y) - (c.y - c.x)) * idx2 + ((b.y - c.y) - (c.y - a.y)) * idy2 + lz1 * iz;
            const double f0 = v.x - mu, f1 = v.y - mu;
            v.x = valid ? f0 - l0 : 0.0;
            v.y = valid ? f1 - l1 : 0.0;
            acc0 += v.x * v.x + v.y * v.y;
            acc1 += valid ? f0 * f0 + f1 * f1 : 0.0;
            accs += v.x + v.y;
            asm volatile("" : "+v"(v.x), "+v"(v.y));
            rcur = rnxt;
            ++rcall;
        } else if constexpr (LM == XL_DIV) {
            // f = (D u*) / s at the cells (2e, 2e + 1) of row (z, y): periodic x and y, w at z-faces
            const int n = 2 * M;
            const size_t rb = (size_t)row * n;   // row offset within the launch's planes
            const double2 uc = ld_stream2<PS_NT_XF>(rin.u + rb + 2 * e);
            const double ur = rin.u[rb + (2 * e + 2 == n ? 0 : 2 * e + 2)];
            const double2 vc = ld_stream2<PS_NT_XF>(rin.v + rb + 2 * e);
            const double2 vp = *reinterpret_cast<const double2*>(rin.v + (rb - (size_t)yr * n) +
                                                                 (size_t)(yr + 1 == ny ? 0 : yr + 1) * n + 2 * e);
            const double2 wc = *reinterpret_cast<const double2*>(rin.w + rb + 2 * e);
            const double2 wp = *reinterpret_cast<const double2*>(rin.w + rb + plane + 2 * e);
            // the same arithmetic as the stored-divergence kernel (reciprocal multiplies)
            const double idx = 1.0 / g.dx, idy = 1.0 / g.dy, idzk = g.idz[zg];
            v.x = rin.div_scale * ((uc.y - uc.x) * idx + (vp.x - vc.x) * idy + (wp.x - wc.x) * idzk);
            v.y = rin.div_scale * ((ur - uc.y) * idx + (vp.y - vc.y) * idy + (wp.y - wc.y) * idzk);
            v.x = valid ? v.x : 0.0;   // selects, not branches: the loads stay unconditional
            v.y = valid ? v.y : 0.0;
            acc0 += v.x + v.y;
        } else if constexpr (LM == XL_ADJ) {
            // f = D (g / V) + (1/s) (g_p / dz - c Dzz (g_p / dz)) at the cells (2e, 2e + 1) of
            // row (z, y): g_u, g_v differenced forward in x / y, g_w / dzc at the cell's
            // interior faces (o = 1/dzc is zero on the walls, which carry none); every load
            // unconditional (a missing z neighbour reads the row itself, its weight o is zero;
            // an absent g_p reads g_u), the row's metrics multiplied (no divisions)
            const int n = 2 * M;
            const size_t rb = (size_t)row * n;
            const bool hi = zg + 1 < g.nz, lo = zg > 0;
            const double2 uc = ld_stream2<PS_NT_XF>(rin.u + rb + 2 * e);
            const double ur = rin.u[rb + (2 * e + 2 == n ? 0 : 2 * e + 2)];
            const double2 vc = ld_stream2<PS_NT_XF>(rin.v + rb + 2 * e);
            const double2 vp = *reinterpret_cast<const double2*>(rin.v + (rb - (size_t)yr * n) +
                                                                 (size_t)(yr + 1 == ny ? 0 : yr + 1) * n + 2 * e);
            const double2 wb = *reinterpret_cast<const double2*>(rin.w + rb + 2 * e);
            const double2 wt = *reinterpret_cast<const double2*>(rin.w + rb + plane + 2 * e);
            const double* hp = rin.gp ? rin.gp : rin.u;
            const double2 h0 = *reinterpret_cast<const double2*>(hp + rb + 2 * e);
            const double2 hu = *reinterpret_cast<const double2*>(hp + rb + (size_t)hi * plane + 2 * e);
            const double2 hd = *reinterpret_cast<const double2*>(hp + rb - (size_t)lo * plane + 2 * e);
            const double idz = g.idz[zg], o_u = g.o[zg + 1], o_d = g.o[zg];
            const double idz_u = g.idz[hi ? zg + 1 : zg], idz_d = g.idz[lo ? zg - 1 : zg];
            const double sx = idz / g.dx, sy = idz / g.dy;
            // the pressure terms are formed unconditionally and weighted by zero without g_p:
            // a term under a branch would sink its loads into the branch, and the wave would
            // wait for them there
            const double gw = rin.gp ? rin.div_scale : 0.0;
            auto cell = [&](double u0, double u1, double v0, double v1, double w0, double w1, double c0, double cu,
                            double cd) {
                const double val = (u1 - u0) * sx + (v1 - v0) * sy + (w1 * o_u - w0 * o_d) * idz;
                const double hc = c0 * idz;
                const double fp = (cu * idz_u - hc) * o_u;
                const double fm = (hc - cd * idz_d) * o_d;
                return val + gw * (hc - rin.adj_c * ((fp - fm) * idz));
            };
            v.x = cell(uc.x, uc.y, vc.x, vp.x, wb.x, wt.x, h0.x, hu.x, hd.x);
            v.y = cell(uc.y, ur, vc.y, vp.y, wb.y, wt.y, h0.y, hu.y, hd.y);
            v.x = valid ? v.x : 0.0;
            v.y = valid ? v.y : 0.0;
            acc0 += v.x + v.y;
        } else {
            v.x = valid ? v.x * zs : 0.0;
            v.y = valid ? v.y * zs : 0.0;
            acc0 += v.x + v.y;
        }
        return cx<T>{(T)v.x, (T)v.y};
    };
    auto st = [&](int e, cx<T> val) { lrow[lds_pad(e)] = val; };
    fft_run<T, M, X::EM, -1>(t, lrow, 1, tw, ld, st);
    __syncthreads();
    // r2c unpack of the R rows into (kx tile, row) order: nkxb = (M + W) / W tiles of W
    // (kx > M are padding).  Fully unrolled, with the twiddle loads unconditional
    // (clamped index), so that they are all in flight together.
    constexpr int NTOT = ((M + W) / W) * R * W;
    constexpr int NIT = (NTOT + X::THREADS - 1) / X::THREADS;
    const int z0 = row0 / ny, y0 = row0 - z0 * ny;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = tid + it * X::THREADS;
        const int w = q % W;
        const int r2 = (q / W) % R;
        const int kxb = q / (W * R);
        const int row2 = row0 + r2;
        const int kx = kxb * W + w;
        const cx<T>* zr = smem + r2 * LROW;
        const int kg = min(max(kx, 1), M - 1);   // general case index, clamped into range
        const cx<T> tw_k = ptw[kg];
        const cx<T> a = zr[lds_pad(kg)];
        const cx<T> b = conjg(zr[lds_pad(M - kg)]);
        const cx<T> zz = zr[0];
        const cx<T> fe = scal(a + b, (T)0.5);
        const cx<T> d = a - b;
        const cx<T> fo = {(T)0.5 * d.y, -(T)0.5 * d.x};
        cx<T> xv = fe + cmul(tw_k, fo);
        if (kx == 0) xv = {zz.x + zz.y, (T)0};
        if (kx == M) xv = {zz.x - zz.y, (T)0};
        if (kx > M) xv = {(T)0, (T)0};
        int z = z0, y = y0 + r2;
        if (y >= ny) {   // the block's rows cross into the next plane(s)
            z += y / ny;
            y -= (y / ny) * ny;
        }
        if (q < NTOT && row2 < nrows && kxb < nkxb)
            st_stream<PS_NT_XF>(out + (((size_t)z * nkxb + kxb) * ny + y) * W + w, xv);
    }
    if constexpr (std::is_same<T, float>::value) {
        // the row's FP64 sum (plain and divergence loaders: acc0 holds it)
        if (rowsum) {
            __shared__ double red[X::THREADS / 64 > 0 ? X::THREADS / 64 : 1];
            const double rs = row_sum<NT>(RESID ? accs : acc0, tid, red);
            if (t == 0 && valid) rowsum[row] = rs;
        }
    }
    if (partial) {
        if constexpr (RESID) {
            double v[2] = {acc0, acc1};   // sum r^2, sum (f - mu)^2
            block_sum_store<2>(v, partial + 2 * blockIdx.x);
        } else {
            double v[1] = {acc0 * dz[row / ny]};   // sum dz f (zero for rows past the end)
            block_sum_store<1>(v, partial + blockIdx.x);
        }
    }
}

// ---------------------------------------------------------------------------
// MODE 0: out = scale * c2r(in).  MODE 1 (accumulate): out += scale * c2r(in) - mu.
template <typename T, int M, int MODE>
__global__ void __launch_bounds__((XShape<T, M, true>::THREADS), PS_XI_WPE)
k_xinv(const cx<T>* __restrict__ in, double* __restrict__ out, int nrows, int ny, int nkxb,
       const cx<T>* __restrict__ tw, const cx<T>* __restrict__ ptw, double scale,
       const double* __restrict__ mu, double mu_scale, const double* __restrict__ scale_z,
       const double* __restrict__ dz, double* __restrict__ partial, const double* __restrict__ col00) {
    using X = XShape<T, M, true>;
    constexpr int NT = X::NT, R = X::R, LROW = X::LROW;
    constexpr int W = TileW<T>::value;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
    __shared__ cx<T> nyq[R];   // X_M of each row (the LDS rows hold k < M)
    const int tid = threadIdx.x;
    // the R rows' half spectra (nkxb = (M + W) / W tiles of W): all loads of a thread are
    // issued before the first is consumed
    constexpr int NTOT = ((M + W) / W) * R * W;
    constexpr int NIT = (NTOT + X::THREADS - 1) / X::THREADS;
    const int row0 = blockIdx.x * R;
    const int z0 = row0 / ny, y0 = row0 - z0 * ny;
    cx<T> buf[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = tid + it * X::THREADS;
        const int w = q % W;
        const int r2 = (q / W) % R;
        const int kxb = q / (W * R);
        // unconditional loads (clamped row and tile; padding columns kx > M are read and
        // dropped), so that all of a thread's loads are in flight together
        const int row2 = min(row0 + r2, nrows - 1);
        const int kxc = min(kxb, nkxb - 1);
        int z = z0, y = y0 + (row2 - row0);
        if (y >= ny) {   // the block's rows cross into the next plane(s)
            z += y / ny;
            y -= (y / ny) * ny;
        }
        buf[it] = ld_stream<PS_NT_XI>(in + (((size_t)z * nkxb + kxc) * ny + y) * W + w);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = tid + it * X::THREADS;
        const int w = q % W;
        const int r2 = (q / W) % R;
        const int kx = (q / (W * R)) * W + w;
        if (q < NTOT && kx < M)
            smem[r2 * LROW + lds_pad(kx)] = buf[it];
        else if (q < NTOT && kx == M)
            nyq[r2] = buf[it];
    }
    __syncthreads();
    const int rl = tid / NT;
    const int t = tid - rl * NT;
    const int row_u = blockIdx.x * R + rl;
    const bool valid = row_u < nrows;
    const int row = valid ? row_u : nrows - 1;   // rows past the end compute, store nothing
    cx<T>* lrow = smem + rl * LROW;
    auto ld = [&](int e) -> cx<T> {
        cx<T> xa, xb;
        if (e == 0) {
            xa = {lrow[0].x, (T)0};
            xb = {nyq[rl].x, (T)0};
        } else {
            xa = lrow[lds_pad(e)];
            xb = lrow[lds_pad(M - e)];
        }
        cx<T> xbc = conjg(xb);
        cx<T> a = xa + xbc;
        cx<T> bb = cmul(xa - xbc, conjg(ptw[e]));
        return cx<T>{a.x - bb.y, a.y + bb.x};
    };
    double* orow = out + (size_t)row * (2 * M);
    const double sc = scale * (scale_z ? scale_z[row / ny] : 1.0);
    const double m0 = MODE == 1 ? mu[0] * mu_scale : 0.0;
    // the FP64 (0,0) coefficient of this plane (FP32 spectra, whose own (0,0) entry is zero)
    const double off = col00 ? col00[row / ny] * sc : 0.0;
    double s_d2 = 0.0, s_o2 = 0.0, s_o = 0.0;
    // MODE 1: the values being accumulated into, loaded before the transform (all in
    // flight together) in the order in which the transform hands out its results:
    // element t + b NT + m Ls of the last radix-r pass, b outer, m inner.
    using Sh = FftShape<M, X::EM>;
    constexpr int E = Sh::E, NP = Sh::NP, RL = Sh::P.r[NP - 1], LS = plan_ls(Sh::P, NP - 1);
    double2 acc_old[MODE == 1 ? E : 1];
    if constexpr (MODE == 1) {
#pragma unroll
        for (int b = 0; b < E / RL; ++b) {
#pragma unroll
            for (int m = 0; m < RL; ++m)
                acc_old[b * RL + m] = *reinterpret_cast<const double2*>(orow + 2 * (t + b * Sh::NT + m * LS));
        }
    }
    int sidx = 0;
    auto st = [&](int e, cx<T> val) {
        double2 r = {(double)val.x * sc + off, (double)val.y * sc + off};
        double2 o;
        if constexpr (MODE == 1) {
            const double2 old = acc_old[sidx++];
            o = {old.x + r.x - m0, old.y + r.y - m0};
        } else {
            o = r;
        }
        if (!valid) return;
        st_stream2<PS_NT_XI>(orow + 2 * e, o);
        s_d2 += r.x * r.x + r.y * r.y;
        s_o2 += o.x * o.x + o.y * o.y;
        s_o += o.x + o.y;
    };
    fft_run<T, M, X::EM, +1>(t, lrow, 1, tw, ld, st);
    if (partial) {
        const double dzr = valid ? dz[row / ny] : 0.0;   // (row clamped: the load is in range)
        double v[3] = {s_d2, s_o2, s_o * dzr};
        block_sum_store<3>(v, partial + 3 * blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// fwd = 1: a -> b (forward transform), fwd = 0: b -> a (inverse transform)
template <typename T, int N, int S>
__global__ void __launch_bounds__((YShape<T, N, S>::THREADS))
k_yfft(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int nzs, int nkxb,
       const cx<T>* __restrict__ tw) {
    using Y = YShape<T, N, S>;
    constexpr int NT = Y::NT, WY = Y::WY, W = TileW<T>::value;
    constexpr int NSUB = W / WY;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* smem = reinterpret_cast<cx<T>*>(smem_raw);
    const int tid = threadIdx.x;
    const int c = tid % WY;
    const int t = tid / WY;
    int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int csub = bid % NSUB;
    bid /= NSUB;
#if PS_Y_ZFAST
    // z fastest: the blocks running together on one XCD touch neighbouring z rows of the
    // same (kx tile, ky) runs of the b layout, so its strided side hits open DRAM pages
    const int nzl = (int)gridDim.x / (NSUB * nkxb);
    const int z = bid % nzl;
    const int kxb = bid / nzl;
#else
    const int kxb = bid % nkxb;
    const int z = bid / nkxb;
#endif
    const int col = csub * WY + c;
    // a-layout address of (z, kxb, e, col) and b-layout address of (kxb, e, z, col)
    const size_t abase = (((size_t)z * nkxb + kxb) * N) * W + col;
    // b has nzs planes per (kxb, ky) column; the pointer is already offset to this launch's first plane
    const size_t bbase = (((size_t)kxb * N) * nzs + z) * W + col;
    const size_t bstride = (size_t)nzs * W;
    constexpr bool kYiLoad = sizeof(T) == 8 ? PS_NT_YI_LOAD64 : PS_NT_YI_LOAD32;
    auto ld = [&](int e) -> cx<T> {
        if constexpr (S < 0)
            return ld_stream<PS_NT_YF>(in + abase + (size_t)e * W);
        else
            return ld_stream<kYiLoad>(in + bbase + (size_t)e * bstride);
    };
    auto st = [&](int e, cx<T> val) {
        if constexpr (S < 0)
            st_stream<PS_NT_YF>(out + bbase + (size_t)e * bstride, val);
        else
            st_stream<PS_NT_YI_STORE>(out + abase + (size_t)e * W, val);
    };
    if constexpr (Y::SPLIT)
        fft_run_split<T, N, Y::EMAX, S>(t, reinterpret_cast<T*>(smem_raw) + c, WY, tw, ld, st);
    else
        fft_run<T, N, kYEmax, S>(t, smem + c, WY, tw, ld, st);
}

// ---------------------------------------------------------------------------
#define PS_FFT_LENGTHS(X) \
    X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
    X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)

#ifdef PS_FFT_PRIMARY
bool fft_length_supported(int n) {
    switch (n) {
#define PS_CASE(L) case L:
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        return true;
        default:
            return false;
    }
}
#endif

template <typename T, int M>
static hipError_t xfwd_launch_t(const GridDev& g, const SpecDev<T>& s, const double* f, const double* scale_z,
                                double* partial, const ResidIn* rin, int mode, hipStream_t st) {
    using X = XShape<T, M>;
    const int nzl = s.nzc > 0 ? s.nzc : g.nz;
    const size_t zoff = (size_t)s.z0 * g.nx * g.ny;
    const int nrows = g.ny * nzl;
    const int nblk = (nrows + X::R - 1) / X::R;
    double* rsum = s.rowsum ? s.rowsum + (size_t)s.z0 * g.ny : nullptr;   // rows of this launch
    if (mode == XL_RESID) {
        // the residual form is used by the refinement, which runs its solves in FP32
        if constexpr (std::is_same<T, float>::value) {
            ResidIn r = *rin;
            r.z0 = s.z0;
            hipLaunchKernelGGL((k_xfwd<T, M, XL_RESID>), dim3(nblk), dim3(X::THREADS), X::LDS, st, f + zoff, s.a,
                               nrows, g.ny, s.nkxb, s.twx, s.ptw, nullptr, g.dz + s.z0, partial, r, g, rsum);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (mode == XL_DIV) {
        ResidIn r = *rin;
        r.z0 = s.z0;
        r.u += zoff;
        r.v += zoff;
        r.w += zoff;
        hipLaunchKernelGGL((k_xfwd<T, M, XL_DIV>), dim3(nblk), dim3(X::THREADS), X::LDS, st, nullptr, s.a, nrows, g.ny,
                           s.nkxb, s.twx, s.ptw, nullptr, g.dz + s.z0, partial, r, g, rsum);
        return hipGetLastError();
    }
    if (mode == XL_ADJ) {
        // the adjoint's fused right-hand side is used on FP64 plans only
        if constexpr (std::is_same<T, double>::value) {
            ResidIn r = *rin;
            r.z0 = s.z0;
            r.u += zoff;
            r.v += zoff;
            r.w += zoff;
            if (r.gp) r.gp += zoff;
            hipLaunchKernelGGL((k_xfwd<T, M, XL_ADJ>), dim3(nblk), dim3(X::THREADS), X::LDS, st, nullptr, s.a, nrows,
                               g.ny, s.nkxb, s.twx, s.ptw, nullptr, g.dz + s.z0, partial, r, g, rsum);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_xfwd<T, M, XL_PLAIN>), dim3(nblk), dim3(X::THREADS), X::LDS, st, f + zoff, s.a, nrows,
                       g.ny, s.nkxb, s.twx, s.ptw, scale_z ? scale_z + s.z0 : nullptr, g.dz + s.z0, partial,
                       ResidIn{}, g, rsum);
    return hipGetLastError();
}

template <typename T, int M>
static hipError_t xinv_launch_t(const GridDev& g, const SpecDev<T>& s, double* out, double scale, int mode,
                                const double* mu, double mu_scale, const double* scale_z, double* partial,
                                hipStream_t st) {
    using X = XShape<T, M, true>;
    const int nzl = s.nzc > 0 ? s.nzc : g.nz;
    const size_t zoff = (size_t)s.z0 * g.nx * g.ny;
    const int nrows = g.ny * nzl;
    const int nblk = (nrows + X::R - 1) / X::R;
    if (mode == 1)
        hipLaunchKernelGGL((k_xinv<T, M, 1>), dim3(nblk), dim3(X::THREADS), X::LDS, st, s.a, out + zoff, nrows,
                           g.ny, s.nkxb, s.twx, s.ptw, scale, mu, mu_scale, scale_z ? scale_z + s.z0 : nullptr,
                           g.dz + s.z0, partial, s.col00 ? s.col00 + s.z0 : nullptr);
    else
        hipLaunchKernelGGL((k_xinv<T, M, 0>), dim3(nblk), dim3(X::THREADS), X::LDS, st, s.a, out + zoff, nrows,
                           g.ny, s.nkxb, s.twx, s.ptw, scale, mu, mu_scale, scale_z ? scale_z + s.z0 : nullptr,
                           g.dz + s.z0, partial, s.col00 ? s.col00 + s.z0 : nullptr);
    return hipGetLastError();
}

template <typename T, int N, int S>
static hipError_t yfft_launch_t(const GridDev& g, const SpecDev<T>& s, hipStream_t st) {
    using Y = YShape<T, N, S>;
    constexpr int NSUB = TileW<T>::value / Y::WY;
    const int nzl = s.nzc > 0 ? s.nzc : g.nz;
    const int nblk = nzl * s.nkxb * NSUB;
    cx<T>* b0 = s.b + (size_t)s.z0 * TileW<T>::value;
    if (S < 0)
        hipLaunchKernelGGL((k_yfft<T, N, S>), dim3(nblk), dim3(Y::THREADS), Y::LDS, st, s.a, b0, g.nz, s.nkxb, s.twy);
    else
        hipLaunchKernelGGL((k_yfft<T, N, S>), dim3(nblk), dim3(Y::THREADS), Y::LDS, st, b0, s.a, g.nz, s.nkxb, s.twy);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_xfwd(const GridDev& g, const SpecDev<T>& s, const double* f, const double* scale_z,
                       double* partial, hipStream_t st, const double* resid_x, const double* resid_mu,
                       double mu_scale) {
    ResidIn rin{resid_x, resid_mu, mu_scale, 0, nullptr, nullptr, nullptr, 0.0};
    const int mode = resid_x ? XL_RESID : XL_PLAIN;
    switch (g.nx / 2) {
#define PS_CASE(L) \
    case L:        \
        return xfwd_launch_t<T, L>(g, s, f, scale_z, partial, &rin, mode, st);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_xfwd_div(const GridDev& g, const SpecDev<T>& s, const double* u, const double* v, const double* w,
                           double div_scale, double* partial, hipStream_t st, bool adjoint, const double* gp,
                           double adj_c) {
    ResidIn rin{nullptr, nullptr, 0.0, 0, u, v, w, div_scale, gp, adj_c};
    const int mode = adjoint ? XL_ADJ : XL_DIV;
    switch (g.nx / 2) {
#define PS_CASE(L) \
    case L:        \
        return xfwd_launch_t<T, L>(g, s, nullptr, nullptr, partial, &rin, mode, st);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_xinv(const GridDev& g, const SpecDev<T>& s, double* out, double scale, int mode,
                       const double* mu, double mu_scale, const double* scale_z, double* partial, hipStream_t st) {
    switch (g.nx / 2) {
#define PS_CASE(L) \
    case L:        \
        return xinv_launch_t<T, L>(g, s, out, scale, mode, mu, mu_scale, scale_z, partial, st);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_yfwd(const GridDev& g, const SpecDev<T>& s, hipStream_t st) {
    switch (g.ny) {
#define PS_CASE(L) \
    case L:        \
        return yfft_launch_t<T, L, -1>(g, s, st);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_yinv(const GridDev& g, const SpecDev<T>& s, hipStream_t st) {
    switch (g.ny) {
#define PS_CASE(L) \
    case L:        \
        return yfft_launch_t<T, L, +1>(g, s, st);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T, int M>
static int xblocks_t(const GridDev& g) {
    return (g.ny * g.nz + XShape<T, M>::R - 1) / XShape<T, M>::R;
}

template <typename T>
int xfwd_blocks(const GridDev& g) {
    switch (g.nx / 2) {
#define PS_CASE(L) \
    case L:        \
        return xblocks_t<T, L>(g);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return 0;
    }
}

template <typename T, int M>
static int xiblocks_t(const GridDev& g) {
    return (g.ny * g.nz + XShape<T, M, true>::R - 1) / XShape<T, M, true>::R;
}

template <typename T>
int xinv_blocks(const GridDev& g) {
    switch (g.nx / 2) {
#define PS_CASE(L) \
    case L:        \
        return xiblocks_t<T, L>(g);
        PS_FFT_LENGTHS(PS_CASE)
#undef PS_CASE
        default:
            return 0;
    }
}

#define PS_INST(T)                                                                                           \
    template hipError_t launch_xfwd<T>(const GridDev&, const SpecDev<T>&, const double*, const double*,     \
                                       double*, hipStream_t, const double*, const double*, double);         \
    template hipError_t launch_xfwd_div<T>(const GridDev&, const SpecDev<T>&, const double*, const double*, \
                                           const double*, double, double*, hipStream_t, bool, const double*,  \
                                           double);                                                           \
    template hipError_t launch_xinv<T>(const GridDev&, const SpecDev<T>&, double*, double, int,             \
                                       const double*, double, const double*, double*, hipStream_t);         \
    template hipError_t launch_yfwd<T>(const GridDev&, const SpecDev<T>&, hipStream_t);                    \
    template hipError_t launch_yinv<T>(const GridDev&, const SpecDev<T>&, hipStream_t);                    \
    template int xfwd_blocks<T>(const GridDev&);                                                            \
    template int xinv_blocks<T>(const GridDev&);

PS_INST(PS_FFT_T)

}  // namespace ps
