// FP64 stencil kernels on the staggered grid (paper Sec. 2.1, Fig. 1):
// divergence, projection / pressure update, flux-form residual, wall-normal
// Crank-Nicolson solves, CFL number (Listing 1), reductions.
//
// Threads map to (x fastest) grid points, so every warp-wide access along x is
// contiguous; neighbours in y and z come from other rows and are served by the
// caches.
#include <algorithm>

#include "ps_internal.h"
#include "reduce.h"

namespace ps {

static inline int nblocks(size_t n, int t) { return (int)((n + t - 1) / t); }

// f = scale * D(u, v, w)
__global__ void __launch_bounds__(256)
k_divergence(const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
             double* __restrict__ f, GridDev g, double scale) {
    int i, j, k;
    if (!stencil_cell(g, i, j, k)) return;
    const size_t id = ((size_t)k * g.ny + j) * g.nx + i;
    const size_t plane = (size_t)g.nx * g.ny;
    const int ip = (i + 1 == g.nx) ? 0 : i + 1;
    const int jp = (j + 1 == g.ny) ? 0 : j + 1;
    const size_t rowb = (size_t)k * plane + (size_t)j * g.nx;
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double du = (u[rowb + ip] - u[id]) * idx;
    const double dv = (v[(size_t)k * plane + (size_t)jp * g.nx + i] - v[id]) * idy;
    const double dw = (w[id + plane] - w[id]) * g.idz[k];
    f[id] = scale * (du + dv + dw);
}

// u -= s (phi_i - phi_{i-1})/dx; v likewise; interior w -= s (phi_k - phi_{k-1})/dzc_k;
// p = ps + phi - c Dzz phi (zero-flux walls; ps is p itself for the in-place update).
__global__ void __launch_bounds__(256)
k_project_update(double* __restrict__ u, double* __restrict__ v, double* __restrict__ w, double* p,
                 const double* ps, const double* __restrict__ phi, GridDev g, double s, double c) {
    int i, j, k;
    if (!stencil_cell(g, i, j, k)) return;
    const size_t id = ((size_t)k * g.ny + j) * g.nx + i;
    const size_t plane = (size_t)g.nx * g.ny;
    const int im = (i == 0) ? g.nx - 1 : i - 1;
    const int jm = (j == 0) ? g.ny - 1 : j - 1;
    // Every load is unconditional (a missing z neighbour reads the cell itself, p absent
    // reads phi) so that they are all in flight together; absent terms are selected away.
    const bool lo = k > 0, hi = k + 1 < g.nz;
    const double pc = phi[id];
    const double pim = phi[(size_t)k * plane + (size_t)j * g.nx + im];
    const double pjm = phi[(size_t)k * plane + (size_t)jm * g.nx + i];
    const double pkm = phi[lo ? id - plane : id];
    const double pkp = phi[hi ? id + plane : id];
    const double uo = u[id], vo = v[id], wo = w[id];
    const double po = (p ? ps : phi)[id];
    u[id] = uo - s * ((pc - pim) * (1.0 / g.dx));
    v[id] = vo - s * ((pc - pjm) * (1.0 / g.dy));
    // fm: the z gradient at face k (o = 1/dzc at interior faces); the bottom wall face keeps
    // its value (w - s * 0)
    const double fm = lo ? (pc - pkm) * g.o[k] : 0.0;
    const double fp = hi ? (pkp - pc) * g.o[k + 1] : 0.0;
    w[id] = wo - s * fm;
    if (p) p[id] = po + (pc - c * ((fp - fm) * g.idz[k]));
}

// out[blockIdx.x * ncomp + c] = sum of partial[b * ncomp + c] over the block's contiguous
// range of b; fixed order for a fixed launch shape.
__global__ void __launch_bounds__(256)
k_reduce(const double* __restrict__ partial, int nblk, int ncomp, int per_block, double* __restrict__ out) {
    const int b0 = blockIdx.x * per_block;
    const int b1 = min(nblk, b0 + per_block);
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) s += partial[(size_t)b * ncomp + c];
        double v[1] = {s};
        block_sum_store<1>(v, out + (size_t)blockIdx.x * ncomp + c);
        __syncthreads();
    }
}

__global__ void k_fill(double* __restrict__ p, size_t n, double v) {
    const size_t id = (size_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id < n) p[id] = v;
}

// out = c * in (out may alias in)
__global__ void k_scale(const double* in, double* out, double c, size_t n) {
    const size_t id = (size_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id < n) out[id] = c * in[id];
}

// out[z][...] = in[z][...] * zs[z] for nplanes planes of `plane` values (out may alias in)
__global__ void k_scale_planes(const double* in, double* out,
                               const double* __restrict__ zs, size_t plane, size_t n) {
    const size_t id = (size_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id < n) out[id] = in[id] * zs[id / plane];
}

// ---- Crank-Nicolson -------------------------------------------------------
// Coefficients of I - beta Dzz (same for all columns) factored once:
// fac = [l (n), invd (n), c (n)] with the LU recurrences of the Thomas method.
// kind 0 (centre): n = nz rows, wall half a cell beyond the end centres.
// kind 1 (face):   n = nz - 1 interior faces.
// The off-diagonal coupling coefficients are formed in parallel into LDS (nz <= 2048),
// then one thread runs the LU recurrence; one block per factorisation (up to four), of C or
// (trans) of its transpose.
__global__ void __launch_bounds__(256) k_cn_factor(GridDev g, CnFactorJobs jobs) {
    __shared__ double am_s[2048], ap_s[2048], sub_s[2048], sup_s[2048];
    const int jy = blockIdx.x;
    const int kind = jy == 0 ? jobs.kind[0] : (jy == 1 ? jobs.kind[1] : (jy == 2 ? jobs.kind[2] : jobs.kind[3]));
    const double beta = jy == 0 ? jobs.beta[0] : (jy == 1 ? jobs.beta[1] : (jy == 2 ? jobs.beta[2] : jobs.beta[3]));
    double* fac = jy == 0 ? jobs.fac[0] : (jy == 1 ? jobs.fac[1] : (jy == 2 ? jobs.fac[2] : jobs.fac[3]));
    const bool tr = jobs.trans != 0;
    const int n = kind == 0 ? g.nz : g.nz - 1;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        if (kind == 0) {
            am_s[r] = 1.0 / (g.dzw[r] * g.dz[r]);
            ap_s[r] = 1.0 / (g.dzw[r + 1] * g.dz[r]);
        } else {
            const int k = r + 1;
            am_s[r] = 1.0 / (g.dz[k - 1] * g.dzc[k]);
            ap_s[r] = 1.0 / (g.dz[k] * g.dzc[k]);
        }
    }
    __syncthreads();
    // C couples row r to r - 1 by -beta am_r and to r + 1 by -beta ap_r; its transpose couples
    // row r to r - 1 by -beta ap_{r-1} and to r + 1 by -beta am_{r+1}.  The couplings are formed
    // in parallel; the LU recurrence then only reads them.
    double* cs = fac + 2 * n;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        sub_s[r] = (r == 0) ? 0.0 : -beta * (tr ? ap_s[r - 1] : am_s[r]);
        const double sup = (r == n - 1) ? 0.0 : -beta * (tr ? am_s[r + 1] : ap_s[r]);
        sup_s[r] = sup;
        cs[r] = sup;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double* l = fac;
    double* invd = fac + n;
    double dprev = 1.0, cprev = 0.0;
    for (int r = 0; r < n; ++r) {
        const double diag = 1.0 + beta * (am_s[r] + ap_s[r]);
        const double lr = (r == 0) ? 0.0 : sub_s[r] / dprev;
        const double d = diag - lr * cprev;
        l[r] = lr;
        invd[r] = 1.0 / d;
        dprev = d;
        cprev = sup_s[r];
    }
}

// Tiled CN solve: a block holds 32 consecutive columns and all n <= 512 rows, split into
// up to 32 z-chunks of KZ rows; each wave holds two chunks (lanes 0-31 and 32-63, each half
// reading 256-byte rows), so a lane keeps KZ = 16 rows of a 512-row column and two blocks
// fit one CU (64 VGPRs): one block's loads run under the other's sweeps (0.96 ms per field
// at 768^2 x 512, against 1.10 ms with 64 columns and 32 rows per lane, one block per CU).
// With the shared LU factors the forward sweep y_r = x_r - l_r y_{r-1} and the backward
// sweep d_r = invd_r (y_r - c_r d_{r+1}) are affine maps whose slopes do not depend on the
// column, so each chunk runs from a zero entry value, the chunk results are combined across
// chunks through LDS, and each row adds (product of slopes) x (true entry value).  Every
// value is read and written once.  The factors are staged in LDS, as are the within-chunk
// slope products; the halves' rows differ, so neither can be a scalar operand.
// Rows past the column's end reuse the last row's factors (its backward coupling is zero,
// so nothing flows back from them): they read zero and are not stored.  One launch per
// field.
//   CN_PUT: out = C^-1 in on the solved rows (face walls untouched; in may alias out)
//   CN_ADD: out += C^-1 in on the solved rows (the old values read in groups of four rows)
//   CN_SET: as CN_PUT, and the two wall rows of face fields zeroed
//   CN_T:   out = C^-T in, given the factors of C^T (the transpose of the solve, which
//           also equals V C^-1 V^-1 with V = dz for centre fields, dzc for interior faces);
//           face walls zeroed; with out2, also out2 = c2 out
constexpr int kCnTiledRows = 512;   // the tallest column the tiled solve holds
using u32x2_t = vec2_t<unsigned int>;
template <int KZ, int MODE, bool O2 = false>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_cn_tiled(GridDev g, int kind, const double* __restrict__ fac, const double* in, double* out, double* out2,
           double c2) {
    __shared__ double bs[32][33];   // (padded: the two halves of a wave write rows 256 B apart)
    __shared__ double pf[kCnTiledRows], pbk[kCnTiledRows];   // running slopes within each chunk
    __shared__ double f_l[kCnTiledRows], f_d[kCnTiledRows], f_c[kCnTiledRows];
    const size_t plane = (size_t)g.nx * g.ny;
    const int n = kind == 0 ? g.nz : g.nz - 1;
    const int ko = kind == 0 ? 0 : 1;
    const int nch = (blockDim.x >> 6) * 2;
    // factors of rows 0 .. nch KZ - 1 (rows past the end repeat the last row's)
    for (int q = threadIdx.x; q < nch * KZ; q += blockDim.x) {
        const int r = min(q, n - 1);
        f_l[q] = fac[r];
        f_d[q] = fac[n + r];
        f_c[q] = fac[2 * n + r];
    }
    const int lane = threadIdx.x & 63, hf = lane >> 5, cl = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ch = 2 * wave + hf;            // this lane's chunk
    const int c0 = xcd_remap(blockIdx.x, gridDim.x) * 32;   // the block's first column
    const bool valid = c0 + cl < (int)plane;
    const int r0 = ch * KZ;
    // this chunk's rows of the staged tables (LDS reads at each use; the barriers between the
    // phases keep them from being held in registers across a phase)
    const double* vl = f_l + r0;
    const double* vd = f_d + r0;
    const double* vc = f_c + r0;
    // Buffer accesses: base at the wave's first row and the block's first column, the lane's
    // offset (its half's chunk, its column) in one register, the row in a scalar offset.  The
    // buffer ends at the column's last row n - 1 (clamped to 4 GiB, which a wave's 2 KZ rows
    // can only exceed when all of them lie inside), so rows past it read zero and their stores
    // are dropped.
    const int rw = 2 * wave * KZ;
    const size_t pb = ((size_t)ko + rw) * plane + c0;
    const size_t lim = n > rw ? (size_t)(n - rw) * plane * sizeof(double) : 0;
    const int nrec = (int)(lim > 0xffffffffull ? 0xffffffffull : lim);
    const int voff = (int)(((size_t)hf * KZ * plane + cl) * sizeof(double));
    const int soff = (int)(plane * sizeof(double));
    const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc((void*)(in + pb), (short)0, nrec, 0x00020000);
    double x[KZ];
#pragma unroll
    for (int i = 0; i < KZ; ++i)
        x[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rin, valid ? voff : 0, i * soff, 0));
#pragma unroll
    for (int i = 0; i < KZ; ++i) anchor(x[i]);
    __syncthreads();   // tables staged
    // The slopes of the affine sweeps do not depend on the column: within each chunk, the
    // product of -l from its first row down to row r (forward) and of -c invd from its last
    // row up to row r (backward), formed once per block; a chunk's whole slope is the
    // product at its far end.
    if (threadIdx.x < nch) {
        const int rb = threadIdx.x * KZ;
        double q = 1.0;
        for (int i = 0; i < KZ; ++i) {
            q *= -f_l[rb + i];
            pf[rb + i] = q;
        }
        q = 1.0;
        for (int i = KZ - 1; i >= 0; --i) {
            q *= -f_c[rb + i] * f_d[rb + i];
            pbk[rb + i] = q;
        }
    }
    // forward sweep from a zero entry value (the table reads are fenced in groups of four, so
    // that the compiler does not hoist a whole phase's reads into registers)
    double b = 0.0;
#pragma unroll
    for (int i = 0; i < KZ; ++i) {
        if (i % 4 == 0) asm volatile("" ::: "memory");
        b = x[i] - vl[i] * b;   // l[0] = 0
        x[i] = b;
    }
    bs[ch][cl] = b;
    __syncthreads();
    double yin = 0.0;
#pragma unroll 4
    for (int v = 0; v < nch - 1; ++v) {
        const double t = pf[v * KZ + KZ - 1] * yin + bs[v][cl];
        yin = v < ch ? t : yin;
    }
    const double* vpf = pf + r0;
#pragma unroll
    for (int i = 0; i < KZ; ++i) {
        if (i % 4 == 0) asm volatile("" ::: "memory");
        x[i] += vpf[i] * yin;
    }
    __syncthreads();
    // backward sweep from a zero entry value (cs[n-1] = 0)
    b = 0.0;
#pragma unroll
    for (int i = KZ - 1; i >= 0; --i) {
        if (i % 4 == 3) asm volatile("" ::: "memory");
        b = (x[i] - vc[i] * b) * vd[i];
        x[i] = b;
    }
    bs[ch][cl] = b;
    __syncthreads();
    double din = 0.0;
#pragma unroll 4
    for (int v = nch - 1; v > 0; --v) {
        const double t = pbk[v * KZ] * din + bs[v][cl];
        din = v > ch ? t : din;
    }
    const double* vpb = pbk + r0;
#pragma unroll
    for (int i = KZ - 1; i >= 0; --i) {
        if (i % 4 == 3) asm volatile("" ::: "memory");
        x[i] += vpb[i] * din;
    }
    if (!valid) return;
    // the second output only in its own instantiation (O2), which keeps it out of the others'
    // registers
    if (!(MODE == CN_T && O2)) out2 = nullptr;
    const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc((void*)(out + pb), (short)0, nrec, 0x00020000);
    if constexpr (MODE == CN_ADD) {
        // rows in groups of four: their old values loaded together, then added and stored
#pragma unroll
        for (int i0 = 0; i0 < KZ; i0 += 4) {
            double ov[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                ov[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rout, voff, (i0 + i) * soff, 0));
#pragma unroll
            for (int i = 0; i < 4; ++i) anchor(ov[i]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, ov[i] + x[i0 + i]), rout, voff,
                                                      (i0 + i) * soff, 0);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < KZ; ++i)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x[i]), rout, voff, i * soff, 0);
    if constexpr (MODE == CN_T && O2) {
        const __amdgpu_buffer_rsrc_t rout2 = __builtin_amdgcn_make_buffer_rsrc((void*)(out2 + pb), (short)0, nrec, 0x00020000);
#pragma unroll
        for (int i = 0; i < KZ; ++i)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, c2 * x[i]), rout2, voff, i * soff, 0);
    }
    const size_t col = (size_t)c0 + cl;
    if (MODE != CN_PUT && kind == 1 && ch == 0) {
        out[col] = 0.0;
        out[(size_t)g.nz * plane + col] = 0.0;
        if (out2) {
            out2[col] = 0.0;
            out2[(size_t)g.nz * plane + col] = 0.0;
        }
    }
}

// Lane-per-column form for columns taller than the tiled kernel holds (nz > 512; one job per
// launch).
//   mode 0: out = C^-1 in on the solved rows (in may alias out; face walls untouched)
//   mode 1: as mode 0 with the factors of C^T, face walls zeroed (and out2 = c2 out when given)
//   mode 2: out += C^-1 in on the solved rows, in used as scratch
__global__ void __launch_bounds__(256) k_cn_column(GridDev g, CnJob jb, int mode) {
    const size_t plane = (size_t)g.nx * g.ny;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    const int kind = jb.kind;
    const int n = kind == 0 ? g.nz : g.nz - 1;
    const int ko = kind == 0 ? 0 : 1;
    const double* l = jb.fac;
    const double* invd = jb.fac + n;
    const double* cs = jb.fac + 2 * n;
    const int trans = mode == 1;
    if (mode == 2) {
        double* r = const_cast<double*>(jb.in) + (size_t)ko * plane + col;
        double* q = jb.out + (size_t)ko * plane + col;
        double y = r[0];
        for (int k = 1; k < n; ++k) {
            y = r[(size_t)k * plane] - l[k] * y;
            r[(size_t)k * plane] = y;
        }
        double d = y * invd[n - 1];
        q[(size_t)(n - 1) * plane] += d;
        for (int k = n - 2; k >= 0; --k) {
            d = (r[(size_t)k * plane] - cs[k] * d) * invd[k];
            q[(size_t)k * plane] += d;
        }
        return;
    }
    const double* r = jb.in + (size_t)ko * plane + col;
    double* x = jb.out + (size_t)ko * plane + col;
    double y = r[0];
    x[0] = y;
    for (int k = 1; k < n; ++k) {
        y = r[(size_t)k * plane] - l[k] * y;
        x[(size_t)k * plane] = y;
    }
    double d = y * invd[n - 1];
    x[(size_t)(n - 1) * plane] = d;
    for (int k = n - 2; k >= 0; --k) {
        d = (x[(size_t)k * plane] - cs[k] * d) * invd[k];
        x[(size_t)k * plane] = d;
    }
    double* x2 = jb.out2 ? jb.out2 + (size_t)ko * plane + col : nullptr;
    if (trans && x2)
        for (int k = 0; k < n; ++k) x2[(size_t)k * plane] = jb.c2 * x[(size_t)k * plane];
    if (trans && kind == 1) {
        jb.out[col] = 0.0;
        jb.out[(size_t)g.nz * plane + col] = 0.0;
        if (jb.out2) {
            jb.out2[col] = 0.0;
            jb.out2[(size_t)g.nz * plane + col] = 0.0;
        }
    }
}

template <int MODE>
static hipError_t cn_tiled_launch(const GridDev& g, const CnJob& j, hipStream_t st) {
    const size_t plane = (size_t)g.nx * g.ny;
    const int n = j.kind == 0 ? g.nz : g.nz - 1;
    const int kz = n <= 128 ? 4 : (n <= 256 ? 8 : 16);
    const int nch = (n + kz - 1) / kz;
    const dim3 grid((unsigned)((plane + 31) / 32));
    const dim3 block(64 * ((nch + 1) / 2));
#define PS_CN_ARGS g, j.kind, j.fac, j.in, j.out, j.out2, j.c2
    bool o2 = false;
    if constexpr (MODE == CN_T) o2 = j.out2 != nullptr;
    if constexpr (MODE == CN_T) if (o2) {
        switch (kz) {
            case 4: hipLaunchKernelGGL((k_cn_tiled<4, MODE, true>), grid, block, 0, st, PS_CN_ARGS); break;
            case 8: hipLaunchKernelGGL((k_cn_tiled<8, MODE, true>), grid, block, 0, st, PS_CN_ARGS); break;
            default: hipLaunchKernelGGL((k_cn_tiled<16, MODE, true>), grid, block, 0, st, PS_CN_ARGS); break;
        }
    }
    if (!o2) {
        switch (kz) {
            case 4: hipLaunchKernelGGL((k_cn_tiled<4, MODE>), grid, block, 0, st, PS_CN_ARGS); break;
            case 8: hipLaunchKernelGGL((k_cn_tiled<8, MODE>), grid, block, 0, st, PS_CN_ARGS); break;
            default: hipLaunchKernelGGL((k_cn_tiled<16, MODE>), grid, block, 0, st, PS_CN_ARGS); break;
        }
    }
#undef PS_CN_ARGS
    return hipGetLastError();
}

// ---- CFL (Listing 1) ------------------------------------------------------
// Each block reduces the maximum over its rows and posts it with one atomic max
// (non-negative doubles order like their bit patterns, and every NaN pattern lies above
// +Inf).  The maximum propagates NaN (fmax would drop it), so a non-finite velocity gives a
// non-finite Courant number.
constexpr int kCflBlocks = 2048;
__device__ __forceinline__ double nan_max(double q, double c) { return (c > q || c != c) ? c : q; }
// Each block walks the rows of one y index upward through one segment of the z range,
// threads along x; the loads of up to four x positions per thread are issued together
// (clamped indices, unused values dropped).  Blocks are numbered so that neighbouring y
// indices run on one XCD: the next-row v values a block reads are its neighbour's own row,
// and the w row of plane k + 1 is read again by the same block at k + 1, both from that
// XCD's L2 (each field then crosses HBM about once).
__global__ void __launch_bounds__(256)
k_cfl(const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w, GridDev g,
      int nseg, unsigned long long* __restrict__ out) {
    __shared__ double wmax[4];
    const size_t plane = (size_t)g.nx * g.ny;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int j = blk % g.ny, seg = blk / g.ny;
    const int jp = (j + 1 == g.ny) ? 0 : j + 1;
    const int kb = (int)((long long)seg * g.nz / nseg), ke = (int)((long long)(seg + 1) * g.nz / nseg);
    constexpr int E = 4;
    double q = 0.0;
    for (int k = kb; k < ke; ++k) {
        const size_t rb = ((size_t)k * g.ny + j) * g.nx, rn = ((size_t)k * g.ny + jp) * g.nx;
        const double dzk = g.dz[k];
        for (int i0 = threadIdx.x; i0 < g.nx; i0 += E * blockDim.x) {
            double uc[E], un[E], vc[E], vn[E], wb[E], wt[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int i = min(i0 + e * (int)blockDim.x, g.nx - 1);
                const int ip = (i + 1 == g.nx) ? 0 : i + 1;
                uc[e] = u[rb + i];
                un[e] = u[rb + ip];
                vc[e] = v[rb + i];
                vn[e] = v[rn + i];
                wb[e] = w[rb + i];
                wt[e] = w[rb + plane + i];
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double c = fabs(wb[e] + wt[e]) / dzk + fabs(vc[e] + vn[e]) / g.dy + fabs(uc[e] + un[e]) / g.dx;
                // positions past the row's end repeat its last point: the maximum is unchanged
                q = nan_max(q, 0.5 * c);
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q = nan_max(q, __shfl_xor(q, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) q = nan_max(q, wmax[wv]);
        atomicMax(out, (unsigned long long)__double_as_longlong(q));
    }
}

// out[0] = max(out[0], max |p| (x zs[plane], when given)) over n values; out[0] must hold a
// non-negative double.  NaN propagates.
__global__ void __launch_bounds__(256)
k_absmax(const double* __restrict__ p, size_t n, size_t plane, const double* __restrict__ zs,
         unsigned long long* __restrict__ out) {
    __shared__ double wmax[4];
    double q = 0.0;
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += (size_t)gridDim.x * blockDim.x) {
        const double v = zs ? p[id] * zs[id / plane] : p[id];
        q = nan_max(q, fabs(v));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q = nan_max(q, __shfl_xor(q, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) q = nan_max(q, wmax[wv]);
        atomicMax(out, (unsigned long long)__double_as_longlong(q));
    }
}

// ---- wall-normal statistics ------------------------------------------------
// Block k sums plane k of T (k = 0..nz) and, for k < nz, the plane of
// wbar Tbar = (w_k + w_{k+1}) (T_k + T_{k+1}) / 4 over cell-centre plane k.
__global__ void __launch_bounds__(1024)
k_plane_sums(const double* __restrict__ w, const double* __restrict__ t, GridDev g, double* __restrict__ sums) {
    const int k = blockIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const double* tk = t + (size_t)k * plane;
    double v[2] = {0.0, 0.0};
    for (size_t q = threadIdx.x; q < plane; q += blockDim.x) {
        const double tc = tk[q];
        v[0] += tc;
        if (k < g.nz) {
            const double wb = 0.5 * (w[(size_t)k * plane + q] + w[(size_t)(k + 1) * plane + q]);
            v[1] += wb * (0.5 * (tc + tk[q + plane]));
        }
    }
    block_sum_store<2>(v, sums + 2 * k);
}

// mean_t[k] = sum_T[k] / (nx ny); flux[k] = sum_wT[k] / (nx ny) - kappa (mean_t[k+1] - mean_t[k]) / dz_k
__global__ void k_heat_flux(const double* __restrict__ sums, GridDev g, double kappa, double* __restrict__ mean_t,
                            double* __restrict__ flux) {
    const double inv = 1.0 / ((double)g.nx * (double)g.ny);
    for (int k = threadIdx.x; k <= g.nz; k += blockDim.x) {
        const double tm = sums[2 * k] * inv;
        mean_t[k] = tm;
        if (k < g.nz) flux[k] = sums[2 * k + 1] * inv - kappa * (sums[2 * (k + 1)] * inv - tm) / g.dz[k];
    }
}

// ---- projection adjoint -----------------------------------------------------
// With Vf = dz on u, v and dzc on interior w, and Vc = dz:
//   g_u* = g_u - Vf G S [ D Vf^-1 g_u + (1/s) (I - c Dzz) Vc^-1 g_p ].
// k_adj_rhs forms the bracket (wall-face cotangents of w are ignored), k_adj_update
// the final combination.
__global__ void __launch_bounds__(256)
k_adj_rhs(const double* __restrict__ gu, const double* __restrict__ gv, const double* __restrict__ gw,
          const double* __restrict__ gp, double* __restrict__ f, GridDev g, double inv_s, double c) {
    int i, j, k;
    if (!stencil_cell(g, i, j, k)) return;
    const size_t id = ((size_t)k * g.ny + j) * g.nx + i;
    const size_t plane = (size_t)g.nx * g.ny;
    const int ip = (i + 1 == g.nx) ? 0 : i + 1;
    const int jp = (j + 1 == g.ny) ? 0 : j + 1;
    // unconditional loads (a missing z neighbour reads the cell itself, gp absent reads
    // gu), absent terms weighted by o = 0 (walls) or selected away: all loads in flight
    // together; the same arithmetic as the fused loader of the x transform
    const bool lo = k > 0, hi = k + 1 < g.nz;
    const double idz = g.idz[k], o_u = g.o[k + 1], o_d = g.o[k];
    const double idz_u = g.idz[hi ? k + 1 : k], idz_d = g.idz[lo ? k - 1 : k];
    const double sx = idz / g.dx, sy = idz / g.dy;
    const double gu0 = gu[id], gu1 = gu[(size_t)k * plane + (size_t)j * g.nx + ip];
    const double gv0 = gv[id], gv1 = gv[(size_t)k * plane + (size_t)jp * g.nx + i];
    const double gwt = gw[id + plane], gwb = gw[id];
    const double* hp = gp ? gp : gu;
    const double h0 = hp[id], hu = hp[hi ? id + plane : id], hd = hp[lo ? id - plane : id];
    const double val = (gu1 - gu0) * sx + (gv1 - gv0) * sy + (gwt * o_u - gwb * o_d) * idz;
    // pressure terms formed unconditionally, weighted by zero without gp (no branch to sink
    // their loads into)
    const double hc = h0 * idz;
    const double fp = (hu * idz_u - hc) * o_u;
    const double fm = (hc - hd * idz_d) * o_d;
    f[id] = val + (gp ? inv_s : 0.0) * (hc - c * ((fp - fm) * idz));
}

__global__ void __launch_bounds__(256)
k_adj_update(const double* __restrict__ gu, const double* __restrict__ gv, const double* __restrict__ gw,
             const double* __restrict__ phi, double* __restrict__ ou, double* __restrict__ ov,
             double* __restrict__ ow, GridDev g) {
    int i, j, k;
    if (!stencil_cell(g, i, j, k)) return;
    const size_t id = ((size_t)k * g.ny + j) * g.nx + i;
    const size_t plane = (size_t)g.nx * g.ny;
    const int im = (i == 0) ? g.nx - 1 : i - 1;
    const int jm = (j == 0) ? g.ny - 1 : j - 1;
    const bool lo = k > 0;
    const double pc = phi[id];
    const double pim = phi[(size_t)k * plane + (size_t)j * g.nx + im];
    const double pjm = phi[(size_t)k * plane + (size_t)jm * g.nx + i];
    const double pkm = phi[lo ? id - plane : id];
    const double gu0 = gu[id], gv0 = gv[id], gw0 = gw[id];
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    ou[id] = gu0 - g.dz[k] * ((pc - pim) * idx);
    ov[id] = gv0 - g.dz[k] * ((pc - pjm) * idy);
    ow[id] = lo ? gw0 - (pc - pkm) : 0.0;
    if (k + 1 == g.nz) ow[id + plane] = 0.0;
}

hipError_t launch_adj_rhs(const GridDev& g, const double* gu, const double* gv, const double* gw, const double* gp,
                          double* f, double inv_s, double c, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_rhs, dim3(stencil_blocks(g)), dim3(kStencilBlock), 0, st, gu, gv, gw, gp, f, g, inv_s, c);
    return hipGetLastError();
}

hipError_t launch_adj_update(const GridDev& g, const double* gu, const double* gv, const double* gw,
                             const double* phi, double* ou, double* ov, double* ow, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_update, dim3(stencil_blocks(g)), dim3(kStencilBlock), 0, st, gu, gv, gw, phi, ou, ov, ow, g);
    return hipGetLastError();
}

// ---- launchers --------------------------------------------------------------
hipError_t launch_divergence(const GridDev& g, const double* u, const double* v, const double* w, double* f,
                             double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_divergence, dim3(stencil_blocks(g)), dim3(kStencilBlock), 0, st, u, v, w, f, g, scale);
    return hipGetLastError();
}

hipError_t launch_project_update(const GridDev& g, double* u, double* v, double* w, double* p, const double* phi,
                                 double s, double c, hipStream_t st, const double* p_src) {
    hipLaunchKernelGGL(k_project_update, dim3(stencil_blocks(g)), dim3(kStencilBlock), 0, st, u, v, w, p,
                       p_src ? p_src : p, phi, g, s, c);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_nonfinite(const double* __restrict__ p, size_t n, unsigned* flag) {
    const size_t id = (size_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    bool bad = false;
    if (id < n) bad = !isfinite(p[id]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

hipError_t launch_nonfinite(const double* p, size_t n, unsigned* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_nonfinite, dim3(nblocks(n, 256)), dim3(256), 0, st, p, n, flag);
    return hipGetLastError();
}

// Two passes when there are many partials: 1024-way split into `scratch`, then one block.
hipError_t launch_reduce2(const double* partial, int nblk, int ncomp, double* scratch, double* out, hipStream_t st) {
    if (nblk > 4096) {
        const int nb1 = 1024;
        const int per = (nblk + nb1 - 1) / nb1;
        hipLaunchKernelGGL(k_reduce, dim3(nb1), dim3(256), 0, st, partial, nblk, ncomp, per, scratch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)scratch, nb1, ncomp, nb1, out);
    } else {
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, partial, nblk, ncomp, nblk, out);
    }
    return hipGetLastError();
}

// Streaming copy: the practical HBM ceiling a one-read / one-write stage is compared
// against.  One 16-byte vector per thread, one pass over the data (no grid-stride loop),
// non-temporal loads and stores; a tail of fewer than 16 bytes goes byte by byte.
// Measured on 4 GiB: 6.47 TB/s, against 4.7-5.0 TB/s for grid-stride loops of 4-32
// blocks per CU with four vectors per thread, and 4.72 TB/s for hipMemcpy.
__global__ void __launch_bounds__(256)
k_stream_copy(const vec2_t<double>* __restrict__ src, vec2_t<double>* __restrict__ dst, size_t nvec) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < nvec) __builtin_nontemporal_store(__builtin_nontemporal_load(src + id), dst + id);
}

__global__ void k_copy_tail(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, size_t n) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) dst[id] = src[id];
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, int ncu, hipStream_t st) {
    (void)ncu;
    const size_t nvec = bytes / 16, tail = bytes - nvec * 16;
    if (nvec) {
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, st,
                           (const vec2_t<double>*)src, (vec2_t<double>*)dst, nvec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tail) {
        hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, st, (const unsigned char*)src + nvec * 16,
                           (unsigned char*)dst + nvec * 16, tail);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_scale(const double* in, double* out, double c, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(nblocks(n, 256)), dim3(256), 0, st, in, out, c, n);
    return hipGetLastError();
}

hipError_t launch_scale_planes(const GridDev& g, const double* in, double* out, const double* zs, int nplanes,
                               size_t plane, hipStream_t st) {
    (void)g;
    const size_t n = (size_t)nplanes * plane;
    hipLaunchKernelGGL(k_scale_planes, dim3(nblocks(n, 256)), dim3(256), 0, st, in, out, zs, plane, n);
    return hipGetLastError();
}

hipError_t launch_heat_flux(const GridDev& g, const double* w, const double* t, double kappa, double* sums,
                            double* mean_t, double* flux, hipStream_t st) {
    hipLaunchKernelGGL(k_plane_sums, dim3(g.nz + 1), dim3(1024), 0, st, w, t, g, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_heat_flux, dim3(1), dim3(256), 0, st, sums, g, kappa, mean_t, flux);
    return hipGetLastError();
}

hipError_t launch_cn_factor(const GridDev& g, const CnFactorJobs& jobs, hipStream_t st) {
    hipLaunchKernelGGL(k_cn_factor, dim3(jobs.n), dim3(256), 0, st, g, jobs);
    return hipGetLastError();
}

hipError_t launch_cn_jobs(const GridDev& g, int mode, const CnJobs& jobs, hipStream_t st) {
    if (jobs.n < 1 || jobs.n > 4) return hipErrorInvalidValue;
    if (g.nz <= kCnTiledRows) {
        for (int q = 0; q < jobs.n; ++q) {
            hipError_t e;
            switch (mode) {
                case CN_PUT: e = cn_tiled_launch<CN_PUT>(g, jobs.j[q], st); break;
                case CN_ADD: e = cn_tiled_launch<CN_ADD>(g, jobs.j[q], st); break;
                case CN_SET: e = cn_tiled_launch<CN_SET>(g, jobs.j[q], st); break;
                default: e = cn_tiled_launch<CN_T>(g, jobs.j[q], st); break;
            }
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const size_t plane = (size_t)g.nx * g.ny;
    for (int q = 0; q < jobs.n; ++q) {
        CnJob jb = jobs.j[q];
        hipLaunchKernelGGL(k_cn_column, dim3(nblocks(plane, 256)), dim3(256), 0, st, g, jb,
                           mode == CN_T ? 1 : (mode == CN_ADD ? 2 : 0));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (mode == CN_SET && jb.kind == 1) {
            if ((e = launch_fill(jb.out, plane, 0.0, st)) != hipSuccess) return e;
            if ((e = launch_fill(jb.out + (size_t)g.nz * plane, plane, 0.0, st)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_cn_solve(const GridDev& g, int kind, const double* fac, double* x, hipStream_t st) {
    CnJobs jobs{};
    jobs.j[0] = CnJob{fac, x, x, nullptr, 0.0, kind};
    jobs.n = 1;
    return launch_cn_jobs(g, CN_SET, jobs, st);
}

hipError_t launch_absmax(const double* p, size_t n, size_t plane, const double* zs, double* out, hipStream_t st) {
    hipError_t e = launch_fill(out, 1, 0.0, st);
    if (e != hipSuccess || n == 0) return e;
    const int nb = (int)std::min<size_t>((size_t)kCflBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(256), 0, st, p, n, plane, zs, reinterpret_cast<unsigned long long*>(out));
    return hipGetLastError();
}

hipError_t launch_cfl(const GridDev& g, const double* u, const double* v, const double* w, double* out,
                      hipStream_t st) {
    hipError_t e = launch_fill(out, 1, 1e-8, st);
    if (e != hipSuccess) return e;
    // z segments per y index: about kCflBlocks blocks in all (one resident round of 256-thread
    // blocks), at least one and at most nz
    const int nseg = std::max(1, std::min(g.nz, kCflBlocks / g.ny));
    const int nb = g.ny * nseg;
    hipLaunchKernelGGL(k_cfl, dim3(nb), dim3(256), 0, st, u, v, w, g, nseg,
                       reinterpret_cast<unsigned long long*>(out));
    return hipGetLastError();
}

}  // namespace ps
