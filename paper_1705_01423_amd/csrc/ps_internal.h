// Internal declarations of the pressure-Poisson library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "fft_engine.h"

namespace ps {

// Marks a loaded value as used at this point (an empty asm reading its register).  Loads
// whose values are only used under a (uniform) branch are otherwise sunk into it by the
// compiler, and a load under a branch is waited for before anything after the branch:
// anchoring keeps a group of loads together, in flight at once, with one wait.
__device__ __forceinline__ void anchor(double v) { asm volatile("" ::"v"(v)); }


// Spectral tile width: W consecutive kx columns are stored together so that
// every row of a tile is one 128-byte segment (8 complex FP64 or 16 complex FP32).
template <typename T>
struct TileW;
template <>
struct TileW<double> {
    static constexpr int value = 8;
};
template <>
struct TileW<float> {
    static constexpr int value = 16;
};

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so that blocks
// with neighbouring logical indices (which share cache lines) run on one XCD and
// share its L2.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    if (nblk % 8 != 0) return bid;
    return (bid % 8) * (nblk / 8) + bid / 8;
}

// Streaming accesses: each value of a stage's input is read once and each output
// written once.  With NT set they carry the non-temporal hint; which stages gain from
// it was measured per kernel (the x transforms and the inverse y transform do, the
// forward y transform and the z solve do not).
template <typename T>
using vec2_t = T __attribute__((ext_vector_type(2)));

template <bool NT, typename T>
__device__ __forceinline__ cx<T> ld_stream(const cx<T>* p) {
    if constexpr (NT) {
        const vec2_t<T> v = __builtin_nontemporal_load(reinterpret_cast<const vec2_t<T>*>(p));
        return cx<T>{v.x, v.y};
    } else {
        return *p;
    }
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(cx<T>* p, cx<T> v) {
    if constexpr (NT) {
        vec2_t<T> w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, reinterpret_cast<vec2_t<T>*>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ double2 ld_stream2(const double* p) {
    if constexpr (NT) {
        const vec2_t<double> v = __builtin_nontemporal_load(reinterpret_cast<const vec2_t<double>*>(p));
        return double2{v.x, v.y};
    } else {
        return *reinterpret_cast<const double2*>(p);
    }
}
template <bool NT>
__device__ __forceinline__ void st_stream2(double* p, double2 v) {
    if constexpr (NT) {
        vec2_t<double> w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, reinterpret_cast<vec2_t<double>*>(p));
    } else {
        *reinterpret_cast<double2*>(p) = v;
    }
}

// Non-temporal choice per stage (build-time overrides for measurement).
#ifndef PS_NT_XF
#define PS_NT_XF 1
#endif
#ifndef PS_NT_YF
#define PS_NT_YF 0
#endif
#ifndef PS_NT_YI_LOAD64
#define PS_NT_YI_LOAD64 1
#endif
#ifndef PS_NT_YI_LOAD32
#define PS_NT_YI_LOAD32 1
#endif
#ifndef PS_NT_YI_STORE
#define PS_NT_YI_STORE 1
#endif
// z solves: the register-tile kernel's tile loads and stores (FP64 1024^2 x 512 z stage
// 1.57 -> 1.45 ms against plain accesses), and the streamed FP32 kernel's stores (refined
// solve 20.44 -> 20.34 ms)
#ifndef PS_NT_Z
#define PS_NT_Z 1
#endif
#ifndef PS_NT_ZPIPE_STORE
#define PS_NT_ZPIPE_STORE 1
#endif
#ifndef PS_NT_XI
#define PS_NT_XI 1
#endif

// Device-side grid tables (FP64).  Built once per plan on the host.
struct GridDev {
    int nx, ny, nz;
    double dx, dy;
    const double* dz;    // nz
    const double* dzc;   // nz+1, interior entries 1..nz-1
    const double* o;     // nz+1, 1/dzc interior, 0 at walls
    const double* dzw;   // nz+1, dzc interior, dz/2 at walls
    const double* lamx;  // nx/2+1
    const double* lamy;  // ny
    const double* idz;   // nz, 1/dz
    const double* idzw;  // nz+1, 1/dzw
};

// Stencil kernels: one thread per cell; a block covers kStencilBlock consecutive x of
// one (y, z) row.  Blocks walk a tile of kStencilTY rows in y, then z, then the next
// tile, so that the z +- 1 (and y +- 1) neighbour rows a block reads were loaded a few
// blocks earlier on the same XCD and are still in its L2.
constexpr int kStencilBlock = 256;
constexpr int kStencilTY = 8;
inline int stencil_blocks(const GridDev& g) {
    const int nxs = (g.nx + kStencilBlock - 1) / kStencilBlock;
    const int nyt = (g.ny + kStencilTY - 1) / kStencilTY;
    return nxs * kStencilTY * g.nz * nyt;
}
// Cell (i, j, k) of this thread; false for the padding threads of ragged rows / tiles.
__device__ __forceinline__ bool stencil_cell(const GridDev& g, int& i, int& j, int& k) {
    int r = xcd_remap(blockIdx.x, gridDim.x);
    const int nxs = (g.nx + kStencilBlock - 1) / kStencilBlock;
    const int xs = r % nxs;
    r /= nxs;
    const int jin = r % kStencilTY;
    r /= kStencilTY;
    k = r % g.nz;
    j = (r / g.nz) * kStencilTY + jin;
    i = xs * kStencilBlock + (int)threadIdx.x;
    return i < g.nx && j < g.ny;
}

// Per-precision spectral machinery: twiddle tables and buffers.
template <typename T>
struct SpecDev {
    int w;                    // tile width
    int nkxb;                 // number of kx tiles
    const cx<T>* twx;         // exp(-2 pi i q / (nx/2)), q < nx/2
    const cx<T>* ptw;         // exp(-2 pi i k / nx), k <= nx/2
    const cx<T>* twy;         // exp(-2 pi i q / ny), q < ny
    cx<T>* a;                 // [nz][nkxb][ny][W]
    cx<T>* b;                 // [nkxb][ny][nz][W]
    T* piv;                   // z-solve pivots, same layout as b (real); tall columns only
    const T* etab = nullptr;  // pivot excess entering each lane chunk of the tiled z solve
    cx<T>* bz = nullptr;      // z solve output in the b layout (nullptr: in place in b)
    // FP32 spectra: the singular (0,0) column is carried in FP64 beside them.  The x transform
    // writes each row's FP64 sum (rowsum, [nz][ny]), the plane sums (psum, [nz]) feed the
    // (0,0) column solve, whose FP64 result (col00, [nz]) the inverse x transform adds to
    // every point of its plane (the spectrum's own (0,0) entry is then zero).
    double* rowsum = nullptr;
    double* psum = nullptr;
    double* col00 = nullptr;
    // Plane range of the x / y stages: planes [z0, z0 + nzc) (nzc = 0: all).  Buffer a
    // is then indexed relative to z0 (it may hold just those planes); b stays absolute.
    int ncu = 0;              // compute units of the plan's device (persistent launches)
    int z0 = 0;
    int nzc = 0;
};

// Launchers (all asynchronous on `st`).  Return hipSuccess or the launch error.
// FFT stages.
// resid_x != NULL (FP32 only): the transformed input is the residual (f - mu) - L x, with
// mu = resid_mu[0] * mu_scale, and partial receives {sum r^2, sum (f - mu)^2} per block.
template <typename T>
hipError_t launch_xfwd(const GridDev& g, const SpecDev<T>& s, const double* f, const double* scale_z,
                       double* partial, hipStream_t st, const double* resid_x = nullptr,
                       const double* resid_mu = nullptr, double mu_scale = 0.0);
// The x transform of the divergence (D u*) * div_scale of a face velocity (u, v: nz planes,
// w: nz + 1 planes), formed while loading; partial (optional) receives sum dz f per block.
// adjoint (FP64 only): instead the projection adjoint's right-hand side from the velocity
// cotangents (u, v, w) and the pressure cotangent gp (or NULL), with 1/s = div_scale and c.
template <typename T>
hipError_t launch_xfwd_div(const GridDev& g, const SpecDev<T>& s, const double* u, const double* v, const double* w,
                           double div_scale, double* partial, hipStream_t st, bool adjoint = false,
                           const double* gp = nullptr, double adj_c = 0.0);
template <typename T>
hipError_t launch_yfwd(const GridDev& g, const SpecDev<T>& s, hipStream_t st);
template <typename T>
hipError_t launch_yinv(const GridDev& g, const SpecDev<T>& s, hipStream_t st);
// mode 0: out = scale * x;  mode 1: out += scale * x - mu[0]
// scale_z (optional): multiply plane z additionally by scale_z[z]
// partial (optional): per-block sums {sum (scale x)^2, sum out^2, sum dz out}
template <typename T>
hipError_t launch_xinv(const GridDev& g, const SpecDev<T>& s, double* out, double scale, int mode,
                       const double* mu, double mu_scale, const double* scale_z, double* partial, hipStream_t st);
template <typename T>
int xfwd_blocks(const GridDev& g);
template <typename T>
int xinv_blocks(const GridDev& g);

// z solves on buffer b (all columns except (0,0)), then the (0,0) column.
template <typename T>
hipError_t launch_zsolve(const GridDev& g, const SpecDev<T>& s, hipStream_t st);
// whether launch_zsolve can write its result to SpecDev::bz instead of in place
template <typename T>
bool zsolve_out_of_place(const GridDev& g);
// The tiled z solve (columns of up to 1024 rows) starts each lane's chunk of rows from the
// pivot excess of the row above it.  The excesses depend only on the grid and the
// wavenumbers, so they are formed once per plan (sequential FP64 recurrence per column) into
// a table of zexcess_elems() entries [kx tile][ky][chunk][W]; 0 entries when the columns are
// too tall for the tiled solve.
template <typename T>
bool zsolve_tiled(const GridDev& g);
template <typename T>
size_t zexcess_elems(const GridDev& g, int nkxb);
template <typename T>
hipError_t launch_zexcess(const GridDev& g, int nkxb, T* etab, hipStream_t st);
template <typename T>
hipError_t launch_zsolve00(const GridDev& g, const SpecDev<T>& s, double* defect, hipStream_t st);

bool fft_length_supported(int n);

// Field kernels (FP64).
hipError_t launch_divergence(const GridDev& g, const double* u, const double* v, const double* w,
                             double* f, double scale, hipStream_t st);
// p_src: the pressure before the update (nullptr: p itself); p = p_src + phi - c Dzz phi
hipError_t launch_project_update(const GridDev& g, double* u, double* v, double* w, double* p,
                                 const double* phi, double s, double c, hipStream_t st,
                                 const double* p_src = nullptr);
// flag[0] |= 1 when some value of p[0..n) is not finite
hipError_t launch_nonfinite(const double* p, size_t n, unsigned* flag, hipStream_t st);
hipError_t launch_adj_rhs(const GridDev& g, const double* gu, const double* gv, const double* gw, const double* gp,
                          double* f, double inv_s, double c, hipStream_t st);
hipError_t launch_adj_update(const GridDev& g, const double* gu, const double* gv, const double* gw,
                             const double* phi, double* ou, double* ov, double* ow, hipStream_t st);
// out[0..ncomp) = sums over nblk blocks of partial[b * ncomp + c]; scratch holds 1024 * ncomp doubles.
hipError_t launch_reduce2(const double* partial, int nblk, int ncomp, double* scratch, double* out, hipStream_t st);
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st);
// dst[0..bytes) = src[0..bytes): 16-byte non-temporal loads and stores (src, dst 16-byte aligned)
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, int ncu, hipStream_t st);
// out[0..n) = c * in[0..n) (out may alias in)
hipError_t launch_scale(const double* in, double* out, double c, size_t n, hipStream_t st);
hipError_t launch_scale_planes(const GridDev& g, const double* in, double* out, const double* zs, int nplanes,
                               size_t plane, hipStream_t st);
// Factorisations of C = I - beta Dzz (or, trans != 0, of C^T) for up to four (kind, beta)
// pairs, one block each: fac[q] = [l (n), invd (n), c (n)], n = nz (centre) or nz - 1 (face).
struct CnFactorJobs {
    double* fac[4];
    double beta[4];
    int kind[4];
    int n;
    int trans;
};
hipError_t launch_cn_factor(const GridDev& g, const CnFactorJobs& jobs, hipStream_t st);
// Crank-Nicolson column solves with factored operators C = I - beta Dzz, up to four fields
// (one launch each).
//   CN_PUT: out = C^-1 in on the solved rows (face walls untouched; in may alias out)
//   CN_ADD: out += C^-1 in on the solved rows (in and out distinct; columns taller than 512
//           rows use in as scratch)
//   CN_SET: as CN_PUT, and the wall rows of face fields zeroed
//   CN_T:   out = C^-T in with the factors of C^T (the transpose of the solve), face walls
//           zeroed; with out2 != NULL also out2 = c2 out
enum { CN_PUT = 0, CN_SET = 1, CN_T = 2, CN_ADD = 3 };
struct CnJob {
    const double* fac;
    const double* in;
    double* out;
    double* out2;
    double c2;
    int kind;
};
struct CnJobs {
    CnJob j[4];
    int n;
};
hipError_t launch_cn_jobs(const GridDev& g, int mode, const CnJobs& jobs, hipStream_t st);
// x = C^-1 x (CN_SET, one field)
hipError_t launch_cn_solve(const GridDev& g, int kind, const double* fac, double* x, hipStream_t st);
// Plane means of T (nz + 1 faces) and total vertical heat flux through the nz centre planes;
// sums: 2 (nz + 1) doubles of scratch.
hipError_t launch_heat_flux(const GridDev& g, const double* w, const double* t, double kappa, double* sums,
                            double* mean_t, double* flux, hipStream_t st);
hipError_t launch_cfl(const GridDev& g, const double* u, const double* v, const double* w, double* out,
                      hipStream_t st);
// out[0] = max |p[id] (x zs[id / plane] when zs != NULL)| over n values (NaN propagates).
hipError_t launch_absmax(const double* p, size_t n, size_t plane, const double* zs, double* out, hipStream_t st);

// RK3 substep (substep_kernels.hip)
struct SubstepArgs {
    const double *u, *v, *w, *t, *p;
    const double *hpu, *hpv, *hpw, *hpt;   // previous H (rho != 0)
    double *ru, *rv, *rw, *rt;             // Crank-Nicolson inputs: C q + rhs (cq = 1) or rhs (cq = 0)
    double *hu, *hv, *hw, *ht;             // this substep's H (optional)
    double dt, nu, ka, gam, rho, alp;
    double bnu, bka;                       // Crank-Nicolson beta of the velocity and of T (0 when cq = 0)
    int cq;
};

struct SubstepAdjArgs {
    const double *u, *v, *w, *t;           // input state (advection is evaluated there)
    const double *lu, *lv, *lw, *lt;       // cotangents of the right-hand sides
    const double *ghu, *ghv, *ghw, *ght;   // cotangent of the substep's H output (all NULL: none)
    const double* dp;                      // direct cotangent of p'
    double *gu, *gv, *gw, *gt, *gp;        // outputs
    double dt, nu, ka, gam, alp;
    double bnu, bka;                       // Crank-Nicolson beta of the velocity and of T
};

hipError_t launch_explicit(const GridDev& g, const SubstepArgs& a, hipStream_t st);
hipError_t launch_explicit_adj(const GridDev& g, const SubstepAdjArgs& a, hipStream_t st);

// Multiple-resolution temperature grid (multires_kernels.hip).
struct MrDev {
    int rx, ry, rz;              // refinement factors
    double dxf, dyf;             // temperature-grid spacings lx / (rx nx), ly / (ry ny)
    const double* dzf;           // temperature-grid cell heights, rz nz
    const double* zhm;           // per momentum level k: zc_k - (zc_{k-1} or the lower wall)
    const double* zhp;           // per momentum level k: (zc_{k+1} or the upper wall) - zc_k
    const double* linv;          // per momentum level k: (L_loc)^+, (rx ry rz)^2 entries
};
struct MrTArgs {
    const double *u0, *v0, *w0;  // temperature-grid velocity at the start of the interval
    const double *u1, *v1, *w1;  // ... and at its end
    const double* t;             // temperature (fine z-faces)
    const double* hp;            // previous substep's H (rho != 0)
    double* rt;                  // Crank-Nicolson input: C T + rhs (C = I - bka Dzz~; cq = 1) or rhs
    double* hout;                // this substep's H (optional; may alias hp)
    double th, dt, ka, gam, rho, alp, bka;
    int cq;
};
bool mr_factors_supported(int rx, int ry, int rz);
hipError_t launch_mr_prolong(const GridDev& g, const MrDev& m, const double* u, const double* v, const double* w,
                             double* uf, double* vf, double* wf, hipStream_t st);
hipError_t launch_mr_restrict(const GridDev& g, const MrDev& m, const double* tf, double* tc, hipStream_t st);
hipError_t launch_mr_explicit_t(const GridDev& gf, const MrTArgs& a, hipStream_t st);

}  // namespace ps
