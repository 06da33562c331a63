// C ABI of the pressure-Poisson library: plan, workspace, entry points.
// Kernels live in fft_kernels.hip, zsolve_kernels.hip, field_kernels.hip and
// substep_kernels.hip; this file validates arguments and sequences launches.
#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ps.h"
#include "ps_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

using namespace ps;

namespace {

thread_local std::string g_last_error;

ps_status fail(ps_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

ps_status hipfail(hipError_t e, const char* where) {
    return fail(e == hipErrorOutOfMemory ? PS_ENOMEM : PS_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define PS_HIP(expr, where)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hipfail(e_, where); \
    } while (0)

// Host-side trace ranges (ROCTx): every entry point, and the phases of the composite ones,
// appear as named ranges in a marker trace (rocprofv3 --marker-trace), so that a timeline
// shows which library call issued which kernels.  Without a tracing tool attached a range
// costs one indirect call.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    // ends this range and opens the next phase's in its place
    void next(const char* name) {
        roctxRangePop();
        roctxRangePushA(name);
    }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
#define PS_RANGE_CAT2(a, b) a##b
#define PS_RANGE_CAT(a, b) PS_RANGE_CAT2(a, b)
#define PS_RANGE(name) Range PS_RANGE_CAT(ps_range_, __LINE__)(name)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// hipMalloc that leaves no error behind on failure: the runtime records a failed
// allocation as its last error, which the next kernel launch's hipGetLastError() would
// otherwise report as a launch failure.
bool dev_alloc(void** ptr, size_t bytes) {
    if (hipMalloc(ptr, bytes) == hipSuccess) return true;
    *ptr = nullptr;
    (void)hipGetLastError();
    return false;
}

bool is_23(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    if (n % 3 == 0) n /= 3;
    return n == 1;
}

}  // namespace

struct ps_plan_s {
    int nx, ny, nz;
    double lx, ly, dx, dy;
    int prec;
    double tol;
    int max_iter;
    unsigned flags;
    int device;
    size_t npts;          // nx * ny * nz
    size_t plane;         // nx * ny
    double sum_dz;
    double dzz_max;       // max over rows of the off-diagonal sum of Dzz (centre and face)
    // host metrics
    std::vector<double> zf, dz, dzc, o, dzw, lamx, lamy, inv_dz, inv_dzw;
    // device tables (one allocation)
    void* d_tables = nullptr;
    double *d_dz, *d_dzc, *d_o, *d_dzw, *d_lamx, *d_lamy, *d_inv_dz, *d_inv_dzw;
    cx<double>*d_twx64, *d_ptw64, *d_twy64;
    cx<float>*d_twx32, *d_ptw32, *d_twy32;
    void* d_etab = nullptr;   // z-solve excess table (tiled solves), in the plan's precision
    // workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    int w_tile, nkxb;
    int ncu = 0;          // compute units of the device
    size_t spec_elems;
    // carved pointers
    void* spec_a;
    void* spec_b;
    void* piv;
    double* fbuf;     // npts
    double* phibuf;   // npts
    double* rbuf;     // npts
    double* rowsum = nullptr;   // FP32 plans: FP64 row sums of the transformed input, ny nz
    double* psum = nullptr;     // FP32 plans: FP64 plane sums, nz
    double* col00 = nullptr;    // FP32 plans: FP64 (0,0) column of the solution, nz
    double* partial;  // nblk_max * 4
    double* red_scratch;  // 1024 * 4
    double* small;    // 64 + cn factors
    double* cnfac;    // 3 (nz+1) * 2
    int nblk_max;
    int chunk = 0;    // planes per x/y chunk (0: whole box per launch)
    // substep temporaries (allocated on first use)
    double* sub_buf = nullptr;
    size_t sub_bytes = 0;
    double* stepadj_buf = nullptr;   // step adjoint temporaries (allocated on first use)
    // host pinned readback
    double* h_res = nullptr;
    GridDev gd;
};

namespace {

// small[] slots
enum {
    R_WSUM = 0,    // sum dz * f  (FP64 weighted sum of the solve input)
    R_DEFECT = 1,  // defect from the (0,0) column
    R_D2 = 2,      // sum (delta)^2
    R_X2 = 3,      // sum phi^2
    R_XW = 4,      // sum dz phi
    R_R2 = 5,      // sum r^2
    R_F2 = 6,      // sum (f - mu)^2
    R_CFL = 8,
    R_FLAG = 9,    // non-finite flag
    R_AMAX = 10,   // max |f| of the solve input (STRICT_COMPAT)
    R_NSLOTS = 16
};

template <typename T>
SpecDev<T> spec_of(ps_plan_t p);

template <>
SpecDev<double> spec_of<double>(ps_plan_t p) {
    SpecDev<double> s;
    s.w = p->w_tile;
    s.nkxb = p->nkxb;
    s.twx = p->d_twx64;
    s.ptw = p->d_ptw64;
    s.twy = p->d_twy64;
    s.a = (cx<double>*)p->spec_a;
    s.b = (cx<double>*)p->spec_b;
    s.piv = (double*)p->piv;
    s.etab = (const double*)p->d_etab;
    s.ncu = p->ncu;
    return s;
}

template <>
SpecDev<float> spec_of<float>(ps_plan_t p) {
    SpecDev<float> s;
    s.w = p->w_tile;
    s.nkxb = p->nkxb;
    s.twx = p->d_twx32;
    s.ptw = p->d_ptw32;
    s.twy = p->d_twy32;
    s.a = (cx<float>*)p->spec_a;
    s.b = (cx<float>*)p->spec_b;
    s.piv = (float*)p->piv;
    s.etab = (const float*)p->d_etab;
    s.ncu = p->ncu;
    s.rowsum = p->rowsum;
    s.psum = p->psum;
    s.col00 = p->col00;
    return s;
}

size_t elem_bytes(int prec) { return prec == PS_FP64 ? sizeof(cx<double>) : sizeof(cx<float>); }
size_t real_bytes(int prec) { return prec == PS_FP64 ? sizeof(double) : sizeof(float); }

size_t workspace_layout(ps_plan_t p, bool carve) {
    size_t off = 0;
    char* base = (char*)p->ws;
    auto take = [&](size_t bytes) -> void* {
        void* ptr = carve ? (void*)(base + off) : nullptr;
        off += align256(bytes);
        return ptr;
    };
    p->spec_a = take(p->spec_elems * elem_bytes(p->prec));
    p->spec_b = take(p->spec_elems * elem_bytes(p->prec));
    // pivot scratch: only the lane-per-column solve of tall columns needs it
    const bool tiled = p->prec == PS_FP64 ? zsolve_tiled<double>(p->gd) : zsolve_tiled<float>(p->gd);
    p->piv = take(tiled ? 0 : p->spec_elems * real_bytes(p->prec));
    p->fbuf = (double*)take(p->npts * sizeof(double));
    p->phibuf = (double*)take(p->npts * sizeof(double));
    p->rbuf = (double*)take(p->npts * sizeof(double));
    const bool fp32 = p->prec != PS_FP64;
    p->rowsum = fp32 ? (double*)take((size_t)p->ny * p->nz * sizeof(double)) : nullptr;
    p->psum = fp32 ? (double*)take((size_t)p->nz * sizeof(double)) : nullptr;
    p->col00 = fp32 ? (double*)take((size_t)p->nz * sizeof(double)) : nullptr;
    p->partial = (double*)take((size_t)p->nblk_max * 4 * sizeof(double));
    p->red_scratch = (double*)take(1024 * 4 * sizeof(double));
    p->small = (double*)take((R_NSLOTS + 9 * (size_t)(p->nz + 1)) * sizeof(double));
    if (carve) p->cnfac = p->small + R_NSLOTS;
    return off;
}

void fill_twiddles(std::vector<cx<double>>& out, int n, int count) {
    out.resize(count);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int q = 0; q < count; ++q) {
        long double a = -2.0L * pi * (long double)q / (long double)n;
        out[q] = {(double)cosl(a), (double)sinl(a)};
    }
}

ps_status upload_tables(ps_plan_t p) {
    const int nxh = p->nx / 2 + 1, M = p->nx / 2;
    std::vector<cx<double>> twx, ptw, twy;
    fill_twiddles(twx, M, M);
    fill_twiddles(ptw, p->nx, M + 1);
    fill_twiddles(twy, p->ny, p->ny);
    const size_t nd = (size_t)p->nz + 4 * (size_t)(p->nz + 1) + nxh + p->ny + p->nz;
    size_t bytes = align256(nd * sizeof(double)) + align256((size_t)(M + M + 1 + p->ny) * sizeof(cx<double>)) +
                   align256((size_t)(M + M + 1 + p->ny) * sizeof(cx<float>));
    if (!dev_alloc(&p->d_tables, bytes)) return fail(PS_ENOMEM, "cannot allocate %zu bytes of tables", bytes);
    std::vector<char> host(bytes, 0);
    double* hd = (double*)host.data();
    size_t o = 0;
    auto putd = [&](const std::vector<double>& v) {
        size_t at = o;
        memcpy(hd + o, v.data(), v.size() * sizeof(double));
        o += v.size();
        return at;
    };
    size_t a_dz = putd(p->dz), a_dzc = putd(p->dzc), a_o = putd(p->o), a_dzw = putd(p->dzw);
    size_t a_lx = putd(p->lamx), a_ly = putd(p->lamy), a_idz = putd(p->inv_dz), a_idzw = putd(p->inv_dzw);
    char* dbase = (char*)p->d_tables;
    p->d_dz = (double*)dbase + a_dz;
    p->d_dzc = (double*)dbase + a_dzc;
    p->d_o = (double*)dbase + a_o;
    p->d_dzw = (double*)dbase + a_dzw;
    p->d_lamx = (double*)dbase + a_lx;
    p->d_lamy = (double*)dbase + a_ly;
    p->d_inv_dz = (double*)dbase + a_idz;
    p->d_inv_dzw = (double*)dbase + a_idzw;
    size_t off64 = align256(nd * sizeof(double));
    cx<double>* h64 = (cx<double>*)(host.data() + off64);
    memcpy(h64, twx.data(), M * sizeof(cx<double>));
    memcpy(h64 + M, ptw.data(), (M + 1) * sizeof(cx<double>));
    memcpy(h64 + 2 * M + 1, twy.data(), p->ny * sizeof(cx<double>));
    p->d_twx64 = (cx<double>*)(dbase + off64);
    p->d_ptw64 = p->d_twx64 + M;
    p->d_twy64 = p->d_twx64 + 2 * M + 1;
    size_t off32 = off64 + align256((size_t)(M + M + 1 + p->ny) * sizeof(cx<double>));
    cx<float>* h32 = (cx<float>*)(host.data() + off32);
    for (int i = 0; i < 2 * M + 1 + p->ny; ++i) h32[i] = {(float)h64[i].x, (float)h64[i].y};
    p->d_twx32 = (cx<float>*)(dbase + off32);
    p->d_ptw32 = p->d_twx32 + M;
    p->d_twy32 = p->d_twx32 + 2 * M + 1;
    PS_HIP(hipMemcpy(p->d_tables, host.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(tables)");
    return PS_OK;
}

ps_status check_ptr(const void* ptr, const char* name, bool allow_null = false) {
    if (!ptr) return allow_null ? PS_OK : fail(PS_EINVAL, "%s is NULL", name);
    if (((uintptr_t)ptr) % 16 != 0) return fail(PS_EINVAL, "%s is not 16-byte aligned", name);
    return PS_OK;
}

#define PS_CHECK(expr)                  \
    do {                                \
        ps_status s_ = (expr);          \
        if (s_ != PS_OK) return s_;     \
    } while (0)

ps_status check_plan(ps_plan_t p) {
    if (!p) return fail(PS_EINVAL, "plan is NULL");
    if (!p->ws) return fail(PS_EINVAL, "plan has no workspace");
    return PS_OK;
}

double inv_den(ps_plan_t p) { return 1.0 / (p->sum_dz * (double)p->nx * (double)p->ny); }

int residual_blocks(ps_plan_t p) { return (int)((p->npts + 255) / 256); }

// Low-storage RK3 coefficients (Rai & Moin / Wray): gamma, rho; alpha = gamma + rho.
const double kGamma[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
const double kRho[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

// Crank-Nicolson factor slots (3 (nz+1) doubles each): 0 centre, 1 face, 2 face (diffusivity)
double* cn_slot(ps_plan_t p, int s) { return p->cnfac + (size_t)s * 3 * (p->nz + 1); }

// Largest beta times Dzz's row sum for which the substep solves q* = C^-1 (C q + rhs): the
// solve's rounding, relative to q, then stays near 1e-13 (eps times the operator's spread).
constexpr double kCnSetFormMax = 256.0;

// Factors of a substep's three Crank-Nicolson operators (one launch): slot 0 the velocity's
// centre rows, slot 1 its face rows (w), slot 2 the temperature's face rows; of their
// transposes for the adjoint.
hipError_t substep_factors(ps_plan_t p, double bnu, double bka, hipStream_t st, bool transpose = false) {
    CnFactorJobs fj{};
    fj.trans = transpose ? 1 : 0;
    fj.fac[0] = cn_slot(p, 0);
    fj.beta[0] = bnu;
    fj.kind[0] = PS_CENTER;
    fj.fac[1] = cn_slot(p, 1);
    fj.beta[1] = bnu;
    fj.kind[1] = PS_FACE;
    fj.fac[2] = cn_slot(p, 2);
    fj.beta[2] = bka;
    fj.kind[2] = PS_FACE;
    fj.n = 3;
    return launch_cn_factor(p->gd, fj, st);
}

constexpr int kSubFields = 8;

// Field-sized temporaries of the substep and its adjoint, allocated on first use.
ps_status ensure_substep_buffers(ps_plan_t p) {
    if (p->sub_buf) return PS_OK;
    const size_t per = align256((p->npts + p->plane) * sizeof(double));
    if (!dev_alloc((void**)&p->sub_buf, per * kSubFields)) {
        p->sub_buf = nullptr;
        return fail(PS_ENOMEM, "cannot allocate %zu bytes of substep temporaries", per * kSubFields);
    }
    p->sub_bytes = per * kSubFields;
    return PS_OK;
}

double* sub_field(ps_plan_t p, int q) {
    const size_t per = align256((p->npts + p->plane) * sizeof(double));
    return (double*)((char*)p->sub_buf + per * q);
}

// A face velocity whose divergence (D u*) * scale is the right-hand side, formed inside the
// x transform instead of being stored.
struct DivSrc {
    const double* u;
    const double* v;
    const double* w;
    double scale;
    // projection adjoint: (u, v, w) are the velocity cotangents, gp the pressure's (or NULL),
    // scale = 1/s, and c the pressure update's Dzz weight
    bool adjoint;
    const double* gp;
    double c;
};

// One spectral solve with the plan's kernels at precision T:
// out = S(in) (mode 0) or out += S(in) - mu (mode 1), scale_in / scale_out per plane (optional).
template <typename T>
ps_status spectral_solve(ps_plan_t p, const double* in, double* out, int mode, const double* mu_dev,
                         double mu_scale, const double* zin, const double* zout, bool want_wsum,
                         bool want_norms, hipStream_t st, const double* resid_x = nullptr,
                         const DivSrc* div = nullptr) {
    // resid_x != NULL: the transformed input is the refinement residual (in - mean) - L resid_x,
    // formed inside the x transform; its norms go to R_R2 / R_F2.
    const GridDev& g = p->gd;
    SpecDev<T> s = spec_of<T>(p);
    const double scale = 1.0 / ((double)p->nx * (double)p->ny);
    // Plane chunks: the x and y stages run chunk by chunk through the first planes of
    // buffer a, so that this small intermediate can stay in the last-level cache.  Each
    // chunk's x-stage blocks write their partial sums after the previous chunks'.
    const int P = (p->chunk > 0 && p->chunk < g.nz) ? p->chunk : g.nz;
    auto chunk_of = [&](int z0, GridDev& gc) {
        SpecDev<T> sc = s;
        gc = g;
        if (P < g.nz) {
            sc.z0 = z0;
            sc.nzc = std::min(P, g.nz - z0);
            gc.nz = sc.nzc;
        }
        return sc;
    };
    int nbx = 0;   // x-forward blocks so far
    for (int z0 = 0; z0 < g.nz; z0 += P) {
        GridDev gc;
        const SpecDev<T> sc = chunk_of(z0, gc);
        if (resid_x)
            PS_HIP(launch_xfwd<T>(g, sc, in, nullptr, p->partial + (size_t)2 * nbx, st, resid_x, p->small + R_WSUM,
                                  inv_den(p)),
                   "x forward FFT (residual)");
        else if (div)
            PS_HIP(launch_xfwd_div<T>(g, sc, div->u, div->v, div->w, div->scale,
                                      want_wsum ? p->partial + (size_t)nbx : nullptr, st, div->adjoint, div->gp,
                                      div->c),
                   "x forward FFT (divergence)");
        else
            PS_HIP(launch_xfwd<T>(g, sc, in, zin, want_wsum ? p->partial + (size_t)nbx : nullptr, st),
                   "x forward FFT");
        nbx += xfwd_blocks<T>(gc);
        PS_HIP(launch_yfwd<T>(g, sc, st), "y forward FFT");
    }
    if (resid_x) PS_HIP(launch_reduce2(p->partial, nbx, 2, p->red_scratch, p->small + R_R2, st), "reduce");
    if (want_wsum) PS_HIP(launch_reduce2(p->partial, nbx, 1, p->red_scratch, p->small + R_WSUM, st), "reduce");
    // Without plane chunks buffer a holds a whole spectrum: the z solve may then write
    // into it (b layout), and the inverse stages run with the two buffers' roles swapped.
    if (P == g.nz && zsolve_out_of_place<T>(g)) {
        SpecDev<T> sz = s;
        sz.bz = s.a;
        PS_HIP(launch_zsolve<T>(g, sz, st), "z solve");
        PS_HIP(launch_zsolve00<T>(g, sz, p->small + R_DEFECT, st), "z solve (0,0)");
        std::swap(s.a, s.b);
    } else {
        PS_HIP(launch_zsolve<T>(g, s, st), "z solve");
        PS_HIP(launch_zsolve00<T>(g, s, p->small + R_DEFECT, st), "z solve (0,0)");
    }
    int nbi = 0;   // x-inverse blocks so far
    for (int z0 = 0; z0 < g.nz; z0 += P) {
        GridDev gc;
        const SpecDev<T> sc = chunk_of(z0, gc);
        PS_HIP(launch_yinv<T>(g, sc, st), "y inverse FFT");
        PS_HIP(launch_xinv<T>(g, sc, out, scale, mode, mu_dev, mu_scale, zout,
                              want_norms ? p->partial + (size_t)3 * nbi : nullptr, st),
               "x inverse FFT");
        nbi += xinv_blocks<T>(gc);
    }
    if (want_norms) PS_HIP(launch_reduce2(p->partial, nbi, 3, p->red_scratch, p->small + R_D2, st), "reduce");
    return PS_OK;
}

ps_status read_small(ps_plan_t p, hipStream_t st) {
    PS_HIP(hipMemcpyAsync(p->h_res, p->small, R_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, st),
           "hipMemcpyAsync(results)");
    PS_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    return PS_OK;
}

ps_status check_finite(ps_plan_t p, const double* f, hipStream_t st);

// Full solve at the plan's precision.  in -> out; zin/zout optional per-plane scalings
// div != NULL (FP64 plans only, no finiteness check): the right-hand side is the divergence
// of div's velocity, formed in the x transform; `in` is then unused.
ps_status solve_impl(ps_plan_t p, const double* in, double* out, const double* zin, const double* zout,
                     hipStream_t st, ps_info* info, const DivSrc* div = nullptr) {
    ps_info loc{};
    loc.rel_residual = -1.0;
    const bool strict = (p->flags & PS_FLAG_STRICT_COMPAT) != 0;
    if (p->flags & PS_FLAG_CHECK_FINITE) PS_CHECK(check_finite(p, in, st));
    // the compatibility test compares the removed mean with max |f| of the (scaled) input
    if (strict) PS_HIP(launch_absmax(in, p->npts, p->plane, zin, p->small + R_AMAX, st), "max |f|");
    ps_status result = PS_OK;
    if (p->prec == PS_FP64) {
        PS_CHECK(spectral_solve<double>(p, in, out, 0, nullptr, 0.0, zin, zout, false, false, st, nullptr, div));
        loc.iterations = 1;
        if (info || strict) {
            PS_CHECK(read_small(p, st));
            loc.compat_defect = p->h_res[R_DEFECT];
        }
    } else {
        // FP32 solves refined on the FP64 residual.  A scaled input is materialised first
        // because the residual needs it.
        const double* f = in;
        if (zin) {
            PS_HIP(launch_scale_planes(p->gd, in, p->fbuf == in ? p->rbuf : p->fbuf, zin, p->nz, p->plane, st),
                   "scale");
            f = (p->fbuf == in) ? p->rbuf : p->fbuf;
        }
        PS_CHECK(spectral_solve<float>(p, f, out, 0, nullptr, 0.0, nullptr, nullptr, true, true, st));
        loc.iterations = 1;
        if (p->prec == PS_FP32_REFINED) {
            // Linear convergence: the error left after correction i is about rho |d_i| with the
            // contraction rho = |d_i| / |d_{i-1}|.  The first correction has no predecessor (|d_1|/|x|
            // measures the FP32 solve's error, not the contraction), so it stops only if |d_1| itself
            // meets the tolerance.
            double prev = 1.0;
            bool converged = false;
            for (int it = 0; it < p->max_iter; ++it) {
                PS_RANGE("refinement correction");
                // correction: residual of the current iterate (formed in the x transform), FP32 solve,
                // FP64 update with the gauge re-imposed
                PS_CHECK(spectral_solve<float>(p, f, out, 1, p->small + R_XW, inv_den(p), nullptr, nullptr, false,
                                               true, st, out));
                loc.iterations++;
                PS_CHECK(read_small(p, st));
                const double d2 = p->h_res[R_D2], x2 = p->h_res[R_X2];
                const double rel = x2 > 0 ? std::sqrt(d2 / x2) : 0.0;
                loc.rel_update = rel;
                const double f2 = p->h_res[R_F2];
                loc.rel_residual = f2 > 0 ? std::sqrt(p->h_res[R_R2] / f2) : 0.0;
                const double rho = rel / prev;
                if (rel <= p->tol || (it > 0 && rho * rel <= p->tol)) {
                    converged = true;
                    break;
                }
                if (rel > 0.5 * prev) break;   // stagnation: rounding floor reached
                prev = rel;
            }
            if (!converged) {
                result = PS_ENOTCONVERGED;
                fail(result, "refinement stopped at ||delta||/||phi|| = %.3e after %d solves (tol %.3e)",
                     loc.rel_update, loc.iterations, p->tol);
            }
        }
        // The iterate is refined unscaled (its residual is f - L x); a per-plane output
        // scaling (the adjoint's Vc) is applied once, in place, at the end.
        if (zout) PS_HIP(launch_scale_planes(p->gd, out, out, zout, p->nz, p->plane, st), "scale");
        if (info || strict) {
            PS_CHECK(read_small(p, st));
            loc.compat_defect = p->h_res[R_WSUM] * inv_den(p);
            loc.gauge_shift = p->h_res[R_XW] * inv_den(p);
        }
    }
    if (strict) {
        // the removed dz-weighted mean against the size of the right-hand side
        const double fmax_abs = p->h_res[R_AMAX];
        if (!(std::fabs(loc.compat_defect) <= 1e-8 * fmax_abs)) {
            if (info) *info = loc;
            return fail(PS_ENOTCOMPAT, "right-hand side incompatible: weighted mean %.3e, max |f| %.3e",
                        loc.compat_defect, fmax_abs);
        }
    }
    if (info) *info = loc;
    return result;
}

// ---- statically allocated scratch (allocation-free entry point) ----------------
// A file-scope device array of kStaticScratchBytes that poisson_solve_static uses as the
// plan's workspace.  Every GPU the library runs on holds its own copy from module load
// to process end.  Host code never names the array except to look up its device address
// (once per device, with that device current); kernels receive that address.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

ps_status static_scratch(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return fail(PS_EDEVICE, "device %d out of range", device);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        PS_HIP(hipGetDevice(&cur), "hipGetDevice");
        if (cur != device) PS_HIP(hipSetDevice(device), "hipSetDevice");
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(PS_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return PS_OK;
}

// The projection; pr_src (nullptr: pr) is the pressure the update starts from, so that a
// substep can write its pressure to another buffer than the one it read.
ps_status project_impl(ps_plan_t p, double* u, double* v, double* w, double* pr, double* phi_out, double s,
                       double c, void* stream, ps_info* info, const double* pr_src) {
    PS_RANGE("project");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(u, "u"));
    PS_CHECK(check_ptr(v, "v"));
    PS_CHECK(check_ptr(w, "w"));
    PS_CHECK(check_ptr(pr, "p", true));
    PS_CHECK(check_ptr(phi_out, "phi_out", true));
    if (!(s > 0) || !std::isfinite(s)) return fail(PS_EINVAL, "s must be positive");
    if (!(c >= 0) || !std::isfinite(c)) return fail(PS_EINVAL, "c must be non-negative");
    hipStream_t st = (hipStream_t)stream;
    double* phi = phi_out ? phi_out : p->phibuf;
    ps_status r;
    if (p->prec == PS_FP64 && !(p->flags & (PS_FLAG_CHECK_FINITE | PS_FLAG_STRICT_COMPAT))) {
        // the divergence is formed inside the x transform and never stored
        const DivSrc d{u, v, w, 1.0 / s, false, nullptr, 0.0};
        r = solve_impl(p, nullptr, phi, nullptr, nullptr, st, info, &d);
    } else {
        // the refinement's residual (and the finiteness and compatibility checks) need the
        // right-hand side stored
        PS_HIP(launch_divergence(p->gd, u, v, w, p->fbuf, 1.0 / s, st), "divergence");
        r = solve_impl(p, p->fbuf, phi, nullptr, nullptr, st, info);
    }
    if (r != PS_OK && r != PS_ENOTCONVERGED) return r;
    PS_HIP(launch_project_update(p->gd, u, v, w, pr, phi, s, c, st, pr_src), "projection update");
    return r;
}

// One substep; advance_t = false leaves T as given (its buoyancy is still applied): the
// momentum part of a step whose temperature is advanced elsewhere.  src (nullptr: in place)
// names the state {u, v, w, T, p} the substep starts from; the new state is written to
// (u, v, w, t, pr), which must not overlap src unless a field is its own source.
ps_status substep_impl(ps_plan_t p, int l, double dt, double nu, double kappa, double* u, double* v, double* w,
                       double* t, double* pr, const double* const* h_prev, double* const* h_out, void* stream,
                       ps_info* info, bool advance_t, const double* const* src = nullptr) {
    PS_CHECK(check_plan(p));
    if (l < 1 || l > 3) return fail(PS_EINVAL, "substep index l=%d must be 1, 2 or 3", l);
    if (!(dt > 0) || !std::isfinite(dt)) return fail(PS_EINVAL, "dt must be positive");
    if (!(nu >= 0) || !(kappa >= 0) || !std::isfinite(nu) || !std::isfinite(kappa))
        return fail(PS_EINVAL, "nu and kappa must be non-negative");
    PS_CHECK(check_ptr(u, "u"));
    PS_CHECK(check_ptr(v, "v"));
    PS_CHECK(check_ptr(w, "w"));
    PS_CHECK(check_ptr(t, "t"));
    PS_CHECK(check_ptr(pr, "p"));
    const double gam = kGamma[l - 1], rho = kRho[l - 1], alp = gam + rho;
    if (rho != 0.0) {
        if (!h_prev) return fail(PS_EINVAL, "h_prev is required for l=%d", l);
        for (int q = 0; q < 4; ++q) PS_CHECK(check_ptr(h_prev[q], "h_prev[q]"));
    }
    if (h_out)
        for (int q = 0; q < 4; ++q) PS_CHECK(check_ptr(h_out[q], "h_out[q]"));
    PS_CHECK(ensure_substep_buffers(p));
    hipStream_t st = (hipStream_t)stream;
    double* ru = sub_field(p, 0);
    double* rv = sub_field(p, 1);
    double* rw = sub_field(p, 2);
    double* rt = sub_field(p, 3);
    if (src)
        for (int q = 0; q < 5; ++q) PS_CHECK(check_ptr(src[q], "src[q]"));
    const double* s_u = src ? src[0] : u;
    const double* s_v = src ? src[1] : v;
    const double* s_w = src ? src[2] : w;
    const double* s_t = src ? src[3] : t;
    const double* s_p = src ? src[4] : pr;
    SubstepArgs a{};
    a.u = s_u;
    a.v = s_v;
    a.w = s_w;
    a.t = s_t;
    a.p = s_p;
    if (rho != 0.0) {
        a.hpu = h_prev[0];
        a.hpv = h_prev[1];
        a.hpw = h_prev[2];
        a.hpt = h_prev[3];
    }
    a.ru = ru;
    a.rv = rv;
    a.rw = rw;
    a.rt = advance_t ? rt : nullptr;
    if (h_out) {
        a.hu = h_out[0];
        a.hv = h_out[1];
        a.hw = h_out[2];
        a.ht = h_out[3];
    }
    a.dt = dt;
    a.nu = nu;
    a.ka = kappa;
    a.gam = gam;
    a.rho = rho;
    a.alp = alp;
    const double bnu = alp * dt * nu / 2.0, bka = alp * dt * kappa / 2.0;
    // q* = C^-1 (C q + rhs) reads one field less than q* = q + C^-1 rhs, but its rounding is
    // relative to q rather than to the increment: it is used while C stays close to the
    // identity (beta times Dzz's largest row sum <= kCnSetFormMax), the add form otherwise
    const bool set_form = std::max(bnu, bka) * p->dzz_max <= kCnSetFormMax;
    a.cq = set_form ? 1 : 0;
    a.bnu = set_form ? bnu : 0.0;
    a.bka = set_form ? bka : 0.0;
    PS_HIP(launch_explicit(p->gd, a, st), "explicit terms");
    PS_HIP(substep_factors(p, bnu, bka, st), "cn factor");
    // the set form writes q* from C q + rhs alone; the add form and an unadvanced T need the
    // old values in the destination first
    const size_t bc = p->npts * sizeof(double), bf = (p->npts + p->plane) * sizeof(double);
    auto seed = [&](double* dst, const double* from, size_t bytes) -> ps_status {
        if (dst != from) PS_HIP(hipMemcpyAsync(dst, from, bytes, hipMemcpyDeviceToDevice, st), "copy state");
        return PS_OK;
    };
    if (!set_form) {
        PS_CHECK(seed(u, s_u, bc));
        PS_CHECK(seed(v, s_v, bc));
        PS_CHECK(seed(w, s_w, bf));
    }
    if (!set_form || !advance_t) PS_CHECK(seed(t, s_t, bf));
    // the set-form solve writes the interior rows of face fields only: their wall planes
    // (w = 0, the wall temperatures) come from the source
    auto seed_walls = [&](double* dst, const double* from) -> ps_status {
        if (dst == from) return PS_OK;
        const size_t pb = p->plane * sizeof(double), top = p->npts;
        PS_HIP(hipMemcpyAsync(dst, from, pb, hipMemcpyDeviceToDevice, st), "copy wall plane");
        PS_HIP(hipMemcpyAsync(dst + top, from + top, pb, hipMemcpyDeviceToDevice, st), "copy wall plane");
        return PS_OK;
    };
    if (set_form) {
        PS_CHECK(seed_walls(w, s_w));
        if (advance_t) PS_CHECK(seed_walls(t, s_t));
    }
    CnJobs jobs{};
    jobs.j[0] = CnJob{cn_slot(p, 0), ru, u, nullptr, 0.0, PS_CENTER};
    jobs.j[1] = CnJob{cn_slot(p, 0), rv, v, nullptr, 0.0, PS_CENTER};
    jobs.j[2] = CnJob{cn_slot(p, 1), rw, w, nullptr, 0.0, PS_FACE};
    jobs.j[3] = CnJob{cn_slot(p, 2), rt, t, nullptr, 0.0, PS_FACE};
    jobs.n = advance_t ? 4 : 3;
    PS_HIP(launch_cn_jobs(p->gd, set_form ? CN_PUT : CN_ADD, jobs, st), "cn solves");
    return project_impl(p, u, v, w, pr, nullptr, alp * dt, bnu, stream, info, s_p);
}

}  // namespace

// ============================================================================
extern "C" {

const char* ps_last_error(void) { return g_last_error.c_str(); }

ps_status poisson_plan_create(ps_plan_t* out, int nx, int ny, int nz, double lx, double ly, const double* zf,
                              int prec, double tol, int max_iter, unsigned flags) {
    PS_RANGE("poisson_plan_create");
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 4 || nx % 2 != 0 || nx > 4096 || !is_23(nx) || !fft_length_supported(nx / 2))
        return fail(PS_EINVAL, "nx=%d: need even 2^a*3^b (b<=1) with 4 <= nx <= 4096", nx);
    if (ny < 2 || ny > 4096 || !fft_length_supported(ny))
        return fail(PS_EINVAL, "ny=%d: need 2^a*3^b (b<=1) with 2 <= ny <= 4096", ny);
    if (nz < 2 || nz > 2048) return fail(PS_EINVAL, "nz=%d: need 2 <= nz <= 2048", nz);
    if (!(lx > 0) || !(ly > 0) || !std::isfinite(lx) || !std::isfinite(ly))
        return fail(PS_EINVAL, "box lengths must be positive and finite");
    if (!zf) return fail(PS_EINVAL, "zf is NULL");
    for (int k = 0; k <= nz; ++k)
        if (!std::isfinite(zf[k])) return fail(PS_EINVAL, "zf[%d] is not finite", k);
    for (int k = 0; k < nz; ++k)
        if (!(zf[k + 1] > zf[k])) return fail(PS_EINVAL, "zf must be strictly increasing (k=%d)", k);
    if (prec != PS_FP64 && prec != PS_FP32_REFINED && prec != PS_FP32)
        return fail(PS_EINVAL, "unknown precision %d", prec);
    ps_plan_t p = new ps_plan_s();
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->lx = lx;
    p->ly = ly;
    p->dx = lx / nx;
    p->dy = ly / ny;
    p->prec = prec;
    p->tol = tol > 0 ? tol : 1e-12;
    p->max_iter = max_iter > 0 ? max_iter : 10;
    p->flags = flags;
    p->npts = (size_t)nx * ny * nz;
    p->plane = (size_t)nx * ny;
    // metrics (same formulas as the problem definition)
    p->zf.assign(zf, zf + nz + 1);
    p->dz.resize(nz);
    for (int k = 0; k < nz; ++k) p->dz[k] = zf[k + 1] - zf[k];
    p->dzc.assign(nz + 1, 0.0);
    p->o.assign(nz + 1, 0.0);
    p->dzw.assign(nz + 1, 0.0);
    for (int k = 1; k < nz; ++k) {
        p->dzc[k] = 0.5 * (p->dz[k - 1] + p->dz[k]);
        p->o[k] = 1.0 / p->dzc[k];
        p->dzw[k] = p->dzc[k];
    }
    p->dzw[0] = 0.5 * p->dz[0];
    p->dzw[nz] = 0.5 * p->dz[nz - 1];
    p->inv_dzw.resize(nz + 1);
    for (int k = 0; k <= nz; ++k) p->inv_dzw[k] = 1.0 / p->dzw[k];
    p->inv_dz.resize(nz);
    double sdz = 0.0;
    for (int k = 0; k < nz; ++k) {
        p->inv_dz[k] = 1.0 / p->dz[k];
        sdz += p->dz[k];
    }
    p->sum_dz = sdz;
    // largest off-diagonal sum of Dzz's rows (centre and interior-face operators): beta times it
    // bounds how far the Crank-Nicolson operator I - beta Dzz is from the identity
    double dmax = 0.0;
    for (int k = 0; k < nz; ++k) dmax = std::max(dmax, 1.0 / (p->dzw[k] * p->dz[k]) + 1.0 / (p->dzw[k + 1] * p->dz[k]));
    for (int k = 1; k < nz; ++k) dmax = std::max(dmax, 1.0 / (p->dz[k - 1] * p->dzc[k]) + 1.0 / (p->dz[k] * p->dzc[k]));
    p->dzz_max = dmax;
    const long double pi = 3.141592653589793238462643383279502884L;
    p->lamx.resize(nx / 2 + 1);
    for (int k = 0; k <= nx / 2; ++k) {
        double sn = (double)sinl(pi * (long double)k / (long double)nx);
        p->lamx[k] = (4.0 / (p->dx * p->dx)) * sn * sn;
    }
    p->lamy.resize(ny);
    for (int k = 0; k < ny; ++k) {
        double sn = (double)sinl(pi * (long double)k / (long double)ny);
        p->lamy[k] = (4.0 / (p->dy * p->dy)) * sn * sn;
    }
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(PS_EDEVICE, "no HIP device");
    }
    if (hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
        p->ncu = 0;
    ps_status s = upload_tables(p);
    if (s != PS_OK) {
        poisson_plan_destroy(p);
        return s;
    }
    p->w_tile = prec == PS_FP64 ? TileW<double>::value : TileW<float>::value;
    p->nkxb = (nx / 2 + 1 + p->w_tile - 1) / p->w_tile;
    p->spec_elems = (size_t)nz * ny * p->nkxb * p->w_tile;
    {
        GridDev& g = p->gd;
        g.nx = nx;
        g.ny = ny;
        g.nz = nz;
        g.dx = p->dx;
        g.dy = p->dy;
        g.dz = p->d_dz;
        g.dzc = p->d_dzc;
        g.o = p->d_o;
        g.dzw = p->d_dzw;
        g.lamx = p->d_lamx;
        g.lamy = p->d_lamy;
        g.idz = p->d_inv_dz;
        g.idzw = p->d_inv_dzw;
    }
    {
        // per-plan z-solve excess table (formed once, on the null stream)
        const size_t ne = prec == PS_FP64 ? zexcess_elems<double>(p->gd, p->nkxb) : zexcess_elems<float>(p->gd, p->nkxb);
        if (ne > 0) {
            if (!dev_alloc(&p->d_etab, ne * real_bytes(prec))) {
                p->d_etab = nullptr;
                poisson_plan_destroy(p);
                return fail(PS_ENOMEM, "cannot allocate the %zu-byte z-solve table", ne * real_bytes(prec));
            }
            hipError_t e = prec == PS_FP64 ? launch_zexcess<double>(p->gd, p->nkxb, (double*)p->d_etab, nullptr)
                                           : launch_zexcess<float>(p->gd, p->nkxb, (float*)p->d_etab, nullptr);
            if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) {
                poisson_plan_destroy(p);
                return hipfail(e, "z-solve table");
            }
        }
    }
    int nbx = prec == PS_FP64 ? xfwd_blocks<double>(p->gd) : xfwd_blocks<float>(p->gd);
    int nbr = (int)((p->npts + 255) / 256);
    // plane chunks may each end with a partly filled x-stage block: one more per plane at most
    nbx += nz;
    p->nblk_max = nbx > nbr ? nbx : nbr;
    if (const char* ev = getenv("PS_CHUNK_PLANES")) p->chunk = atoi(ev);
    p->ws_bytes = workspace_layout(p, false);
    if (!dev_alloc(&p->ws, p->ws_bytes)) {
        p->ws = nullptr;
        poisson_plan_destroy(p);
        return fail(PS_ENOMEM, "cannot allocate %zu bytes of workspace", p->ws_bytes);
    }
    p->ws_owned = true;
    workspace_layout(p, true);
    if (hipHostMalloc((void**)&p->h_res, R_NSLOTS * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        p->h_res = nullptr;
        (void)hipGetLastError();
        poisson_plan_destroy(p);
        return fail(PS_ENOMEM, "cannot allocate pinned host memory");
    }
    *out = p;
    return PS_OK;
}

size_t poisson_plan_workspace_bytes(ps_plan_t p) { return p ? p->ws_bytes : 0; }

ps_status poisson_plan_set_workspace(ps_plan_t p, void* dev, size_t bytes) {
    PS_RANGE("poisson_plan_set_workspace");
    if (!p) return fail(PS_EINVAL, "plan is NULL");
    if (dev) {
        if (bytes < p->ws_bytes) return fail(PS_EINVAL, "workspace too small: %zu < %zu", bytes, p->ws_bytes);
        if (((uintptr_t)dev) % 256 != 0) return fail(PS_EINVAL, "workspace not 256-byte aligned");
    }
    if (p->ws_owned && p->ws) hipFree(p->ws);
    p->ws = nullptr;
    p->ws_owned = false;
    if (dev) {
        p->ws = dev;
    } else {
        if (!dev_alloc(&p->ws, p->ws_bytes)) {
            p->ws = nullptr;
            return fail(PS_ENOMEM, "cannot allocate %zu bytes of workspace", p->ws_bytes);
        }
        p->ws_owned = true;
    }
    workspace_layout(p, true);
    return PS_OK;
}

ps_status poisson_plan_destroy(ps_plan_t p) {
    PS_RANGE("poisson_plan_destroy");
    if (!p) return PS_OK;
    if (p->ws_owned && p->ws) hipFree(p->ws);
    if (p->d_tables) hipFree(p->d_tables);
    if (p->d_etab) hipFree(p->d_etab);
    if (p->sub_buf) hipFree(p->sub_buf);
    if (p->stepadj_buf) hipFree(p->stepadj_buf);
    if (p->h_res) hipHostFree(p->h_res);
    delete p;
    return PS_OK;
}

ps_status poisson_solve(ps_plan_t p, const double* f, double* phi, void* stream, ps_info* info) {
    PS_RANGE("poisson_solve");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(f, "f"));
    PS_CHECK(check_ptr(phi, "phi"));
    if ((const void*)f == (const void*)phi) return fail(PS_EINVAL, "phi may not alias f");
    return solve_impl(p, f, phi, nullptr, nullptr, (hipStream_t)stream, info);
}

ps_status poisson_solve_adjoint(ps_plan_t p, const double* g_phi, double* g_rhs, void* stream, ps_info* info) {
    PS_RANGE("poisson_solve_adjoint");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(g_phi, "g_phi"));
    PS_CHECK(check_ptr(g_rhs, "g_rhs"));
    if ((const void*)g_phi == (const void*)g_rhs) return fail(PS_EINVAL, "g_rhs may not alias g_phi");
    return solve_impl(p, g_phi, g_rhs, p->d_inv_dz, p->d_dz, (hipStream_t)stream, info);
}

ps_status poisson_solve_static(ps_plan_t p, const double* f, double* phi, void* stream, ps_info* info) {
    PS_RANGE("poisson_solve_static");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(f, "f"));
    PS_CHECK(check_ptr(phi, "phi"));
    if ((const void*)f == (const void*)phi) return fail(PS_EINVAL, "phi may not alias f");
    if (p->ws_bytes > kStaticScratchBytes)
        return fail(PS_EINVAL, "box needs %zu bytes of scratch, more than the %zu of the static array", p->ws_bytes,
                    kStaticScratchBytes);
    void* sp = nullptr;
    PS_CHECK(static_scratch(p->device, &sp));
    // run the solve with the plan's buffers carved out of the static array, then restore
    // the plan's own (the kernels already enqueued hold the static addresses)
    void* own = p->ws;
    p->ws = sp;
    workspace_layout(p, true);
    const ps_status r = solve_impl(p, f, phi, nullptr, nullptr, (hipStream_t)stream, info);
    p->ws = own;
    workspace_layout(p, true);
    return r;
}

ps_status project(ps_plan_t p, double* u, double* v, double* w, double* pr, double* phi_out, double s, double c,
                  void* stream, ps_info* info) {
    return project_impl(p, u, v, w, pr, phi_out, s, c, stream, info, nullptr);
}

ps_status project_adjoint(ps_plan_t p, const double* g_u, const double* g_v, const double* g_w, const double* g_p,
                          double* gu_star, double* gv_star, double* gw_star, double s, double c, void* stream,
                          ps_info* info) {
    PS_RANGE("project_adjoint");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(g_u, "g_u"));
    PS_CHECK(check_ptr(g_v, "g_v"));
    PS_CHECK(check_ptr(g_w, "g_w"));
    PS_CHECK(check_ptr(g_p, "g_p", true));
    PS_CHECK(check_ptr(gu_star, "gu_star"));
    PS_CHECK(check_ptr(gv_star, "gv_star"));
    PS_CHECK(check_ptr(gw_star, "gw_star"));
    if (!(s > 0) || !std::isfinite(s)) return fail(PS_EINVAL, "s must be positive");
    if (!(c >= 0) || !std::isfinite(c)) return fail(PS_EINVAL, "c must be non-negative");
    const void* ins[4] = {g_u, g_v, g_w, g_p};
    const void* outs[3] = {gu_star, gv_star, gw_star};
    for (const void* a : ins)
        for (const void* b : outs)
            if (a && a == b) return fail(PS_EINVAL, "outputs may not alias inputs");
    hipStream_t st = (hipStream_t)stream;
    ps_status r;
    if (p->prec == PS_FP64 && !(p->flags & (PS_FLAG_CHECK_FINITE | PS_FLAG_STRICT_COMPAT))) {
        // the solve's right-hand side is formed inside the x transform and never stored
        const DivSrc d{g_u, g_v, g_w, 1.0 / s, true, g_p, c};
        r = solve_impl(p, nullptr, p->phibuf, nullptr, nullptr, st, info, &d);
    } else {
        PS_HIP(launch_adj_rhs(p->gd, g_u, g_v, g_w, g_p, p->fbuf, 1.0 / s, c, st), "adjoint rhs");
        r = solve_impl(p, p->fbuf, p->phibuf, nullptr, nullptr, st, info);
    }
    if (r != PS_OK && r != PS_ENOTCONVERGED) return r;
    PS_HIP(launch_adj_update(p->gd, g_u, g_v, g_w, p->phibuf, gu_star, gv_star, gw_star, st), "adjoint update");
    return r;
}

ps_status cn_solve(ps_plan_t p, int kind, double beta, double* x, void* stream) {
    PS_RANGE("cn_solve");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(x, "rhs_inout"));
    if (kind != PS_CENTER && kind != PS_FACE) return fail(PS_EINVAL, "unknown kind %d", kind);
    if (!(beta >= 0) || !std::isfinite(beta)) return fail(PS_EINVAL, "beta must be non-negative");
    hipStream_t st = (hipStream_t)stream;
    double* fac = cn_slot(p, kind == PS_CENTER ? 0 : 1);
    CnFactorJobs fj{};
    fj.fac[0] = fac;
    fj.beta[0] = beta;
    fj.kind[0] = kind;
    fj.n = 1;
    PS_HIP(launch_cn_factor(p->gd, fj, st), "cn factor");
    PS_HIP(launch_cn_solve(p->gd, kind, fac, x, st), "cn solve");
    return PS_OK;
}

ps_status ps_cfl(ps_plan_t p, const double* u, const double* v, const double* w, double* cfl_dev, void* stream) {
    PS_RANGE("ps_cfl");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(u, "u"));
    PS_CHECK(check_ptr(v, "v"));
    PS_CHECK(check_ptr(w, "w"));
    if (!cfl_dev || ((uintptr_t)cfl_dev) % 8 != 0) return fail(PS_EINVAL, "cfl_dev must be an aligned device pointer");
    PS_HIP(launch_cfl(p->gd, u, v, w, cfl_dev, (hipStream_t)stream), "cfl");
    return PS_OK;
}

ps_status rk3_substep(ps_plan_t p, int l, double dt, double nu, double kappa, double* u, double* v, double* w,
                      double* t, double* pr, const double* const* h_prev, double* const* h_out, void* stream,
                      ps_info* info) {
    PS_RANGE("rk3_substep");
    return substep_impl(p, l, dt, nu, kappa, u, v, w, t, pr, h_prev, h_out, stream, info, true);
}

ps_status rk3_step(ps_plan_t p, double dt, double cfl_target, double dt_max, double nu, double kappa, double* u,
                   double* v, double* w, double* t, double* pr, double* dt_used, void* stream, ps_info* info) {
    PS_RANGE("rk3_step");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(u, "u"));
    PS_CHECK(check_ptr(v, "v"));
    PS_CHECK(check_ptr(w, "w"));
    PS_CHECK(check_ptr(t, "t"));
    PS_CHECK(check_ptr(pr, "p"));
    if (!(nu >= 0) || !(kappa >= 0) || !std::isfinite(nu) || !std::isfinite(kappa))
        return fail(PS_EINVAL, "nu and kappa must be non-negative");
    hipStream_t st = (hipStream_t)stream;
    if (!(dt > 0)) {
        if (!(cfl_target > 0) || !std::isfinite(cfl_target)) return fail(PS_EINVAL, "cfl_target must be positive");
        if (!(dt_max > 0)) return fail(PS_EINVAL, "dt_max must be positive");
        // Courant number of the current state, read back once
        PS_HIP(launch_cfl(p->gd, u, v, w, p->small + R_CFL, st), "cfl");
        PS_CHECK(read_small(p, st));
        const double c = p->h_res[R_CFL];
        if (!std::isfinite(c)) return fail(PS_ENONFINITE, "Courant number is not finite");
        dt = std::min(dt_max, cfl_target / std::max(c, 1e-8));
    }
    if (!std::isfinite(dt)) return fail(PS_EINVAL, "dt must be finite");
    PS_CHECK(ensure_substep_buffers(p));
    // H^l of substep l is read by substep l + 1 and overwritten in place (each point's
    // explicit terms are read before they are written, by the same thread)
    double* h[4] = {sub_field(p, 4), sub_field(p, 5), sub_field(p, 6), sub_field(p, 7)};
    const double* hc[4] = {h[0], h[1], h[2], h[3]};
    ps_info acc{};
    ps_status result = PS_OK;
    std::string first_msg;
    for (int l = 1; l <= 3; ++l) {
        ps_info li{};
        // the last substep's H is not needed by anyone
        const ps_status r = rk3_substep(p, l, dt, nu, kappa, u, v, w, t, pr, l > 1 ? hc : nullptr,
                                        l < 3 ? h : nullptr, stream, info ? &li : nullptr);
        if (r != PS_OK && r != PS_ENOTCONVERGED) return r;
        // a refinement that stopped above the tolerance still completes the step (its phi is
        // written); the step then reports the first such substep
        if (r == PS_ENOTCONVERGED && result == PS_OK) {
            result = r;
            first_msg = g_last_error;
        }
        acc.iterations += li.iterations;
        acc.rel_update = std::max(acc.rel_update, li.rel_update);
        acc.rel_residual = std::max(acc.rel_residual, li.rel_residual);
        acc.compat_defect = li.compat_defect;
        acc.gauge_shift = li.gauge_shift;
    }
    if (dt_used) *dt_used = dt;
    if (info) *info = acc;
    if (result != PS_OK) return fail(result, "%s", first_msg.c_str());
    return PS_OK;
}

ps_status ps_heat_flux(ps_plan_t p, const double* w, const double* t, double kappa, double* mean_t, double* flux,
                       void* stream) {
    PS_RANGE("ps_heat_flux");
    PS_CHECK(check_plan(p));
    PS_CHECK(check_ptr(w, "w"));
    PS_CHECK(check_ptr(t, "t"));
    if (!mean_t || !flux || ((uintptr_t)mean_t) % 8 || ((uintptr_t)flux) % 8)
        return fail(PS_EINVAL, "mean_t and flux must be aligned device pointers");
    if (!(kappa >= 0) || !std::isfinite(kappa)) return fail(PS_EINVAL, "kappa must be non-negative");
    PS_HIP(launch_heat_flux(p->gd, w, t, kappa, p->partial, mean_t, flux, (hipStream_t)stream), "heat flux");
    return PS_OK;
}

ps_status rk3_substep_adjoint(ps_plan_t p, int l, double dt, double nu, double kappa, const double* u,
                              const double* v, const double* w, const double* t, const double* pr,
                              const double* const* g_out, const double* const* g_hout, double* const* g_in,
                              double* const* g_hprev, void* stream, ps_info* info) {
    PS_RANGE("rk3_substep_adjoint");
    PS_CHECK(check_plan(p));
    if (l < 1 || l > 3) return fail(PS_EINVAL, "substep index l=%d must be 1, 2 or 3", l);
    if (!(dt > 0) || !std::isfinite(dt)) return fail(PS_EINVAL, "dt must be positive");
    if (!(nu >= 0) || !(kappa >= 0) || !std::isfinite(nu) || !std::isfinite(kappa))
        return fail(PS_EINVAL, "nu and kappa must be non-negative");
    PS_CHECK(check_ptr(u, "u"));
    PS_CHECK(check_ptr(v, "v"));
    PS_CHECK(check_ptr(w, "w"));
    PS_CHECK(check_ptr(t, "t"));
    PS_CHECK(check_ptr(pr, "p"));
    if (!g_out || !g_in) return fail(PS_EINVAL, "g_out and g_in are required");
    for (int q = 0; q < 5; ++q) {
        PS_CHECK(check_ptr(g_out[q], "g_out[q]"));
        PS_CHECK(check_ptr(g_in[q], "g_in[q]"));
        for (int r = 0; r < 5; ++r)
            if ((const void*)g_in[q] == (const void*)g_out[r]) return fail(PS_EINVAL, "g_in may not alias g_out");
    }
    if (g_hout)
        for (int q = 0; q < 4; ++q) {
            PS_CHECK(check_ptr(g_hout[q], "g_hout[q]"));
            for (int r = 0; r < 5; ++r)
                if ((const void*)g_hout[q] == (const void*)g_in[r]) return fail(PS_EINVAL, "g_in may not alias g_hout");
        }
    if (g_hprev)
        for (int q = 0; q < 4; ++q) {
            PS_CHECK(check_ptr(g_hprev[q], "g_hprev[q]"));
            for (int r = 0; r < 5; ++r)
                if ((const void*)g_hprev[q] == (const void*)g_in[r] || (const void*)g_hprev[q] == (const void*)g_out[r])
                    return fail(PS_EINVAL, "g_hprev may not alias g_in or g_out");
        }
    PS_CHECK(ensure_substep_buffers(p));
    hipStream_t st = (hipStream_t)stream;
    const double gam = kGamma[l - 1], rho = kRho[l - 1], alp = gam + rho;
    const double bnu = alp * dt * nu / 2.0, bka = alp * dt * kappa / 2.0;
    double* du = sub_field(p, 0);
    double* dv = sub_field(p, 1);
    double* dw = sub_field(p, 2);
    double* lu = sub_field(p, 3);
    double* lv = sub_field(p, 4);
    double* lw = sub_field(p, 5);
    double* lt = sub_field(p, 6);
    // projection (linear in u*): cotangents of u*, v*, w*
    ps_status r = project_adjoint(p, g_out[0], g_out[1], g_out[2], g_out[4], du, dv, dw, alp * dt, bnu, stream, info);
    if (r != PS_OK && r != PS_ENOTCONVERGED) return r;
    // Crank-Nicolson solves (linear): cotangents of the right-hand sides
    // The previous substep's H enters the right-hand sides as dt rho H^{l-1}: its cotangent is
    // dt rho lambda, written by the same launch unless it shares memory with g_hout (which the
    // explicit adjoint below still reads; then it is scaled after that kernel).
    bool hprev_shared = false;
    if (g_hprev && g_hout)
        for (int q = 0; q < 4; ++q)
            for (int r = 0; r < 4; ++r) hprev_shared |= (const void*)g_hprev[q] == (const void*)g_hout[r];
    const bool hprev_fused = g_hprev && !hprev_shared;
    double* h2[4] = {nullptr, nullptr, nullptr, nullptr};
    if (hprev_fused)
        for (int q = 0; q < 4; ++q) h2[q] = g_hprev[q];
    const double crho = dt * rho;
    PS_HIP(substep_factors(p, bnu, bka, st, true), "cn factor (transposed)");
    CnJobs jobs{};
    jobs.j[0] = CnJob{cn_slot(p, 0), du, lu, h2[0], crho, PS_CENTER};
    jobs.j[1] = CnJob{cn_slot(p, 0), dv, lv, h2[1], crho, PS_CENTER};
    jobs.j[2] = CnJob{cn_slot(p, 1), dw, lw, h2[2], crho, PS_FACE};
    jobs.j[3] = CnJob{cn_slot(p, 2), g_out[3], lt, h2[3], crho, PS_FACE};
    jobs.n = 4;
    PS_HIP(launch_cn_jobs(p->gd, CN_T, jobs, st), "cn adjoint solves");
    // explicit terms (bilinear advection at the input state, linear operators, buoyancy, pressure)
    SubstepAdjArgs a{};
    a.u = u;
    a.v = v;
    a.w = w;
    a.t = t;
    a.lu = lu;
    a.lv = lv;
    a.lw = lw;
    a.lt = lt;
    a.dp = g_out[4];
    a.gu = g_in[0];
    a.gv = g_in[1];
    a.gw = g_in[2];
    a.gt = g_in[3];
    a.gp = g_in[4];
    a.dt = dt;
    a.nu = nu;
    a.ka = kappa;
    a.gam = gam;
    a.alp = alp;
    a.bnu = bnu;
    a.bka = bka;
    // the cotangent of this substep's H output joins dt gamma lambda wherever H acts
    if (g_hout) {
        a.ghu = g_hout[0];
        a.ghv = g_hout[1];
        a.ghw = g_hout[2];
        a.ght = g_hout[3];
    }
    PS_HIP(launch_explicit_adj(p->gd, a, st), "explicit adjoint");
    if (g_hprev && !hprev_fused) {
        // g_hprev shares memory with g_hout: written now that the explicit adjoint has read it
        const size_t nc = p->npts, nf = p->npts + p->plane;
        PS_HIP(launch_scale(lu, g_hprev[0], crho, nc, st), "h_prev adjoint");
        PS_HIP(launch_scale(lv, g_hprev[1], crho, nc, st), "h_prev adjoint");
        PS_HIP(launch_scale(lw, g_hprev[2], crho, nf, st), "h_prev adjoint");
        PS_HIP(launch_scale(lt, g_hprev[3], crho, nf, st), "h_prev adjoint");
    }
    return r;
}

// Field-sized temporaries of the step adjoint (allocated on first use): the states after
// substeps 1 and 2 (five fields each), the H hand-over (four), two sets of state
// cotangents (five each) and two H cotangents (four each: substep 2 reads one while its
// Crank-Nicolson adjoint writes the other).
constexpr int kStepAdjFields = 32;

ps_status rk3_step_adjoint(ps_plan_t p, double dt, double nu, double kappa, const double* u, const double* v,
                           const double* w, const double* t, const double* pr, const double* const* g_out,
                           double* const* g_in, void* stream, ps_info* info) {
    PS_RANGE("rk3_step_adjoint");
    PS_CHECK(check_plan(p));
    if (!(dt > 0) || !std::isfinite(dt)) return fail(PS_EINVAL, "dt must be positive (the step adjoint takes dt fixed)");
    if (!(nu >= 0) || !(kappa >= 0) || !std::isfinite(nu) || !std::isfinite(kappa))
        return fail(PS_EINVAL, "nu and kappa must be non-negative");
    const double* in[5] = {u, v, w, t, pr};
    for (int q = 0; q < 5; ++q) PS_CHECK(check_ptr(in[q], "state"));
    if (!g_out || !g_in) return fail(PS_EINVAL, "g_out and g_in are required");
    for (int q = 0; q < 5; ++q) {
        PS_CHECK(check_ptr(g_out[q], "g_out[q]"));
        PS_CHECK(check_ptr(g_in[q], "g_in[q]"));
        for (int r = 0; r < 5; ++r)
            if ((const void*)g_in[q] == (const void*)g_out[r]) return fail(PS_EINVAL, "g_in may not alias g_out");
    }
    PS_CHECK(ensure_substep_buffers(p));
    const size_t per = align256((p->npts + p->plane) * sizeof(double));
    if (!p->stepadj_buf) {
        if (!dev_alloc((void**)&p->stepadj_buf, per * kStepAdjFields))
            return fail(PS_ENOMEM, "cannot allocate %zu bytes of step-adjoint temporaries", per * kStepAdjFields);
    }
    auto fld = [&](int q) { return (double*)((char*)p->stepadj_buf + per * q); };
    double* s1[5] = {fld(0), fld(1), fld(2), fld(3), fld(4)};
    double* s2[5] = {fld(5), fld(6), fld(7), fld(8), fld(9)};
    double* h[4] = {fld(10), fld(11), fld(12), fld(13)};
    double* ga[5] = {fld(14), fld(15), fld(16), fld(17), fld(18)};
    double* gb[5] = {fld(19), fld(20), fld(21), fld(22), fld(23)};
    double* gh[4] = {fld(24), fld(25), fld(26), fld(27)};
    double* gh2[4] = {fld(28), fld(29), fld(30), fld(31)};
    const double* hc[4] = {h[0], h[1], h[2], h[3]};
    const double* ghc[4] = {gh[0], gh[1], gh[2], gh[3]};
    const double* gh2c[4] = {gh2[0], gh2[1], gh2[2], gh2[3]};
    hipStream_t st = (hipStream_t)stream;
    // forward recomputation from the stored input: states after substeps 1 and 2 (each substep
    // reads the state before it and writes the next one to its own buffers)
    Range phase("forward recomputation");
    ps_status worst = PS_OK;
    auto note = [&](ps_status r) {
        if (r == PS_ENOTCONVERGED && worst == PS_OK) worst = r;
        return r == PS_OK || r == PS_ENOTCONVERGED;
    };
    const double* s1c[5] = {s1[0], s1[1], s1[2], s1[3], s1[4]};
    ps_status r = substep_impl(p, 1, dt, nu, kappa, s1[0], s1[1], s1[2], s1[3], s1[4], nullptr, h, stream, nullptr,
                               true, in);
    if (!note(r)) return r;
    r = substep_impl(p, 2, dt, nu, kappa, s2[0], s2[1], s2[2], s2[3], s2[4], hc, nullptr, stream, nullptr, true,
                     s1c);
    if (!note(r)) return r;
    phase.next("reverse sweep");
    // reverse sweep: substep 3 at s2, substep 2 at s1 (with the cotangent of H^2), substep 1
    // at the input (with the cotangent of H^1); the two H cotangents in separate buffers
    const double* go[5] = {g_out[0], g_out[1], g_out[2], g_out[3], g_out[4]};
    const double* gac[5] = {ga[0], ga[1], ga[2], ga[3], ga[4]};
    const double* gbc[5] = {gb[0], gb[1], gb[2], gb[3], gb[4]};
    r = rk3_substep_adjoint(p, 3, dt, nu, kappa, s2[0], s2[1], s2[2], s2[3], s2[4], go, nullptr, ga, gh, stream,
                            nullptr);
    if (!note(r)) return r;
    r = rk3_substep_adjoint(p, 2, dt, nu, kappa, s1[0], s1[1], s1[2], s1[3], s1[4], gac, ghc, gb, gh2, stream,
                            nullptr);
    if (!note(r)) return r;
    r = rk3_substep_adjoint(p, 1, dt, nu, kappa, u, v, w, t, pr, gbc, gh2c, g_in, nullptr, stream, info);
    if (!note(r)) return r;
    if (worst != PS_OK) return fail(worst, "a Poisson refinement of the step adjoint stopped above the tolerance");
    return PS_OK;
}

ps_status ps_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    PS_RANGE("ps_stream_copy");
    if (!dst || !src || ((uintptr_t)dst) % 16 || ((uintptr_t)src) % 16)
        return fail(PS_EINVAL, "src and dst must be 16-byte aligned device pointers");
    const char* s0 = (const char*)src;
    const char* d0 = (const char*)dst;
    if (d0 < s0 + bytes && s0 < d0 + bytes && bytes) return fail(PS_EINVAL, "src and dst overlap");
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        ncu = 0;
    }
    PS_HIP(launch_stream_copy(dst, src, bytes, ncu, (hipStream_t)stream), "stream copy");
    return PS_OK;
}

ps_status ps_spectral_layout(ps_plan_t p, int* w_tile, int* nkxb) {
    if (!p) return fail(PS_EINVAL, "plan is NULL");
    if (w_tile) *w_tile = p->w_tile;
    if (nkxb) *nkxb = p->nkxb;
    return PS_OK;
}

size_t ps_spectral_elems(ps_plan_t p) { return p ? p->spec_elems : 0; }

ps_status ps_debug_stage(ps_plan_t p, int stage, const void* in, void* out, void* stream) {
    PS_RANGE("ps_debug_stage");
    PS_CHECK(check_plan(p));
    hipStream_t st = (hipStream_t)stream;
    const size_t eb = elem_bytes(p->prec);
    const size_t sb = p->spec_elems * eb;
    // stage inputs are copied into the plan's buffers, outputs copied out, so the
    // kernels run on their usual buffers
    auto copy_in = [&](void* dst) -> ps_status {
        if (in && in != dst) PS_HIP(hipMemcpyAsync(dst, in, sb, hipMemcpyDeviceToDevice, st), "copy in");
        return PS_OK;
    };
    auto copy_out = [&](void* src) -> ps_status {
        if (out && out != src) PS_HIP(hipMemcpyAsync(out, src, sb, hipMemcpyDeviceToDevice, st), "copy out");
        return PS_OK;
    };
    const bool f64 = p->prec == PS_FP64;
    const GridDev& g = p->gd;
    // each stage alone, on the spectrum as it stands: FP32 stages keep the (0,0) entry in
    // the spectrum (no FP64 side column)
    SpecDev<float> sf = spec_of<float>(p);
    sf.rowsum = sf.psum = sf.col00 = nullptr;
    switch (stage) {
        case 0:
            PS_CHECK(check_ptr(in, "in"));
            PS_HIP(f64 ? launch_xfwd<double>(g, spec_of<double>(p), (const double*)in, nullptr, nullptr, st)
                       : launch_xfwd<float>(g, sf, (const double*)in, nullptr, nullptr, st),
                   "x forward FFT");
            return copy_out(p->spec_a);
        case 1:
            PS_CHECK(copy_in(p->spec_a));
            PS_HIP(f64 ? launch_yfwd<double>(g, spec_of<double>(p), st) : launch_yfwd<float>(g, sf, st),
                   "y forward FFT");
            return copy_out(p->spec_b);
        case 2: {
            // as in poisson_solve: out of place from B into A where that path applies
            PS_CHECK(copy_in(p->spec_b));
            const bool whole = p->chunk <= 0 || p->chunk >= g.nz;
            const bool oop = whole && (f64 ? zsolve_out_of_place<double>(g) : zsolve_out_of_place<float>(g));
            if (f64) {
                SpecDev<double> sz = spec_of<double>(p);
                if (oop) sz.bz = sz.a;
                PS_HIP(launch_zsolve<double>(g, sz, st), "z solve");
                PS_HIP(launch_zsolve00<double>(g, sz, p->small + R_DEFECT, st), "z solve (0,0)");
            } else {
                SpecDev<float> sz = sf;
                if (oop) sz.bz = sz.a;
                PS_HIP(launch_zsolve<float>(g, sz, st), "z solve");
                PS_HIP(launch_zsolve00<float>(g, sz, p->small + R_DEFECT, st), "z solve (0,0)");
            }
            return copy_out(oop ? p->spec_a : p->spec_b);
        }
        case 3:
            PS_CHECK(copy_in(p->spec_b));
            PS_HIP(f64 ? launch_yinv<double>(g, spec_of<double>(p), st) : launch_yinv<float>(g, sf, st),
                   "y inverse FFT");
            return copy_out(p->spec_a);
        case 4: {
            PS_CHECK(copy_in(p->spec_a));
            PS_CHECK(check_ptr(out, "out"));
            const double scale = 1.0 / ((double)p->nx * (double)p->ny);
            PS_HIP(f64 ? launch_xinv<double>(g, spec_of<double>(p), (double*)out, scale, 0, nullptr, 0.0, nullptr, nullptr, st)
                       : launch_xinv<float>(g, sf, (double*)out, scale, 0, nullptr, 0.0, nullptr, nullptr, st),
                   "x inverse FFT");
            return PS_OK;
        }
        default:
            return fail(PS_EINVAL, "unknown stage %d", stage);
    }
}

}  // extern "C"

namespace {
ps_status check_finite(ps_plan_t p, const double* f, hipStream_t st) {
    unsigned* flag = reinterpret_cast<unsigned*>(p->small + R_FLAG);
    PS_HIP(launch_fill(p->small + R_FLAG, 1, 0.0, st), "fill");
    PS_HIP(launch_nonfinite(f, p->npts, flag, st), "finite check");
    PS_CHECK(read_small(p, st));
    unsigned hv;
    memcpy(&hv, p->h_res + R_FLAG, sizeof(hv));
    if (hv) return fail(PS_ENONFINITE, "input holds NaN or Inf");
    return PS_OK;
}
}  // namespace

// ============================================================================
// Multiple-resolution temperature grid (Sec. 6)
struct ps_mr_s {
    ps_plan_t plan;
    int rx, ry, rz, nsub;
    int nxf, nyf, nzf;
    size_t fc, ff;        // values per fine centre / face field
    GridDev gf;           // temperature grid
    MrDev md;
    void* d_tab = nullptr;
    double* cnfac;        // Crank-Nicolson factors of the temperature grid, 3 (nzf + 1)
    double dzz_max;       // max over interior faces of Dzz's off-diagonal sum on the temperature grid
    double* buf = nullptr;
    double *u0, *v0, *w0, *u1, *v1, *w1, *rt, *h, *tc;
};

namespace {

// (L_loc)^+ of the rx x ry x rz sub-cells of one coarse cell (spacings hx, hy, hz, closed outer
// faces), from the eigenvectors of the one-dimensional Neumann Laplacians:
// v_p[n] = cos(pi p (n + 1/2) / r), eigenvalue -(4 / h^2) sin^2(pi p / (2 r)).
void local_pinv(int rx, int ry, int rz, double hx, double hy, double hz, double* out) {
    const int ns = rx * ry * rz;
    const long double pi = 3.141592653589793238462643383279502884L;
    auto vec = [&](int r, int p, int n) { return (double)cosl(pi * p * (n + 0.5L) / r); };
    auto mu = [&](int r, int p, double h) {
        const double sn = (double)sinl(pi * p / (2.0L * r));
        return -(4.0 / (h * h)) * sn * sn;
    };
    for (int q = 0; q < ns * ns; ++q) out[q] = 0.0;
    for (int pz = 0; pz < rz; ++pz)
        for (int py = 0; py < ry; ++py)
            for (int px = 0; px < rx; ++px) {
                if (px == 0 && py == 0 && pz == 0) continue;
                const double lam = mu(rx, px, hx) + mu(ry, py, hy) + mu(rz, pz, hz);
                const double nrm = (px ? rx / 2.0 : rx) * (py ? ry / 2.0 : ry) * (pz ? rz / 2.0 : rz);
                std::vector<double> e(ns);
                for (int c = 0; c < rz; ++c)
                    for (int b = 0; b < ry; ++b)
                        for (int a = 0; a < rx; ++a)
                            e[(c * ry + b) * rx + a] = vec(rx, px, a) * vec(ry, py, b) * vec(rz, pz, c);
                for (int s = 0; s < ns; ++s)
                    for (int t = 0; t < ns; ++t) out[s * ns + t] += e[s] * e[t] / (nrm * lam);
            }
}

ps_status check_mr(ps_mr_t m) {
    if (!m) return fail(PS_EINVAL, "multi-resolution object is NULL");
    return check_plan(m->plan);
}

}  // namespace

extern "C" {

ps_status mr_create(ps_mr_t* out, ps_plan_t p, int rx, int ry, int rz, int nsub) {
    PS_RANGE("mr_create");
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    PS_CHECK(check_plan(p));
    if (!mr_factors_supported(rx, ry, rz))
        return fail(PS_EINVAL, "refinement factors (%d, %d, %d): each must be 1 or 2", rx, ry, rz);
    if (nsub < 1 || nsub > 64) return fail(PS_EINVAL, "nsub=%d: need 1 <= nsub <= 64", nsub);
    const int nzf = p->nz * rz;
    if (nzf > 2048) return fail(PS_EINVAL, "temperature grid of %d levels: at most 2048", nzf);
    ps_mr_t m = new ps_mr_s();
    m->plan = p;
    m->rx = rx;
    m->ry = ry;
    m->rz = rz;
    m->nsub = nsub;
    m->nxf = p->nx * rx;
    m->nyf = p->ny * ry;
    m->nzf = nzf;
    const size_t planef = (size_t)m->nxf * m->nyf;
    m->fc = planef * nzf;
    m->ff = planef * (nzf + 1);
    // temperature-grid faces: every momentum cell split into rz equal sub-cells
    const int nz = p->nz;
    std::vector<double> zff(nzf + 1);
    for (int k = 0; k < nz; ++k)
        for (int q = 0; q < rz; ++q) zff[k * rz + q] = p->zf[k] + ((double)q / rz) * p->dz[k];
    zff[nzf] = p->zf[nz];
    std::vector<double> dzf(nzf), dzcf(nzf + 1, 0.0), of(nzf + 1, 0.0), dzwf(nzf + 1, 0.0), idzf(nzf),
        idzwf(nzf + 1);
    for (int k = 0; k < nzf; ++k) {
        dzf[k] = zff[k + 1] - zff[k];
        idzf[k] = 1.0 / dzf[k];
    }
    for (int k = 1; k < nzf; ++k) {
        dzcf[k] = 0.5 * (dzf[k - 1] + dzf[k]);
        of[k] = 1.0 / dzcf[k];
        dzwf[k] = dzcf[k];
    }
    dzwf[0] = 0.5 * dzf[0];
    dzwf[nzf] = 0.5 * dzf[nzf - 1];
    for (int k = 0; k <= nzf; ++k) idzwf[k] = 1.0 / dzwf[k];
    m->dzz_max = 0.0;
    for (int k = 1; k < nzf; ++k) m->dzz_max = std::max(m->dzz_max, 1.0 / (dzf[k - 1] * dzcf[k]) + 1.0 / (dzf[k] * dzcf[k]));
    // slope stencil distances and local pseudo-inverses per momentum level
    const int ns = rx * ry * rz;
    std::vector<double> zc(nz), zhm(nz), zhp(nz), linv((size_t)nz * ns * ns);
    for (int k = 0; k < nz; ++k) zc[k] = 0.5 * (p->zf[k] + p->zf[k + 1]);
    for (int k = 0; k < nz; ++k) {
        zhm[k] = zc[k] - (k > 0 ? zc[k - 1] : p->zf[0]);
        zhp[k] = (k + 1 < nz ? zc[k + 1] : p->zf[nz]) - zc[k];
        local_pinv(rx, ry, rz, p->lx / m->nxf, p->ly / m->nyf, p->dz[k] / rz, linv.data() + (size_t)k * ns * ns);
    }
    // one device table: fine metrics, mr tables, CN factors
    std::vector<double> host;
    auto put = [&](const std::vector<double>& vv) {
        const size_t at = host.size();
        host.insert(host.end(), vv.begin(), vv.end());
        while (host.size() % 32) host.push_back(0.0);
        return at;
    };
    const size_t a_dz = put(dzf), a_dzc = put(dzcf), a_o = put(of), a_dzw = put(dzwf), a_idz = put(idzf),
                 a_idzw = put(idzwf), a_hm = put(zhm), a_hp = put(zhp), a_li = put(linv);
    const size_t a_cn = host.size();
    host.resize(host.size() + 3 * (size_t)(nzf + 1) + 32, 0.0);
    if (!dev_alloc(&m->d_tab, host.size() * sizeof(double))) {
        delete m;
        return fail(PS_ENOMEM, "cannot allocate the temperature-grid tables");
    }
    if (hipMemcpy(m->d_tab, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        hipFree(m->d_tab);
        delete m;
        return fail(PS_EDEVICE, "cannot upload the temperature-grid tables");
    }
    const double* d = (const double*)m->d_tab;
    GridDev& g = m->gf;
    g.nx = m->nxf;
    g.ny = m->nyf;
    g.nz = nzf;
    g.dx = p->lx / m->nxf;
    g.dy = p->ly / m->nyf;
    g.dz = d + a_dz;
    g.dzc = d + a_dzc;
    g.o = d + a_o;
    g.dzw = d + a_dzw;
    g.lamx = nullptr;
    g.lamy = nullptr;
    g.idz = d + a_idz;
    g.idzw = d + a_idzw;
    m->md.rx = rx;
    m->md.ry = ry;
    m->md.rz = rz;
    m->md.dxf = g.dx;
    m->md.dyf = g.dy;
    m->md.dzf = g.dz;
    m->md.zhm = d + a_hm;
    m->md.zhp = d + a_hp;
    m->md.linv = d + a_li;
    m->cnfac = (double*)m->d_tab + a_cn;
    // fields: two temperature-grid velocities, the temperature right-hand side and H, and the
    // temperature the momentum equations see
    const size_t per = align256(m->ff * sizeof(double));
    const size_t coarse = align256((p->npts + p->plane) * sizeof(double));
    if (!dev_alloc((void**)&m->buf, per * 8 + coarse)) {
        hipFree(m->d_tab);
        delete m;
        return fail(PS_ENOMEM, "cannot allocate %zu bytes of temperature-grid fields", per * 8 + coarse);
    }
    double* f[9];
    for (int q = 0; q < 9; ++q) f[q] = (double*)((char*)m->buf + per * q);
    m->u0 = f[0];
    m->v0 = f[1];
    m->w0 = f[2];
    m->u1 = f[3];
    m->v1 = f[4];
    m->w1 = f[5];
    m->rt = f[6];
    m->h = f[7];
    m->tc = f[8];
    *out = m;
    return PS_OK;
}

ps_status mr_destroy(ps_mr_t m) {
    PS_RANGE("mr_destroy");
    if (!m) return PS_OK;
    if (m->buf) hipFree(m->buf);
    if (m->d_tab) hipFree(m->d_tab);
    delete m;
    return PS_OK;
}

ps_status mr_shape(ps_mr_t m, int* nxf, int* nyf, int* nzf) {
    if (!m) return fail(PS_EINVAL, "multi-resolution object is NULL");
    if (nxf) *nxf = m->nxf;
    if (nyf) *nyf = m->nyf;
    if (nzf) *nzf = m->nzf;
    return PS_OK;
}

ps_status mr_prolong_velocity(ps_mr_t m, const double* u, const double* v, const double* w, double* uf, double* vf,
                              double* wf, void* stream) {
    PS_RANGE("mr_prolong_velocity");
    PS_CHECK(check_mr(m));
    const void* ps[6] = {u, v, w, uf, vf, wf};
    const char* names[6] = {"u", "v", "w", "uf", "vf", "wf"};
    for (int q = 0; q < 6; ++q) PS_CHECK(check_ptr(ps[q], names[q]));
    for (int q = 0; q < 3; ++q)
        for (int r = 3; r < 6; ++r)
            if (ps[q] == ps[r]) return fail(PS_EINVAL, "outputs may not alias inputs");
    PS_HIP(launch_mr_prolong(m->plan->gd, m->md, u, v, w, uf, vf, wf, (hipStream_t)stream), "prolongation");
    return PS_OK;
}

ps_status mr_restrict_temperature(ps_mr_t m, const double* tf, double* tc, void* stream) {
    PS_RANGE("mr_restrict_temperature");
    PS_CHECK(check_mr(m));
    PS_CHECK(check_ptr(tf, "tf"));
    PS_CHECK(check_ptr(tc, "tc"));
    if ((const void*)tf == (const void*)tc) return fail(PS_EINVAL, "tc may not alias tf");
    PS_HIP(launch_mr_restrict(m->plan->gd, m->md, tf, tc, (hipStream_t)stream), "restriction");
    return PS_OK;
}

}  // extern "C"

namespace {

// nsub RK3 steps of dt / nsub for the temperature on its grid; stage velocity linear in time
// between vel0 and vel1 at the stage's start time.
ps_status mr_tstep(ps_mr_t m, double dt, double kappa, const double* const* v0, const double* const* v1, double* tf,
                   hipStream_t st) {
    const double start[3] = {0.0, 8.0 / 15.0, 2.0 / 3.0};
    const double dts = dt / m->nsub;
    for (int s = 0; s < m->nsub; ++s)
        for (int l = 1; l <= 3; ++l) {
            const double gam = kGamma[l - 1], rho = kRho[l - 1], alp = gam + rho;
            MrTArgs a{};
            a.u0 = v0[0];
            a.v0 = v0[1];
            a.w0 = v0[2];
            a.u1 = v1[0];
            a.v1 = v1[1];
            a.w1 = v1[2];
            a.t = tf;
            a.hp = m->h;
            a.rt = m->rt;
            a.hout = l < 3 ? m->h : nullptr;
            a.th = (s + start[l - 1]) / m->nsub;
            a.dt = dts;
            a.ka = kappa;
            a.gam = gam;
            a.rho = rho;
            a.alp = alp;
            const double bka = alp * dts * kappa / 2.0;
            const bool set_form = bka * m->dzz_max <= kCnSetFormMax;   // as in the momentum substep
            a.cq = set_form ? 1 : 0;
            a.bka = set_form ? bka : 0.0;
            PS_HIP(launch_mr_explicit_t(m->gf, a, st), "temperature explicit terms");
            CnFactorJobs fj{};
            fj.fac[0] = m->cnfac;
            fj.beta[0] = bka;
            fj.kind[0] = PS_FACE;
            fj.n = 1;
            PS_HIP(launch_cn_factor(m->gf, fj, st), "cn factor");
            // rt holds C T + rhs (T* = C^-1 rt) or rhs alone (T* = T + C^-1 rt)
            CnJobs jobs{};
            jobs.j[0] = CnJob{m->cnfac, m->rt, tf, nullptr, 0.0, PS_FACE};
            jobs.n = 1;
            PS_HIP(launch_cn_jobs(m->gf, set_form ? CN_PUT : CN_ADD, jobs, st), "cn solve T");
        }
    return PS_OK;
}

}  // namespace

extern "C" {

ps_status mr_temperature_step(ps_mr_t m, double dt, double kappa, const double* const* vel0,
                              const double* const* vel1, double* tf, void* stream) {
    PS_RANGE("mr_temperature_step");
    PS_CHECK(check_mr(m));
    if (!(dt > 0) || !std::isfinite(dt)) return fail(PS_EINVAL, "dt must be positive");
    if (!(kappa >= 0) || !std::isfinite(kappa)) return fail(PS_EINVAL, "kappa must be non-negative");
    if (!vel0 || !vel1) return fail(PS_EINVAL, "vel0 and vel1 are required");
    for (int q = 0; q < 3; ++q) {
        PS_CHECK(check_ptr(vel0[q], "vel0[q]"));
        PS_CHECK(check_ptr(vel1[q], "vel1[q]"));
        if ((const void*)vel0[q] == (const void*)tf || (const void*)vel1[q] == (const void*)tf)
            return fail(PS_EINVAL, "tf may not alias a velocity");
    }
    PS_CHECK(check_ptr(tf, "tf"));
    return mr_tstep(m, dt, kappa, vel0, vel1, tf, (hipStream_t)stream);
}

ps_status rk3_step_mr(ps_mr_t m, double dt, double cfl_target, double dt_max, double nu, double kappa, double* u,
                      double* v, double* w, double* pr, double* tf, double* dt_used, void* stream, ps_info* info) {
    PS_RANGE("rk3_step_mr");
    PS_CHECK(check_mr(m));
    ps_plan_t p = m->plan;
    PS_CHECK(check_ptr(u, "u"));
    PS_CHECK(check_ptr(v, "v"));
    PS_CHECK(check_ptr(w, "w"));
    PS_CHECK(check_ptr(pr, "p"));
    PS_CHECK(check_ptr(tf, "tf"));
    if (!(nu >= 0) || !(kappa >= 0) || !std::isfinite(nu) || !std::isfinite(kappa))
        return fail(PS_EINVAL, "nu and kappa must be non-negative");
    hipStream_t st = (hipStream_t)stream;
    if (!(dt > 0)) {
        if (!(cfl_target > 0) || !std::isfinite(cfl_target)) return fail(PS_EINVAL, "cfl_target must be positive");
        if (!(dt_max > 0)) return fail(PS_EINVAL, "dt_max must be positive");
        PS_HIP(launch_cfl(p->gd, u, v, w, p->small + R_CFL, st), "cfl");
        PS_CHECK(read_small(p, st));
        const double c = p->h_res[R_CFL];
        if (!std::isfinite(c)) return fail(PS_ENONFINITE, "Courant number is not finite");
        dt = std::min(dt_max, cfl_target / std::max(c, 1e-8));
    }
    if (!std::isfinite(dt)) return fail(PS_EINVAL, "dt must be finite");
    PS_CHECK(ensure_substep_buffers(p));
    // buoyancy: the temperature restricted to the momentum grid, frozen over the step
    Range phase("restriction and prolongation");
    PS_HIP(launch_mr_restrict(p->gd, m->md, tf, m->tc, st), "restriction");
    PS_HIP(launch_mr_prolong(p->gd, m->md, u, v, w, m->u0, m->v0, m->w0, st), "prolongation");
    phase.next("momentum substeps");
    double* h[4] = {sub_field(p, 4), sub_field(p, 5), sub_field(p, 6), sub_field(p, 7)};
    const double* hc[4] = {h[0], h[1], h[2], h[3]};
    ps_info acc{};
    ps_status result = PS_OK;
    std::string first_msg;
    for (int l = 1; l <= 3; ++l) {
        ps_info li{};
        const ps_status r = substep_impl(p, l, dt, nu, kappa, u, v, w, m->tc, pr, l > 1 ? hc : nullptr,
                                         l < 3 ? h : nullptr, stream, info ? &li : nullptr, false);
        if (r != PS_OK && r != PS_ENOTCONVERGED) return r;
        if (r == PS_ENOTCONVERGED && result == PS_OK) {
            result = r;
            first_msg = g_last_error;
        }
        acc.iterations += li.iterations;
        acc.rel_update = std::max(acc.rel_update, li.rel_update);
        acc.rel_residual = std::max(acc.rel_residual, li.rel_residual);
        acc.compat_defect = li.compat_defect;
        acc.gauge_shift = li.gauge_shift;
    }
    phase.next("temperature step");
    PS_HIP(launch_mr_prolong(p->gd, m->md, u, v, w, m->u1, m->v1, m->w1, st), "prolongation");
    const double* v0[3] = {m->u0, m->v0, m->w0};
    const double* v1[3] = {m->u1, m->v1, m->w1};
    PS_CHECK(mr_tstep(m, dt, kappa, v0, v1, tf, st));
    if (dt_used) *dt_used = dt;
    if (info) *info = acc;
    if (result != PS_OK) return fail(result, "%s", first_msg.c_str());
    return PS_OK;
}

}  // extern "C"
