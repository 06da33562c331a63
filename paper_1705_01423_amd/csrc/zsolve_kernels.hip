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
    const size_t ncol = (size_t)s.nkxb * g.ny * W;
    const int nblk = (int)((ncol + 255) / 256);
    hipLaunchKernelGGL((k_zsolve_seq<T>), dim3(nblk), dim3(256), 0, st, s.b, s.piv, g.nz, g.ny, s.nkxb,
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
