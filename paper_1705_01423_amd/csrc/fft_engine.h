// Register-blocked Stockham FFT engine for gfx950 (wave64, LDS exchange).
//
// A length-N complex transform is computed by NT = N/E cooperating threads,
// each holding E elements in registers.  Each pass p applies radix r_p
// butterflies in registers (each thread owns E/r_p of them); between passes
// the elements are exchanged through LDS.  The first pass reads its inputs
// through a loader functor and the last pass hands its outputs (natural
// order) to a storer functor, so global memory is touched exactly once each
// way.  Butterflies of radix 2..16 are fully unrolled at compile time with
// constant twiddles (all radices divide 48); inter-pass twiddles come from a
// table exp(-2 pi i q / N), q < N, built in FP64 on the host.
//
// Stockham indexing (self-sorting): at pass p with radix r and sub-length
// Ls = r_0 ... r_{p-1}, butterfly j in [0, N/r) reads x[j + m N/r], applies
// w^m with w = exp(sign 2 pi i (j mod Ls) / (Ls r)), transforms, and writes
// x[(j - j mod Ls) r + j mod Ls + m Ls], m = 0..r-1.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

namespace ps {

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> scal(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// cos(2 pi m / 48) for the first quadrant, m = 0..12 (FP64, correctly rounded)
__host__ __device__ constexpr double cq48(int m) {
    constexpr double t[13] = {1.0, 0.9914448613738104, 0.9659258262890683, 0.9238795325112867,
                              0.8660254037844386, 0.7933533402912352, 0.7071067811865476,
                              0.6087614290087207, 0.5, 0.3826834323650898, 0.25881904510252074,
                              0.1305261922200516, 0.0};
    return t[m];
}
__host__ __device__ constexpr double cos48(int m) {
    m = ((m % 48) + 48) % 48;
    if (m <= 12) return cq48(m);
    if (m <= 24) return -cq48(24 - m);
    if (m <= 36) return -cq48(m - 24);
    return cq48(48 - m);
}
__host__ __device__ constexpr double sin48(int m) { return cos48(m - 12); }

// a * exp(S * 2 pi i M / 48), S = +1 / -1, with the quarter turns done exactly
template <int S, int M, typename T>
__device__ __forceinline__ cx<T> tw48(cx<T> a) {
    constexpr int m = ((M % 48) + 48) % 48;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 12) {
        return S > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
    } else if constexpr (m == 24) {
        return cx<T>{-a.x, -a.y};
    } else if constexpr (m == 36) {
        return S > 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
    } else {
        constexpr T c = (T)cos48(m);
        constexpr T s = (T)(S * sin48(m));
        return cx<T>{a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

template <int I, int End, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < End) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, End>(f);
    }
}

// ---- in-register DFTs, x[0..R) natural order in and out, sign S ----------
template <int R, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<1, S, T> {
    __device__ __forceinline__ static void run(cx<T>*) {}
};

template <int S, typename T>
struct Dft<2, S, T> {
    __device__ __forceinline__ static void run(cx<T>* x) {
        cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    }
};

template <int S, typename T>
struct Dft<3, S, T> {
    __device__ __forceinline__ static void run(cx<T>* x) {
        constexpr T h = (T)0.8660254037844386;   // sqrt(3)/2
        cx<T> t1 = x[1] + x[2];
        cx<T> t2 = {x[0].x - (T)0.5 * t1.x, x[0].y - (T)0.5 * t1.y};
        cx<T> d = x[1] - x[2];
        // i * S * h * d
        cx<T> t3 = {-(T)S * h * d.y, (T)S * h * d.x};
        x[0] = x[0] + t1;
        x[1] = t2 + t3;
        x[2] = t2 - t3;
    }
};

template <int S, typename T>
struct Dft<4, S, T> {
    __device__ __forceinline__ static void run(cx<T>* x) {
        cx<T> a = x[0] + x[2], b = x[0] - x[2];
        cx<T> c = x[1] + x[3], d = x[1] - x[3];
        cx<T> id = S > 0 ? cx<T>{-d.y, d.x} : cx<T>{d.y, -d.x};   // S i d
        x[0] = a + c;
        x[2] = a - c;
        x[1] = b + id;
        x[3] = b - id;
    }
};

__host__ __device__ constexpr int first_split(int r) { return (r % 4 == 0 && r > 4) ? 4 : (r % 2 == 0 ? 2 : 3); }

// composite radix R = R1 * R2, Cooley-Tukey in registers: n = R2 n1 + n2, k = k1 + R1 k2
template <int R, int S, typename T>
struct Dft {
    static constexpr int R1 = first_split(R);
    static constexpr int R2 = R / R1;
    __device__ __forceinline__ static void run(cx<T>* x) {
        cx<T> y[R];
        static_for<0, R2>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            cx<T> a[R1];
            static_for<0, R1>([&](auto n1c) {
                constexpr int n1 = decltype(n1c)::value;
                a[n1] = x[R2 * n1 + n2];
            });
            Dft<R1, S, T>::run(a);
            static_for<0, R1>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                y[n2 * R1 + k1] = tw48<S, (48 / R) * n2 * k1>(a[k1]);
            });
        });
        static_for<0, R1>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            cx<T> b[R2];
            static_for<0, R2>([&](auto n2c) {
                constexpr int n2 = decltype(n2c)::value;
                b[n2] = y[n2 * R1 + k1];
            });
            Dft<R2, S, T>::run(b);
            static_for<0, R2>([&](auto k2c) {
                constexpr int k2 = decltype(k2c)::value;
                x[k1 + R1 * k2] = b[k2];
            });
        });
    }
};

// ---- compile-time pass schedule ------------------------------------------
struct RadixPlan {
    int n, e, np;
    int r[24];
};

__host__ __device__ constexpr RadixPlan make_plan(int n, int e) {
    RadixPlan p{n, e, 0, {}};
    int rem = n;
    const int cand[7] = {16, 12, 8, 6, 4, 3, 2};
    while (rem > 1) {
        int pick = 0;
        for (int i = 0; i < 7; ++i) {
            if (e % cand[i] == 0 && rem % cand[i] == 0) {
                pick = cand[i];
                break;
            }
        }
        if (pick == 0) {
            p.np = -1;
            return p;
        }
        p.r[p.np++] = pick;
        rem /= pick;
    }
    if (p.np == 0) {   // n == 1
        p.r[0] = 1;
        p.np = 1;
    }
    return p;
}

__host__ __device__ constexpr int plan_ls(RadixPlan p, int i) {
    int l = 1;
    for (int q = 0; q < i; ++q) l *= p.r[q];
    return l;
}

// elements per thread: the largest E <= emax dividing n for which a schedule exists
__host__ __device__ constexpr int choose_e(int n, int emax) {
    const int cand[9] = {32, 16, 12, 8, 6, 4, 3, 2, 1};
    for (int i = 0; i < 9; ++i) {
        int e = cand[i];
        if (e <= emax && n % e == 0 && make_plan(n, e).np > 0) return e;
    }
    return 1;
}

template <int N, int EMAX>
struct FftShape {
    static constexpr int E = choose_e(N, EMAX);
    static constexpr int NT = N / E;
    static constexpr RadixPlan P = make_plan(N, E);
    static constexpr int NP = P.np;
};

// twiddle power table: pw[m] = w^m, m < R, built with few products
template <int R, typename T>
__device__ __forceinline__ void powers(cx<T> w, cx<T>* pw) {
    pw[0] = {(T)1, (T)0};
    if constexpr (R > 1) pw[1] = w;
    static_for<2, R>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        if constexpr (m % 2 == 0)
            pw[m] = cmul(pw[m / 2], pw[m / 2]);
        else
            pw[m] = cmul(pw[m - 1], w);
    });
}

// One radix pass (twiddle + butterflies) on the registers of thread t.
// tw: table exp(-2 pi i q / N); the inverse transform uses its conjugate.
template <typename T, int N, int EMAX, int S, int I>
__device__ __forceinline__ void pass_compute(cx<T>* v, int t, const cx<T>* __restrict__ tw) {
    using Sh = FftShape<N, EMAX>;
    constexpr int r = Sh::P.r[I];
    constexpr int Ls = plan_ls(Sh::P, I);
    constexpr int NT = Sh::NT;
#pragma unroll
    for (int b = 0; b < Sh::E / r; ++b) {
        if constexpr (Ls > 1) {
            const int j = t + b * NT;
            const int k = j % Ls;
            cx<T> w = tw[k * (N / (Ls * r))];
            if (S > 0) w.y = -w.y;
            cx<T> pw[r];
            powers<r, T>(w, pw);
#pragma unroll
            for (int m = 1; m < r; ++m) v[b * r + m] = cmul(v[b * r + m], pw[m]);
        }
        Dft<r, S, T>::run(v + b * r);
    }
}

// LDS slot of element e: one padding slot after every 16 elements, so that the
// stride-r writes after a radix-r pass (r <= 16) spread over the LDS banks.
__host__ __device__ constexpr int lds_pad(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int lds_len(int n) { return n + (n >> 4) + 1; }

// Full transform.  base/stride address this transform's LDS scratch
// (element e at base[lds_pad(e) * stride], lds_len(N) slots).  All threads of
// the block must call this (it synchronises the block between passes).
template <typename T, int N, int EMAX, int S, class Ld, class St>
__device__ __forceinline__ void fft_run(int t, cx<T>* base, int stride, const cx<T>* __restrict__ tw,
                                        Ld&& ld, St&& st) {
    using Sh = FftShape<N, EMAX>;
    constexpr int E = Sh::E;
    constexpr int NT = Sh::NT;
    constexpr int NP = Sh::NP;
    cx<T> v[E];
    {
        constexpr int r = Sh::P.r[0];
#pragma unroll
        for (int b = 0; b < E / r; ++b) {
#pragma unroll
            for (int m = 0; m < r; ++m) v[b * r + m] = ld(t + b * NT + m * (N / r));
        }
    }
    pass_compute<T, N, EMAX, S, 0>(v, t, tw);
    static_for<1, NP>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr int rp = Sh::P.r[I - 1];
        constexpr int Lp = plan_ls(Sh::P, I - 1);
        constexpr int r = Sh::P.r[I];
        __syncthreads();
#pragma unroll
        for (int b = 0; b < E / rp; ++b) {
            const int j = t + b * NT;
            const int k = j % Lp;
            const int o0 = (j - k) * rp + k;
#pragma unroll
            for (int m = 0; m < rp; ++m) base[lds_pad(o0 + m * Lp) * stride] = v[b * rp + m];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < E / r; ++b) {
#pragma unroll
            for (int m = 0; m < r; ++m) v[b * r + m] = base[lds_pad(t + b * NT + m * (N / r)) * stride];
        }
        pass_compute<T, N, EMAX, S, I>(v, t, tw);
    });
    {
        constexpr int r = Sh::P.r[NP - 1];
        constexpr int Ls = plan_ls(Sh::P, NP - 1);
        static_assert(Ls * r == N, "schedule");
#pragma unroll
        for (int b = 0; b < E / r; ++b) {
#pragma unroll
            for (int m = 0; m < r; ++m) st(t + b * NT + m * Ls, v[b * r + m]);
        }
    }
}

// The same transform with the LDS exchange done in two halves, real parts then imaginary
// parts, through a T (not cx<T>) scratch of lds_len(N) slots per transform: half the LDS,
// two more barriers per exchange.
template <typename T, int N, int EMAX, int S, class Ld, class St>
__device__ __forceinline__ void fft_run_split(int t, T* base, int stride, const cx<T>* __restrict__ tw, Ld&& ld,
                                              St&& st) {
    using Sh = FftShape<N, EMAX>;
    constexpr int E = Sh::E;
    constexpr int NT = Sh::NT;
    constexpr int NP = Sh::NP;
    cx<T> v[E];
    {
        constexpr int r = Sh::P.r[0];
#pragma unroll
        for (int b = 0; b < E / r; ++b) {
#pragma unroll
            for (int m = 0; m < r; ++m) v[b * r + m] = ld(t + b * NT + m * (N / r));
        }
    }
    pass_compute<T, N, EMAX, S, 0>(v, t, tw);
    static_for<1, NP>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr int rp = Sh::P.r[I - 1];
        constexpr int Lp = plan_ls(Sh::P, I - 1);
        constexpr int r = Sh::P.r[I];
        // half q = 0: real parts, q = 1: imaginary parts; each value is read back into the
        // same component it came from, the other component still holding the old order
        static_for<0, 2>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            __syncthreads();
#pragma unroll
            for (int b = 0; b < E / rp; ++b) {
                const int j = t + b * NT;
                const int k = j % Lp;
                const int o0 = (j - k) * rp + k;
#pragma unroll
                for (int m = 0; m < rp; ++m) base[lds_pad(o0 + m * Lp) * stride] = q == 0 ? v[b * rp + m].x : v[b * rp + m].y;
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < E / r; ++b) {
#pragma unroll
                for (int m = 0; m < r; ++m) {
                    const T x = base[lds_pad(t + b * NT + m * (N / r)) * stride];
                    if (q == 0)
                        v[b * r + m].x = x;
                    else
                        v[b * r + m].y = x;
                }
            }
        });
        pass_compute<T, N, EMAX, S, I>(v, t, tw);
    });
    {
        constexpr int r = Sh::P.r[NP - 1];
        constexpr int Ls = plan_ls(Sh::P, NP - 1);
        static_assert(Ls * r == N, "schedule");
#pragma unroll
        for (int b = 0; b < E / r; ++b) {
#pragma unroll
            for (int m = 0; m < r; ++m) st(t + b * NT + m * Ls, v[b * r + m]);
        }
    }
}

}  // namespace ps
