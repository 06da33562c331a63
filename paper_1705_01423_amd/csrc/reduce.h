// Deterministic block reductions (fixed order for a fixed launch shape).
#pragma once

#include <hip/hip_runtime.h>

namespace ps {

// Sums NC values over the block; thread 0 writes them to out[0..NC).
// Every thread of the block must call it.
template <int NC>
__device__ __forceinline__ void block_sum_store(double (&v)[NC], double* out) {
    __shared__ double red[NC][16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] += __shfl_down(v[c], off, 64);
    }
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) red[c][wid] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[c][w];
            out[c] = s;
        }
    }
}

}  // namespace ps
