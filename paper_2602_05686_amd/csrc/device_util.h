// Device-side helpers: wave64 / block reductions with a fixed combination
// order (run-to-run deterministic), last-block finalisation of FP64 sums.
#pragma once

#include "common.h"
#include "kernels.h"

namespace matamg {

__device__ __forceinline__ double wave_sum(double v) {
    // lane 0 ends with the sum; the combination tree depends only on lane ids
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_sumf(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// sum over a 256-thread block, result valid on thread 0; sh: >= 4 doubles
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        t = sh[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    }
    __syncthreads();
    return t;
}

// Store this block's partial; the last block to arrive sums all partials in
// index order (fixed tree for a fixed grid) and writes *result.
__device__ __forceinline__ void finalize_sum(double block_total, const DotTarget& dt, double* sh) {
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        dt.partial[blockIdx.x] = block_total;
        __threadfence();
        unsigned t = atomicAdd(dt.counter, 1u);
        s_last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (s_last) {
        __threadfence();
        double v = 0.0;
        for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x)
            v += __hip_atomic_load(dt.partial + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = block_sum(v, sh);
        if (threadIdx.x == 0) {
            *dt.result = v;
            __hip_atomic_store(dt.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace matamg
