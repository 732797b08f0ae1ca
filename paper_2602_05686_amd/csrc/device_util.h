// Device-side helpers: wave64 / block reductions with a fixed combination
// order (run-to-run deterministic), last-block finalisation of FP64 sums.
#pragma once

#include "common.h"
#include "kernels.h"

namespace matamg {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup g runs on
// XCD g % 8).  Remapping so that each XCD walks one contiguous eighth of the
// row blocks keeps the gathered neighbours of consecutive blocks in that
// XCD's L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int nblk) {
    const int per = (nblk + kXcds - 1) / kXcds;
    return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}
inline int xcd_grid(int nblk) { return ((nblk + kXcds - 1) / kXcds) * kXcds; }

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

// Store this block's partial sum (valid on thread 0).  A second, one-block
// kernel (finish_sum) adds the partials in index order; the kernel boundary
// makes them visible without device-scope fences, and the order is fixed
// for a fixed grid.
__device__ __forceinline__ void store_partial(double block_total, const DotTarget& dt) {
    if (threadIdx.x == 0) dt.partial[blockIdx.x] = block_total;
}

}  // namespace matamg
