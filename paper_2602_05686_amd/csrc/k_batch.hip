// Batched solve-path kernels (see batch.h): a block finds its segment by a
// binary search over the launch's segment starts, loads that segment's
// argument record and runs the shared device body with its block index
// within the segment.  Streaming launches keep the XCD-aware block order
// over the whole launch, so each XCD walks one contiguous run of segments.
#include "batch.h"

namespace matamg {
namespace {

// largest j with starts[j] <= gb (starts ascending, starts[0] = 0)
__device__ __forceinline__ int find_segment(const int* starts, int nseg, int gb) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= gb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T, int MODE, bool HAS_DOT, int G>
__global__ __launch_bounds__(kBlock) void k_stream_batch(const SArgs<T>* args, const int* starts, int nseg,
                                                         int total) {
    __shared__ StreamShared<T> S;
    const int gb = xcd_block(total);
    if (gb >= total) return;
    const int j = find_segment(starts, nseg, gb);
    const SArgs<T> a = args[j];
    stream_block<T, MODE, HAS_DOT, G>(a, gb - starts[j], S);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_smooth_first_batch(const SmoothFirstArgs<T>* args, const int* starts,
                                                               int nseg) {
    const int j = find_segment(starts, nseg, blockIdx.x);
    const SmoothFirstArgs<T> a = args[j];
    smooth_first_body(a, blockIdx.x - starts[j], starts[j + 1] - starts[j]);
}

__global__ __launch_bounds__(kBlock) void k_cg_direction_batch(const CgDirArgs* args, const int* starts, int nseg) {
    const int j = find_segment(starts, nseg, blockIdx.x);
    const CgDirArgs a = args[j];
    cg_direction_body(a, blockIdx.x - starts[j], starts[j + 1] - starts[j]);
}

__global__ __launch_bounds__(kBlock) void k_cg_update_batch(const CgUpdArgs* args, const int* starts, int nseg) {
    __shared__ double sh[kBlock / 64];
    const int j = find_segment(starts, nseg, blockIdx.x);
    const CgUpdArgs a = args[j];
    cg_update_body(a, blockIdx.x - starts[j], starts[j + 1] - starts[j], sh);
}

__global__ __launch_bounds__(kFinishThreads) void k_finish_batch(const FinishArgs* args) {
    __shared__ double sh[kFinishThreads / 64];
    const FinishArgs a = args[blockIdx.x];
    finish_body(a, sh);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gemv_batch(const GemvArgs<T>* args, const int* starts, int nseg) {
    const int j = find_segment(starts, nseg, blockIdx.x);
    const GemvArgs<T> a = args[j];
    gemv_body(a, blockIdx.x - starts[j]);
}

template <typename T, int MODE, bool HAS_DOT>
void stream_batch_t(int group, const SArgs<T>* args, const int* starts, int nseg, int total, hipStream_t s) {
    if (group == 1)
        hipLaunchKernelGGL((k_stream_batch<T, MODE, HAS_DOT, 1>), dim3(xcd_grid(total)), dim3(kBlock), 0, s, args,
                           starts, nseg, total);
    else
        hipLaunchKernelGGL((k_stream_batch<T, MODE, HAS_DOT, 8>), dim3(xcd_grid(total)), dim3(kBlock), 0, s, args,
                           starts, nseg, total);
    MATAMG_LAUNCH_CHECK();
}
}  // namespace

template <typename T>
void stream_batch(int mode, bool has_dot, int group, const SArgs<T>* args, const int* starts, int nseg, int total,
                  hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    if (group != 1 && group != 8) fail(AMG_ERR_INVALID_ARG, "batched SpMV: group must be 1 or 8");
    switch (mode) {
        case M_PLAIN: return stream_batch_t<T, M_PLAIN, false>(group, args, starts, nseg, total, s);
        case M_RESID: return stream_batch_t<T, M_RESID, false>(group, args, starts, nseg, total, s);
        case M_ADD: return stream_batch_t<T, M_ADD, false>(group, args, starts, nseg, total, s);
        case M_SMOOTH:
            if (has_dot) return stream_batch_t<T, M_SMOOTH, true>(group, args, starts, nseg, total, s);
            return stream_batch_t<T, M_SMOOTH, false>(group, args, starts, nseg, total, s);
        case M_DOTPQ: return stream_batch_t<T, M_DOTPQ, true>(group, args, starts, nseg, total, s);
        case M_RESNORM: return stream_batch_t<T, M_RESNORM, true>(group, args, starts, nseg, total, s);
        default: fail(AMG_ERR_INVALID_ARG, "batched SpMV: unsupported mode");
    }
}
template void stream_batch<float>(int, bool, int, const SArgs<float>*, const int*, int, int, hipStream_t);
template void stream_batch<double>(int, bool, int, const SArgs<double>*, const int*, int, int, hipStream_t);

template <typename T>
void smooth_first_batch(const SmoothFirstArgs<T>* args, const int* starts, int nseg, int total, hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    hipLaunchKernelGGL(k_smooth_first_batch<T>, dim3(total), dim3(kBlock), 0, s, args, starts, nseg);
    MATAMG_LAUNCH_CHECK();
}
template void smooth_first_batch<float>(const SmoothFirstArgs<float>*, const int*, int, int, hipStream_t);
template void smooth_first_batch<double>(const SmoothFirstArgs<double>*, const int*, int, int, hipStream_t);

void cg_direction_batch(const CgDirArgs* args, const int* starts, int nseg, int total, hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    hipLaunchKernelGGL(k_cg_direction_batch, dim3(total), dim3(kBlock), 0, s, args, starts, nseg);
    MATAMG_LAUNCH_CHECK();
}

void cg_update_batch(const CgUpdArgs* args, const int* starts, int nseg, int total, hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    hipLaunchKernelGGL(k_cg_update_batch, dim3(total), dim3(kBlock), 0, s, args, starts, nseg);
    MATAMG_LAUNCH_CHECK();
}

void finish_batch(const FinishArgs* args, int nseg, hipStream_t s) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_finish_batch, dim3(nseg), dim3(kFinishThreads), 0, s, args);
    MATAMG_LAUNCH_CHECK();
}

template <typename T>
void gemv_batch(const GemvArgs<T>* args, const int* starts, int nseg, int total, hipStream_t s) {
    if (nseg <= 0 || total <= 0) return;
    hipLaunchKernelGGL(k_gemv_batch<T>, dim3(total), dim3(kBlock), 0, s, args, starts, nseg);
    MATAMG_LAUNCH_CHECK();
}
template void gemv_batch<float>(const GemvArgs<float>*, const int*, int, int, hipStream_t);
template void gemv_batch<double>(const GemvArgs<double>*, const int*, int, int, hipStream_t);

}  // namespace matamg
