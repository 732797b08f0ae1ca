// Solve-path kernels: streaming CSR SpMV with fused smoother / residual /
// transfer epilogues, deterministic FP64 reductions, CG vector updates,
// dense coarse-level GEMV, and the integer prefix scan used by setup.
//
// Streaming CSR layout: rows are cut into blocks of at most kStreamCap
// stored entries and kMaxRowsPerBlock rows; a row longer than
// long_row_limit(1) gets a block of its own.  A 256-thread block first
// streams its contiguous val/col range (fully coalesced) and stores
// val*x[col] in LDS, then one thread per row sums its products in ascending
// stored order and applies the epilogue; rows wider than kWideRow are summed
// by 8-lane groups of their thread's wavefront (lane-strided partial sums, a
// fixed butterfly) so that a few wide rows do not hold up the block.  A long
// row is reduced by the whole block: strided partial sums and a fixed tree.
// Every sum therefore has a fixed order for a given matrix: results are
// bitwise reproducible run to run.
#include "solve_device.h"

namespace matamg {

// ===================================================================== scan
namespace {
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ int block_exclusive_scan(int v, int* sh, int* total) {
    // inclusive scan within the wave
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int wave_off = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        if (i < w) wave_off += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return wave_off + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_partials(const int* in, int64_t n, int* sums) {
    __shared__ int sh[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    int tot;
    (void)block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(int* sums, int nb) {
    __shared__ int sh[kBlock / 64];
    int carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        int i = base + threadIdx.x;
        int v = (i < nb) ? sums[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int* in, int* out, int64_t n, const int* sums,
                                                       int nb) {
    __shared__ int sh[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, sh, &tot) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = sums[nb];
}
}  // namespace

// inputs up to this length are scanned by one block of kScanOneThreads threads
constexpr int kScanOneThreads = 1024;
constexpr int64_t kScanOneMax = 1 << 16;

namespace {
// the whole scan in one block: tiles of kScanOneThreads * kScanItems
// consecutive values, each thread kScanItems of them, with a running carry
__global__ __launch_bounds__(kScanOneThreads) void k_scan_one(const int* in, int* out, int64_t n) {
    __shared__ int sh[kScanOneThreads / 64];
    int carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += (int64_t)kScanOneThreads * kScanItems) {
        const int64_t base = t0 + (int64_t)threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t i = base + k;
            v[k] = (i < n) ? in[i] : 0;
            sum += v[k];
        }
        int tot;
        int ex = block_exclusive_scan(sum, sh, &tot) + carry;
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t i = base + k;
            if (i < n) out[i] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_zero_words(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_zero_bytes(uint8_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
}  // namespace

void zero_async(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0 || p == nullptr) return;
    if (((uintptr_t)p & 3u) == 0 && (bytes & 3u) == 0) {
        const int64_t n = (int64_t)(bytes / 4);
        hipLaunchKernelGGL(k_zero_words, dim3(std::min<int64_t>(ceil_div(n, kBlock), 2048)), dim3(kBlock), 0, s,
                           (uint32_t*)p, n);
    } else {
        const int64_t n = (int64_t)bytes;
        hipLaunchKernelGGL(k_zero_bytes, dim3(std::min<int64_t>(ceil_div(n, kBlock), 2048)), dim3(kBlock), 0, s,
                           (uint8_t*)p, n);
    }
    MATAMG_LAUNCH_CHECK();
}

size_t scan_tmp_size(int64_t n) { return (size_t)ceil_div(n > 0 ? n : 1, kScanTile) + 1; }

void exclusive_scan(const int* in, int* out, int64_t n, int* tmp, hipStream_t s) {
    if (n <= 0) {
        zero_async(out, sizeof(int), s);
        return;
    }
    if (n <= kScanOneMax) {
        hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneThreads), 0, s, in, out, n);
        MATAMG_LAUNCH_CHECK();
        return;
    }
    int nb = ceil_div(n, kScanTile);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kBlock), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, s, in, out, n, tmp, nb);
    MATAMG_LAUNCH_CHECK();
}

// ====================================================================== dot
namespace {
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot(const T* a, const T* b, int64_t n, DotTarget dt) {
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        v += (double)a[i] * (double)b[i];
    double t = block_sum(v, sh);
    store_partial(t, dt);
}

__global__ __launch_bounds__(kFinishThreads) void k_finish_sum(FinishArgs a) {
    __shared__ double sh[kFinishThreads / 64];
    finish_body(a, sh);
}
}  // namespace

void finish_sum(const DotTarget& dt, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kFinishThreads), 0, s, FinishArgs{nblocks, dt.partial, dt.result});
    MATAMG_LAUNCH_CHECK();
}

template <typename T>
void dot(const T* a, const T* b, int64_t n, double* partial, unsigned* counter, double* result, hipStream_t s) {
    DotTarget dt{partial, counter, result};
    const int g = vec_grid(n);
    hipLaunchKernelGGL(k_dot<T>, dim3(g), dim3(kBlock), 0, s, a, b, n, dt);
    MATAMG_LAUNCH_CHECK();
    finish_sum(dt, g, s);
}
template void dot<double>(const double*, const double*, int64_t, double*, unsigned*, double*, hipStream_t);
template void dot<float>(const float*, const float*, int64_t, double*, unsigned*, double*, hipStream_t);

// =============================================================== streaming
int stream_group(const int* rp, int n) {
    int max_len = 0;
    int64_t wide = 0;
    for (int i = 0; i < n; ++i) {
        const int len = rp[i + 1] - rp[i];
        max_len = std::max(max_len, len);
        if (len > kWideRow) wide += len;
    }
    return stream_group_rule(max_len, wide, n > 0 ? rp[n] : 0);
}

std::vector<int> stream_blocks(const int* rp, int n, int group, int cap) {
    const int max_rows = max_block_rows(group);
    const int long_len = long_row_limit(group);
    std::vector<int> blk;
    blk.reserve((size_t)n / 32 + 2);
    blk.push_back(0);
    int cur = 0, rows = 0;
    for (int r = 0; r < n; ++r) {
        int len = rp[r + 1] - rp[r];
        if (len > long_len) {
            if (rows > 0) blk.push_back(r);
            blk.push_back(r + 1);
            cur = 0;
            rows = 0;
            continue;
        }
        if (rows > 0 && (cur + len > cap || rows == max_rows)) {
            blk.push_back(r);
            cur = 0;
            rows = 0;
        }
        cur += len;
        rows++;
    }
    if (blk.back() != n) blk.push_back(n);
    return blk;
}

namespace {
template <typename T, int MODE, bool HAS_DOT, int G, int CAP = kStreamCap>
__global__ __launch_bounds__(kBlock) void k_stream(SArgs<T> a, int nblk) {
    __shared__ StreamShared<T, CAP> S;
    const int bid = xcd_block(nblk);
    if (bid >= nblk) return;
    stream_block<T, MODE, HAS_DOT, G, CAP>(a, bid, S);
}

template <typename T, int MODE, bool HAS_DOT>
void launch_stream(const DCsr& A, const SArgs<T>& a, hipStream_t s) {
    if (A.nblk <= 0) return;
    if (A.group == 1 && A.cap == kStreamCapWide)
        hipLaunchKernelGGL((k_stream<T, MODE, HAS_DOT, 1, kStreamCapWide>), dim3(xcd_grid(A.nblk)), dim3(kBlock), 0, s,
                           a, A.nblk);
    else if (A.group == 1)
        hipLaunchKernelGGL((k_stream<T, MODE, HAS_DOT, 1>), dim3(xcd_grid(A.nblk)), dim3(kBlock), 0, s, a, A.nblk);
    else
        hipLaunchKernelGGL((k_stream<T, MODE, HAS_DOT, 8>), dim3(xcd_grid(A.nblk)), dim3(kBlock), 0, s, a, A.nblk);
    MATAMG_LAUNCH_CHECK();
    if constexpr (HAS_DOT) finish_sum(a.dt, stream_partials(A), s);
}

template <typename T>
SArgs<T> base_args(const DCsr& A, const T* val, const T* x) {
    SArgs<T> a{};
    a.rowptr = A.rowptr.get();
    a.col = A.col.get();
    a.col16 = A.col16.get();
    a.cbase = A.cbase.get();
    a.val = val;
    a.blk = A.blk.get();
    a.blkk = A.blkk.get();
    a.ustart = A.ustart.get();
    a.uoff = A.uoff.get();
    a.urun = A.urun.get();
    a.x = x;
    return a;
}
}  // namespace

template <typename T>
void spmv(const DCsr& A, const T* val, const T* x, T* y, hipStream_t s) {
    auto a = base_args<T>(A, val, x);
    a.y = y;
    launch_stream<T, M_PLAIN, false>(A, a, s);
}

template <typename T>
void spmv_resid(const DCsr& A, const T* val, const T* x, const T* b, T* y, hipStream_t s) {
    auto a = base_args<T>(A, val, x);
    a.b = b;
    a.y = y;
    launch_stream<T, M_RESID, false>(A, a, s);
}

template <typename T>
void spmv_add(const DCsr& A, const T* val, const T* x, const T* y_in, T* y, hipStream_t s) {
    auto a = base_args<T>(A, val, x);
    a.yin = y_in;
    a.y = y;
    launch_stream<T, M_ADD, false>(A, a, s);
}

template <typename T>
void spmv_smooth(const DCsr& A, const T* val, const T* x, const T* b, const T* dinv, T* d, T c1, T c2, T* out,
                 double* out64, const double* dotvec, DotTarget dt, hipStream_t s) {
    auto a = base_args<T>(A, val, x);
    a.b = b;
    a.yin = x;
    a.dinv = dinv;
    a.d = d;
    a.c1 = c1;
    a.c2 = c2;
    a.y = out;
    a.y64 = out64;
    a.dotvec = dotvec;
    a.dt = dt;
    if (dotvec) launch_stream<T, M_SMOOTH, true>(A, a, s);
    else launch_stream<T, M_SMOOTH, false>(A, a, s);
}

template <typename T>
void spmv_restrict_first(const DCsr& R, const T* val, const T* r, T* bc, const T* dinv_c, T c2, T* d_c, T* x_c,
                         hipStream_t s) {
    auto a = base_args<T>(R, val, r);
    a.y = bc;
    a.dinv = dinv_c;
    a.c2 = c2;
    a.d = d_c;
    a.xo = x_c;
    launch_stream<T, M_RESTRICT, false>(R, a, s);
}

void spmv_dot(const DCsr& A, const double* p, double* q, DotTarget dt, hipStream_t s) {
    auto a = base_args<double>(A, A.val.get(), p);
    a.y = q;
    a.dt = dt;
    launch_stream<double, M_DOTPQ, true>(A, a, s);
}

void spmv_resid_norm(const DCsr& A, const double* x, const double* b, double* y, DotTarget dt, hipStream_t s) {
    auto a = base_args<double>(A, A.val.get(), x);
    a.b = b;
    a.y = y;
    a.dt = dt;
    launch_stream<double, M_RESNORM, true>(A, a, s);
}

void spmv_scale_norm(const DCsr& A, const double* x, const double* dscale, double* y, DotTarget dt,
                     hipStream_t s) {
    auto a = base_args<double>(A, A.val.get(), x);
    a.dinv = dscale;
    a.y = y;
    a.dt = dt;
    launch_stream<double, M_SCALENORM, true>(A, a, s);
}

#define INST(T)                                                                                        \
    template void spmv<T>(const DCsr&, const T*, const T*, T*, hipStream_t);                          \
    template void spmv_resid<T>(const DCsr&, const T*, const T*, const T*, T*, hipStream_t);          \
    template void spmv_add<T>(const DCsr&, const T*, const T*, const T*, T*, hipStream_t);            \
    template void spmv_smooth<T>(const DCsr&, const T*, const T*, const T*, const T*, T*, T, T, T*,   \
                                 double*, const double*, DotTarget, hipStream_t);                      \
    template void spmv_restrict_first<T>(const DCsr&, const T*, const T*, T*, const T*, T, T*, T*,    \
                                         hipStream_t);
INST(double)
INST(float)
#undef INST

// ================================================================= vectors
namespace {
template <typename T>
__global__ __launch_bounds__(kBlock) void k_smooth_first(SmoothFirstArgs<T> a) {
    smooth_first_body(a, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_scale_inv_norm(int64_t n, const double* nrm2, const double* in,
                                                           double* out) {
    const double inv = 1.0 / sqrt(*nrm2);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = in[i] * inv;
}

__global__ __launch_bounds__(kBlock) void k_cg_update(CgUpdArgs a) {
    __shared__ double sh[kBlock / 64];
    cg_update_body(a, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(kBlock) void k_cg_direction(CgDirArgs a) {
    cg_direction_body(a, blockIdx.x, gridDim.x);
}

template <typename A, typename B>
__global__ __launch_bounds__(kBlock) void k_cast(int64_t n, const A* in, B* out) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = (B)in[i];
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_seeded_uniform(int64_t n, uint64_t key, double* v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        uint64_t h = splitmix64(key ^ (uint64_t)i);
        double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
        v[i] = 2.0 * u - 1.0;
    }
}
}  // namespace

template <typename T>
void smooth_first(int64_t n, const double* b64, T* b, const T* dinv, T c2, T* d, T* x, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_smooth_first<T>, dim3(vec_grid(n)), dim3(kBlock), 0, s,
                       SmoothFirstArgs<T>{n, b64, b, dinv, c2, d, x});
    MATAMG_LAUNCH_CHECK();
}
template void smooth_first<double>(int64_t, const double*, double*, const double*, double, double*, double*,
                                   hipStream_t);
template void smooth_first<float>(int64_t, const double*, float*, const float*, float, float*, float*,
                                  hipStream_t);

void scale_by_inv_norm(int64_t n, const double* nrm2, const double* in, double* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_inv_norm, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, nrm2, in, out);
    MATAMG_LAUNCH_CHECK();
}

void cg_update(int64_t n, double* x, double* r, const double* p, const double* q, const double* rz,
               const double* pq, DotTarget rr, hipStream_t s) {
    const int g = vec_grid(n);
    hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(kBlock), 0, s, CgUpdArgs{n, x, r, p, q, rz, pq, rr.partial});
    MATAMG_LAUNCH_CHECK();
    finish_sum(rr, g, s);
}

void cg_direction(int64_t n, double* p, const double* z, const double* rz_new, const double* rz_old,
                  hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cg_direction, dim3(vec_grid(n)), dim3(kBlock), 0, s, CgDirArgs{n, p, z, rz_new, rz_old});
    MATAMG_LAUNCH_CHECK();
}

template <typename A, typename B>
void cast_vec(int64_t n, const A* in, B* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_cast<A, B>), dim3(vec_grid(n)), dim3(kBlock), 0, s, n, in, out);
    MATAMG_LAUNCH_CHECK();
}
template void cast_vec<double, float>(int64_t, const double*, float*, hipStream_t);
template void cast_vec<float, double>(int64_t, const float*, double*, hipStream_t);

void fill_seeded_uniform(int64_t n, uint64_t key, double* v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_seeded_uniform, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, key, v);
    MATAMG_LAUNCH_CHECK();
}

// =================================================================== dense
namespace {
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(GemvArgs<T> a) {
    gemv_body(a, blockIdx.x);
}
}  // namespace

template <typename T>
void dense_gemv(int n, const double* M, const T* in, T* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_dense_gemv<T>, dim3(gemv_grid(n)), dim3(kBlock), 0, s, GemvArgs<T>{n, M, in, out});
    MATAMG_LAUNCH_CHECK();
}
template void dense_gemv<double>(int, const double*, const double*, double*, hipStream_t);
template void dense_gemv<float>(int, const double*, const float*, float*, hipStream_t);

}  // namespace matamg
