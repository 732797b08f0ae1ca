// Row-block partition of a CSR matrix for the streaming kernels, computed on
// the device.
//
// The partition is the greedy one: walking the rows in order, a block takes
// rows while it holds fewer than 256/G rows and its stored entries stay
// within kStreamCap; a row longer than long_row_limit(G) forms a block of its
// own.  The walk is sequential, but the block that starts at row r ends at a
// row next(r) that depends on r alone, so every next(r) is computed in
// parallel (binary searches over the row pointer and the list of long rows)
// and the block starts -- the orbit of row 0 under next -- are marked by
// pointer doubling: after round k every start within 2^(k+1) blocks of row 0
// is marked.  The result equals the host walk exactly.
#include "device_util.h"
#include "kernels.h"

namespace matamg {
namespace {

inline int grid1(int64_t n) {
    int g = ceil_div(n > 0 ? n : 1, kBlock);
    return g < 65535 ? g : 65535;
}

#define FOR_ROWS(i, n) for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kBlock)

__global__ void k_max_row_len(int n, const int* rp, int* out) {
    int m = 0;
    FOR_ROWS(i, n) m = max(m, rp[i + 1] - rp[i]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

__global__ void k_long_flags(int n, const int* rp, int limit, int* flags) {
    FOR_ROWS(i, n) flags[i] = (rp[i + 1] - rp[i] > limit) ? 1 : 0;
}

__global__ void k_long_list(int n, const int* flags, const int* pos, int* list) {
    FOR_ROWS(i, n) if (flags[i]) list[pos[i]] = (int)i;
}

// end (exclusive) of the block that starts at row r; next[n] = n
__global__ void k_block_next(int n, const int* rp, int limit, int max_rows, const int* longs, const int* nlong,
                             int* next) {
    const int nl = *nlong;
    FOR_ROWS(r64, (int64_t)n + 1) {
        const int r = (int)r64;
        if (r == n) {
            next[r] = n;
            continue;
        }
        if (rp[r + 1] - rp[r] > limit) {
            next[r] = r + 1;
            continue;
        }
        int e = min(n, r + max_rows);
        // largest j in (r, e] with rp[j] - rp[r] <= kStreamCap (j = r + 1 always qualifies)
        const int cap = rp[r] + kStreamCap;
        int lo = r + 1, hi = e;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= cap) lo = mid;
            else hi = mid - 1;
        }
        e = lo;
        // first long row after r
        int a = 0, b = nl;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (longs[mid] <= r) a = mid + 1;
            else b = mid;
        }
        if (a < nl && longs[a] < e) e = longs[a];
        next[r] = e;
    }
}

__global__ void k_mark_start(int* mark) { mark[0] = 1; }

__global__ void k_mark_jump(int n, const int* jump, int* mark) {
    FOR_ROWS(p, (int64_t)n + 1) if (mark[p]) mark[jump[p]] = 1;
}

__global__ void k_jump_square(int n, const int* jump, int* out) {
    FOR_ROWS(p, (int64_t)n + 1) out[p] = jump[jump[p]];
}

__global__ void k_fill_starts(int n, const int* mark, const int* pos, int* blk) {
    FOR_ROWS(i, n) if (mark[i]) blk[pos[i]] = (int)i;
    if (blockIdx.x == 0 && threadIdx.x == 0) blk[pos[n]] = n;
}

}  // namespace

void stream_partition(DCsr& A, MemCounter* mc, hipStream_t s) {
    const int n = A.n;
    if (n <= 0) {
        A.group = 1;
        A.nblk = 0;
        A.blk.alloc(1, mc);
        MATAMG_HIP(hipMemsetAsync(A.blk.get(), 0, sizeof(int), s));
        MATAMG_HIP(hipStreamSynchronize(s));
        return;
    }
    const int* rp = A.rowptr.get();
    DBuf<int> one(2, mc);
    MATAMG_HIP(hipMemsetAsync(one.get(), 0, 2 * sizeof(int), s));
    hipLaunchKernelGGL(k_max_row_len, dim3(grid1(n)), dim3(kBlock), 0, s, n, rp, one.get());
    MATAMG_LAUNCH_CHECK();
    int max_len = 0;
    d2h(&max_len, one.get(), 1, s);
    A.group = stream_group(max_len);
    const int limit = long_row_limit(A.group);
    const int max_rows = max_block_rows(A.group);

    const size_t n1 = (size_t)n + 1;
    DBuf<int> flags(n1, mc), pos(n1, mc), tmp(scan_tmp_size(n1), mc), longs(n1, mc);
    hipLaunchKernelGGL(k_long_flags, dim3(grid1(n)), dim3(kBlock), 0, s, n, rp, limit, flags.get());
    exclusive_scan(flags.get(), pos.get(), n, tmp.get(), s);
    hipLaunchKernelGGL(k_long_list, dim3(grid1(n)), dim3(kBlock), 0, s, n, flags.get(), pos.get(), longs.get());
    DBuf<int> ja(n1, mc), jb(n1, mc);
    hipLaunchKernelGGL(k_block_next, dim3(grid1(n1)), dim3(kBlock), 0, s, n, rp, limit, max_rows, longs.get(),
                       pos.get() + n, ja.get());
    MATAMG_LAUNCH_CHECK();
    // pointer doubling from row 0 (flags reused as the start marks)
    MATAMG_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int) * n1, s));
    hipLaunchKernelGGL(k_mark_start, dim3(1), dim3(1), 0, s, flags.get());
    int* cur = ja.get();
    int* nxt = jb.get();
    for (int64_t span = 1; span <= (int64_t)n; span <<= 1) {
        hipLaunchKernelGGL(k_mark_jump, dim3(grid1(n1)), dim3(kBlock), 0, s, n, (const int*)cur, flags.get());
        if ((span << 1) <= (int64_t)n) {
            hipLaunchKernelGGL(k_jump_square, dim3(grid1(n1)), dim3(kBlock), 0, s, n, (const int*)cur, nxt);
            std::swap(cur, nxt);
        }
    }
    MATAMG_LAUNCH_CHECK();
    exclusive_scan(flags.get(), pos.get(), n, tmp.get(), s);
    int nblk = 0;
    d2h(&nblk, pos.get() + n, 1, s);
    A.nblk = nblk;
    A.blk.alloc((size_t)nblk + 1, mc);
    hipLaunchKernelGGL(k_fill_starts, dim3(grid1(n)), dim3(kBlock), 0, s, n, (const int*)flags.get(),
                       (const int*)pos.get(), A.blk.get());
    MATAMG_LAUNCH_CHECK();
    MATAMG_HIP(hipStreamSynchronize(s));
}

}  // namespace matamg
