// Row-block partition of a CSR matrix for the streaming kernels, computed on
// the device.
//
// The partition is the greedy one: walking the rows in order, a block takes
// rows while it holds fewer than max_block_rows(G) rows and its stored
// entries stay within the cap (kStreamCap, or kStreamCapWide); a row longer
// than long_row_limit(G) forms a
// block of its own.  The walk is sequential, but the block that starts at row r ends at a
// row next(r) that depends on r alone, so every next(r) is computed in
// parallel (binary searches over the row pointer and the list of long rows)
// and the block starts -- the orbit of row 0 under next -- are marked by
// radix-8 pointer jumping: after round k every start within 8^(k+1) blocks
// of row 0 is marked.  The result equals the host walk exactly.
#include <algorithm>

#include "device_util.h"
#include "kernels.h"

namespace matamg {
namespace {

inline int grid1(int64_t n) {
    int g = ceil_div(n > 0 ? n : 1, kBlock);
    return g < 65535 ? g : 65535;
}

#define FOR_ROWS(i, n) for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kBlock)

// longest row (out[0]) and the entries in rows wider than kWideRow (out[6]);
// launched with a small grid so that few blocks meet at the atomics (both
// results are order-independent)
__global__ __launch_bounds__(kBlock) void k_max_row_len(int n, const int* rp, int* out) {
    __shared__ int sm[kBlock / 64], sw[kBlock / 64];
    int m = 0, w = 0;
    FOR_ROWS(i, n) {
        const int len = rp[i + 1] - rp[i];
        m = max(m, len);
        if (len > kWideRow) w += len;
    }
    for (int off = 32; off > 0; off >>= 1) {
        m = max(m, __shfl_xor(m, off, 64));
        w += __shfl_xor(w, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = m;
        sw[threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; ++k) {
            m = max(m, sm[k]);
            w += sw[k];
        }
        if (m > 0) atomicMax(out, m);
        if (w > 0) atomicAdd(out + 6, w);
    }
}

// par[0] = longest row, par[6] = entries in wide rows -> par[1] = threads per
// row, par[2] = long-row limit, par[3] = most rows per block (the host's
// stream_group rule)
__global__ void k_group_params(int n, const int* rp, int* par) {
    const int group = stream_group_rule(par[0], par[6], rp[n]);
    par[1] = group;
    par[2] = long_row_limit(group);
    par[3] = max_block_rows(group);
}

__global__ void k_long_flags(int n, const int* rp, const int* par, int* flags) {
    const int limit = par[2];
    FOR_ROWS(i, n) flags[i] = (rp[i + 1] - rp[i] > limit) ? 1 : 0;
}

__global__ void k_long_list(int n, const int* flags, const int* pos, int* list) {
    FOR_ROWS(i, n) if (flags[i]) list[pos[i]] = (int)i;
}

// end (exclusive) of the block that starts at row r; next[n] = n
__global__ void k_block_next(int n, const int* rp, const int* par, const int* longs, const int* nlong, int bcap,
                             int* next) {
    const int nl = *nlong;
    const int limit = par[2], max_rows = par[3];
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
        // largest j in (r, e] with rp[j] - rp[r] <= bcap (j = r + 1 always qualifies)
        const int cap = rp[r] + bcap;
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

// mark[p] = (p == 0): row 0 starts the first block
__global__ void k_mark_init(int n, int* mark) {
    FOR_ROWS(p, (int64_t)n + 1) mark[p] = (p == 0) ? 1 : 0;
}

// One round of radix-8 doubling with jump = J: every marked start p marks
// J(p), J^2(p), ..., J^7(p), and (if out is set) out = J^8.  A mark set by
// another thread of the same round may be seen early; that only marks a
// true start sooner (marks are only ever set on the orbit of row 0), so
// after the round at least the starts within eight times the span are
// marked, as with the rounds apart.
__global__ void k_mark_pow8(int n, const int* jump, int* mark, int* out) {
    FOR_ROWS(p, (int64_t)n + 1) {
        const bool mk = mark[p] != 0;
        int q = (int)p;
        for (int t = 1; t < 8; ++t) {
            q = jump[q];
            if (mk) mark[q] = 1;
        }
        if (out) out[p] = jump[q];
    }
}

// out[0] = number of blocks, out[1] = threads per row
__global__ void k_partition_result(int n, const int* pos, const int* par, int* out) {
    out[0] = pos[n];
    out[1] = par[1];
}

__global__ void k_fill_starts(int n, const int* mark, const int* pos, int* blk) {
    FOR_ROWS(i, n) if (mark[i]) blk[pos[i]] = (int)i;
    if (blockIdx.x == 0 && threadIdx.x == 0) blk[pos[n]] = n;
}

// cbase[b] = smallest column of block b; flag = 1 if a block's columns span
// 2^16 values or more (the block count *nblk_dev is read on the device)
__global__ __launch_bounds__(kBlock) void k_block_col_range(const int* nblk_dev, const int* rp, const int* col,
                                                            const int* blk, int* cbase, int* flag) {
    __shared__ int smin[kBlock / 64], smax[kBlock / 64];
    const int nblk = *nblk_dev;
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int k0 = rp[blk[b]], k1 = rp[blk[b + 1]];
        int lo = 0x7fffffff, hi = -1;
        for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) {
            const int c = col[k];
            lo = min(lo, c);
            hi = max(hi, c);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off, 64));
            hi = max(hi, __shfl_xor(hi, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            smin[threadIdx.x >> 6] = lo;
            smax[threadIdx.x >> 6] = hi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kBlock / 64; ++w) {
                lo = min(lo, smin[w]);
                hi = max(hi, smax[w]);
            }
            cbase[b] = k1 > k0 ? lo : 0;
            if (k1 > k0 && hi - lo > 0xffff) *flag = 1;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_pack_cols(int nblk, const int* rp, const int* col, const int* blk,
                                                      const int* cbase, uint16_t* col16) {
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int k0 = rp[blk[b]], k1 = rp[blk[b + 1]], base = cbase[b];
        for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) col16[k] = (uint16_t)(col[k] - base);
    }
}

// Distinct packed columns of a block: a bitmap over the 2^16 offsets a
// packed block can hold (2048 words in LDS), set by the block's entries.
constexpr int kColWords = 65536 / 32;

__device__ __forceinline__ bool long_row_block(int r0, int r1, int k0, int k1, int group) {
    return r1 - r0 == 1 && k1 - k0 > long_row_limit(group);
}

__device__ __forceinline__ void mark_columns(unsigned* bits, const uint16_t* col16, int k0, int k1) {
    for (int w = threadIdx.x; w < kColWords; w += kBlock) bits[w] = 0u;
    __syncthreads();
    for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) {
        const unsigned c = col16[k];
        atomicOr(&bits[c >> 5], 1u << (c & 31u));
    }
    __syncthreads();
}

// exclusive prefix over the block's threads of v (block-wide, 256 threads);
// *total receives the sum
__device__ __forceinline__ int block_exclusive(int v, int* red, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) red[wv] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < wv) woff += red[i];
        tot += red[i];
    }
    __syncthreads();
    *total = tot;
    return woff + incl - v;
}

// Per block b: the number of distinct columns and of runs of consecutive
// columns among them.  A block is staged when it is not one long row, has
// at most ucap distinct columns and at most kUniqueReusePct percent as many
// as entries (too little reuse does not pay for the staging).  A staged
// block with at most kMaxRuns runs gets its run record (urun); any other
// staged block a list of ucnt[b] = its distinct count (0 otherwise).
__global__ __launch_bounds__(kBlock) void k_block_uniques_count(int nblk, const int* blk, const int* blkk,
                                                                const uint16_t* col16, int group, int ucap,
                                                                int* ucnt, uint32_t* urun, int* nstaged) {
    __shared__ unsigned bits[kColWords];
    __shared__ int red[kBlock / 64];
    __shared__ int rs[kMaxRuns], re[kMaxRuns];
    constexpr int kPer = kColWords / kBlock;  // words per thread, contiguous
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int r0 = blk[b], r1 = blk[b + 1], k0 = blkk[b], k1 = blkk[b + 1];
        const bool skip = long_row_block(r0, r1, k0, k1, group);
        mark_columns(bits, col16, k0, skip ? k0 : k1);
        int c = 0, ns = 0, ne = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int w = threadIdx.x * kPer + i;
            const unsigned m = bits[w];
            const unsigned prev = w > 0 ? bits[w - 1] >> 31 : 0u;
            const unsigned next = w + 1 < kColWords ? (bits[w + 1] & 1u) << 31 : 0u;
            c += __popc(m);
            ns += __popc(m & ~((m << 1) | prev));
            ne += __popc(m & ~((m >> 1) | next));
        }
        int total = 0, runs = 0, tmp = 0;
        (void)block_exclusive(c, red, &total);
        const int s0 = block_exclusive(ns, red, &runs);
        const int e0 = block_exclusive(ne, red, &tmp);
        const bool staged = !skip && total <= ucap && total * 100 <= kUniqueReusePct * (k1 - k0) && total > 0;
        const bool use_runs = staged && runs <= kMaxRuns;
        if (use_runs) {
            // the run starts and ends in column order (threads own contiguous words)
            int si = s0, ei = e0;
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int w = threadIdx.x * kPer + i;
                const unsigned m = bits[w];
                const unsigned prev = w > 0 ? bits[w - 1] >> 31 : 0u;
                const unsigned next = w + 1 < kColWords ? (bits[w + 1] & 1u) << 31 : 0u;
                unsigned st = m & ~((m << 1) | prev), en = m & ~((m >> 1) | next);
                while (st) {
                    rs[si++] = w * 32 + __builtin_ctz(st);
                    st &= st - 1u;
                }
                while (en) {
                    re[ei++] = w * 32 + __builtin_ctz(en);
                    en &= en - 1u;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < kRunWords) {
            uint32_t word = 0u;
            if (use_runs) {
                const int t = (int)threadIdx.x;
                if (t == 0) word = (uint32_t)runs;
                else if (t == 1) word = (uint32_t)total;
                else if (t - 2 < runs) word = (uint32_t)rs[t - 2] | ((uint32_t)(re[t - 2] - rs[t - 2] + 1) << 16);
            }
            urun[(size_t)b * kRunWords + threadIdx.x] = word;
        }
        if (threadIdx.x == 0) {
            ucnt[b] = (staged && !use_runs) ? total : 0;
            if (staged) atomicAdd(nstaged, 1);
        }
        __syncthreads();
    }
}

// the lists (ascending offsets) and every staged entry's index into its
// block's distinct columns (list or runs: the same ascending order)
__global__ __launch_bounds__(kBlock) void k_block_uniques_fill(int nblk, const int* blkk, const int* ustart,
                                                               const uint32_t* urun, uint16_t* col16,
                                                               uint16_t* uoff) {
    __shared__ unsigned bits[kColWords];
    __shared__ int wpre[kColWords];
    __shared__ int red[kBlock / 64];
    constexpr int kPer = kColWords / kBlock;  // words per thread
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int u0 = ustart[b];
        const bool list = ustart[b + 1] > u0;
        if (!list && urun[(size_t)b * kRunWords] == 0u) continue;  // block-uniform: not staged
        const int k0 = blkk[b], k1 = blkk[b + 1];
        mark_columns(bits, col16, k0, k1);
        // exclusive prefix of the set-bit counts over the words, thread t
        // owning words [t kPer, (t + 1) kPer)
        int loc[kPer];
        int sum = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            loc[i] = sum;
            sum += __popc(bits[threadIdx.x * kPer + i]);
        }
        int tot = 0;
        const int base = block_exclusive(sum, red, &tot);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int w = threadIdx.x * kPer + i;
            wpre[w] = base + loc[i];
            if (list) {
                unsigned m = bits[w];
                int r = base + loc[i];
                while (m) {
                    uoff[u0 + r] = (uint16_t)(w * 32 + __builtin_ctz(m));
                    ++r;
                    m &= m - 1u;
                }
            }
        }
        __syncthreads();
        for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) {
            const unsigned c = col16[k];
            const unsigned m = bits[c >> 5] & ((1u << (c & 31u)) - 1u);
            col16[k] = (uint16_t)(wpre[c >> 5] + __popc(m));
        }
        __syncthreads();
    }
}

// blkk[b] = rp[blk[b]] for b <= nblk
__global__ void k_block_entries(int nblk, const int* rp, const int* blk, int* blkk) {
    FOR_ROWS(b, (int64_t)nblk + 1) blkk[b] = rp[blk[b]];
}

}  // namespace

void stream_partition(DCsr& A, MemCounter* mc, hipStream_t s, bool pack, int cap) {
    const int n = A.n;
    A.col16.release();
    A.cbase.release();
    A.ustart.release();
    A.uoff.release();
    A.urun.release();
    A.nuniq = 0;
    A.sblk.release();
    A.snblk = 0;
    A.cap = cap;
    if (n <= 0) {
        A.group = 1;
        A.nblk = 0;
        A.blk.alloc(1, mc);
        A.blkk.alloc(1, mc);
        zero_async(A.blk.get(), sizeof(int), s);
        zero_async(A.blkk.get(), sizeof(int), s);
        MATAMG_HIP(hipStreamSynchronize(s));
        return;
    }
    const int* rp = A.rowptr.get();
    // threads per row from the longest row, decided on the device: the
    // only read-back is the block count at the end
    DBuf<int> par(8, mc);
    zero_async(par.get(), 8 * sizeof(int), s);
    hipLaunchKernelGGL(k_max_row_len, dim3(std::min(grid1(n), 256)), dim3(kBlock), 0, s, n, rp, par.get());
    hipLaunchKernelGGL(k_group_params, dim3(1), dim3(1), 0, s, n, rp, par.get());
    MATAMG_LAUNCH_CHECK();

    const size_t n1 = (size_t)n + 1;
    DBuf<int> flags(n1, mc), pos(n1, mc), tmp(scan_tmp_size(n1), mc), longs(n1, mc);
    hipLaunchKernelGGL(k_long_flags, dim3(grid1(n)), dim3(kBlock), 0, s, n, rp, (const int*)par.get(), flags.get());
    exclusive_scan(flags.get(), pos.get(), n, tmp.get(), s);
    hipLaunchKernelGGL(k_long_list, dim3(grid1(n)), dim3(kBlock), 0, s, n, flags.get(), pos.get(), longs.get());
    DBuf<int> ja(n1, mc), jb(n1, mc);
    hipLaunchKernelGGL(k_block_next, dim3(grid1(n1)), dim3(kBlock), 0, s, n, rp, (const int*)par.get(), longs.get(),
                       pos.get() + n, cap, ja.get());
    MATAMG_LAUNCH_CHECK();
    // pointer doubling from row 0 (flags reused as the start marks)
    hipLaunchKernelGGL(k_mark_init, dim3(grid1(n1)), dim3(kBlock), 0, s, n, flags.get());
    int* cur = ja.get();
    int* nxt = jb.get();
    for (int64_t span = 1; span <= (int64_t)n; span <<= 3) {
        const bool more = (span << 3) <= (int64_t)n;
        hipLaunchKernelGGL(k_mark_pow8, dim3(grid1(n1)), dim3(kBlock), 0, s, n, (const int*)cur, flags.get(),
                           more ? nxt : (int*)nullptr);
        if (more) std::swap(cur, nxt);
    }
    MATAMG_LAUNCH_CHECK();
    exclusive_scan(flags.get(), pos.get(), n, tmp.get(), s);
    // block starts (at most n blocks) and, for packing, every block's
    // column range, all before the one read-back of {blocks, group, wide}
    DBuf<int> blk(n1 + 1, mc), cbase;
    hipLaunchKernelGGL(k_fill_starts, dim3(grid1(n)), dim3(kBlock), 0, s, n, (const int*)flags.get(),
                       (const int*)pos.get(), blk.get());
    if (pack && A.nnz > 0) {
        cbase.alloc(n1, mc);
        hipLaunchKernelGGL(k_block_col_range, dim3(std::min(grid1(n) * 4, 65535)), dim3(kBlock), 0, s,
                           (const int*)pos.get() + n, rp, A.col.get(), (const int*)blk.get(), cbase.get(),
                           par.get() + 7);
    }
    hipLaunchKernelGGL(k_partition_result, dim3(1), dim3(1), 0, s, n, (const int*)pos.get(), (const int*)par.get(),
                       par.get() + 4);
    MATAMG_LAUNCH_CHECK();
    int res[4] = {0, 0, 0, 0};
    d2h(res, par.get() + 4, 4, s);
    const int nblk = res[0];
    A.group = res[1];
    A.nblk = nblk;
    A.blk.alloc((size_t)nblk + 1, mc);
    MATAMG_HIP(hipMemcpyAsync(A.blk.get(), blk.get(), sizeof(int) * ((size_t)nblk + 1), hipMemcpyDeviceToDevice, s));
    A.blkk.alloc((size_t)nblk + 1, mc);
    hipLaunchKernelGGL(k_block_entries, dim3(grid1((int64_t)nblk + 1)), dim3(kBlock), 0, s, nblk, rp,
                       (const int*)A.blk.get(), A.blkk.get());
    MATAMG_LAUNCH_CHECK();
    if (pack && A.nnz > 0 && res[3] == 0) {
        A.cbase.alloc((size_t)nblk, mc);
        MATAMG_HIP(hipMemcpyAsync(A.cbase.get(), cbase.get(), sizeof(int) * (size_t)nblk, hipMemcpyDeviceToDevice, s));
        A.col16.alloc((size_t)A.nnz, mc);
        hipLaunchKernelGGL(k_pack_cols, dim3(std::min(nblk, 65535)), dim3(kBlock), 0, s, nblk, rp, A.col.get(),
                           (const int*)A.blk.get(), (const int*)A.cbase.get(), A.col16.get());
        MATAMG_LAUNCH_CHECK();
        block_uniques(A, mc, s);
    }
}

void block_uniques(DCsr& A, MemCounter* mc, hipStream_t s) {
    A.ustart.release();
    A.uoff.release();
    A.urun.release();
    A.nuniq = 0;
    const int nblk = A.nblk;
    if (!A.col16 || nblk <= 0) return;
    DBuf<int> cnt((size_t)nblk + 2, mc), tmp(scan_tmp_size((int64_t)nblk + 1), mc);
    A.urun.alloc((size_t)nblk * kRunWords, mc);
    zero_async(cnt.get() + nblk + 1, sizeof(int), s);
    const int grid = std::min(nblk, 8192);
    hipLaunchKernelGGL(k_block_uniques_count, dim3(grid), dim3(kBlock), 0, s, nblk, (const int*)A.blk.get(),
                       (const int*)A.blkk.get(), (const uint16_t*)A.col16.get(), A.group, unique_cap(A.cap),
                       cnt.get(), A.urun.get(), cnt.get() + nblk + 1);
    MATAMG_LAUNCH_CHECK();
    A.ustart.alloc((size_t)nblk + 1, mc);
    exclusive_scan(cnt.get(), A.ustart.get(), nblk, tmp.get(), s);
    int res[2] = {0, 0};  // list length, staged blocks
    MATAMG_HIP(hipMemcpyAsync(cnt.get() + nblk, A.ustart.get() + nblk, sizeof(int), hipMemcpyDeviceToDevice, s));
    d2h(res, cnt.get() + nblk, 2, s);
    const int total = res[0];
    if (res[1] == 0) {
        // nothing staged: the streaming kernels read no per-block tables
        A.ustart.release();
        A.urun.release();
        return;
    }
    A.nuniq = total;
    A.uoff.alloc((size_t)(total > 0 ? total : 1), mc);
    hipLaunchKernelGGL(k_block_uniques_fill, dim3(grid), dim3(kBlock), 0, s, nblk, (const int*)A.blkk.get(),
                       (const int*)A.ustart.get(), (const uint32_t*)A.urun.get(), A.col16.get(), A.uoff.get());
    MATAMG_LAUNCH_CHECK();
}

}  // namespace matamg
