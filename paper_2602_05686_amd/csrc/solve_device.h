// Device bodies of the solve-path kernels, shared by the one-hierarchy
// launchers (k_solve.hip) and the batched launchers that run the same work
// for many hierarchies in one launch (k_batch.hip).  Each body takes its
// block index and grid size within its own problem explicitly, so a block
// computes exactly the same thing whether it is launched alone or as one
// segment of a batch: results do not depend on what else is in the batch.
#pragma once

#include "device_util.h"
#include "kernels.h"

namespace matamg {

__host__ __device__ inline int vec_grid(int64_t n) {
    const int64_t g = (n > 0 ? n : 1) / kBlock + (((n > 0 ? n : 1) % kBlock) ? 1 : 0);
    return g < 2048 ? (int)g : 2048;
}

// ----------------------------------------------------------- streaming SpMV
enum StreamMode {
    M_PLAIN = 0,
    M_RESID = 1,
    M_ADD = 2,
    M_SMOOTH = 3,
    M_DOTPQ = 4,
    M_RESNORM = 5,
    M_SCALENORM = 6,
    M_RESTRICT = 7  // y = A x, then the first smoother step on y as right-hand side
};

template <typename T>
struct SArgs {
    const int* rowptr;
    const int* col;
    const uint16_t* col16;  // packed columns (or null): col = cbase[block] + col16
    const int* cbase;
    const T* val;
    const int* blk;
    const int* blkk;   // first entry of each block (rowptr at its first row)
    const int* ustart;       // packed blocks' distinct-column lists (or null):
    const uint16_t* uoff;    // block b's are uoff[ustart[b] .. ustart[b+1])
    const uint32_t* urun;    // or their runs (DCsr::urun; null: none)
    const T* x;        // gathered operand
    const T* b;        // right-hand side (RESID, SMOOTH, RESNORM)
    const T* yin;      // ADD: base vector; SMOOTH: iterate at the row
    const T* dinv;     // SMOOTH: inverse diagonal; SCALENORM: row scale
    T* d;              // SMOOTH: direction (in/out); RESTRICT: direction (out)
    T* y;              // output
    T* xo;             // RESTRICT: first smoother iterate
    double* y64;       // SMOOTH: FP64 output instead of y
    const double* dotvec;  // SMOOTH: fused dot partner
    T c1, c2;
    DotTarget dt;
};

// Per-row operands of the epilogue, loaded before the row's sum is known so
// that their latency overlaps the streaming of the block's entries.
template <typename T>
struct RowOperands {
    T b, dinv, d, xin;
};

template <typename T, int MODE>
__device__ __forceinline__ RowOperands<T> row_operands(const SArgs<T>& a, int r) {
    RowOperands<T> o{};
    if constexpr (MODE == M_RESID || MODE == M_RESNORM) o.b = a.b[r];
    if constexpr (MODE == M_ADD) o.xin = a.yin[r];
    if constexpr (MODE == M_SMOOTH) {
        o.b = a.b[r];
        o.dinv = a.dinv[r];
        o.d = a.d[r];
        o.xin = a.yin[r];
    }
    if constexpr (MODE == M_DOTPQ) o.xin = a.x[r];
    if constexpr (MODE == M_SCALENORM || MODE == M_RESTRICT) o.dinv = a.dinv[r];
    return o;
}

template <typename T, int MODE, bool HAS_DOT>
__device__ __forceinline__ double epilogue(const SArgs<T>& a, int r, T s, const RowOperands<T>& o) {
    double dp = 0.0;
    if constexpr (MODE == M_PLAIN) {
        a.y[r] = s;
    } else if constexpr (MODE == M_RESID) {
        a.y[r] = o.b - s;
    } else if constexpr (MODE == M_ADD) {
        a.y[r] = o.xin + s;
    } else if constexpr (MODE == M_SMOOTH) {
        T res = o.b - s;
        T dn = a.c1 * o.d + a.c2 * (o.dinv * res);
        a.d[r] = dn;
        T xn = o.xin + dn;
        if (a.y64) a.y64[r] = (double)xn;
        else a.y[r] = xn;
        if constexpr (HAS_DOT) dp = (double)xn * a.dotvec[r];
    } else if constexpr (MODE == M_DOTPQ) {
        a.y[r] = s;
        dp = (double)o.xin * (double)s;
    } else if constexpr (MODE == M_RESNORM) {
        T v = o.b - s;
        a.y[r] = v;
        dp = (double)v * (double)v;
    } else if constexpr (MODE == M_SCALENORM) {
        T v = o.dinv * s;
        a.y[r] = v;
        dp = (double)v * (double)v;
    } else if constexpr (MODE == M_RESTRICT) {
        // the coarse right-hand side, and the first smoother step from a
        // zero iterate (the same operations as smooth_first_body)
        a.y[r] = s;
        T di = a.c2 * (o.dinv * s);
        a.d[r] = di;
        a.xo[r] = di;
    }
    return dp;
}

constexpr int kPerThread = kStreamCap / kBlock;

// LDS of one streaming block of at most CAP stored entries: the products
// (first holding the block's distinct gathered values), reduction scratch
template <typename T, int CAP = kStreamCap>
struct StreamShared {
    T prod[CAP];
    double sh[kBlock / 64];
    T shr[kBlock / 64];
};

// prod[t] = val[k0 + t] * x[col[k0 + t]] for t < cnt, with NU = ceil(cnt /
// kBlock) strides per thread: all loads first (indices past the end clamped
// to the last entry, results discarded), then the gathers, then the stores.
// PACKED: the columns come from the 16-bit col16 plus the block's base.
// packed columns, two entries per load: the block's entries from its first
// even position are read as aligned pairs (a pair of values, a pair of
// 16-bit columns), NP = ceil(pairs / kBlock) strides per thread; an entry left
// over at either end (odd start, odd length) is read alone by thread 0 or 1.
template <typename T>
struct PairOf;
template <>
struct PairOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct PairOf<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int stage_head(int k0, int cnt) { return cnt > 0 ? (k0 & 1) : 0; }

template <typename T, int NP, int UQ>
__device__ __forceinline__ void stage_pairs(const SArgs<T>& a, int bid, int k0, int cnt, T* prod) {
    using P2 = typename PairOf<T>::type;
    const int base = a.cbase[bid];
    const int head = stage_head(k0, cnt);  // entry 0 alone when the block starts at an odd position
    const int body = cnt - head;
    const int np = body >> 1;  // whole pairs from the even position k0 + head
    const int kp = k0 + head;
    const int tid = (int)threadIdx.x;
    // the block's distinct columns (block-uniform): runs, a list, or none
    // (gathers)
    const uint32_t* rec = a.urun ? a.urun + (size_t)bid * kRunWords : nullptr;
    const int nruns = rec ? (int)rec[0] : 0;
    const int u0 = a.ustart ? a.ustart[bid] : 0;
    const int nu = nruns > 0 ? (int)rec[1] : (a.ustart ? a.ustart[bid + 1] - u0 : 0);
    u16x2 c[NP > 0 ? NP : 1];
    P2 v[NP > 0 ? NP : 1];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int p = tid + u * kBlock;
        const int pc = p < np ? p : np - 1;
        c[u] = __builtin_nontemporal_load(reinterpret_cast<const u16x2*>(a.col16 + kp + 2 * pc));
        v[u] = __builtin_nontemporal_load(reinterpret_cast<const P2*>(a.val + kp + 2 * pc));
    }
    // the single entries: the head (thread 0) and, for an odd body, the tail (thread 1)
    int ts = -1;
    if (tid == 0 && head) ts = 0;
    if (tid == 1 && (body & 1)) ts = cnt - 1;
    int cs = 0;
    T vs = 0;
    if (ts >= 0) {
        cs = (int)a.col16[k0 + ts];
        vs = a.val[k0 + ts];
    }
    T x0[NP > 0 ? NP : 1], x1[NP > 0 ? NP : 1];
    T xsng = T(0);
    if (UQ > 0 && nu > 0) {
        // the block's distinct values of the gathered vector, read in
        // ascending column order (coalesced along the list), staged in the
        // product array (nu <= unique_cap(CAP) <= CAP entries); the entries'
        // col16 index the list.  Every thread takes its values into
        // registers before the products overwrite the array.
        T* xs = prod;
        int off[UQ > 0 ? UQ : 1];
        if (nruns > 0) {
            // list index j lies in the run whose prefix of lengths it reaches
            uint32_t rw[kMaxRuns];
#pragma unroll
            for (int r = 0; r < kMaxRuns; ++r) rw[r] = rec[2 + r];
#pragma unroll
            for (int q = 0; q < UQ; ++q) {
                const int j0 = tid + q * kBlock;
                const int j = j0 < nu ? j0 : nu - 1;
                int pos = (int)(rw[0] & 0xffffu) + j, pre = 0;
#pragma unroll
                for (int r = 0; r < kMaxRuns - 1; ++r) {
                    pre += (int)(rw[r] >> 16);
                    if (r + 1 < nruns && j >= pre) pos = (int)(rw[r + 1] & 0xffffu) + (j - pre);
                }
                off[q] = pos;
            }
        } else {
#pragma unroll
            for (int q = 0; q < UQ; ++q) {
                const int j = tid + q * kBlock;
                off[q] = (int)a.uoff[u0 + (j < nu ? j : nu - 1)];
            }
        }
        T xv[UQ > 0 ? UQ : 1];
#pragma unroll
        for (int q = 0; q < UQ; ++q) xv[q] = a.x[base + off[q]];
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const int j = tid + q * kBlock;
            if (j < nu) xs[j] = xv[q];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            x0[u] = xs[(int)c[u].x];
            x1[u] = xs[(int)c[u].y];
        }
        if (ts >= 0) xsng = xs[cs];
        __syncthreads();
    } else {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            x0[u] = a.x[base + (int)c[u].x];
            x1[u] = a.x[base + (int)c[u].y];
        }
        if (ts >= 0) xsng = a.x[base + cs];
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int p = tid + u * kBlock;
        if (p < np) {
            prod[head + 2 * p] = v[u].x * x0[u];
            prod[head + 2 * p + 1] = v[u].y * x1[u];
        }
    }
    if (ts >= 0) prod[ts] = vs * xsng;
}

template <typename T, int NU, bool PACKED>
__device__ __forceinline__ void stage_products(const SArgs<T>& a, int bid, int k0, int cnt, T* prod) {
    int c[NU];
    T v[NU];
    const int base = PACKED ? a.cbase[bid] : 0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int t = (int)threadIdx.x + u * kBlock;
        const int tc = t < cnt ? t : cnt - 1;
        if constexpr (PACKED) c[u] = base + (int)__builtin_nontemporal_load(a.col16 + k0 + tc);
        else c[u] = __builtin_nontemporal_load(a.col + k0 + tc);
        v[u] = __builtin_nontemporal_load(a.val + k0 + tc);
    }
    T xv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) xv[u] = a.x[c[u]];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int t = (int)threadIdx.x + u * kBlock;
        if (t < cnt) prod[t] = v[u] * xv[u];
    }
}

// s + prod[k0] + prod[k0 + step] + ... (k < k1), added one at a time in
// that order; the LDS reads go out eight at a time so that their latencies
// overlap (the additions, and so the result, are those of the plain loop)
template <typename T, int STEP>
__device__ __forceinline__ T ordered_sum(const T* prod, int k0, int k1, T s) {
    int k = k0;
    for (; k + 7 * STEP < k1; k += 8 * STEP) {
        T p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = prod[k + u * STEP];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += p[u];
    }
    for (; k < k1; k += STEP) s += prod[k];
    return s;
}

// Row block `bid` of the matrix in `a`: stream its val/col range into LDS
// products, reduce each row with G threads (or the whole block for a long
// row), apply the epilogue, and store the block's dot partial (its
// wavefront sums in wavefront order) at a.dt.partial[bid].
//
// Every load of the streaming phase is unconditional: indices past the
// block's end are clamped to its last entry (or row) and the results are
// discarded, so the compiler issues all of them back to back with no
// branch, and no wait, between them.
template <typename T, int MODE, bool HAS_DOT, int G, int CAP = kStreamCap>
__device__ __forceinline__ void stream_block(const SArgs<T>& a, int bid, StreamShared<T, CAP>& S) {
    // rows and entries of the block from the two tables: the loads of the
    // entries do not wait for the row pointer
    const int r0 = a.blk[bid], r1 = a.blk[bid + 1];
    const int k0 = a.blkk[bid], k1 = a.blkk[bid + 1];
    const int cnt = k1 - k0;
    double dp = 0.0;
    if (!(r1 - r0 == 1 && cnt > long_row_limit(G))) {
        const int gl = (int)threadIdx.x % G;
        const int r = r0 + (int)threadIdx.x / G;
        const bool owner = r < r1;
        const int rc = owner ? r : r1 - 1;
        const int e0 = a.rowptr[rc], e1 = a.rowptr[rc + 1];
        // one thread per row: every thread prefetches its row's operands;
        // with G > 1 every thread prefetches the row bounds of its group's
        // rows_per_group(G) rows and the group's first thread their operands,
        // so that none of these loads waits behind the reduction
        RowOperands<T> ops{};
        if constexpr (G == 1) ops = row_operands<T, MODE>(a, rc);
        constexpr int RQ = G == 1 ? 1 : rows_per_group(G);
        int gf0[RQ], gf1[RQ];
        RowOperands<T> gops[RQ];
        if constexpr (G > 1) {
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int rq = r + q * (kBlock / G);
                const int rqc = rq < r1 ? rq : r1 - 1;
                gf0[q] = a.rowptr[rqc] - k0;
                gf1[q] = a.rowptr[rqc + 1] - k0;
                gops[q] = RowOperands<T>{};
                if (gl == 0) gops[q] = row_operands<T, MODE>(a, rqc);
            }
        }
        // ceil(cnt / kBlock) strides of the block's entries (block-uniform),
        // from packed or plain columns (uniform per matrix)
        const int nu = (cnt + kBlock - 1) / kBlock;
        constexpr int kUQ = unique_cap(CAP) / kBlock;  // distinct values per thread
        if (a.col16) {
            // pairs of entries: ceil(pairs / kBlock) strides (block-uniform)
            switch (((cnt - stage_head(k0, cnt)) / 2 + kBlock - 1) / kBlock) {
                case 0: stage_pairs<T, 0, kUQ>(a, bid, k0, cnt, S.prod); break;
                case 1: stage_pairs<T, 1, kUQ>(a, bid, k0, cnt, S.prod); break;
                case 2: stage_pairs<T, 2, kUQ>(a, bid, k0, cnt, S.prod); break;
                case 3: stage_pairs<T, 3, kUQ>(a, bid, k0, cnt, S.prod); break;
                case 4: stage_pairs<T, 4, kUQ>(a, bid, k0, cnt, S.prod); break;
                default:
                    if constexpr (CAP > kStreamCap) {
                        switch (((cnt - stage_head(k0, cnt)) / 2 + kBlock - 1) / kBlock) {
                            case 5: stage_pairs<T, 5, kUQ>(a, bid, k0, cnt, S.prod); break;
                            case 6: stage_pairs<T, 6, kUQ>(a, bid, k0, cnt, S.prod); break;
                            case 7: stage_pairs<T, 7, kUQ>(a, bid, k0, cnt, S.prod); break;
                            case 8: stage_pairs<T, 8, kUQ>(a, bid, k0, cnt, S.prod); break;
                            default: break;
                        }
                    }
                    break;
            }
        } else if constexpr (CAP == kStreamCap) {
            // (wide blocks are only made for packed matrices)
            switch (nu) {
                case 1: stage_products<T, 1, false>(a, bid, k0, cnt, S.prod); break;
                case 2: stage_products<T, 2, false>(a, bid, k0, cnt, S.prod); break;
                case 3: stage_products<T, 3, false>(a, bid, k0, cnt, S.prod); break;
                case 4: stage_products<T, 4, false>(a, bid, k0, cnt, S.prod); break;
                case 5: stage_products<T, 5, false>(a, bid, k0, cnt, S.prod); break;
                case 6: stage_products<T, 6, false>(a, bid, k0, cnt, S.prod); break;
                case 7: stage_products<T, 7, false>(a, bid, k0, cnt, S.prod); break;
                case 8: stage_products<T, 8, false>(a, bid, k0, cnt, S.prod); break;
                default: break;
            }
        }
        __syncthreads();
        if constexpr (G == 1) {
            // a row up to kWideRow wide is summed by its own thread; the
            // wider rows of a wavefront (at most long_row_limit(1) wide) by
            // 8-lane groups of it, eight rows at a time: lane-strided
            // partial sums, then a butterfly that leaves the same bits in
            // the group's eight lanes
            const bool wide = owner && (e1 - e0) > kWideRow;
            T s = 0;
            if (owner && !wide) s = ordered_sum<T, 1>(S.prod, e0 - k0, e1 - k0, s);
            const int lane = (int)threadIdx.x & 63, grp = lane >> 3, gl = lane & 7;
            unsigned long long wm = __ballot(wide);
            // rank of this lane's row among the wide rows of the wavefront
            const int rank = __popcll(wm & ((1ull << lane) - 1ull));
            for (int base = 0; wm; base += 8) {
                unsigned long long m = wm;
                for (int j = 0; j < grp; ++j) m &= m - 1ull;  // the grp-th remaining wide row
                const int l = m ? __builtin_ctzll(m) : 0;
                const int f0 = __shfl(e0, l, 64) - k0, f1 = __shfl(e1, l, 64) - k0;
                T ps = 0;
                if (m) ps = ordered_sum<T, 8>(S.prod, f0 + gl, f1, ps);
                for (int off = 4; off > 0; off >>= 1) ps += __shfl_xor(ps, off, 64);
                const int src = (rank >= base && rank < base + 8) ? (rank - base) * 8 : 0;
                const T got = __shfl(ps, src, 64);
                if (wide && rank >= base && rank < base + 8) s = got;
                for (int j = 0; j < 8; ++j) wm &= wm - 1ull;
            }
            if (owner) dp = epilogue<T, MODE, HAS_DOT>(a, r, s, ops);
        } else {
            // G threads per row, rows_per_group(G) rows per group: strided
            // partial sums, then a fixed shuffle tree, row after row
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int rq = r + q * (kBlock / G);
                const bool own = rq < r1;
                T s = 0;
                if (own) s = ordered_sum<T, G>(S.prod, gf0[q] + gl, gf1[q], s);
                for (int off = G / 2; off > 0; off >>= 1) s += __shfl_down(s, off, G);
                if (gl == 0 && own) dp += epilogue<T, MODE, HAS_DOT>(a, rq, s, gops[q]);
            }
        }
    } else {
        // one long row (a block of its own): strided partial sums, fixed
        // tree.  Each thread adds its entries t, t + kBlock, ... in order;
        // four strides at a time have their loads, then their gathers, in
        // flight together.  A long row's block is never staged, so packed
        // columns hold plain offsets from the block's base.
        T s = 0;
        const int* col = a.col16 ? nullptr : a.col;
        const int base = a.col16 ? a.cbase[bid] : 0;
        int t = (int)threadIdx.x;
        for (; t + 3 * kBlock < cnt; t += 4 * kBlock) {
            int c[4];
            T v[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + t + u * kBlock;
                c[u] = col ? col[k] : base + (int)a.col16[k];
                v[u] = a.val[k];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = a.x[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) s += v[u] * xv[u];
        }
        for (; t < cnt; t += kBlock) {
            const int k = k0 + t;
            s += a.val[k] * a.x[col ? col[k] : base + (int)a.col16[k]];
        }
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) S.shr[w] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            T t = S.shr[0];
            for (int i = 1; i < kBlock / 64; ++i) t += S.shr[i];
            dp = epilogue<T, MODE, HAS_DOT>(a, r0, t, row_operands<T, MODE>(a, r0));
        }
    }
    if constexpr (HAS_DOT) {
        // the block's partial: wavefront sums added in wavefront order
        const double t = wave_sum(dp);
        if ((threadIdx.x & 63) == 0) S.sh[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double u = S.sh[0];
            for (int w = 1; w < kBlock / 64; ++w) u += S.sh[w];
            a.dt.partial[bid] = u;
        }
    }
}

// ------------------------------------------------------------ vector bodies
// Grid-stride loops over one problem's vectors: block `lb` of `grid`.

template <typename T>
struct SmoothFirstArgs {
    int64_t n;
    const double* b64;  // if set: b = (T) b64 is stored first
    T* b;
    const T* dinv;
    T c2;
    T* d;
    T* x;
};

template <typename T>
__device__ __forceinline__ void smooth_first_body(const SmoothFirstArgs<T>& a, int lb, int grid) {
    for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < a.n; i += (int64_t)grid * kBlock) {
        T bi;
        if (a.b64) {
            bi = (T)a.b64[i];
            a.b[i] = bi;
        } else {
            bi = a.b[i];
        }
        T di = a.c2 * (a.dinv[i] * bi);
        a.d[i] = di;
        a.x[i] = di;
    }
}

struct CgDirArgs {
    int64_t n;
    double* p;
    const double* z;
    const double* rz_new;
    const double* rz_old;  // null: p = z
};

__device__ __forceinline__ void cg_direction_body(const CgDirArgs& a, int lb, int grid) {
    const double beta = a.rz_old ? (*a.rz_new / *a.rz_old) : 0.0;
    for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < a.n; i += (int64_t)grid * kBlock)
        a.p[i] = a.rz_old ? a.z[i] + beta * a.p[i] : a.z[i];
}

struct CgUpdArgs {
    int64_t n;
    double* x;
    double* r;
    const double* p;
    const double* q;
    const double* rz;
    const double* pq;
    double* partial;  // r.r partial of block lb at partial[lb]
};

__device__ __forceinline__ void cg_update_body(const CgUpdArgs& a, int lb, int grid, double* sh) {
    // a non-positive or non-finite curvature is a breakdown: leave x and r
    // unchanged so the caller keeps the last iterate
    const double pqv = *a.pq, rzv = *a.rz;
    const double alpha = (pqv > 0.0 && isfinite(pqv) && isfinite(rzv)) ? rzv / pqv : 0.0;
    double v = 0.0;
    for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < a.n; i += (int64_t)grid * kBlock) {
        a.x[i] = a.x[i] + alpha * a.p[i];
        double ri = a.r[i] - alpha * a.q[i];
        a.r[i] = ri;
        v += ri * ri;
    }
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) a.partial[lb] = t;
}

// *result = sum of partial[0..nb) (one block of kFinishThreads threads).
// Thread t adds partial[t], partial[t + T], ... in ascending order, four
// independent loads in flight at a time; the per-thread sums are combined
// by a fixed tree.  The order depends on nb only.
constexpr int kFinishThreads = 1024;

struct FinishArgs {
    int nb;
    const double* partial;
    double* result;
};

__device__ __forceinline__ void finish_body(const FinishArgs& a, double* sh /* kFinishThreads / 64 */) {
    constexpr int T = kFinishThreads;
    double v = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * T < a.nb; i += 4 * T) {
        const double p0 = a.partial[i], p1 = a.partial[i + T], p2 = a.partial[i + 2 * T], p3 = a.partial[i + 3 * T];
        v += p0;
        v += p1;
        v += p2;
        v += p3;
    }
    for (; i < a.nb; i += T) v += a.partial[i];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int k = 1; k < T / 64; ++k) t += sh[k];
        *a.result = t;
    }
}

// ------------------------------------------------------------- dense GEMV
// out = M in, one wavefront per row of the row-major n x n FP64 matrix
template <typename T>
struct GemvArgs {
    int n;
    const double* M;
    const T* in;
    T* out;
};

template <typename T>
__device__ __forceinline__ void gemv_body(const GemvArgs<T>& a, int lb) {
    const int lane = threadIdx.x & 63;
    const int row = lb * (kBlock / 64) + (threadIdx.x >> 6);
    if (row >= a.n) return;
    const double* m = a.M + (size_t)row * a.n;
    const int n = a.n;
    // lane-strided sum (columns lane, lane + 64, ... in order) over chunks of
    // sixteen columns per lane; the next chunk's loads are issued before the
    // current chunk is summed, so a row costs about one memory latency
    // instead of one per chunk.  Indices past the row's end are clamped to
    // its last column and their products skipped.
    constexpr int U = 16;
    double mv[U], iv[U];
    auto load = [&](int j0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(j0 + u * 64, n - 1);
            mv[u] = m[j];
            iv[u] = (double)a.in[j];
        }
    };
    double s = 0.0;
    load(lane);
    for (int j0 = lane; j0 < n; j0 += U * 64) {
        double cm[U], ci[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cm[u] = mv[u];
            ci[u] = iv[u];
        }
        if (j0 + U * 64 < n) load(j0 + U * 64);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u * 64 < n) s += cm[u] * ci[u];
    }
    s = wave_sum(s);
    if (lane == 0) a.out[row] = (T)s;
}

inline int gemv_grid(int n) { return ceil_div(n, kBlock / 64); }

}  // namespace matamg
