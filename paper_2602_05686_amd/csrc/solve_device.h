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
enum StreamMode { M_PLAIN = 0, M_RESID = 1, M_ADD = 2, M_SMOOTH = 3, M_DOTPQ = 4, M_RESNORM = 5, M_SCALENORM = 6 };

template <typename T>
struct SArgs {
    const int* rowptr;
    const int* col;
    const T* val;
    const int* blk;
    const T* x;        // gathered operand
    const T* b;        // right-hand side (RESID, SMOOTH, RESNORM)
    const T* yin;      // ADD: base vector; SMOOTH: iterate at the row
    const T* dinv;     // SMOOTH: inverse diagonal; SCALENORM: row scale
    T* d;              // SMOOTH: direction (in/out)
    T* y;              // output
    double* y64;       // SMOOTH: FP64 output instead of y
    const double* dotvec;  // SMOOTH: fused dot partner
    T c1, c2;
    DotTarget dt;
};

template <typename T, int MODE, bool HAS_DOT>
__device__ __forceinline__ double epilogue(const SArgs<T>& a, int r, T s) {
    double dp = 0.0;
    if constexpr (MODE == M_PLAIN) {
        a.y[r] = s;
    } else if constexpr (MODE == M_RESID) {
        a.y[r] = a.b[r] - s;
    } else if constexpr (MODE == M_ADD) {
        a.y[r] = a.yin[r] + s;
    } else if constexpr (MODE == M_SMOOTH) {
        T res = a.b[r] - s;
        T dn = a.c1 * a.d[r] + a.c2 * (a.dinv[r] * res);
        a.d[r] = dn;
        T xn = a.yin[r] + dn;
        if (a.y64) a.y64[r] = (double)xn;
        else a.y[r] = xn;
        if constexpr (HAS_DOT) dp = (double)xn * a.dotvec[r];
    } else if constexpr (MODE == M_DOTPQ) {
        a.y[r] = s;
        dp = (double)a.x[r] * (double)s;
    } else if constexpr (MODE == M_RESNORM) {
        T v = a.b[r] - s;
        a.y[r] = v;
        dp = (double)v * (double)v;
    } else if constexpr (MODE == M_SCALENORM) {
        T v = a.dinv[r] * s;
        a.y[r] = v;
        dp = (double)v * (double)v;
    }
    return dp;
}

constexpr int kPerThread = kStreamCap / kBlock;

// LDS of one streaming block
template <typename T>
struct StreamShared {
    T prod[kStreamCap];
    double sh[kBlock / 64];
    T shr[kBlock / 64];
};

// Row block `bid` of the matrix in `a`: stream its val/col range into LDS
// products, reduce each row with G threads (or the whole block for a long
// row), apply the epilogue, and store each wavefront's dot partial at
// a.dt.partial[bid * kStreamPartials + wave] (no block-wide step at the end,
// so the waves of a block retire independently).
template <typename T, int MODE, bool HAS_DOT, int G>
__device__ __forceinline__ void stream_block(const SArgs<T>& a, int bid, StreamShared<T>& S) {
    const int r0 = a.blk[bid], r1 = a.blk[bid + 1];
    const int k0 = a.rowptr[r0], k1 = a.rowptr[r1];
    const int cnt = k1 - k0;
    double dp = 0.0;
    if (!(r1 - r0 == 1 && cnt > long_row_limit(G))) {
        // issue every load of this thread's share before using any of them
        int c[kPerThread];
        T v[kPerThread];
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            const int t = (int)threadIdx.x + u * kBlock;
            if (t < cnt) {
                c[u] = __builtin_nontemporal_load(a.col + k0 + t);
                v[u] = __builtin_nontemporal_load(a.val + k0 + t);
            }
        }
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            const int t = (int)threadIdx.x + u * kBlock;
            if (t < cnt) S.prod[t] = v[u] * a.x[c[u]];
        }
        __syncthreads();
        // G threads per row: strided partial sums, then a fixed shuffle tree
        const int gl = (int)threadIdx.x % G;
        const int r = r0 + (int)threadIdx.x / G;
        T s = 0;
        if (r < r1) {
            const int s0 = a.rowptr[r] - k0, s1 = a.rowptr[r + 1] - k0;
            for (int k = s0 + gl; k < s1; k += G) s += S.prod[k];
        }
        if constexpr (G > 1) {
            for (int off = G / 2; off > 0; off >>= 1) s += __shfl_down(s, off, G);
        }
        if (gl == 0 && r < r1) dp = epilogue<T, MODE, HAS_DOT>(a, r, s);
    } else {
        // one long row (a block of its own): strided partial sums, fixed tree
        T s = 0;
        for (int t = threadIdx.x; t < cnt; t += kBlock) {
            const int k = k0 + t;
            s += a.val[k] * a.x[a.col[k]];
        }
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) S.shr[w] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            T t = S.shr[0];
            for (int i = 1; i < kBlock / 64; ++i) t += S.shr[i];
            dp = epilogue<T, MODE, HAS_DOT>(a, r0, t);
        }
    }
    if constexpr (HAS_DOT) {
        const double t = wave_sum(dp);
        if ((threadIdx.x & 63) == 0) a.dt.partial[bid * kStreamPartials + (threadIdx.x >> 6)] = t;
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
    double s = 0.0;
    for (int j = lane; j < a.n; j += 64) s += m[j] * (double)a.in[j];
    s = wave_sum(s);
    if (lane == 0) a.out[row] = (T)s;
}

inline int gemv_grid(int n) { return ceil_div(n, kBlock / 64); }

}  // namespace matamg
