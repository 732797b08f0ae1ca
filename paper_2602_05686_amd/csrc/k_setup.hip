// Setup-phase kernels.  This file is compiled with -ffp-contract=off: the
// strength-of-connection arithmetic, the Clement means and the aggregate
// means are evaluated one IEEE-754 operation at a time in a fixed order, so
// the drop masks and aggregates they decide are bit-reproducible and equal to
// any other evaluation of the same operation sequence.
//
// Paper references: Clement interpolant and auxiliary transfer (section 3,
// eq. auxiliary_transfer); distance Laplacian and pointwise dropping
// (section 2.1); material distance (section 3); aggregation and tentative
// prolongator (section 2); filtered matrix and 1-norm diagonal (section 2.2,
// eqs. filtered_matrix and 1_norm_diagonal).
#pragma clang fp contract(off)

#include "device_util.h"
#include "kernels.h"
#include <algorithm>

#include "setup_kernels.h"

namespace matamg {
namespace {

constexpr double kRowNoise = 1.4210854715202004e-14;  // 2^-46

inline int grid_for(int64_t n) {
    int g = ceil_div(n > 0 ? n : 1, kBlock);
    return g;
}

#define ROW_LOOP(i, n) for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kBlock)

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// --------------------------------------------------------------- incidence
__global__ void k_count_elem_nodes(const int* en, int64_t total, int n, int* cnt, int* flag) {
    ROW_LOOP(e, total) {
        int i = en[e];
        if (i < 0 || i >= n) {
            *flag = 1;
            continue;
        }
        atomicAdd(cnt + i, 1);
    }
}

__global__ void k_fill_elem_nodes(const int* en, int64_t total, int npe, int n, const int* rowptr, int* fill,
                                  int* items) {
    ROW_LOOP(e, total) {
        int i = en[e];
        if (i < 0 || i >= n) continue;
        int pos = rowptr[i] + atomicAdd(fill + i, 1);
        items[pos] = (int)(e / npe);
    }
}

__global__ void k_count_agg(const int* agg, int n, int* cnt) {
    ROW_LOOP(i, n) {
        int a = agg[i];
        if (a >= 0) atomicAdd(cnt + a, 1);
    }
}

__global__ void k_fill_agg(const int* agg, int n, const int* rowptr, int* fill, int* items) {
    ROW_LOOP(i, n) {
        int a = agg[i];
        if (a < 0) continue;
        int pos = rowptr[a] + atomicAdd(fill + a, 1);
        items[pos] = (int)i;
    }
}

// ascending order within each list (insertion sort; lists are short)
__global__ void k_sort_lists(int nt, const int* rowptr, int* items) {
    ROW_LOOP(t, nt) {
        int lo = rowptr[t], hi = rowptr[t + 1];
        for (int a = lo + 1; a < hi; ++a) {
            int v = items[a], b = a - 1;
            while (b >= lo && items[b] > v) {
                items[b + 1] = items[b];
                --b;
            }
            items[b + 1] = v;
        }
    }
}

// ------------------------------------------------------------------- level 1
__global__ void k_detect_dirichlet(int n, const int* rowptr, const int* col, const double* val, uint8_t* dir) {
    ROW_LOOP(i, n) {
        int any = 0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] != i && val[k] != 0.0) {
                any = 1;
                break;
            }
        dir[i] = any ? 0 : 1;
    }
}

// nodal tensor = arithmetic mean of the incident element tensors, summed in
// ascending element id, one divide per component
__global__ void k_clement(int n, int dim, const int* rowptr, const int* elems, const double* es, double* sig) {
    const int nc = dim * (dim + 1) / 2;
    ROW_LOOP(i, n) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        const int lo = rowptr[i], hi = rowptr[i + 1];
        for (int k = lo; k < hi; ++k) {
            const double* s = es + (size_t)elems[k] * dim * dim;
            int c = 0;
            for (int p = 0; p < dim; ++p)
                for (int q = p; q < dim; ++q) acc[c++] += s[p * dim + q];
        }
        const int cnt = hi - lo;
        for (int c = 0; c < nc; ++c) sig[(size_t)i * nc + c] = cnt > 0 ? acc[c] / (double)cnt : acc[c];
    }
}

// sigma^{-1} by adjugate / determinant
__global__ void k_tensor_inverse(int n, int dim, const double* sig, double* minv, int* flag) {
    const int nc = dim * (dim + 1) / 2;
    ROW_LOOP(i, n) {
        const double* s = sig + (size_t)i * nc;
        double* m = minv + (size_t)i * nc;
        bool ok;
        if (dim == 1) {
            ok = s[0] > 0.0;
            m[0] = 1.0 / s[0];
        } else if (dim == 2) {
            double s00 = s[0], s01 = s[1], s11 = s[2];
            double det = s00 * s11 - s01 * s01;
            ok = (det > 0.0) && (s00 > 0.0);
            m[0] = s11 / det;
            m[1] = (-s01) / det;
            m[2] = s00 / det;
        } else {
            double s00 = s[0], s01 = s[1], s02 = s[2], s11 = s[3], s12 = s[4], s22 = s[5];
            double c00 = s11 * s22 - s12 * s12;
            double c01 = s02 * s12 - s01 * s22;
            double c02 = s01 * s12 - s02 * s11;
            double c11 = s00 * s22 - s02 * s02;
            double c12 = s01 * s02 - s00 * s12;
            double c22 = s00 * s11 - s01 * s01;
            double det = (s00 * c00 + s01 * c01) + s02 * c02;
            ok = (det > 0.0) && (s00 > 0.0) && (c22 > 0.0);
            m[0] = c00 / det;
            m[1] = c01 / det;
            m[2] = c02 / det;
            m[3] = c11 / det;
            m[4] = c12 / det;
            m[5] = c22 / det;
        }
        if (!ok) *flag = 1;
    }
}


// ------------------------------------------------------- streamed row blocks
// The kernels below walk the same row blocks as the streaming SpMV: a block
// stages its contiguous range of stored entries through LDS with coalesced
// loads, works per entry in parallel, and finishes per row with one thread
// per row in ascending stored order.  A long row has a block of its own.
struct RowBlock {
    int r0, r1, k0, k1, cnt;
    bool longrow;
};

__device__ __forceinline__ RowBlock row_block(const int* rowptr, const int* blk, int bid) {
    RowBlock rb;
    rb.r0 = blk[bid];
    rb.r1 = blk[bid + 1];
    rb.k0 = rowptr[rb.r0];
    rb.k1 = rowptr[rb.r1];
    rb.cnt = rb.k1 - rb.k0;
    rb.longrow = (rb.r1 - rb.r0 == 1) && rb.cnt > kLongRow;
    return rb;
}

// rowof[t] = row of stored entry k0 + t, for a block of short rows
__device__ __forceinline__ void fill_row_ids(const int* rowptr, const RowBlock& rb, int* rowof) {
    const int r = rb.r0 + (int)threadIdx.x;
    if (r < rb.r1)
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) rowof[k - rb.k0] = r;
    __syncthreads();
}

__device__ __forceinline__ double quad_form(int dim, const double* m, const double* d) {
    if (dim == 1) return d[0] * (m[0] * d[0]);
    if (dim == 2) {
        double t0 = m[0] * d[0] + m[1] * d[1];
        double t1 = m[1] * d[0] + m[2] * d[1];
        return d[0] * t0 + d[1] * t1;
    }
    double t0 = (m[0] * d[0] + m[1] * d[1]) + m[2] * d[2];
    double t1 = (m[1] * d[0] + m[3] * d[1]) + m[4] * d[2];
    double t2 = (m[2] * d[0] + m[4] * d[1]) + m[5] * d[2];
    return (d[0] * t0 + d[1] * t1) + d[2] * t2;
}

struct SocArgs {
    const int* rowptr;
    const int* col;
    const double* val;
    const int* blk;
    int nblk, dim, soc;
    const double* x;
    const double* minv;
    const uint8_t* dir;
    double* lval;
    double* ldiag;
};

// |L_ij| = 1 / max(q_i, q_j) for a stored off-diagonal between non-Dirichlet
// nodes (q = d^T sigma^{-1} d from either end); 0 on the diagonal and on
// Dirichlet edges; -1 for coincident points; |A_ij| for the classical measure
__device__ __forceinline__ double edge_l(const SocArgs& a, int i, int k) {
    const int j = a.col[k];
    if (j == i) return 0.0;
    if (a.dir && (a.dir[i] || a.dir[j])) return 0.0;
    if (a.soc == AMG_SOC_SA) return fabs(a.val[k]);
    const int dim = a.dim, nc = dim * (dim + 1) / 2;
    double d[3];
    for (int c = 0; c < dim; ++c) d[c] = a.x[(size_t)j * dim + c] - a.x[(size_t)i * dim + c];
    double qi, qj;
    if (a.soc == AMG_SOC_MATERIAL) {
        qi = quad_form(dim, a.minv + (size_t)i * nc, d);
        qj = quad_form(dim, a.minv + (size_t)j * nc, d);
    } else {
        const double id[6] = {1.0, 0.0, dim == 2 ? 1.0 : 0.0, 1.0, 0.0, 1.0};
        const double id2[3] = {1.0, 0.0, 1.0};
        const double* m = dim == 3 ? id : (dim == 2 ? id2 : id);
        qi = quad_form(dim, m, d);
        qj = qi;
    }
    const double q = qi > qj ? qi : qj;
    if (!(q > 0.0) || !isfinite(q)) return -1.0;
    return 1.0 / q;
}

// s plus the positive values of l[lo..hi) in ascending order, the loads of
// eight values issued before any is added
__device__ __forceinline__ double positive_sum(const double* l, int lo, int hi, double s) {
    int k = lo;
    for (; k + 8 <= hi; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = l[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (v[u] > 0.0) s += v[u];
    }
    for (; k < hi; ++k)
        if (l[k] > 0.0) s += l[k];
    return s;
}

// the row's L_ii: ascending sum of the positive |L_ij| (or |A_ii| for the classical measure)
__device__ __forceinline__ double row_diag(const SocArgs& a, int i, const double* l, int base) {
    const int lo = a.rowptr[i], hi = a.rowptr[i + 1];
    if (a.soc == AMG_SOC_SA) {
        double ad = 0.0;
        for (int k = lo; k < hi; ++k)
            if (a.col[k] == i) ad = fabs(a.val[k]);
        return ad;
    }
    return positive_sum(l, lo - base, hi - base, 0.0);
}

__global__ __launch_bounds__(kBlock) void k_soc_values(SocArgs a) {
    __shared__ double lv[kStreamCap];
    __shared__ int rowof[kStreamCap];
    const int bid = xcd_block(a.nblk);
    if (bid >= a.nblk) return;
    const RowBlock rb = row_block(a.rowptr, a.blk, bid);
    if (!rb.longrow) {
        fill_row_ids(a.rowptr, rb, rowof);
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) {
            const double l = edge_l(a, rowof[t], rb.k0 + t);
            a.lval[rb.k0 + t] = l;
            lv[t] = l;
        }
        __syncthreads();
        const int r = rb.r0 + (int)threadIdx.x;
        if (r < rb.r1) a.ldiag[r] = row_diag(a, r, lv, rb.k0);
    } else {
        // one long row, kStreamCap entries at a time: the block computes a
        // piece's values into memory and LDS, then thread 0 continues the
        // row's ascending sum over the piece from LDS (the order row_diag
        // adds in); the classical measure's |A_ii| is the diagonal entry's
        __shared__ double li;
        const int i = rb.r0;
        if (threadIdx.x == 0) li = 0.0;
        for (int c0 = 0; c0 < rb.cnt; c0 += kStreamCap) {
            const int cn = rb.cnt - c0 < kStreamCap ? rb.cnt - c0 : kStreamCap;
            __syncthreads();  // the previous piece has been summed
            for (int t = threadIdx.x; t < cn; t += kBlock) {
                const int k = rb.k0 + c0 + t;
                const double l = edge_l(a, i, k);
                a.lval[k] = l;
                lv[t] = l;
                if (a.soc == AMG_SOC_SA && a.col[k] == i) li = fabs(a.val[k]);
            }
            __syncthreads();
            if (threadIdx.x == 0 && a.soc != AMG_SOC_SA) li = positive_sum(lv, 0, cn, li);
        }
        __syncthreads();
        if (threadIdx.x == 0) a.ldiag[i] = li;
    }
}

struct MaskArgs {
    const int* rowptr;
    const int* col;
    const int* blk;
    int nblk;
    const uint8_t* dir;
    const double* lval;
    const double* ldiag;
    double th2;
    double* S;
    uint8_t* mask;
};

// S_ij = l / sqrt(L_ii L_jj); keep iff l*l >= (theta*theta) * (L_ii * L_jj)
__device__ __forceinline__ void mask_entry(const MaskArgs& a, int i, int k) {
    const int j = a.col[k];
    double sv;
    uint8_t m;
    if (j == i) {
        sv = 1.0;
        m = 1;
    } else if (a.dir && (a.dir[i] || a.dir[j])) {
        sv = 0.0;
        m = 0;
    } else if (a.lval[k] < 0.0) {
        sv = 1.0;
        m = 1;
    } else {
        const double l = a.lval[k];
        const double prod = a.ldiag[i] * a.ldiag[j];
        sv = (prod > 0.0) ? l / sqrt(prod) : 1.0;
        m = (l * l >= a.th2 * prod) ? 1 : 0;
    }
    if (a.S) a.S[k] = sv;
    a.mask[k] = m;
}

__global__ __launch_bounds__(kBlock) void k_soc_mask(MaskArgs a) {
    __shared__ int rowof[kStreamCap];
    const int bid = xcd_block(a.nblk);
    if (bid >= a.nblk) return;
    const RowBlock rb = row_block(a.rowptr, a.blk, bid);
    if (!rb.longrow) {
        fill_row_ids(a.rowptr, rb, rowof);
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) mask_entry(a, rowof[t], rb.k0 + t);
    } else {
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) mask_entry(a, rb.r0, rb.k0 + t);
    }
}

// ---------------------------------------------------------------- cut-drop
// Cut-drop criterion (strength-of-connection section): row i keeps the
// entries whose strength is at least s_k, s_k the first value of the
// decreasingly ordered row with theta * s_k >= s_{k+1} (all if none).  The
// row's strengths are compared through t_ij = (l_ij * l_ij) / L_jj (S_ij^2 L_ii
// with the common L_ii dropped), t = L_ii for coincident points, and the test
// is (theta*theta) * t_k >= t_{k+1}.  Only off-diagonal entries are ordered
// (the diagonal is always kept), so the strongest connection of a row always
// survives the row's own cut.  Instead of sorting,
// every ordered entry a finds the next smaller key nxt(a) in its row: a gap
// sits after a iff th2 * t_a >= nxt(a), and the first gap in decreasing order
// is the one with the largest t_a.  One wavefront per row.
__device__ __forceinline__ double cut_key(const int* col, const uint8_t* dir, const double* lval,
                                          const double* ldiag, int i, double lii, int k, int hi) {
    if (k >= hi) return -1.0;
    const int j = col[k];
    if (j == i) return -1.0;         // the diagonal is not ordered (always kept)
    if (dir && dir[j]) return -1.0;  // not ordered, never kept
    const double l = lval[k];
    if (l < 0.0) return lii;         // coincident points: S = 1
    const double ljj = ldiag[j];
    return ljj > 0.0 ? (l * l) / ljj : lii;
}

__global__ __launch_bounds__(kBlock) void k_cut_keep(int n, const int* rowptr, const int* col, const uint8_t* dir,
                                                     const double* lval, const double* ldiag, double th2,
                                                     uint8_t* keep) {
    const int lane = threadIdx.x & 63;
    const int waves = (int)(gridDim.x * blockDim.x) >> 6;
    for (int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); i < n; i += waves) {
        const int lo = rowptr[i], hi = rowptr[i + 1];
        if (dir && dir[i]) {
            for (int k = lo + lane; k < hi; k += 64) keep[k] = col[k] == i;
            continue;
        }
        const double lii = ldiag[i];
        double cut = -1.0;  // keep every ordered entry
        if (lii > 0.0) {
            double best = -1.0;
            for (int a0 = lo; a0 < hi; a0 += 64) {
                const double ta = cut_key(col, dir, lval, ldiag, i, lii, a0 + lane, hi);
                double nxt = -1.0;
                for (int b0 = lo; b0 < hi; b0 += 64) {
                    const double tb = cut_key(col, dir, lval, ldiag, i, lii, b0 + lane, hi);
                    const int m = min(64, hi - b0);
                    for (int q = 0; q < m; ++q) {
                        const double v = __shfl(tb, q, 64);  // every lane takes part
                        if (v >= 0.0 && v < ta && v > nxt) nxt = v;
                    }
                }
                if (ta >= 0.0 && nxt >= 0.0 && th2 * ta >= nxt && ta > best) best = ta;
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double o = __shfl_xor(best, off, 64);
                best = o > best ? o : best;
            }
            cut = best;
        }
        for (int k0 = lo; k0 < hi; k0 += 64) {
            const int k = k0 + lane;
            const double t = cut_key(col, dir, lval, ldiag, i, lii, k, hi);
            if (k < hi) keep[k] = (col[k] == i) || (t >= 0.0 && t >= cut);
        }
    }
}

// mask_ij = keep_ij and keep_ji (the entry (j, i) found by binary search)
__global__ void k_cut_symmetric(int n, const int* rowptr, const int* col, const uint8_t* keep, uint8_t* mask) {
    ROW_LOOP(i, n) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = col[k];
            if (j == (int)i) {
                mask[k] = 1;
                continue;
            }
            int lo = rowptr[j], hi = rowptr[j + 1] - 1, kt = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int c = col[mid];
                if (c == (int)i) {
                    kt = mid;
                    break;
                }
                if (c < (int)i) lo = mid + 1;
                else hi = mid - 1;
            }
            mask[k] = (keep[k] && kt >= 0 && keep[kt]) ? 1 : 0;
        }
    }
}

// ---------------------------------------------------------------------- MIS
__device__ __forceinline__ uint64_t tuple_of(uint8_t state, uint64_t key, int i) {
    const uint64_t prio = splitmix64(key ^ (uint64_t)i) >> 34;   // top 30 bits
    return ((uint64_t)state << 62) | (prio << 32) | (uint64_t)(uint32_t)i;
}

__global__ void k_mis_init(int n, const uint8_t* dir, uint8_t* state) {
    ROW_LOOP(i, n) state[i] = (dir && dir[i]) ? MIS_OUT : MIS_UND;
}

// T_out(i) = max over i and its kept neighbours of T_in, where T_in is the
// packed tuple of the node state (FIRST) or the previous hop's result
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_mis_hop(const int* rowptr, const int* col, const uint8_t* mask,
                                                    const int* blk, int nblk, uint64_t key, const uint8_t* state,
                                                    const uint64_t* tin, uint64_t* tout) {
    __shared__ uint64_t tv[kStreamCap];
    __shared__ uint64_t tred[kBlock / 64];
    const int bid = xcd_block(nblk);
    if (bid >= nblk) return;
    const RowBlock rb = row_block(rowptr, blk, bid);
    auto tuple_at = [&](int j) -> uint64_t { return FIRST ? tuple_of(state[j], key, j) : tin[j]; };
    if (!rb.longrow) {
        // all column and mask loads first (indices past the block's end
        // clamped to its last entry), then all neighbour gathers, then the
        // stores: three memory latencies per block instead of three per
        // stride; the diagonal's own tuple is harmless
        constexpr int U = kStreamCap / kBlock;
        if (rb.cnt > 0) {
            int c[U];
            uint8_t m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = (int)threadIdx.x + u * kBlock;
                const int k = rb.k0 + (t < rb.cnt ? t : rb.cnt - 1);
                c[u] = col[k];
                m[u] = mask ? mask[k] : (uint8_t)1;
            }
            uint64_t v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = tuple_at(c[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = (int)threadIdx.x + u * kBlock;
                if (t < rb.cnt) tv[t] = m[u] ? v[u] : 0ull;
            }
        }
        __syncthreads();
        const int r = rb.r0 + (int)threadIdx.x;
        if (r < rb.r1) {
            uint64_t best = tuple_at(r);
            for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
                const uint64_t v = tv[k - rb.k0];
                best = v > best ? v : best;
            }
            tout[r] = best;
        }
    } else {
        uint64_t best = 0ull;
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) {
            const int k = rb.k0 + t;
            if (!mask || mask[k]) {
                const uint64_t v = tuple_at(col[k]);
                best = v > best ? v : best;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_down(best, off, 64);
            best = o > best ? o : best;
        }
        if ((threadIdx.x & 63) == 0) tred[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t b = tuple_at(rb.r0);
            for (int w = 0; w < kBlock / 64; ++w) b = tred[w] > b ? tred[w] : b;
            tout[rb.r0] = b;
        }
    }
}

__global__ void k_mis_update(int n, uint64_t key, const uint64_t* t2, uint8_t* state, int* undecided) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    ROW_LOOP(i, n) {
        uint8_t st = state[i];
        if (st != MIS_UND) continue;
        const uint64_t own = tuple_of(st, key, (int)i);
        const uint64_t t = t2[i];
        if (t == own) st = MIS_IN;
        else if ((t >> 62) == MIS_IN) st = MIS_OUT;
        state[i] = st;
        local += (st == MIS_UND);
    }
    if (local) atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(undecided, cnt);
}

__global__ void k_root_flags(int n, const uint8_t* state, int* flags) {
    ROW_LOOP(i, n) flags[i] = (state[i] == MIS_IN) ? 1 : 0;
}

__global__ void k_agg_phase2(int n, const int* rowptr, const int* col, const uint8_t* mask, const uint8_t* dir,
                             const uint8_t* state, const int* rank, int* phase2, int* list, int* nlist) {
    ROW_LOOP(i, n) {
        int a = -1;
        if (state[i] == MIS_IN) {
            a = rank[i];
        } else if (!(dir && dir[i])) {
            // the first kept neighbour (ascending stored order) that is a
            // root; the row is read eight entries at a time, each chunk's
            // columns and masks, then their states, loaded together.  Rows
            // longer than kLongRow are listed for k_agg_phase2_long instead.
            const int lo = rowptr[i], hi = rowptr[i + 1];
            if (hi - lo > kLongRow) {
                list[atomicAdd(nlist, 1)] = (int)i;
                continue;
            }
            int root = -1;
            for (int k0 = lo; k0 < hi && root < 0; k0 += 8) {
                int c[8];
                uint8_t m[8], st[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = min(k0 + u, hi - 1);
                    c[u] = col[k];
                    m[u] = mask ? mask[k] : (uint8_t)1;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) st[u] = state[c[u]];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (root < 0 && k0 + u < hi && c[u] != i && m[u] && st[u] == MIS_IN) root = c[u];
            }
            if (root >= 0) a = rank[root];
        }
        phase2[i] = a;
    }
}

// Phase 2 of the rows listed above, a wavefront each: the first kept
// neighbour in stored order that is a root, as the row's thread would find
// it.  Each lane takes the first match among its entries (four strides of
// columns and masks, then their states, loaded together) and the smallest
// position over the lanes wins.
__global__ void k_agg_phase2_long(const int* rowptr, const int* col, const uint8_t* mask, const uint8_t* state,
                                  const int* rank, const int* list, const int* nlist, int* phase2) {
    const int lane = threadIdx.x & 63;
    const int nl = *nlist;
    const int nw = (int)((gridDim.x * blockDim.x) >> 6);
    for (int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); w < nl; w += nw) {
        const int i = list[w];
        const int lo = rowptr[i], hi = rowptr[i + 1];
        int kf = hi;
        for (int k0 = lo + lane; k0 < hi && kf == hi; k0 += 4 * 64) {
            int c[4];
            uint8_t m[4], st[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = min(k0 + u * 64, hi - 1);
                c[u] = col[k];
                m[u] = mask ? mask[k] : (uint8_t)1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) st[u] = state[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (kf == hi && k0 + u * 64 < hi && c[u] != i && m[u] && st[u] == MIS_IN) kf = k0 + u * 64;
        }
        for (int off = 32; off > 0; off >>= 1) kf = min(kf, __shfl_xor(kf, off, 64));
        if (lane == 0) phase2[i] = kf < hi ? rank[col[kf]] : -1;
    }
}

// Phase 3: a node left unassigned by phase 2 joins the phase-2 aggregate
// that holds most of its kept neighbours (ties: smallest aggregate id).
// The first kernel settles every other node and lists the unassigned ones;
// the second gives each listed node a wavefront, which visits the distinct
// aggregates among the row's kept neighbours, counts each with ballots and
// keeps (largest count, smallest id).  The outcome of a node
// depends only on phase 2, so the list order does not matter.
// every lane with `want` set appends `value` to list (length *nlist): one
// atomic per wavefront, the lanes in lane order after the wavefront's base
__device__ __forceinline__ void wave_append(bool want, int value, int* list, int* nlist) {
    const unsigned long long m = __ballot(want);
    if (!want) return;
    const int lane = (int)(threadIdx.x & 63);
    const int leader = __builtin_ctzll(m);
    int base = 0;
    if (lane == leader) base = atomicAdd(nlist, __popcll(m));
    base = __shfl(base, leader, 64);
    list[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

__global__ void k_agg_phase3_split(int n, const uint8_t* dir, const int* phase2, int* agg, int* list, int* nlist) {
    ROW_LOOP(i, n) {
        const int a = phase2[i];
        const bool left = a < 0 && !(dir && dir[i]);
        if (!left) agg[i] = a;
        wave_append(left, (int)i, list, nlist);
    }
}

__device__ __forceinline__ int phase3_candidate(const int* col, const uint8_t* mask, const int* phase2, int i, int k,
                                                int hi) {
    if (k >= hi) return -1;
    const int j = col[k];
    if (j == i || (mask && !mask[k])) return -1;
    return phase2[j];  // -1 if j is unassigned too
}

__global__ __launch_bounds__(kBlock) void k_agg_phase3_rows(const int* rowptr, const int* col, const uint8_t* mask,
                                                            const int* phase2, const int* list, const int* nlist,
                                                            int* agg) {
    const int lane = threadIdx.x & 63;
    const int waves = (int)(gridDim.x * blockDim.x) >> 6;
    const int nl = *nlist;
    // the row and its bounds are the same in every lane; reading them through
    // the first lane keeps every loop below wave-uniform
    for (int w = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6)); w < nl;
         w += waves) {
        const int i = __builtin_amdgcn_readfirstlane(list[w]);
        const int lo = __builtin_amdgcn_readfirstlane(rowptr[i]), hi = __builtin_amdgcn_readfirstlane(rowptr[i + 1]);
        const bool one_chunk = hi - lo <= 64;
        int bestc = -1, bestn = 0;
        for (int k0 = lo; k0 < hi; k0 += 64) {
            const int c = phase3_candidate(col, mask, phase2, i, k0 + lane, hi);
            // visit each distinct candidate of this chunk once: take the lowest
            // lane still pending, count its aggregate over the whole row with
            // ballots, then retire every lane that holds the same aggregate
            uint64_t pending = __ballot(c >= 0);
            while (pending) {
                const int v = __builtin_amdgcn_readlane(c, __builtin_ctzll(pending));
                const uint64_t same = __ballot(c == v);
                int cnt = __popcll(same);
                if (!one_chunk) {
                    cnt = 0;
                    for (int k1 = lo; k1 < hi; k1 += 64)
                        cnt += __popcll(__ballot(phase3_candidate(col, mask, phase2, i, k1 + lane, hi) == v));
                }
                pending &= ~same;
                if (cnt > bestn || (cnt == bestn && v < bestc)) {
                    bestn = cnt;
                    bestc = v;
                }
            }
        }
        if (lane == 0) agg[i] = bestc;
    }
}

// ------------------------------------------------------------- prolongator
__global__ __launch_bounds__(kBlock) void k_filter_count(const int* rowptr, const int* col, const uint8_t* mask,
                                                         const int* blk, int nblk, int* cnt) {
    __shared__ int cs[kStreamCap];
    __shared__ uint8_t ms[kStreamCap];
    __shared__ int red[kBlock / 64];
    const int bid = xcd_block(nblk);
    if (bid >= nblk) return;
    const RowBlock rb = row_block(rowptr, blk, bid);
    if (!rb.longrow) {
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) {
            cs[t] = col[rb.k0 + t];
            ms[t] = mask[rb.k0 + t];
        }
        __syncthreads();
        const int r = rb.r0 + (int)threadIdx.x;
        if (r < rb.r1) {
            int c = 0;
            for (int k = rowptr[r] - rb.k0; k < rowptr[r + 1] - rb.k0; ++k) c += (cs[k] == r || ms[k]) ? 1 : 0;
            cnt[r] = c;
        }
    } else {
        int c = 0;
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) {
            const int k = rb.k0 + t;
            c += (col[k] == rb.r0 || mask[k]) ? 1 : 0;
        }
        for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) cnt[rb.r0] = red[0] + red[1] + red[2] + red[3];
    }
}

// filtered row (kept entries in order, lumped diagonal), its 1-norm, and the
// rows that are not smoothed (1-norm diagonal zero, prolongator row = the
// tentative one):
//  - isolated rows: a non-Dirichlet row whose kept off-diagonals weigh at
//    most 2^-46 of its 1-norm in A.  Its lumped diagonal is the row sum of
//    A, zero in exact arithmetic on interior rows and rounding noise of any
//    size on coarse levels, and the 1-norm scaling would turn its sign into a
//    (1 -+ omega) factor; the drop mask decides instead, reproducibly;
//  - empty rows: a filtered row whose 1-norm is at most 2^-46 of that.
// Both sums run in ascending stored order, one IEEE operation at a time.
// running state of one row's filtering (its entries may come in pieces)
struct FilterAcc {
    int p0, p, diagpos;
    double lump, rowabs, keptabs;
};

__device__ __forceinline__ FilterAcc filter_begin(int p) { return FilterAcc{p, p, -1, 0.0, 0.0, 0.0}; }

// one entry of the row, in stored order
__device__ __forceinline__ void filter_entry(int i, int j, double v, uint8_t m, FilterAcc& f, int* fcol,
                                             double* fval) {
    f.rowabs += fabs(v);
    if (j == i || m) {
        if (j == i) f.diagpos = f.p;
        else f.keptabs += fabs(v);
        fcol[f.p] = j;
        fval[f.p] = v;
        f.p++;
    } else {
        f.lump += v;
    }
}

// the row's entries lo..hi of cs/vs/ms, next in stored order; the LDS loads
// of eight entries are issued before any of them is used
__device__ __forceinline__ void filter_entries(int i, const int* cs, const double* vs, const uint8_t* ms, int lo,
                                               int hi, FilterAcc& f, int* fcol, double* fval) {
    int k = lo;
    for (; k + 8 <= hi; k += 8) {
        int j[8];
        double v[8];
        uint8_t m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            j[u] = cs[k + u];
            v[u] = vs[k + u];
            m[u] = ms[k + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) filter_entry(i, j[u], v[u], m[u], f, fcol, fval);
    }
    for (; k < hi; ++k) filter_entry(i, cs[k], vs[k], ms[k], f, fcol, fval);
}

__device__ __forceinline__ void filter_end(int i, bool dirichlet, const FilterAcc& f, double* fval, double* dt,
                                           double* dtinv) {
    if (f.diagpos >= 0) fval[f.diagpos] = fval[f.diagpos] + f.lump;
    // the filtered row read back in order, eight loads in flight at a time
    double s = 0.0;
    int q = f.p0;
    for (; q + 8 <= f.p; q += 8) {
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = fval[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += fabs(w[u]);
    }
    for (; q < f.p; ++q) s += fabs(fval[q]);
    const bool isolated = !dirichlet && !(f.keptabs > kRowNoise * f.rowabs);
    if (isolated || !(s > kRowNoise * f.rowabs)) s = 0.0;
    dt[i] = s;
    dtinv[i] = s > 0.0 ? 1.0 / s : 0.0;
}

__device__ __forceinline__ void filter_row(int i, const int* cs, const double* vs, const uint8_t* ms, int lo, int hi,
                                           int p, bool dirichlet, int* fcol, double* fval, double* dt, double* dtinv) {
    FilterAcc f = filter_begin(p);
    filter_entries(i, cs, vs, ms, lo, hi, f, fcol, fval);
    filter_end(i, dirichlet, f, fval, dt, dtinv);
}

__global__ __launch_bounds__(kBlock) void k_filter_fill(const int* rowptr, const int* col, const double* val,
                                                        const uint8_t* mask, const uint8_t* dir, const int* blk,
                                                        int nblk, const int* frowptr, int* fcol, double* fval,
                                                        double* dt, double* dtinv) {
    __shared__ int cs[kStreamCap];
    __shared__ double vs[kStreamCap];
    __shared__ uint8_t ms[kStreamCap];
    const int bid = xcd_block(nblk);
    if (bid >= nblk) return;
    const RowBlock rb = row_block(rowptr, blk, bid);
    if (!rb.longrow) {
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) {
            cs[t] = col[rb.k0 + t];
            vs[t] = val[rb.k0 + t];
            ms[t] = mask[rb.k0 + t];
        }
        __syncthreads();
        const int r = rb.r0 + (int)threadIdx.x;
        if (r < rb.r1)
            filter_row(r, cs, vs, ms, rowptr[r] - rb.k0, rowptr[r + 1] - rb.k0, frowptr[r], dir[r] != 0, fcol, fval,
                       dt, dtinv);
    } else {
        // one long row: the block stages it through LDS kStreamCap entries
        // at a time, and thread 0 filters each piece in stored order (the
        // same operations as a row of a short block)
        FilterAcc f = filter_begin(frowptr[rb.r0]);
        for (int c0 = 0; c0 < rb.cnt; c0 += kStreamCap) {
            const int cn = rb.cnt - c0 < kStreamCap ? rb.cnt - c0 : kStreamCap;
            __syncthreads();  // the previous piece has been filtered
            for (int t = threadIdx.x; t < cn; t += kBlock) {
                cs[t] = col[rb.k0 + c0 + t];
                vs[t] = val[rb.k0 + c0 + t];
                ms[t] = mask[rb.k0 + c0 + t];
            }
            __syncthreads();
            if (threadIdx.x == 0) filter_entries(rb.r0, cs, vs, ms, 0, cn, f, fcol, fval);
        }
        if (threadIdx.x == 0) filter_end(rb.r0, dir[rb.r0] != 0, f, fval, dt, dtinv);
    }
}

__global__ void k_phat_counts(int n, const int* agg, int* cnt) {
    ROW_LOOP(i, n) cnt[i] = agg[i] >= 0 ? 1 : 0;
}

__global__ void k_phat_fill(int n, const int* agg, const int* prowptr, int* pcol, double* pval) {
    ROW_LOOP(i, n) {
        if (agg[i] >= 0) {
            pcol[prowptr[i]] = agg[i];
            pval[prowptr[i]] = 1.0;
        }
    }
}

// P = P^ - omega Dt^{-1} (A_F P^), on the pattern of A_F P^
__global__ void k_prolongator_finalize(int n, const int* prowptr, const int* pcol, double* pval, const int* agg,
                                       const double* dt, double omega) {
    ROW_LOOP(i, n) {
        const double di = dt[i];
        for (int k = prowptr[i]; k < prowptr[i + 1]; ++k) {
            const double delta = (pcol[k] == agg[i]) ? 1.0 : 0.0;
            const double corr = (di > 0.0) ? (omega * pval[k]) / di : 0.0;
            pval[k] = delta - corr;
        }
    }
}

// coarse coordinates / tensors: member sums in ascending node id, one divide
__global__ void k_coarse_aux(int nc, int dim, const int* rowptr, const int* members, const double* x,
                             const double* sig, double* xc, double* sigc) {
    const int ncomp = dim * (dim + 1) / 2;
    ROW_LOOP(j, nc) {
        double ax[3] = {0, 0, 0}, as[6] = {0, 0, 0, 0, 0, 0};
        const int lo = rowptr[j], hi = rowptr[j + 1];
        for (int k = lo; k < hi; ++k) {
            const int i = members[k];
            for (int a = 0; a < dim; ++a) ax[a] += x[(size_t)i * dim + a];
            for (int c = 0; c < ncomp; ++c) as[c] += sig[(size_t)i * ncomp + c];
        }
        const double cnt = (double)(hi - lo);
        for (int a = 0; a < dim; ++a) xc[(size_t)j * dim + a] = ax[a] / cnt;
        for (int c = 0; c < ncomp; ++c) sigc[(size_t)j * ncomp + c] = as[c] / cnt;
    }
}

__global__ void k_diag_inverse(int n, const int* rowptr, const int* col, const double* val, double* dinv) {
    ROW_LOOP(i, n) {
        double d = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i) d = val[k];
        dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
    }
}

// the same over the streaming row blocks: the block's columns are staged in
// LDS with coalesced loads, then each row's thread finds its diagonal there
__global__ __launch_bounds__(kBlock) void k_diag_inverse_blocks(const int* rowptr, const int* col, const double* val,
                                                                const int* blk, int nblk, double* dinv) {
    __shared__ int cs[kStreamCap];
    const int bid = xcd_block(nblk);
    if (bid >= nblk) return;
    const RowBlock rb = row_block(rowptr, blk, bid);
    if (!rb.longrow) {
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) cs[t] = col[rb.k0 + t];
        __syncthreads();
        const int r = rb.r0 + (int)threadIdx.x;
        if (r < rb.r1) {
            double d = 0.0;
            for (int k = rowptr[r]; k < rowptr[r + 1]; ++k)
                if (cs[k - rb.k0] == r) d = val[k];
            dinv[r] = d != 0.0 ? 1.0 / d : 0.0;
        }
    } else {
        // one long row: the lane that holds the diagonal writes it (the
        // columns are distinct), after the row is set to "none"
        const int i = rb.r0;
        if (threadIdx.x == 0) dinv[i] = 0.0;
        __syncthreads();
        for (int t = threadIdx.x; t < rb.cnt; t += kBlock) {
            const int k = rb.k0 + t;
            if (col[k] == i) dinv[i] = val[k] != 0.0 ? 1.0 / val[k] : 0.0;
        }
    }
}

__global__ void k_densify(int n, const int* rowptr, const int* col, const double* val, double* D) {
    ROW_LOOP(i, n) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) D[(size_t)i * n + col[k]] = val[k];
    }
}

// *flag = 1 if any of v[0..n) is a NaN or an infinity
__global__ void k_check_finite(const double* v, int64_t n, int* flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(v[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) *flag = 1;
}

// eight lanes per row, so neighbouring lanes read neighbouring entries
__global__ void k_validate_csr(int n, const int* rowptr, const int* col, int64_t nnz, int* flag) {
    const int sub = threadIdx.x & 7;
    const int64_t groups = (int64_t)gridDim.x * (kBlock / 8);
    for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 3; i < n; i += groups) {
        const int lo = rowptr[i], hi = rowptr[i + 1];
        if (lo < 0 || hi < lo || hi > nnz) {
            *flag = 1;
            continue;
        }
        for (int k = lo + sub; k < hi; k += 8) {
            const int c = col[k];
            if (c < 0 || c >= n || (k > lo && c <= col[k - 1])) {
                *flag = 1;
                break;
            }
        }
    }
}

// flag = 1 where the two byte arrays differ
__global__ void k_bytes_differ(int n, const uint8_t* a, const uint8_t* b, int* flag) {
    ROW_LOOP(i, n) if (a[i] != b[i]) *flag = 1;
}

}  // namespace

#define LAUNCH(kern, n, ...)                                                              \
    do {                                                                                  \
        if ((n) > 0) {                                                                    \
            hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(kBlock), 0, s, __VA_ARGS__); \
            MATAMG_LAUNCH_CHECK();                                                        \
        }                                                                                 \
    } while (0)

static void finish_incidence(Incidence& out, DBuf<int>& cnt, int nt, MemCounter* mc, hipStream_t s) {
    out.rowptr.alloc((size_t)nt + 1, mc);
    DBuf<int> tmp(scan_tmp_size(nt), mc);
    exclusive_scan(cnt.get(), out.rowptr.get(), nt, tmp.get(), s);
    zero_async(cnt.get(), sizeof(int) * (size_t)(nt > 0 ? nt : 1), s);
}

void build_node_elements(const int* en, int64_t nelem, int npe, int n, Incidence& out, int* flag, MemCounter* mc,
                         hipStream_t s) {
    const int64_t total = nelem * npe;
    DBuf<int> cnt((size_t)n, mc);
    zero_async(cnt.get(), sizeof(int) * (size_t)n, s);
    LAUNCH(k_count_elem_nodes, total, en, total, n, cnt.get(), flag);
    finish_incidence(out, cnt, n, mc, s);
    out.items.alloc((size_t)(total > 0 ? total : 1), mc);
    LAUNCH(k_fill_elem_nodes, total, en, total, npe, n, out.rowptr.get(), cnt.get(), out.items.get());
    LAUNCH(k_sort_lists, n, n, out.rowptr.get(), out.items.get());
    out.ntarget = n;
}

void build_aggregate_members(const int* agg, int n, int nagg, Incidence& out, MemCounter* mc, hipStream_t s) {
    DBuf<int> cnt((size_t)(nagg > 0 ? nagg : 1), mc);
    zero_async(cnt.get(), sizeof(int) * (size_t)(nagg > 0 ? nagg : 1), s);
    LAUNCH(k_count_agg, n, agg, n, cnt.get());
    finish_incidence(out, cnt, nagg, mc, s);
    out.items.alloc((size_t)(n > 0 ? n : 1), mc);
    LAUNCH(k_fill_agg, n, agg, n, out.rowptr.get(), cnt.get(), out.items.get());
    LAUNCH(k_sort_lists, nagg, nagg, out.rowptr.get(), out.items.get());
    out.ntarget = nagg;
}

void detect_dirichlet(int n, const int* rowptr, const int* col, const double* val, uint8_t* dir, hipStream_t s) {
    LAUNCH(k_detect_dirichlet, n, n, rowptr, col, val, dir);
}

void clement(int n, int dim, const Incidence& inc, const double* es, double* sig, hipStream_t s) {
    LAUNCH(k_clement, n, n, dim, inc.rowptr.get(), inc.items.get(), es, sig);
}

void tensor_inverse(int n, int dim, const double* sig, double* minv, int* flag, hipStream_t s) {
    LAUNCH(k_tensor_inverse, n, n, dim, sig, minv, flag);
}

void soc_values(const DCsr& A, int dim, const double* x, const double* minv, const uint8_t* dir, int soc,
                double* lval, double* ldiag, hipStream_t s) {
    if (A.setup_nblk() <= 0) return;
    SocArgs a{A.rowptr.get(), A.col.get(), A.val.get(), A.setup_blk(), A.setup_nblk(), dim, soc, x, minv, dir, lval, ldiag};
    hipLaunchKernelGGL(k_soc_values, dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, a);
    MATAMG_LAUNCH_CHECK();
}

void soc_mask(const DCsr& A, const uint8_t* dir, const double* lval, const double* ldiag, double theta, double* S,
              uint8_t* mask, hipStream_t s) {
    if (A.setup_nblk() <= 0) return;
    MaskArgs a{A.rowptr.get(), A.col.get(), A.setup_blk(), A.setup_nblk(), dir, lval, ldiag, theta * theta, S, mask};
    hipLaunchKernelGGL(k_soc_mask, dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, a);
    MATAMG_LAUNCH_CHECK();
}

void cut_drop(const DCsr& A, const uint8_t* dir, const double* lval, const double* ldiag, double theta,
              uint8_t* keep, uint8_t* mask, hipStream_t s) {
    const int n = A.n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cut_keep, dim3(std::min(ceil_div(n, kBlock / 64), 8192)), dim3(kBlock), 0, s, n,
                       A.rowptr.get(), A.col.get(), dir, lval, ldiag, theta * theta, keep);
    LAUNCH(k_cut_symmetric, n, n, A.rowptr.get(), A.col.get(), (const uint8_t*)keep, mask);
}

void mis_init(int n, const uint8_t* dir, uint8_t* state, hipStream_t s) { LAUNCH(k_mis_init, n, n, dir, state); }

void mis_round(const DCsr& A, const uint8_t* mask, uint64_t key, uint8_t* state, uint64_t* t1, uint64_t* t2,
               int* undecided, hipStream_t s) {
    const int n = A.n;
    if (A.setup_nblk() > 0) {
        hipLaunchKernelGGL((k_mis_hop<true>), dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, A.rowptr.get(),
                           A.col.get(), mask, A.setup_blk(), A.setup_nblk(), key, (const uint8_t*)state, (const uint64_t*)nullptr,
                           t1);
        hipLaunchKernelGGL((k_mis_hop<false>), dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, A.rowptr.get(),
                           A.col.get(), mask, A.setup_blk(), A.setup_nblk(), key, (const uint8_t*)state, (const uint64_t*)t1,
                           t2);
        MATAMG_LAUNCH_CHECK();
    }
    LAUNCH(k_mis_update, n, n, key, t2, state, undecided);
}

void agg_root_flags(int n, const uint8_t* state, int* flags, hipStream_t s) {
    LAUNCH(k_root_flags, n, n, state, flags);
}

void agg_assign(int n, const int* rowptr, const int* col, const uint8_t* mask, const uint8_t* dir,
                const uint8_t* state, const int* root_rank, int* phase2, int* agg, int* list, int* nlist,
                hipStream_t s) {
    zero_async(nlist, sizeof(int), s);
    LAUNCH(k_agg_phase2, n, n, rowptr, col, mask, dir, state, root_rank, phase2, list, nlist);
    if (n > 0) {
        hipLaunchKernelGGL(k_agg_phase2_long, dim3(std::min(ceil_div(n, kBlock / 64), 1024)), dim3(kBlock), 0, s,
                           rowptr, col, mask, state, root_rank, (const int*)list, (const int*)nlist, phase2);
        MATAMG_LAUNCH_CHECK();
    }
    zero_async(nlist, sizeof(int), s);
    LAUNCH(k_agg_phase3_split, n, n, dir, phase2, agg, list, nlist);
    if (n > 0) {
        hipLaunchKernelGGL(k_agg_phase3_rows, dim3(std::min(ceil_div(n, kBlock / 64), 8192)), dim3(kBlock), 0, s,
                           rowptr, col, mask, phase2,
                           (const int*)list, (const int*)nlist, agg);
        MATAMG_LAUNCH_CHECK();
    }
}

void filter_count(const DCsr& A, const uint8_t* mask, int* cnt, hipStream_t s) {
    if (A.setup_nblk() <= 0) return;
    hipLaunchKernelGGL(k_filter_count, dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, A.rowptr.get(), A.col.get(), mask,
                       A.setup_blk(), A.setup_nblk(), cnt);
    MATAMG_LAUNCH_CHECK();
}

void filter_fill(const DCsr& A, const uint8_t* mask, const uint8_t* dir, const int* frowptr, int* fcol, double* fval,
                 double* dt, double* dtinv, hipStream_t s) {
    if (A.setup_nblk() <= 0) return;
    hipLaunchKernelGGL(k_filter_fill, dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, A.rowptr.get(), A.col.get(),
                       A.val.get(), mask, dir, A.setup_blk(), A.setup_nblk(), frowptr, fcol, fval, dt, dtinv);
    MATAMG_LAUNCH_CHECK();
}

void phat_counts(int n, const int* agg, int* cnt, hipStream_t s) { LAUNCH(k_phat_counts, n, n, agg, cnt); }

void phat_fill(int n, const int* agg, const int* prowptr, int* pcol, double* pval, hipStream_t s) {
    LAUNCH(k_phat_fill, n, n, agg, prowptr, pcol, pval);
}

void prolongator_finalize(int n, const int* prowptr, const int* pcol, double* pval, const int* agg,
                          const double* dt, double omega, hipStream_t s) {
    LAUNCH(k_prolongator_finalize, n, n, prowptr, pcol, pval, agg, dt, omega);
}

void coarse_aux(int nc, int dim, const Incidence& m, const double* x, const double* sig, double* xc, double* sigc,
                hipStream_t s) {
    LAUNCH(k_coarse_aux, nc, nc, dim, m.rowptr.get(), m.items.get(), x, sig, xc, sigc);
}

void diag_inverse_blocks(const DCsr& A, double* dinv, hipStream_t s) {
    if (A.setup_nblk() <= 0) return;
    hipLaunchKernelGGL(k_diag_inverse_blocks, dim3(xcd_grid(A.setup_nblk())), dim3(kBlock), 0, s, A.rowptr.get(),
                       A.col.get(), A.val.get(), A.setup_blk(), A.setup_nblk(), dinv);
    MATAMG_LAUNCH_CHECK();
}

void bytes_differ(int n, const uint8_t* a, const uint8_t* b, int* flag, hipStream_t s) {
    LAUNCH(k_bytes_differ, n, n, a, b, flag);
}

void diag_inverse(int n, const int* rowptr, const int* col, const double* val, double* dinv, hipStream_t s) {
    LAUNCH(k_diag_inverse, n, n, rowptr, col, val, dinv);
}

void densify(int n, const int* rowptr, const int* col, const double* val, double* D, hipStream_t s) {
    LAUNCH(k_densify, n, n, rowptr, col, val, D);
}

void check_finite(const double* v, int64_t n, int* flag, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_check_finite, dim3(std::min<int64_t>(ceil_div(n, kBlock), 4096)), dim3(kBlock), 0, s, v, n,
                       flag);
    MATAMG_LAUNCH_CHECK();
}

void validate_csr(int n, const int* rowptr, const int* col, int64_t nnz, int* flag, hipStream_t s) {
    LAUNCH(k_validate_csr, (int64_t)n * 8, n, rowptr, col, nnz, flag);
}

}  // namespace matamg
