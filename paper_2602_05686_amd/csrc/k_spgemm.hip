// Sparse matrix-matrix product C = A * B (Galerkin product R (A P) and the
// smoothed prolongator A_F P^) and the CSR transpose P -> R = P^T.
//
// One wavefront per output row.  The row's products are enumerated in the
// canonical order (A's row ascending, then B's row order), 64 at a time: the
// lanes scan the B-row lengths of up to 64 A-entries, then each product
// index is mapped to its (A entry, B entry) pair by a binary search over the
// scanned offsets.  Symbolic phase: product columns go into an open-addressed
// hash set in LDS (1024 slots per wave, at most 512 distinct columns); rows
// that overflow it are redone with a table in global memory sized from the
// row's product count.  Numeric phase: the products are accumulated strictly
// in canonical order, A entry after A entry (the products of one A entry
// have distinct columns and are added at once), so every entry is the same
// sequence of IEEE additions as a serial row-by-row product.  On LDS tables a
// single walk adds each product to its column's hash-slot sum and the slots
// are ranked by column (ascending output positions) afterwards; the global
// tables rank the columns first and accumulate by rank in a second walk.
// Overflow rows of at most kDBig columns run their numeric phase in a large
// LDS table shared by a workgroup's wavefronts, the others in global memory.

#pragma clang fp contract(off)

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "device_util.h"
#include "kernels.h"
#include "setup_kernels.h"

namespace matamg {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kHS = 1024;     // LDS hash slots per wave
constexpr int kDMax = 512;    // max distinct columns on the LDS path
constexpr int kHSSmall = 256; // LDS hash slots per wave for rows of at most 128 distinct columns
constexpr int kRankTile = 1024;  // LDS tile of the column list when ranking long rows
constexpr int kRankKeys = 8;     // keys per lane per ranking pass
constexpr int kDBig = 4096;      // overflow rows with at most this many columns: numeric phase in LDS
constexpr int kHSBig = 8192;     // their LDS hash slots (one workgroup per row)
// dynamic LDS of the large-table workgroup: a key, a list entry and a running sum per slot
constexpr size_t kBigLds = (sizeof(int) * 2 + sizeof(double)) * kHSBig;
// numeric phase of the wavefront path: LDS table per wavefront (rows of at
// most kDMax columns) or global-memory table (overflow rows of more than
// kDBig columns); the overflow rows in between take numeric_row_big
enum NumericMode { N_LDS = 0, N_GLOBAL = 1 };

__device__ __forceinline__ unsigned hash_slot(int key, unsigned mask) {
    return ((unsigned)key * 2654435761u) & mask;
}

// insert key; returns 1 if newly inserted, 0 if present, -1 if the table is full
__device__ __forceinline__ int hash_insert(int* keys, unsigned mask, int key) {
    unsigned h = hash_slot(key, mask);
    for (unsigned probe = 0; probe <= mask; ++probe) {
        int old = atomicCAS(keys + h, -1, key);
        if (old == -1) return 1;
        if (old == key) return 0;
        h = (h + 1) & mask;
    }
    return -1;
}

// slot of key, inserting it if absent (the table has room for every key of
// the row: at least twice as many slots)
__device__ __forceinline__ unsigned hash_insert_slot(int* keys, unsigned mask, int key) {
    unsigned h = hash_slot(key, mask);
    for (unsigned probe = 0; probe <= mask; ++probe) {
        const int old = atomicCAS(keys + h, -1, key);
        if (old == -1 || old == key) return h;
        h = (h + 1) & mask;
    }
    return 0;
}

// Enumerate the products of row i of A*B in canonical order, 64 per step
// (with stride > 1, only the steps s with s % stride == offset).
// f(valid, colB, value, t0, total, seg) is called by every lane for each step
// of 64 products starting at t0; lanes past the end get valid = false.  seg
// is the index of the product's A entry within the current chunk of 64 A
// entries: it does not decrease with the lane, and the products of one A
// entry (one B row) have distinct columns.  All cross-lane traffic uses
// shuffles, so every lane executes the same steps.  f returns whether to go
// on; its answer must be the same on every lane.
template <bool NEED_VAL, typename F>
__device__ void for_each_product(const int* arp, const int* acol, const double* aval, const int* brp,
                                 const int* bcol, const double* bval, int i, F&& f, int stride = 1, int offset = 0) {
    const int lane = threadIdx.x & 63;
    const int a0 = arp[i], a1 = arp[i + 1];
    int step = 0;  // steps of the row so far: only those with step % stride == offset are taken
    for (int c0 = a0; c0 < a1; c0 += 64) {
        const int ka = c0 + lane;
        int blen = 0, bstart = 0;
        double av = 0.0;
        if (ka < a1) {
            const int k = acol[ka];
            bstart = brp[k];
            blen = brp[k + 1] - bstart;
            if (NEED_VAL) av = aval[ka];
        }
        int incl = blen;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        const int excl = incl - blen;
        const int total = __shfl(incl, 63, 64);
        for (int t0 = 0; t0 < total; t0 += 64, ++step) {
            if (stride > 1 && step % stride != offset) continue;
            const int t = t0 + lane;
            const bool valid = t < total;
            // source = last lane whose exclusive offset is <= t (empty B rows
            // share their offset with the next non-empty one, which wins)
            int lo = 0, hi = 63;
            for (int it = 0; it < 6; ++it) {
                const int mid = (lo + hi + 1) >> 1;
                const int om = __shfl(excl, mid, 64);
                if (om <= t) lo = mid;
                else hi = mid - 1;
            }
            const int sb = __shfl(bstart, lo, 64);
            const int so = __shfl(excl, lo, 64);
            const double sa = NEED_VAL ? __shfl(av, lo, 64) : 0.0;
            int colB = 0;
            double pv = 0.0;
            if (valid) {
                const int kb = sb + (t - so);
                colB = bcol[kb];
                if (NEED_VAL) pv = sa * bval[kb];
            }
            if (!f(valid, colB, pv, t0, total, lo)) return;
        }
    }
}

// number of products of row i (sum of the B-row lengths over A's row), on every lane
__device__ __forceinline__ int row_products(const int* arp, const int* acol, const int* brp, int i) {
    const int lane = threadIdx.x & 63;
    int m = 0;
    for (int ka = arp[i] + lane; ka < arp[i + 1]; ka += 64) {
        const int k = acol[ka];
        m += brp[k + 1] - brp[k];
    }
    for (int off = 32; off > 0; off >>= 1) m += __shfl_xor(m, off, 64);
    return m;
}

// LDS table size for m keys (products in the symbolic phase, distinct
// columns in the numeric one): a power of two >= 2m, 64..kHS
__device__ __forceinline__ unsigned lds_table_mask(int m) {
    unsigned t = 64;
    while (t < 2u * (unsigned)m && t < (unsigned)kHS) t <<= 1;
    return t - 1;
}

__device__ __forceinline__ int ld_key(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Memory ordering between the phases of one wavefront's row.  A row's hash
// table (LDS, or global memory for long rows) is private to one wavefront,
// which runs on one CU: workgroup scope orders its accesses.
template <bool GLOBAL>
__device__ __forceinline__ void phase_fence() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

template <bool GLOBAL>
__device__ __forceinline__ int key_at(const int* keys, unsigned h) {
    if constexpr (GLOBAL) return ld_key(keys + h);
    else return keys[h];
}

// slot of a key known to be present; the probe count is bounded by the table size
template <bool GLOBAL>
__device__ __forceinline__ unsigned hash_find_fresh(const int* keys, unsigned mask, int key) {
    unsigned h = hash_slot(key, mask);
    for (unsigned probe = 0; probe <= mask; ++probe) {
        if (key_at<GLOBAL>(keys, h) == key) return h;
        h = (h + 1) & mask;
    }
    return 0;
}

// one row (list position ridx) of the symbolic phase, by one wavefront
template <bool GLOBAL>
__device__ void symbolic_row(int ridx, const int* rows, const int* arp, const int* acol, const int* brp,
                             const int* bcol, int* cnt, int* gkeys, const int64_t* goff, int* pcount, int dmax,
                             int* lds_keys) {
    const int lane = threadIdx.x & 63;
    const int i = rows ? rows[ridx] : ridx;
    int* keys;
    unsigned mask;
    if (GLOBAL) {
        const int64_t o = goff[ridx];
        keys = gkeys + o;
        mask = (unsigned)(goff[ridx + 1] - o) - 1;
    } else {
        keys = lds_keys;
        const int m = row_products(arp, acol, brp, i);
        if (lane == 0) pcount[i] = m;
        mask = lds_table_mask(m);
    }
    for (unsigned h = lane; h <= mask; h += 64) keys[h] = -1;
    phase_fence<GLOBAL>();
    // distinct columns so far (the same on every lane); the LDS path stops as
    // soon as the row cannot fit, so its table never fills up
    int added = 0;
    bool full = false;
    for_each_product<false>(arp, acol, nullptr, brp, bcol, nullptr, i,
                            [&](bool valid, int c, double, int, int, int) {
                                int r = 0;
                                if (valid) r = hash_insert(keys, mask, c);
                                added += __popcll(__ballot(r > 0));
                                const bool overflow = __ballot(r < 0) != 0;
                                full = full || overflow;
                                return GLOBAL || !(full || added > dmax);
                            });
    if (lane == 0) {
        if (!GLOBAL && (full || added > dmax)) cnt[i] = -1;
        else cnt[i] = added;
    }
}

// rows [0, nrows) of the list (all rows if rows is null), a wavefront per
// row, grid-stride; nrows_dev (if set) holds the row count on the device
template <bool GLOBAL>
__global__ __launch_bounds__(kBlock) void k_spgemm_symbolic(int nrows, const int* nrows_dev, const int* rows,
                                                            const int* arp, const int* acol, const int* brp,
                                                            const int* bcol, int* cnt, int* gkeys,
                                                            const int64_t* goff, int* pcount, int dmax) {
    __shared__ int skeys[GLOBAL ? 1 : kWaves][GLOBAL ? 1 : kHS];
    const int w = threadIdx.x >> 6;
    const int nr = nrows_dev ? *nrows_dev : nrows;
    for (int ridx = blockIdx.x * kWaves + w; ridx < nr; ridx += gridDim.x * kWaves)
        symbolic_row<GLOBAL>(ridx, rows, arp, acol, brp, bcol, cnt, gkeys, goff, pcount, dmax,
                             skeys[GLOBAL ? 0 : w]);
}

// one row (list position ridx) of the numeric phase, by one wavefront
template <int MODE, int HS>
__device__ void numeric_row(int ridx, const int* rows, const int* arp, const int* acol, const double* aval,
                            const int* brp, const int* bcol, const double* bval, const int* crp, int* ccol,
                            double* cval, const int* skip, int* gkeys, int* gvals, double* gacc, const int64_t* goff,
                            const int* pcount, int mlo, int mhi, int* lds_keys, int* lds_vals, double* lds_acc,
                            int* lds_tile) {
    constexpr bool GLOBAL = MODE == N_GLOBAL;
    const int lane = threadIdx.x & 63;
    const int i = rows ? rows[ridx] : ridx;
    if constexpr (MODE == N_LDS) {
        // routed by the row's distinct columns (known from the symbolic
        // phase): a table of at least twice as many slots holds them all, so
        // rows of many products but few columns take the small tables
        if (skip && skip[i]) return;
        const int dc = crp[i + 1] - crp[i];
        if (dc <= mlo || dc > mhi) return;
    } else {
        // overflow rows of up to mlo columns take the large LDS table
        if (crp[i + 1] - crp[i] <= mlo) return;
    }
    int *keys, *vals;
    double* acc;
    unsigned mask;
    if (GLOBAL) {
        const int64_t o = goff[ridx];
        keys = gkeys + o;
        vals = gvals + o;
        acc = gacc + o;
        mask = (unsigned)(goff[ridx + 1] - o) - 1;
    } else {
        keys = lds_keys;
        vals = lds_vals;
        acc = lds_acc;
        mask = lds_table_mask(crp[i + 1] - crp[i]);
    }
    if constexpr (MODE == N_LDS) {
        // One walk over the products: each takes its column's hash slot
        // (inserting the column on first sight) and is added to that slot's
        // running sum in canonical order, the segments of a step one after
        // the other as below; then the occupied slots are ranked by column
        // and written out.  Every entry receives the same additions in the
        // same order as on the two-walk path (a zeroed sum plus the first
        // product, then the others).
        for (unsigned h = lane; h <= mask; h += 64) {
            keys[h] = -1;
            acc[h] = 0.0;
        }
        phase_fence<false>();
        for_each_product<true>(arp, acol, aval, brp, bcol, bval, i,
                               [&](bool valid, int c, double pv, int t0, int total, int seg) {
                                   const unsigned h = valid ? hash_insert_slot(keys, mask, c) : 0u;
                                   const int m = min(64, total - t0);
                                   const int s0 = __shfl(seg, 0, 64), s1 = __shfl(seg, m - 1, 64);
                                   for (int sg = s0; sg <= s1; ++sg) {
                                       if (valid && seg == sg) acc[h] += pv;
                                       phase_fence<false>();
                                   }
                                   return true;
                               });
        phase_fence<false>();
        const int base = crp[i];
        const int d = crp[i + 1] - base;
        int* lst = vals;  // the row's columns, compacted (arbitrary order)
        int filled = 0;
        for (unsigned h0 = 0; h0 <= mask; h0 += 64) {
            const unsigned h = h0 + lane;
            const int key = (h <= mask) ? keys[h] : -1;
            const bool occ = key >= 0;
            const uint64_t bal = __ballot(occ);
            const int before = __popcll(bal & ((1ull << lane) - 1ull));
            if (occ && filled + before < d) lst[filled + before] = key;
            filled += __popcll(bal);
        }
        phase_fence<false>();
        for (int e = lane; e < d; e += 64) {
            const int c = lst[e];
            int r = 0;
            for (int q = 0; q < d; ++q) r += (lst[q] < c);
            ccol[base + r] = c;
            cval[base + r] = acc[hash_find_fresh<false>(keys, mask, c)];
        }
        phase_fence<false>();  // the tables are reused by the wavefront's next row
        return;
    }
    for (unsigned h = lane; h <= mask; h += 64) {
        keys[h] = -1;
        vals[h] = 0;
    }
    phase_fence<GLOBAL>();
    for_each_product<false>(arp, acol, nullptr, brp, bcol, nullptr, i,
                            [&](bool valid, int c, double, int, int, int) {
                                if (valid) (void)hash_insert(keys, mask, c);
                                return true;
                            });
    phase_fence<GLOBAL>();
    // compact the occupied slots (arbitrary order): into LDS on the LDS path
    // (the accumulator's space, unused until the ranks are known), into the
    // output column range otherwise
    const int base = crp[i];
    const int d = crp[i + 1] - base;
    int* cl = ccol + base;
    int* lst = GLOBAL ? cl : reinterpret_cast<int*>(acc);
    int filled = 0;
    for (unsigned h0 = 0; h0 <= mask; h0 += 64) {
        const unsigned h = h0 + lane;
        const int key = (h <= mask) ? key_at<GLOBAL>(keys, h) : -1;
        const bool occ = key >= 0;
        const uint64_t bal = __ballot(occ);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (occ && filled + before < d) lst[filled + before] = key;
        filled += __popcll(bal);
    }
    phase_fence<GLOBAL>();
    // rank of each column among the row's columns = its output position
    if constexpr (MODE == N_LDS) {
        for (int e = lane; e < d; e += 64) {
            const int c = lst[e];
            int r = 0;
            for (int q = 0; q < d; ++q) r += (lst[q] < c);
            vals[hash_find_fresh<GLOBAL>(keys, mask, c)] = r;
        }
    } else {
        // long rows: kRankKeys keys per lane at a time, compared against the
        // list staged through LDS in tiles
        int* tile = lds_tile;
        for (int e0 = 0; e0 < d; e0 += 64 * kRankKeys) {
            int c[kRankKeys], r[kRankKeys];
#pragma unroll
            for (int u = 0; u < kRankKeys; ++u) {
                const int e = e0 + u * 64 + lane;
                c[u] = e < d ? lst[e] : -1;
                r[u] = 0;
            }
            for (int t0 = 0; t0 < d; t0 += kRankTile) {
                const int tn = min(kRankTile, d - t0);
                for (int q = lane; q < tn; q += 64) tile[q] = lst[t0 + q];
                phase_fence<false>();
                for (int q = 0; q < tn; ++q) {
                    const int v = tile[q];
#pragma unroll
                    for (int u = 0; u < kRankKeys; ++u) r[u] += (v < c[u]) ? 1 : 0;
                }
                phase_fence<false>();
            }
#pragma unroll
            for (int u = 0; u < kRankKeys; ++u)
                if (c[u] >= 0) vals[hash_find_fresh<GLOBAL>(keys, mask, c[u])] = r[u];
        }
    }
    phase_fence<GLOBAL>();
    for (unsigned h = lane; h <= mask; h += 64) {
        const int key = key_at<GLOBAL>(keys, h);
        const int r = vals[h];
        if (key >= 0 && r >= 0 && r < d) cl[r] = key;
    }
    for (int e = lane; e < d; e += 64) acc[e] = 0.0;
    phase_fence<GLOBAL>();
    // Accumulate in canonical product order.  The products of one A entry
    // (a segment) have distinct columns, so a segment's lanes add their
    // products to their columns' running values at once; the segments of a
    // step go one after the other in order, and steps follow each other in
    // product order.  Every entry therefore receives exactly the sequence of
    // additions of a serial row product.
    for_each_product<true>(arp, acol, aval, brp, bcol, bval, i,
                           [&](bool valid, int c, double pv, int t0, int total, int seg) {
                               int r = valid ? vals[hash_find_fresh<GLOBAL>(keys, mask, c)] : 0;
                               r = (r >= 0 && r < d) ? r : 0;
                               const int m = min(64, total - t0);
                               const int s0 = __shfl(seg, 0, 64), s1 = __shfl(seg, m - 1, 64);
                               for (int sg = s0; sg <= s1; ++sg) {
                                   if (valid && seg == sg) acc[r] += pv;
                                   phase_fence<GLOBAL>();
                               }
                               return true;
                           });
    phase_fence<GLOBAL>();
    for (int e = lane; e < d; e += 64) cval[base + e] = acc[e];
}

// LDS path (N_LDS): the rows of the list whose distinct column count lies in
// (mlo, mhi] and that did not overflow (skip), with HS >= 2 * mhi hash slots
// per wave; N_GLOBAL: the listed overflow rows with
// more than mlo (at most kDBig) columns.  A wavefront per row, grid-stride; nrows_dev (if
// set) holds the count.
template <int MODE, int HS>
__global__ __launch_bounds__(kBlock) void k_spgemm_numeric(int nrows, const int* nrows_dev, const int* rows,
                                                           const int* arp, const int* acol, const double* aval,
                                                           const int* brp, const int* bcol, const double* bval,
                                                           const int* crp, int* ccol, double* cval, const int* skip,
                                                           int* gkeys, int* gvals, double* gacc,
                                                           const int64_t* goff, const int* pcount, int mlo, int mhi) {
    constexpr bool GLOBAL = MODE == N_GLOBAL;
    __shared__ int skeys[GLOBAL ? 1 : kWaves][GLOBAL ? 1 : HS];
    __shared__ int svals[GLOBAL ? 1 : kWaves][GLOBAL ? 1 : HS];
    __shared__ double sacc[GLOBAL ? 1 : kWaves][GLOBAL ? 1 : HS];  // one running sum per hash slot
    __shared__ int stile[GLOBAL ? kWaves : 1][GLOBAL ? kRankTile : 1];
    const int w = threadIdx.x >> 6;
    const int nr = nrows_dev ? *nrows_dev : nrows;
    for (int ridx = blockIdx.x * kWaves + w; ridx < nr; ridx += gridDim.x * kWaves)
        numeric_row<MODE, HS>(ridx, rows, arp, acol, aval, brp, bcol, bval, crp, ccol, cval, skip, gkeys, gvals,
                              gacc, goff, pcount, mlo, mhi, skeys[GLOBAL ? 0 : w], svals[GLOBAL ? 0 : w],
                              sacc[GLOBAL ? 0 : w], stile[GLOBAL ? w : 0]);
}

// Overflow row i with at most kDBig columns, by a whole workgroup of kWaves
// wavefronts on one table in LDS.  Within each chunk of 64 A entries the
// wavefronts take the chunk's steps of 64 products in turn (wavefront w the
// steps w, w + kWaves, ...): in a round each loads its step's products and
// takes their columns' hash slots (inserting a column on first sight), then
// the round's steps are added to the slots' running sums in step order, one
// wavefront after the other between barriers, each step's segments one
// after the other.  Every entry thus receives the additions of a serial row
// product in the same order (a zeroed sum plus the first product, then the
// others), while kWaves steps' loads are in flight at once.  The occupied
// slots are then ranked by column and written out.
__device__ void numeric_row_big(int i, const int* arp, const int* acol, const double* aval, const int* brp,
                                const int* bcol, const double* bval, const int* crp, int* ccol, double* cval,
                                int* keys, int* vals, double* acc) {
    const int tid = (int)threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int base = crp[i];
    const int d = crp[i + 1] - base;
    unsigned tsz = 64;
    while (tsz < 2u * (unsigned)d) tsz <<= 1;
    const unsigned mask = tsz - 1;
    for (unsigned h = tid; h <= mask; h += kBlock) {
        keys[h] = -1;
        acc[h] = 0.0;
    }
    __syncthreads();
    const int a0 = arp[i], a1 = arp[i + 1];
    for (int c0 = a0; c0 < a1; c0 += 64) {
        const int ka = c0 + lane;
        int blen = 0, bstart = 0;
        double av = 0.0;
        if (ka < a1) {
            const int k = acol[ka];
            bstart = brp[k];
            blen = brp[k + 1] - bstart;
            av = aval[ka];
        }
        int incl = blen;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        const int excl = incl - blen;
        const int total = __shfl(incl, 63, 64);
        const int nsteps = (total + 63) / 64;  // the same in every wavefront
        for (int sr = 0; sr < nsteps; sr += kWaves) {
            const int st = sr + w;
            const int t0 = st * 64;
            const int t = t0 + lane;
            const bool valid = st < nsteps && t < total;
            // source A entry of product t: the last lane whose exclusive
            // offset is <= t (empty B rows lose to the next non-empty one)
            int lo = 0, hi = 63;
            for (int it = 0; it < 6; ++it) {
                const int mid = (lo + hi + 1) >> 1;
                const int om = __shfl(excl, mid, 64);
                if (om <= t) lo = mid;
                else hi = mid - 1;
            }
            const int sb = __shfl(bstart, lo, 64);
            const int so = __shfl(excl, lo, 64);
            const double sa = __shfl(av, lo, 64);
            unsigned h = 0;
            double pv = 0.0;
            if (valid) {
                const int kb = sb + (t - so);
                h = hash_insert_slot(keys, mask, bcol[kb]);
                pv = sa * bval[kb];
            }
            const int m = st < nsteps ? min(64, total - t0) : 0;
            const int s0 = __shfl(lo, 0, 64), s1 = __shfl(lo, m > 0 ? m - 1 : 0, 64);
            for (int q = 0; q < kWaves; ++q) {
                if (q == w && m > 0) {
                    for (int sg = s0; sg <= s1; ++sg) {
                        if (valid && lo == sg) acc[h] += pv;
                        phase_fence<false>();
                    }
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    // compact the occupied slots' columns (wavefront 0)
    int* lst = vals;
    if (w == 0) {
        int filled = 0;
        for (unsigned h0 = 0; h0 <= mask; h0 += 64) {
            const unsigned h = h0 + lane;
            const int key = (h <= mask) ? keys[h] : -1;
            const bool occ = key >= 0;
            const uint64_t bal = __ballot(occ);
            const int before = __popcll(bal & ((1ull << lane) - 1ull));
            if (occ && filled + before < d) lst[filled + before] = key;
            filled += __popcll(bal);
        }
    }
    __syncthreads();
    // ranks: kRankKeys keys per lane at a time, the wavefronts taking turns;
    // each column goes to its rank's output position with its slot's sum
    for (int e0 = w * 64 * kRankKeys; e0 < d; e0 += kWaves * 64 * kRankKeys) {
        int c[kRankKeys], r[kRankKeys];
#pragma unroll
        for (int u = 0; u < kRankKeys; ++u) {
            const int e = e0 + u * 64 + lane;
            c[u] = e < d ? lst[e] : -1;
            r[u] = 0;
        }
        for (int q = 0; q < d; ++q) {
            const int v = lst[q];
#pragma unroll
            for (int u = 0; u < kRankKeys; ++u) r[u] += (v < c[u]) ? 1 : 0;
        }
#pragma unroll
        for (int u = 0; u < kRankKeys; ++u)
            if (c[u] >= 0 && r[u] < d) {
                ccol[base + r[u]] = c[u];
                cval[base + r[u]] = acc[hash_find_fresh<false>(keys, mask, c[u])];
            }
    }
    __syncthreads();  // the tables are reused by the workgroup's next row
}

// the listed overflow rows with at most kDBig columns: a workgroup per row,
// with a kHSBig-slot hash table and one running sum per slot in 128 KB of
// dynamic LDS
__global__ __launch_bounds__(kBlock) void k_spgemm_numeric_big(int nrows, const int* rows, const int* arp,
                                                               const int* acol, const double* aval, const int* brp,
                                                               const int* bcol, const double* bval, const int* crp,
                                                               int* ccol, double* cval, int dbig) {
    extern __shared__ __align__(16) unsigned char big_lds[];
    double* sacc = reinterpret_cast<double*>(big_lds);
    int* skeys = reinterpret_cast<int*>(sacc + kHSBig);
    int* svals = skeys + kHSBig;
    for (int ridx = blockIdx.x; ridx < nrows; ridx += gridDim.x) {
        const int i = rows[ridx];
        if (crp[i + 1] - crp[i] > dbig) continue;  // block-uniform
        numeric_row_big(i, arp, acol, aval, brp, bcol, bval, crp, ccol, cval, skeys, svals, sacc);
    }
}

// --------------------------------------------------- one thread per row
// Rows with at most kThreadCols distinct output columns (most rows of the
// finer levels' products) are multiplied by one thread each: the thread walks
// its row's products in the canonical order and keeps the distinct columns,
// in order of first appearance, in registers with their running sums; the
// sorted output position of each is its rank among them.  Every entry
// therefore gets the same additions, in the same order, as on the wavefront
// path.  A row with more than kThreadProducts products takes the wavefront
// path even when its columns would fit: each product costs a thread a
// compare against every register slot, a wavefront one hash probe per lane
// (the coarse levels' Galerkin rows collapse hundreds of products into few
// columns).
constexpr int kThreadCols = 32;
constexpr int kThreadProducts = 64;
constexpr int kThreadRow = -3;  // pcount marker of a row on the thread path

// add product (c, v) to the row's column list key/acc[0..d) of S slots (v
// when VAL); returns false when a new column does not fit
template <bool VAL, int S>
__device__ __forceinline__ bool thread_row_add(int (&key)[S], double (&acc)[S], int& d, int c, double v) {
    bool found = false;
#pragma unroll
    for (int j = 0; j < S; ++j)
        if (key[j] == c) {
            found = true;
            if constexpr (VAL) acc[j] += v;
        }
    if (found) return true;
    if (d == S) return false;
#pragma unroll
    for (int j = 0; j < S; ++j)
        if (j == d) {
            key[j] = c;
            if constexpr (VAL) acc[j] = 0.0 + v;  // as the wavefront path: a zeroed sum plus the first product
        }
    ++d;
    return true;
}

// the products of row i in canonical order, f(column, value): A's row in
// chunks of CH entries whose column, B-row bounds and first B entry are all
// loaded before any is used (P rows mostly hold one entry), so a chunk costs
// three memory latencies instead of three per entry.  f returns whether to
// go on.
template <bool VAL, int CH, typename F>
__device__ __forceinline__ void thread_row_products(const int* arp, const int* acol, const double* aval,
                                                    const int* brp, const int* bcol, const double* bval, int i,
                                                    F&& f) {
    const int a0 = arp[i], a1 = arp[i + 1];
    for (int c0 = a0; c0 < a1; c0 += CH) {
        int kk[CH], b0[CH], b1[CH], fc[CH];
        double av[CH], fv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int ka = min(c0 + u, a1 - 1);
            kk[u] = acol[ka];
            av[u] = VAL ? aval[ka] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            b0[u] = brp[kk[u]];
            b1[u] = brp[kk[u] + 1];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int kb = b0[u] < b1[u] ? b0[u] : 0;
            fc[u] = bcol[kb];
            fv[u] = VAL ? bval[kb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (c0 + u >= a1 || b0[u] >= b1[u]) continue;
            if (!f(fc[u], VAL ? av[u] * fv[u] : 0.0)) return;
            for (int kb = b0[u] + 1; kb < b1[u]; ++kb)
                if (!f(bcol[kb], VAL ? av[u] * bval[kb] : 0.0)) return;
        }
    }
}

// symbolic: cnt[i] = distinct columns and pcount[i] = kThreadRow for rows
// that fit (at most kThreadCols columns from at most kThreadProducts
// products); wide[i] = 1 (and cnt[i] untouched) for the others, whose walk
// stops where they stop fitting
__global__ __launch_bounds__(kBlock) void k_spgemm_symbolic_thread(int n, const int* arp, const int* acol,
                                                                   const int* brp, const int* bcol, int* cnt,
                                                                   int* pcount, int* wide, int tprod) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int key[kThreadCols];
        double acc[kThreadCols];
#pragma unroll
        for (int j = 0; j < kThreadCols; ++j) key[j] = -1;
        int d = 0, m = 0;
        bool fits = true;
        thread_row_products<false, 8>(arp, acol, nullptr, brp, bcol, nullptr, i, [&](int c, double) {
            fits = ++m <= tprod && thread_row_add<false, kThreadCols>(key, acc, d, c, 0.0);
            return fits;
        });
        wide[i] = fits ? 0 : 1;
        if (fits) {
            cnt[i] = d;
            pcount[i] = kThreadRow;
        }
    }
}

// numeric for the rows the thread symbolic pass kept whose column count
// lies in (dlo, S], with S register slots (fewer slots for narrower rows:
// fewer registers and compares per product; the additions are the same)
template <int S>
__global__ __launch_bounds__(kBlock) void k_spgemm_numeric_thread(int n, const int* arp, const int* acol,
                                                                  const double* aval, const int* brp,
                                                                  const int* bcol, const double* bval,
                                                                  const int* pcount, const int* crp, int* ccol,
                                                                  double* cval, int dlo) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (pcount[i] != kThreadRow) continue;
        const int base = crp[i];
        const int dr = crp[i + 1] - base;
        if (dr <= dlo || dr > S) continue;
        int key[S];
        double acc[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            key[j] = -1;
            acc[j] = 0.0;
        }
        int d = 0;
        thread_row_products<true, 4>(arp, acol, aval, brp, bcol, bval, i, [&](int c, double v) {
            (void)thread_row_add<true, S>(key, acc, d, c, v);
            return true;
        });
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (key[j] < 0) continue;
            int r = 0;
#pragma unroll
            for (int q = 0; q < S; ++q) r += (key[q] >= 0 && key[q] < key[j]) ? 1 : 0;
            ccol[base + r] = key[j];
            cval[base + r] = acc[j];
        }
    }
}

__global__ void k_list_flagged(int n, const int* flags, const int* pos, int* list) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (flags[i]) list[pos[i]] = i;
}

// product-count upper bound of each listed row, as a hash table size (power
// of two >= 2*m): a wavefront per row, lane-strided over its A entries
__global__ __launch_bounds__(kBlock) void k_row_table_size(int nrows, const int* rows, const int* arp,
                                                           const int* acol, const int* brp, int ncols,
                                                           int64_t* size) {
    const int w = (int)threadIdx.x >> 6;
    for (int r = blockIdx.x * kWaves + w; r < nrows; r += gridDim.x * kWaves) {
        int64_t m = row_products(arp, acol, brp, rows[r]);
        if (m > ncols) m = ncols;
        int64_t t = 64;
        while (t < 2 * m) t <<= 1;
        if ((threadIdx.x & 63) == 0) size[r] = t;
    }
}

// flags[i] = row i overflowed the LDS table; cntc[i] = its count, 0 if it did
__global__ void k_overflow_flags(int n, const int* cnt, int* flags, int* cntc) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        flags[i] = cnt[i] < 0 ? 1 : 0;
        cntc[i] = cnt[i] < 0 ? 0 : cnt[i];
    }
}

// out = {*a, *b}, for one read-back of two device values
__global__ void k_pair(const int* a, const int* b, int* out) {
    out[0] = *a;
    out[1] = *b;
}

__global__ void k_overflow_list(int n, const int* flags, const int* pos, int* list) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (flags[i]) list[pos[i]] = i;
}

// exclusive scan of n 64-bit values by one block, kBlock at a time with a
// running carry (overflow rows are few)
__global__ __launch_bounds__(kBlock) void k_scan64(int n, const int64_t* in, int64_t* out) {
    __shared__ int64_t sh[kBlock];
    int64_t carry = 0;
    for (int b = 0; b < n; b += kBlock) {
        const int i = b + (int)threadIdx.x;
        const int64_t v = i < n ? in[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        // inclusive Hillis-Steele scan in LDS
        for (int off = 1; off < kBlock; off <<= 1) {
            const int64_t y = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < n) out[i] = carry + sh[threadIdx.x] - v;
        carry += sh[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// ---------------------------------------------------------------- transpose
__global__ void k_col_counts(int64_t nnz, const int* col, int* cnt) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(cnt + col[k], 1);
}

// the transpose's entries, in the order the atomic slots hand out within
// each row, with each entry's row
__global__ void k_transpose_fill(int n, const int* rp, const int* col, const double* val, const int* trp,
                                 int* fill, int* tcol, double* tval, int* trow) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int c = col[k];
            const int p = trp[c] + atomicAdd(fill + c, 1);
            tcol[p] = i;
            tval[p] = val[k];
            trow[p] = c;
        }
    }
}

// Rows of the transpose up to this long are put in column order by ranking;
// longer ones are sorted in place afterwards
constexpr int kRankRow = 256;

// Each entry to its place in column order.  A row's columns (the source
// rows) are distinct, so an entry's place is the number of the row's
// columns below its own: one thread per entry, reading the row with
// independent loads.  Entries of longer rows are copied where they are.
__global__ void k_rank_place(int64_t nnz, const int* trp, const int* trow, const int* tcol, const double* tval,
                             int* col, double* val) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = trow[e];
        const int lo = trp[j], hi = trp[j + 1];
        const int c = tcol[e];
        int64_t pos = e;
        if (hi - lo <= kRankRow) {
            int r = 0;
            for (int k = lo; k < hi; ++k) r += tcol[k] < c ? 1 : 0;
            pos = lo + r;
        }
        col[pos] = c;
        val[pos] = tval[e];
    }
}

// insertion sort of the rows longer than kRankRow, one thread per row
__global__ void k_sort_pairs(int n, const int* rp, int* col, double* val) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int lo = rp[i], hi = rp[i + 1];
        if (hi - lo <= kRankRow) continue;
        for (int a = lo + 1; a < hi; ++a) {
            const int c = col[a];
            const double v = val[a];
            int b = a - 1;
            while (b >= lo && col[b] > c) {
                col[b + 1] = col[b];
                val[b + 1] = val[b];
                --b;
            }
            col[b + 1] = c;
            val[b + 1] = v;
        }
    }
}

inline int g1(int64_t n) {
    int g = ceil_div(n > 0 ? n : 1, kBlock);
    return g < 65535 ? g : 65535;
}

// The rows' routes: at most tprod products (and kThreadCols columns) for one
// thread, at most dmax columns for a wavefront's LDS table, at most dbig for
// a workgroup's, a global-memory table beyond.  MATAMG_SPGEMM_ROUTE=t,d,b
// lowers them (the tests send rows down every path: every route adds the
// same products in the same order).
struct Route {
    int tprod = kThreadProducts, dmax = kDMax, dbig = kDBig;
};

Route spgemm_route() {
    Route r;
    const char* e = std::getenv("MATAMG_SPGEMM_ROUTE");
    int t = 0, d = 0, b = 0;
    if (e && std::sscanf(e, "%d,%d,%d", &t, &d, &b) == 3) {
        r.tprod = std::max(0, std::min(t, kThreadProducts));
        r.dmax = std::max(0, std::min(d, kDMax));
        r.dbig = std::max(0, std::min(b, kDBig));
    }
    return r;
}

}  // namespace

void spgemm(const DCsr& A, const DCsr& B, DCsr& C, MemCounter* mc, hipStream_t s) {
    const Route route = spgemm_route();
    const int n = A.n;
    C.n = n;
    C.m = B.m;
    const int nn = n > 0 ? n : 1;
    DBuf<int> cnt((size_t)nn, mc), flags((size_t)nn, mc), pos((size_t)n + 1, mc), pcount((size_t)nn, mc);
    // cntc also takes the pair {overflow rows, stored entries} read back below
    DBuf<int> wide((size_t)nn, mc), wpos((size_t)n + 1, mc), wl((size_t)nn, mc), cntc((size_t)std::max(nn, 2), mc);
    DBuf<int> tmp(scan_tmp_size(n), mc);
    C.rowptr.alloc((size_t)n + 1, mc);
    // wavefront launches loop over a row list whose length stays on the device
    const int wgrid = std::max(1, std::min(ceil_div(nn, kWaves), 8192));
    const int* nwide_dev = wpos.get() + n;
    if (n > 0) {
        // one thread per row where at most kThreadCols columns come out; the
        // remaining (wide) rows take a wavefront each
        hipLaunchKernelGGL(k_spgemm_symbolic_thread, dim3(g1(n)), dim3(kBlock), 0, s, n, A.rowptr.get(),
                           A.col.get(), B.rowptr.get(), B.col.get(), cnt.get(), pcount.get(), wide.get(), route.tprod);
        exclusive_scan(wide.get(), wpos.get(), n, tmp.get(), s);
        hipLaunchKernelGGL(k_list_flagged, dim3(g1(n)), dim3(kBlock), 0, s, n, (const int*)wide.get(),
                           (const int*)wpos.get(), wl.get());
        hipLaunchKernelGGL((k_spgemm_symbolic<false>), dim3(wgrid), dim3(kBlock), 0, s, 0, nwide_dev,
                           (const int*)wl.get(), A.rowptr.get(), A.col.get(), B.rowptr.get(), B.col.get(), cnt.get(),
                           (int*)nullptr, (const int64_t*)nullptr, pcount.get(), route.dmax);
        // overflow flags, and the row pointer as if no row overflowed
        hipLaunchKernelGGL(k_overflow_flags, dim3(g1(n)), dim3(kBlock), 0, s, n, (const int*)cnt.get(), flags.get(),
                           cntc.get());
        MATAMG_LAUNCH_CHECK();
    }
    exclusive_scan(flags.get(), pos.get(), n, tmp.get(), s);
    exclusive_scan(cntc.get(), C.rowptr.get(), n, tmp.get(), s);
    int head[2] = {0, 0};  // overflow rows, stored entries
    hipLaunchKernelGGL(k_pair, dim3(1), dim3(1), 0, s, (const int*)pos.get() + n, (const int*)C.rowptr.get() + n,
                       cntc.get());
    d2h(head, cntc.get(), 2, s);
    const int novf = head[0];
    int nnz = head[1];
    DBuf<int> list;
    DBuf<int64_t> tsize, toff;
    DBuf<int> gkeys, gvals;
    DBuf<double> gacc;
    if (novf > 0) {
        // rows with more distinct columns than the LDS table holds
        list.alloc((size_t)novf, mc);
        hipLaunchKernelGGL(k_overflow_list, dim3(g1(n)), dim3(kBlock), 0, s, n, flags.get(), pos.get(), list.get());
        tsize.alloc((size_t)novf, mc);
        toff.alloc((size_t)novf + 1, mc);
        hipLaunchKernelGGL(k_row_table_size, dim3(std::min(ceil_div(novf, kWaves), 8192)), dim3(kBlock), 0, s, novf,
                           list.get(), A.rowptr.get(), A.col.get(), B.rowptr.get(), B.m, tsize.get());
        hipLaunchKernelGGL(k_scan64, dim3(1), dim3(kBlock), 0, s, novf, tsize.get(), toff.get());
        int64_t tot = 0;
        d2h(&tot, toff.get() + novf, 1, s);
        gkeys.alloc((size_t)tot, mc);
        gvals.alloc((size_t)tot, mc);
        gacc.alloc((size_t)tot, mc);
        hipLaunchKernelGGL((k_spgemm_symbolic<true>), dim3(ceil_div(novf, kWaves)), dim3(kBlock), 0, s, novf,
                           (const int*)nullptr, list.get(), A.rowptr.get(), A.col.get(), B.rowptr.get(), B.col.get(),
                           cnt.get(), gkeys.get(), toff.get(), (int*)nullptr, route.dmax);
        MATAMG_LAUNCH_CHECK();
        exclusive_scan(cnt.get(), C.rowptr.get(), n, tmp.get(), s);
        d2h(&nnz, C.rowptr.get() + n, 1, s);
    }
    C.nnz = nnz;
    C.col.alloc((size_t)(nnz > 0 ? nnz : 1), mc);
    C.val.alloc((size_t)(nnz > 0 ? nnz : 1), mc);
    if (n > 0) {
        hipLaunchKernelGGL(k_spgemm_numeric_thread<kThreadCols / 2>, dim3(g1(n)), dim3(kBlock), 0, s, n,
                           A.rowptr.get(), A.col.get(), A.val.get(), B.rowptr.get(), B.col.get(), B.val.get(),
                           (const int*)pcount.get(), C.rowptr.get(), C.col.get(), C.val.get(), -1);
        hipLaunchKernelGGL(k_spgemm_numeric_thread<kThreadCols>, dim3(g1(n)), dim3(kBlock), 0, s, n, A.rowptr.get(),
                           A.col.get(), A.val.get(), B.rowptr.get(), B.col.get(), B.val.get(),
                           (const int*)pcount.get(), C.rowptr.get(), C.col.get(), C.val.get(), kThreadCols / 2);
        // wide rows with few distinct columns: small tables, so more
        // wavefronts fit a CU
        hipLaunchKernelGGL((k_spgemm_numeric<N_LDS, kHSSmall>), dim3(wgrid), dim3(kBlock), 0, s, 0, nwide_dev,
                           (const int*)wl.get(), A.rowptr.get(), A.col.get(), A.val.get(), B.rowptr.get(), B.col.get(),
                           B.val.get(), C.rowptr.get(), C.col.get(), C.val.get(), (const int*)flags.get(),
                           (int*)nullptr, (int*)nullptr, (double*)nullptr, (const int64_t*)nullptr,
                           (const int*)pcount.get(), -1, kHSSmall / 2);
        hipLaunchKernelGGL((k_spgemm_numeric<N_LDS, kHS>), dim3(wgrid), dim3(kBlock), 0, s, 0, nwide_dev,
                           (const int*)wl.get(), A.rowptr.get(), A.col.get(), A.val.get(), B.rowptr.get(), B.col.get(),
                           B.val.get(), C.rowptr.get(), C.col.get(), C.val.get(), (const int*)flags.get(),
                           (int*)nullptr, (int*)nullptr, (double*)nullptr, (const int64_t*)nullptr,
                           (const int*)pcount.get(), kHSSmall / 2, 0x7fffffff);
        MATAMG_LAUNCH_CHECK();
    }
    if (novf > 0) {
        // the dynamic LDS limit, raised once per process (thread-safe static)
        static const bool big_lds_set = [] {
            MATAMG_HIP(hipFuncSetAttribute((const void*)k_spgemm_numeric_big,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBigLds));
            return true;
        }();
        (void)big_lds_set;
        hipLaunchKernelGGL(k_spgemm_numeric_big, dim3(std::min(novf, 4096)), dim3(kBlock), kBigLds, s, novf,
                           (const int*)list.get(), A.rowptr.get(), A.col.get(), A.val.get(), B.rowptr.get(),
                           B.col.get(), B.val.get(), (const int*)C.rowptr.get(), C.col.get(), C.val.get(),
                           route.dbig);
        hipLaunchKernelGGL((k_spgemm_numeric<N_GLOBAL, 1>), dim3(ceil_div(novf, kWaves)), dim3(kBlock), 0, s, novf,
                           (const int*)nullptr, list.get(), A.rowptr.get(), A.col.get(), A.val.get(), B.rowptr.get(),
                           B.col.get(), B.val.get(), C.rowptr.get(), C.col.get(), C.val.get(), (const int*)nullptr,
                           gkeys.get(), gvals.get(), gacc.get(), toff.get(), (const int*)nullptr, route.dbig, 0);
        MATAMG_LAUNCH_CHECK();
    }
    // no synchronisation: temporaries go back to the pool in stream order
}

void transpose(const DCsr& A, DCsr& T, MemCounter* mc, hipStream_t s) {
    const int n = A.n, m = A.m;
    T.n = m;
    T.m = n;
    T.nnz = A.nnz;
    DBuf<int> cnt((size_t)(m > 0 ? m : 1), mc);
    zero_async(cnt.get(), sizeof(int) * (size_t)(m > 0 ? m : 1), s);
    if (A.nnz > 0)
        hipLaunchKernelGGL(k_col_counts, dim3(g1(A.nnz)), dim3(kBlock), 0, s, A.nnz, A.col.get(), cnt.get());
    T.rowptr.alloc((size_t)m + 1, mc);
    DBuf<int> tmp(scan_tmp_size(m), mc);
    exclusive_scan(cnt.get(), T.rowptr.get(), m, tmp.get(), s);
    zero_async(cnt.get(), sizeof(int) * (size_t)(m > 0 ? m : 1), s);
    const size_t nz = (size_t)(A.nnz > 0 ? A.nnz : 1);
    T.col.alloc(nz, mc);
    T.val.alloc(nz, mc);
    DBuf<int> tcol(nz, mc), trow(nz, mc);
    DBuf<double> tval(nz, mc);
    if (n > 0)
        hipLaunchKernelGGL(k_transpose_fill, dim3(g1(n)), dim3(kBlock), 0, s, n, A.rowptr.get(), A.col.get(),
                           A.val.get(), T.rowptr.get(), cnt.get(), tcol.get(), tval.get(), trow.get());
    if (A.nnz > 0)
        hipLaunchKernelGGL(k_rank_place, dim3(g1(A.nnz)), dim3(kBlock), 0, s, A.nnz, (const int*)T.rowptr.get(),
                           (const int*)trow.get(), (const int*)tcol.get(), (const double*)tval.get(), T.col.get(),
                           T.val.get());
    if (m > 0)
        hipLaunchKernelGGL(k_sort_pairs, dim3(g1(m)), dim3(kBlock), 0, s, m, T.rowptr.get(), T.col.get(),
                           T.val.get());
    MATAMG_LAUNCH_CHECK();
}

}  // namespace matamg
