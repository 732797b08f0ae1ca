// Host-side launchers of the library's HIP kernels (gfx950, wave64).
#pragma once

#include "common.h"

namespace matamg {

// ----------------------------------------------------------------- prims ---
// exclusive scan of `n` int32 counts into out[0..n]; out[n] = total.
// `tmp` must hold scan_tmp_size(n) ints.  Returns nothing; total stays on device.
size_t scan_tmp_size(int64_t n);
void exclusive_scan(const int* in, int* out, int64_t n, int* tmp, hipStream_t s);
// bytes zero bytes at p, by a kernel on s (cheaper to issue than a runtime memset)
void zero_async(void* p, size_t bytes, hipStream_t s);

// deterministic dot product sum_i a_i b_i in FP64 (fixed reduction tree for a given n)
// written to *result (device).  partial: >= kMaxPartials doubles, counter: zeroed uint.
constexpr int kMaxPartials = 4096;
template <typename T>
void dot(const T* a, const T* b, int64_t n, double* partial, unsigned* counter, double* result, hipStream_t s);

// --------------------------------------------------------------- streaming ---
// row blocks for the streaming CSR kernels, computed from a host row pointer
std::vector<int> stream_blocks(const int* rowptr_host, int n, int group, int cap = kStreamCap);
// threads per row for a matrix (host row pointer): stream_group_rule
int stream_group(const int* rowptr_host, int n);
// A.group, A.nblk and A.blk from A's device row pointer (the same greedy
// partition as stream_blocks, computed on the device), and with `pack`
// A.col16 and A.cbase when every block's columns span fewer than 2^16
// values (otherwise both stay empty); reads back the block count, so s is
// synchronised once
// (blocks of at most `cap` stored entries; A.cap records it)
void stream_partition(DCsr& A, MemCounter* mc, hipStream_t s, bool pack, int cap = kStreamCap);
// the distinct-column lists of A's packed streaming blocks (see DCsr::ustart)
void block_uniques(DCsr& A, MemCounter* mc, hipStream_t s);

// dot partials of a streaming launch: one per row block
constexpr int kStreamPartials = 1;  // dot partials per streaming block
inline int stream_partials(const DCsr& A) { return A.nblk * kStreamPartials; }

// dot-fusion target: per-block partial sums, reduced by finish_sum into *result
struct DotTarget {
    double* partial = nullptr;
    unsigned* counter = nullptr;
    double* result = nullptr;
};
// *dt.result = sum of dt.partial[0..nblocks) in index order (one block)
void finish_sum(const DotTarget& dt, int nblocks, hipStream_t s);

// y = A x
template <typename T>
void spmv(const DCsr& A, const T* val, const T* x, T* y, hipStream_t s);
// y = b - A x
template <typename T>
void spmv_resid(const DCsr& A, const T* val, const T* x, const T* b, T* y, hipStream_t s);
// y = y_in + A x  (prolongation x += P e when y == y_in)
template <typename T>
void spmv_add(const DCsr& A, const T* val, const T* x, const T* y_in, T* y, hipStream_t s);
// smoother step: res = b - A x; d = c1 d + c2 dinv res; out = x + d.
// out64 (if non-null) receives the FP64 iterate instead of out; dotvec (if
// non-null) fuses sum_i out_i * dotvec_i into `dt`.
template <typename T>
void spmv_smooth(const DCsr& A, const T* val, const T* x, const T* b, const T* dinv, T* d, T c1, T c2, T* out,
                 double* out64, const double* dotvec, DotTarget dt, hipStream_t s);
// restriction fused with the next level's first smoother step from zero:
// bc = R r; d_c = c2 * dinv_c .* bc; x_c = d_c (as smooth_first on bc)
template <typename T>
void spmv_restrict_first(const DCsr& R, const T* val, const T* r, T* bc, const T* dinv_c, T c2, T* d_c, T* x_c,
                         hipStream_t s);
// q = A p and sum_i p_i q_i (FP64)
void spmv_dot(const DCsr& A, const double* p, double* q, DotTarget dt, hipStream_t s);
// y = b - A x and sum_i y_i^2
void spmv_resid_norm(const DCsr& A, const double* x, const double* b, double* y, DotTarget dt, hipStream_t s);
// y = dscale .* (A x) and sum y_i^2 (power method)
void spmv_scale_norm(const DCsr& A, const double* x, const double* dscale, double* y, DotTarget dt,
                     hipStream_t s);

// --------------------------------------------------------------- vectors ---
// first smoother step from zero: d = c2 * dinv .* b; x = d.  If b64 is given,
// b = (T) b64 is also stored to `b`.
template <typename T>
void smooth_first(int64_t n, const double* b64, T* b, const T* dinv, T c2, T* d, T* x, hipStream_t s);
// v = v / sqrt(*nrm2)
void scale_by_inv_norm(int64_t n, const double* nrm2, const double* in, double* out, hipStream_t s);
// CG: alpha = rz/pq; x += alpha p; r -= alpha q; rr = r.r
void cg_update(int64_t n, double* x, double* r, const double* p, const double* q, const double* rz,
               const double* pq, DotTarget rr, hipStream_t s);
// CG: p = z + (rz_new / rz_old) p  (rz_old == nullptr: p = z)
void cg_direction(int64_t n, double* p, const double* z, const double* rz_new, const double* rz_old,
                  hipStream_t s);
template <typename A, typename B>
void cast_vec(int64_t n, const A* in, B* out, hipStream_t s);
void fill_seeded_uniform(int64_t n, uint64_t key, double* v, hipStream_t s);

// ----------------------------------------------------------------- dense ---
// out = Minv * in for a dense row-major n x n FP64 matrix; in/out of type T
template <typename T>
void dense_gemv(int n, const double* M, const T* in, T* out, hipStream_t s);
// A (n x n, row-major, symmetric) -> A^{-1} in place via blocked Cholesky,
// enqueued on s; *flag (device int, set to 0 here) becomes 1 if the matrix is
// not positive definite, and A then holds no inverse.  work: n*n doubles.
void dense_spd_inverse(int n, double* A, double* work, int* flag, hipStream_t s);

}  // namespace matamg
