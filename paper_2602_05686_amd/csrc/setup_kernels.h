// Launchers of the setup-phase kernels (strength of connection, aggregation,
// prolongator, Galerkin product, auxiliary transfer).
#pragma once

#include "common.h"

namespace matamg {

enum MisState : uint8_t { MIS_OUT = 0, MIS_UND = 1, MIS_IN = 2 };

// entry k of a row-wise incidence list with `count` items per source;
// builds the CSR of target -> sources with sources ascending per target.
// map(e) gives the target of item e (or -1 to skip); items per source fixed.
struct Incidence {
    DBuf<int> rowptr, items;
    int ntarget = 0;
};

// element -> node incidence to node -> element lists (ascending element id)
void build_node_elements(const int* elem_nodes, int64_t nelem, int npe, int n, Incidence& out, int* flag,
                         MemCounter* mc, hipStream_t s);
// node -> aggregate map to aggregate -> member lists (ascending node id)
void build_aggregate_members(const int* agg, int n, int nagg, Incidence& out, MemCounter* mc, hipStream_t s);

void detect_dirichlet(int n, const int* rowptr, const int* col, const double* val, uint8_t* dir, hipStream_t s);
void clement(int n, int dim, const Incidence& inc, const double* elem_sigma, double* sig, hipStream_t s);
void tensor_inverse(int n, int dim, const double* sig, double* minv, int* flag, hipStream_t s);
// lval[k] = |L_ij| (0 for diagonal / Dirichlet edges, -1 for coincident
// points), ldiag[i] = sum of lval over the row (ascending)
void soc_values(const DCsr& A, int dim, const double* x, const double* minv, const uint8_t* dir, int soc,
                double* lval, double* ldiag, hipStream_t s);
void soc_mask(const DCsr& A, const uint8_t* dir, const double* lval, const double* ldiag, double theta, double* S,
              uint8_t* mask, hipStream_t s);

// cut-drop criterion in place of the pointwise mask: keep (nnz bytes of
// scratch) holds each row's own choice, mask the symmetric result
void cut_drop(const DCsr& A, const uint8_t* dir, const double* lval, const double* ldiag, double theta,
              uint8_t* keep, uint8_t* mask, hipStream_t s);
void mis_init(int n, const uint8_t* dir, uint8_t* state, hipStream_t s);
// one synchronous round over the entries mask keeps (nullptr: every stored
// entry); *undecided (device, zero on entry) receives the number of nodes
// still undecided
void mis_round(const DCsr& A, const uint8_t* mask, uint64_t key, uint8_t* state, uint64_t* t1, uint64_t* t2,
               int* undecided, hipStream_t s);
void agg_root_flags(int n, const uint8_t* state, int* flags, hipStream_t s);
// phase 2 (neighbours of roots) and phase 3 (leftovers) over the entries
// mask keeps (nullptr: every stored entry); list: n ints and nlist: one int
// of device scratch
void agg_assign(int n, const int* rowptr, const int* col, const uint8_t* mask, const uint8_t* dir,
                const uint8_t* state, const int* root_rank, int* phase2, int* agg, int* list, int* nlist,
                hipStream_t s);

// *flag = 1 (device int) if any value of v[0..n) is not finite
void check_finite(const double* v, int64_t n, int* flag, hipStream_t s);

// filtered matrix A_F (diagonal + kept entries, lumped diagonal) and its 1-norm
// diagonal (zero on isolated and empty rows); dir: Dirichlet flags of the level
void filter_count(const DCsr& A, const uint8_t* mask, int* cnt, hipStream_t s);
void filter_fill(const DCsr& A, const uint8_t* mask, const uint8_t* dir, const int* frowptr, int* fcol, double* fval,
                 double* dt, double* dtinv, hipStream_t s);
void phat_counts(int n, const int* agg, int* cnt, hipStream_t s);
void phat_fill(int n, const int* agg, const int* prowptr, int* pcol, double* pval, hipStream_t s);
void prolongator_finalize(int n, const int* prowptr, const int* pcol, double* pval, const int* agg,
                          const double* dt, double omega, hipStream_t s);
void coarse_aux(int nc, int dim, const Incidence& members, const double* x, const double* sig, double* xc,
                double* sigc, hipStream_t s);
void diag_inverse(int n, const int* rowptr, const int* col, const double* val, double* dinv, hipStream_t s);
// the same over A's streaming row blocks (A.blk must be set)
void diag_inverse_blocks(const DCsr& A, double* dinv, hipStream_t s);
void densify(int n, const int* rowptr, const int* col, const double* val, double* D, hipStream_t s);
// CSR sanity: columns in range and strictly ascending; *flag set on violation
void validate_csr(int n, const int* rowptr, const int* col, int64_t nnz, int* flag, hipStream_t s);
// *flag = 1 if a[i] != b[i] for some i < n (flag is not cleared)
void bytes_differ(int n, const uint8_t* a, const uint8_t* b, int* flag, hipStream_t s);

// ----------------------------------------------------------------- SpGEMM ---
// C = A * B with the symbolic pattern (zeros kept), ascending columns, and
// every entry accumulated in the order (k ascending in A's row, B's row order)
void spgemm(const DCsr& A, const DCsr& B, DCsr& C, MemCounter* mc, hipStream_t s);
// T = A^T, entries of each output row in ascending source row
void transpose(const DCsr& A, DCsr& T, MemCounter* mc, hipStream_t s);

}  // namespace matamg
