/*
 * Serial FP64 reference of material-aware smoothed-aggregation AMG and the
 * AMG-preconditioned CG it accelerates.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: a plain, slow, serial
 * implementation written to be checked by eye against the paper
 * (Firmbach, Phillips, Glusa, Popp, Siefert, Mayr, "Smoothed aggregation
 * algebraic multigrid for problems with heterogeneous and anisotropic
 * materials").  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or table with the HIP
 * library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (every floating-point
 * operation is a separate IEEE-754 double operation; no fused multiply-add).
 *
 * Where the paper is silent the reading taken is stated at the function.
 * Parity pins live in the CPU tests; every function below is pinned there.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status codes (numeric values mirror the library's public ones) */
enum {
    ORC_OK = 0,
    ORC_INVALID_ARG = 1,
    ORC_OUT_OF_MEMORY = 2,
    ORC_NOT_SPD = 4,
    ORC_STAGNATED = 5,
    ORC_NOT_CONVERGED = 6,
    ORC_BREAKDOWN = 7,
};

enum { SOC_MATERIAL = 0, SOC_DISTANCE = 1, SOC_SA = 2 };
enum { DROP_POINTWISE = 0, DROP_CUT = 1 };
enum { SMOOTH_CHEBYSHEV = 0, SMOOTH_JACOBI = 1, SMOOTH_JACOBI_SCALED = 2 };

typedef struct {
    int32_t dim;
    double theta;
    int32_t soc;
    int32_t drop;
    int32_t smoother;
    int32_t max_coarse;
    int32_t max_levels;
    int32_t cheb_degree;
    double cheb_ratio;
    double cheb_boost;
    int32_t power_iters;
    double omega_sym;
    double jacobi_omega;
    int32_t jacobi_sweeps;
    uint64_t seed;
} OrcOptions;

typedef struct {
    int n, m; /* rows, columns */
    int *rowptr, *col;
    double *val;
} Csr;

typedef struct {
    Csr A;
    int dim;
    double *x;            /* [n*dim] coordinates */
    double *sig;          /* [n*ncomp] symmetric tensor, upper triangle row-wise */
    unsigned char *dir;   /* Dirichlet flags (only ever set on the finest level) */
    double *lval;         /* |L_ij| per stored entry (0 on the diagonal) */
    double *ldiag;        /* L_ii */
    double *S;            /* strength values per stored entry */
    unsigned char *mask;  /* dropping criterion C(S) per stored entry */
    int *agg;             /* aggregate id or -1 */
    int nc;
    int mis_rounds;
    Csr P, R;
    double lam_pf, omega; /* prolongator smoothing */
    double lam_cheb;      /* spectral estimate of D^{-1} A for the smoother */
    double *dinv;
} Level;

typedef struct {
    OrcOptions opt;
    int nlev;
    Level lev[16];
    double *chol; /* dense lower Cholesky factor of the coarsest operator */
    int nL;
    double *work;
} Hier;

/* ------------------------------------------------------------------------ */
/* counter-based generator: splitmix64 (Steele, Lea, Flood, OOPSLA 2014)      */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* stream keys: MIS-2 priorities, prolongator power method, smoother power method */
static uint64_t stream_key(uint64_t seed, uint64_t purpose, int level)
{
    return splitmix64(seed + purpose + (uint64_t)level);
}
#define PURPOSE_MIS 1ull
/* 2^-46 = 64 * DBL_EPSILON: relative size of round-off noise in a row sum */
#define ROW_NOISE 1.4210854715202004e-14
#define PURPOSE_PF 101ull
#define PURPOSE_CHEB 201ull

/* uniform draw in [-1, 1) for index i of a stream */
static double uniform_pm1(uint64_t key, uint64_t i)
{
    uint64_t h = splitmix64(key ^ i);
    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0); /* [0,1) */
    return 2.0 * u - 1.0;
}

/* ------------------------------------------------------------------------ */
/* helpers                                                                   */
/* ------------------------------------------------------------------------ */
static int ncomp_of(int dim) { return dim * (dim + 1) / 2; }

static void csr_free(Csr *a)
{
    free(a->rowptr);
    free(a->col);
    free(a->val);
    memset(a, 0, sizeof(*a));
}

/* y = A x, each row summed in ascending stored order */
static void spmv(const Csr *a, const double *x, double *y)
{
    for (int i = 0; i < a->n; ++i) {
        double s = 0.0;
        for (int k = a->rowptr[i]; k < a->rowptr[i + 1]; ++k) s += a->val[k] * x[a->col[k]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* C = A * B for CSR matrices; the product pattern is the symbolic one
 * (every structurally reachable column, zeros kept), columns ascending, and
 * each entry accumulated in the order (k ascending in A's row, then B's row). */
static int spgemm(const Csr *a, const Csr *b, Csr *c)
{
    int n = a->n, m = b->m;
    int *mark = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    double *acc = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    int *list = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    c->rowptr = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    if (!mark || !acc || !list || !c->rowptr) {
        free(mark); free(acc); free(list); free(c->rowptr); c->rowptr = NULL;
        return ORC_OUT_OF_MEMORY;
    }
    for (int j = 0; j < m; ++j) mark[j] = -1;
    /* symbolic */
    long long total = 0;
    c->rowptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        int cnt = 0;
        for (int ka = a->rowptr[i]; ka < a->rowptr[i + 1]; ++ka) {
            int k = a->col[ka];
            for (int kb = b->rowptr[k]; kb < b->rowptr[k + 1]; ++kb) {
                int j = b->col[kb];
                if (mark[j] != i) { mark[j] = i; ++cnt; }
            }
        }
        total += cnt;
        if (total > 2147483647LL) { free(mark); free(acc); free(list); return ORC_OUT_OF_MEMORY; }
        c->rowptr[i + 1] = (int)total;
    }
    c->n = n; c->m = m;
    c->col = (int *)malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
    c->val = (double *)malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    if (!c->col || !c->val) { free(mark); free(acc); free(list); return ORC_OUT_OF_MEMORY; }
    for (int j = 0; j < m; ++j) mark[j] = -1;
    /* numeric */
    for (int i = 0; i < n; ++i) {
        int cnt = 0;
        for (int ka = a->rowptr[i]; ka < a->rowptr[i + 1]; ++ka) {
            int k = a->col[ka];
            double av = a->val[ka];
            for (int kb = b->rowptr[k]; kb < b->rowptr[k + 1]; ++kb) {
                int j = b->col[kb];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; list[cnt++] = j; }
                acc[j] += av * b->val[kb];
            }
        }
        /* ascending columns: insertion sort of the touched list */
        for (int s = 1; s < cnt; ++s) {
            int v = list[s], t = s - 1;
            while (t >= 0 && list[t] > v) { list[t + 1] = list[t]; --t; }
            list[t + 1] = v;
        }
        int base = c->rowptr[i];
        for (int s = 0; s < cnt; ++s) {
            c->col[base + s] = list[s];
            c->val[base + s] = acc[list[s]];
        }
    }
    free(mark); free(acc); free(list);
    return ORC_OK;
}

/* transpose; within each output row the entries are in ascending source row */
static int transpose(const Csr *a, Csr *t)
{
    int n = a->n, m = a->m, nnz = a->rowptr[n];
    t->n = m; t->m = n;
    t->rowptr = (int *)calloc((size_t)m + 1, sizeof(int));
    t->col = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    t->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int *fill = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    if (!t->rowptr || !t->col || !t->val || !fill) { free(fill); return ORC_OUT_OF_MEMORY; }
    for (int k = 0; k < nnz; ++k) t->rowptr[a->col[k] + 1]++;
    for (int j = 0; j < m; ++j) t->rowptr[j + 1] += t->rowptr[j];
    for (int j = 0; j < m; ++j) fill[j] = t->rowptr[j];
    for (int i = 0; i < n; ++i)
        for (int k = a->rowptr[i]; k < a->rowptr[i + 1]; ++k) {
            int p = fill[a->col[k]]++;
            t->col[p] = i;
            t->val[p] = a->val[k];
        }
    free(fill);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Clement interpolant of element-wise tensors (section "A material based    */
/* strength-of-connection measure", paragraph on low-regularity sigma).      */
/* Reading: the degree-0 Clement operator on meshes of equal-measure         */
/* elements, i.e. the arithmetic mean of sigma_e over the elements e that    */
/* contain node i, summed in ascending element id and divided once.          */
/* ------------------------------------------------------------------------ */
int orc_clement(int n, int dim, int nelem, int npe, const int32_t *elem_nodes,
                const double *elem_sigma, double *sig_out)
{
    if (n <= 0 || dim < 1 || dim > 3 || nelem < 0 || npe <= 0) return ORC_INVALID_ARG;
    int nc = ncomp_of(dim);
    int *count = (int *)calloc((size_t)n, sizeof(int));
    if (!count) return ORC_OUT_OF_MEMORY;
    for (int i = 0; i < n * nc; ++i) sig_out[i] = 0.0;
    for (int e = 0; e < nelem; ++e) {          /* ascending element id */
        const double *s = elem_sigma + (size_t)e * dim * dim;
        for (int a = 0; a < npe; ++a) {
            int i = elem_nodes[(size_t)e * npe + a];
            if (i < 0 || i >= n) { free(count); return ORC_INVALID_ARG; }
            int c = 0;
            for (int p = 0; p < dim; ++p)
                for (int q = p; q < dim; ++q) sig_out[(size_t)i * nc + c++] += s[p * dim + q];
            count[i]++;
        }
    }
    for (int i = 0; i < n; ++i)
        if (count[i] > 0)
            for (int c = 0; c < nc; ++c) sig_out[(size_t)i * nc + c] = sig_out[(size_t)i * nc + c] / (double)count[i];
    free(count);
    return ORC_OK;
}

/* sigma^{-1} by the adjugate over the determinant, one IEEE op at a time.
 * Components are stored as the upper triangle row by row:
 * 1D (m00); 2D (m00, m01, m11); 3D (m00, m01, m02, m11, m12, m22). */
static int tensor_inverse(int dim, const double *s, double *m)
{
    if (dim == 1) {
        if (!(s[0] > 0.0)) return ORC_NOT_SPD;
        m[0] = 1.0 / s[0];
        return ORC_OK;
    }
    if (dim == 2) {
        double s00 = s[0], s01 = s[1], s11 = s[2];
        double det = s00 * s11 - s01 * s01;
        if (!(det > 0.0) || !(s00 > 0.0)) return ORC_NOT_SPD;
        m[0] = s11 / det;
        m[1] = (-s01) / det;
        m[2] = s00 / det;
        return ORC_OK;
    }
    double s00 = s[0], s01 = s[1], s02 = s[2], s11 = s[3], s12 = s[4], s22 = s[5];
    double c00 = s11 * s22 - s12 * s12;
    double c01 = s02 * s12 - s01 * s22;
    double c02 = s01 * s12 - s02 * s11;
    double c11 = s00 * s22 - s02 * s02;
    double c12 = s01 * s02 - s00 * s12;
    double c22 = s00 * s11 - s01 * s01;
    double det = (s00 * c00 + s01 * c01) + s02 * c02;
    if (!(det > 0.0) || !(s00 > 0.0) || !(c22 > 0.0)) return ORC_NOT_SPD;
    m[0] = c00 / det; m[1] = c01 / det; m[2] = c02 / det;
    m[3] = c11 / det; m[4] = c12 / det; m[5] = c22 / det;
    return ORC_OK;
}

/* squared material distance from one endpoint: q = delta^T M delta,
 * evaluated as sum_a delta_a * (sum_b M_ab delta_b), left to right */
static double quad_form(int dim, const double *m, const double *d)
{
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

/* Dirichlet rows: every stored off-diagonal value is exactly zero (or absent). */
int orc_detect_dirichlet(int n, const int32_t *rowptr, const int32_t *col, const double *val,
                         unsigned char *dir)
{
    for (int i = 0; i < n; ++i) {
        int any = 0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] != i && val[k] != 0.0) { any = 1; break; }
        dir[i] = any ? 0 : 1;
    }
    return ORC_OK;
}

/*
 * Strength of connection and pointwise dropping (sections "Strength-of-
 * connection measures and dropping criteria" and "A material based
 * strength-of-connection measure").
 *
 * Material distance Laplacian: for a stored off-diagonal (i, j) the distance is
 *   d_sigma(x_i, x_j)^2 = max(q_i, q_j),  q_i = (x_j-x_i)^T sigma_i^{-1} (x_j-x_i),
 * reading the symmetrisation as the maximum of the two one-sided distances
 * (the printed definition repeats one argument; the low/high scaling argument
 * needs the two orders).  L_ij = -1/d^2, L_ii = -sum_{j != i} L_ij (summed in
 * ascending column order), S = D^{-1/2} L D^{-1/2}.  With SOC_DISTANCE sigma is
 * the identity (Euclidean distance Laplacian); with SOC_SA the classical
 * S_ij = |A_ij| / sqrt(|A_ii| |A_jj|).
 *
 * "A_ij != 0" in the distance Laplacian is read as "structurally stored".
 * Edges touching a Dirichlet node carry no strength and are always dropped.
 * Coincident points (max(q_i, q_j) not positive) are read as a strong edge:
 * they are kept and left out of L_ii.
 *
 * Pointwise criterion |S_ij| >= theta is evaluated in the square-free form
 *   l_ij * l_ij >= (theta*theta) * (L_ii * L_jj),   l_ij = |L_ij|,
 * which is the same inequality for positive quantities and involves no square
 * root.  S itself is reported with the square root.  drop = DROP_CUT applies
 * the cut-drop criterion instead (cut_drop below).
 */
static int cut_drop(int n, const int32_t *rowptr, const int32_t *col, const unsigned char *dir,
                    const double *lval, const double *ldiag, const unsigned char *coinc, double theta,
                    unsigned char *mask);

int orc_strength(int n, const int32_t *rowptr, const int32_t *col, const double *val, int dim,
                 const double *x, const double *sig, const unsigned char *dir, int soc, int drop, double theta,
                 double *lval, double *ldiag, double *S, unsigned char *mask)
{
    if (drop != DROP_POINTWISE && drop != DROP_CUT) return ORC_INVALID_ARG;
    if (dim < 1 || dim > 3) return ORC_INVALID_ARG;
    int nc = ncomp_of(dim);
    int nnz = rowptr[n];
    double *minv = NULL;
    unsigned char *coinc = (unsigned char *)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
    if (!coinc) return ORC_OUT_OF_MEMORY;
    if (soc == SOC_MATERIAL) {
        minv = (double *)malloc(sizeof(double) * (size_t)n * nc);
        if (!minv) { free(coinc); return ORC_OUT_OF_MEMORY; }
        for (int i = 0; i < n; ++i) {
            int rc = tensor_inverse(dim, sig + (size_t)i * nc, minv + (size_t)i * nc);
            if (rc != ORC_OK) { free(minv); free(coinc); return rc; }
        }
    }
    double ident[6];
    for (int c = 0; c < 6; ++c) ident[c] = 0.0;
    if (dim == 1) ident[0] = 1.0;
    if (dim == 2) { ident[0] = 1.0; ident[2] = 1.0; }
    if (dim == 3) { ident[0] = 1.0; ident[3] = 1.0; ident[5] = 1.0; }

    double *adiag = NULL;
    if (soc == SOC_SA) {
        adiag = (double *)calloc((size_t)n, sizeof(double));
        if (!adiag) { free(minv); free(coinc); return ORC_OUT_OF_MEMORY; }
        for (int i = 0; i < n; ++i)
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == i) adiag[i] = fabs(val[k]);
    }

    /* off-diagonal magnitudes and the diagonal */
    for (int i = 0; i < n; ++i) {
        double li = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            lval[k] = 0.0;
            if (j == i) continue;
            if (dir && (dir[i] || dir[j])) continue;
            if (soc == SOC_SA) {
                lval[k] = fabs(val[k]);
                continue;
            }
            double d[3];
            for (int a = 0; a < dim; ++a) d[a] = x[(size_t)j * dim + a] - x[(size_t)i * dim + a];
            const double *mi = (soc == SOC_MATERIAL) ? minv + (size_t)i * nc : ident;
            const double *mj = (soc == SOC_MATERIAL) ? minv + (size_t)j * nc : ident;
            double qi = quad_form(dim, mi, d);
            double qj = quad_form(dim, mj, d);
            double q = qi > qj ? qi : qj;
            if (!(q > 0.0) || !isfinite(q)) {
                coinc[k] = 1;
                continue;
            }
            lval[k] = 1.0 / q;
            li += lval[k];
        }
        ldiag[i] = li;
    }
    if (soc == SOC_SA)
        for (int i = 0; i < n; ++i) ldiag[i] = adiag[i];

    double th2 = theta * theta;
    for (int i = 0; i < n; ++i) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            if (j == i) {
                S[k] = 1.0;
                mask[k] = 1;
                continue;
            }
            if (dir && (dir[i] || dir[j])) {
                S[k] = 0.0;
                mask[k] = 0;
                continue;
            }
            if (coinc[k]) {
                S[k] = 1.0;
                mask[k] = 1;
                continue;
            }
            double l = lval[k];
            double prod = ldiag[i] * ldiag[j];
            S[k] = (prod > 0.0) ? l / sqrt(prod) : 1.0;
            mask[k] = (l * l >= th2 * prod) ? 1 : 0;
        }
    }
    int rc = ORC_OK;
    if (drop == DROP_CUT) rc = cut_drop(n, rowptr, col, dir, lval, ldiag, coinc, theta, mask);
    free(adiag);
    free(minv);
    free(coinc);
    return rc;
}

static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/*
 * Cut-drop criterion (section "Strength-of-connection measures and dropping
 * criteria"): order the strengths of row i decreasingly, s_1 >= s_2 >= ...,
 * let k be the first position with theta * s_k >= s_{k+1}, and keep the
 * entries whose strength is at least s_k; drop nothing when no such k exists.
 *
 * Readings (the paper leaves them open):
 *  - the ordered row holds the off-diagonal entries only; the diagonal is
 *    always kept.  The two-domain study reports cut-drop as the robust
 *    criterion at large tolerances, where the pointwise one stagnates: that
 *    holds only if the strongest off-diagonal entry always survives, which
 *    an ordered diagonal (S_ii = 1 above every S_ij) would prevent;
 *  - the row's strengths are compared through the square-free key
 *      t_ij = (l_ij * l_ij) / L_jj   (= S_ij^2 L_ii, L_ii common to the row),
 *    with t = L_ii for coincident points (S = 1), and
 *    theta * s_k >= s_{k+1} as (theta*theta) * t_k >= t_{k+1};  an entry with
 *    L_jj <= 0 has S = 1 like the pointwise form, so t = L_ii;
 *  - a row with L_ii <= 0 (no positive coupling) keeps every entry;
 *  - edges touching a Dirichlet node stay dropped and are not ordered;
 *  - the result is made symmetric by keeping (i, j) only if both rows keep it.
 */
static int cut_drop(int n, const int32_t *rowptr, const int32_t *col, const unsigned char *dir,
                    const double *lval, const double *ldiag, const unsigned char *coinc, double theta,
                    unsigned char *mask)
{
    const int nnz = rowptr[n];
    unsigned char *keep = (unsigned char *)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
    double *tk = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *ord = NULL;
    int maxlen = 0;
    for (int i = 0; i < n; ++i) {
        int len = rowptr[i + 1] - rowptr[i];
        if (len > maxlen) maxlen = len;
    }
    ord = (double *)malloc(sizeof(double) * (size_t)(maxlen > 0 ? maxlen : 1));
    if (!keep || !tk || !ord) {
        free(keep);
        free(tk);
        free(ord);
        return ORC_OUT_OF_MEMORY;
    }
    const double th2 = theta * theta;
    for (int i = 0; i < n; ++i) {
        const int k0 = rowptr[i], k1 = rowptr[i + 1];
        if (dir && dir[i]) {
            for (int k = k0; k < k1; ++k) keep[k] = (col[k] == i);
            continue;
        }
        const double lii = ldiag[i];
        int m = 0;
        for (int k = k0; k < k1; ++k) {
            const int j = col[k];
            tk[k] = -1.0;  /* not ordered */
            if (j == i) continue;
            if (coinc[k]) tk[k] = lii;
            else if (dir && dir[j]) continue;
            else tk[k] = (ldiag[j] > 0.0) ? (lval[k] * lval[k]) / ldiag[j] : lii;
            ord[m++] = tk[k];
        }
        double cut = -1.0;  /* keep everything */
        if (lii > 0.0) {
            qsort(ord, (size_t)m, sizeof(double), cmp_desc);
            for (int p = 0; p + 1 < m; ++p)
                if (th2 * ord[p] >= ord[p + 1]) {
                    cut = ord[p];
                    break;
                }
        }
        for (int k = k0; k < k1; ++k) keep[k] = (col[k] == i) || (tk[k] >= 0.0 && tk[k] >= cut);
    }
    for (int i = 0; i < n; ++i) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = col[k];
            if (j == i) {
                mask[k] = 1;
                continue;
            }
            /* the entry (j, i): binary search in row j's sorted columns */
            int lo = rowptr[j], hi = rowptr[j + 1] - 1, kt = -1;
            while (lo <= hi) {
                int mid = (lo + hi) / 2;
                if (col[mid] == i) { kt = mid; break; }
                if (col[mid] < i) lo = mid + 1;
                else hi = mid - 1;
            }
            mask[k] = (keep[k] && kt >= 0 && keep[kt]) ? 1 : 0;
        }
    }
    free(keep);
    free(tk);
    free(ord);
    return ORC_OK;
}

/*
 * Aggregation on the filtered graph G_C (section "Smoothed aggregation
 * algebraic multigrid methods").  The paper defers the aggregation algorithm;
 * the reading here is a distance-2 maximal independent set (Bell, Dalton,
 * Olson, SIAM J. Sci. Comput. 2012, MIS(k) with k = 2) grown into aggregates:
 *
 *   tuple(i) = (state, priority, i) ordered lexicographically, with
 *   state OUT=0 < UNDECIDED=1 < IN=2 and priority the top 30 bits of
 *   splitmix64(stream ^ i).  Dirichlet nodes start OUT.
 *   Round: T0 = tuples; T1(i) = max over i and its kept neighbours of T0;
 *   T2 likewise from T1.  An undecided i whose T2 is its own tuple becomes IN;
 *   otherwise, if T2's state is IN, it becomes OUT.  Rounds repeat until no
 *   node is undecided.
 *
 *   Roots (IN nodes) are numbered by ascending node index.  Every non-root,
 *   non-Dirichlet node adjacent to a root joins it (phase 2, unique because
 *   roots are at distance >= 3).  Each remaining non-Dirichlet node joins the
 *   aggregate with the most kept neighbours among the phase-2 nodes, ties to
 *   the smallest aggregate id (phase 3).  Dirichlet nodes get -1.
 */
typedef struct { int state; uint32_t prio; uint32_t id; } Tup;

static int tup_gt(Tup a, Tup b)
{
    if (a.state != b.state) return a.state > b.state;
    if (a.prio != b.prio) return a.prio > b.prio;
    return a.id > b.id;
}

int orc_aggregate(int n, const int32_t *rowptr, const int32_t *col, const unsigned char *mask,
                  const unsigned char *dir, uint64_t seed, int level, int32_t *agg, int32_t *nagg_out,
                  int32_t *rounds_out, unsigned char *root_out)
{
    enum { OUT = 0, UND = 1, IN = 2 };
    int *state = (int *)malloc(sizeof(int) * (size_t)n);
    Tup *t0 = (Tup *)malloc(sizeof(Tup) * (size_t)n);
    Tup *t1 = (Tup *)malloc(sizeof(Tup) * (size_t)n);
    Tup *t2 = (Tup *)malloc(sizeof(Tup) * (size_t)n);
    int *phase2 = (int *)malloc(sizeof(int) * (size_t)n);
    if (!state || !t0 || !t1 || !t2 || !phase2) {
        free(state); free(t0); free(t1); free(t2); free(phase2);
        return ORC_OUT_OF_MEMORY;
    }
    uint64_t key = stream_key(seed, PURPOSE_MIS, level);
    for (int i = 0; i < n; ++i) state[i] = (dir && dir[i]) ? OUT : UND;
    int rounds = 0;
    for (;;) {
        int undecided = 0;
        for (int i = 0; i < n; ++i) undecided += (state[i] == UND);
        if (!undecided) break;
        ++rounds;
        for (int i = 0; i < n; ++i) {
            t0[i].state = state[i];
            t0[i].prio = (uint32_t)(splitmix64(key ^ (uint64_t)i) >> 34);
            t0[i].id = (uint32_t)i;
        }
        for (int i = 0; i < n; ++i) {
            Tup best = t0[i];
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                int j = col[k];
                if (j == i || !mask[k]) continue;
                if (tup_gt(t0[j], best)) best = t0[j];
            }
            t1[i] = best;
        }
        for (int i = 0; i < n; ++i) {
            Tup best = t1[i];
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                int j = col[k];
                if (j == i || !mask[k]) continue;
                if (tup_gt(t1[j], best)) best = t1[j];
            }
            t2[i] = best;
        }
        for (int i = 0; i < n; ++i) {
            if (state[i] != UND) continue;
            if (t2[i].id == (uint32_t)i && t2[i].state == UND) state[i] = IN;
            else if (t2[i].state == IN) state[i] = OUT;
        }
    }
    int nagg = 0;
    for (int i = 0; i < n; ++i) {
        agg[i] = -1;
        if (state[i] == IN) agg[i] = nagg++;
        if (root_out) root_out[i] = (state[i] == IN);
    }
    /* phase 2: neighbours of roots */
    for (int i = 0; i < n; ++i) {
        phase2[i] = agg[i];
        if (agg[i] >= 0 || (dir && dir[i])) continue;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            if (j == i || !mask[k]) continue;
            if (state[j] == IN) { phase2[i] = agg[j]; break; }
        }
    }
    /* phase 3: the remaining nodes, reading only phase-2 assignments */
    for (int i = 0; i < n; ++i) {
        agg[i] = phase2[i];
        if (phase2[i] >= 0 || (dir && dir[i])) continue;
        int best = -1, bestcnt = 0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            if (j == i || !mask[k] || phase2[j] < 0) continue;
            int c = phase2[j], cnt = 0;
            for (int k2 = rowptr[i]; k2 < rowptr[i + 1]; ++k2) {
                int j2 = col[k2];
                if (j2 == i || !mask[k2]) continue;
                if (phase2[j2] == c) cnt++;
            }
            if (cnt > bestcnt || (cnt == bestcnt && c < best)) { best = c; bestcnt = cnt; }
        }
        agg[i] = best; /* -1 only if the node is unreachable, which MIS-2 rules out */
    }
    free(state); free(t0); free(t1); free(t2); free(phase2);
    *nagg_out = nagg;
    if (rounds_out) *rounds_out = rounds;
    return ORC_OK;
}

/* power method: after `iters` steps of v <- B v / ||B v||_2 from a seeded
 * start, returns ||B v||_2 for the last unit v.  B = diag(dscale) * A. */
static double power_method(const Csr *a, const double *dscale, int iters, uint64_t key, double *v, double *w)
{
    int n = a->n;
    for (int i = 0; i < n; ++i) v[i] = uniform_pm1(key, (uint64_t)i);
    double nv = sqrt(dot(n, v, v));
    if (!(nv > 0.0)) return 0.0;
    for (int i = 0; i < n; ++i) v[i] = v[i] / nv;
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        spmv(a, v, w);
        for (int i = 0; i < n; ++i) w[i] = dscale[i] * w[i];
        lam = sqrt(dot(n, w, w));
        if (!(lam > 0.0)) return 0.0;
        for (int i = 0; i < n; ++i) v[i] = w[i] / lam;
    }
    return lam;
}

/*
 * Smoothed prolongator (section "Prolongator smoothing and matrix filtering").
 * Tentative P^(i, agg(i)) = 1 (near null space = ones, no orthonormalisation).
 * Filtered matrix A_F keeps the diagonal and the kept off-diagonals, and lumps
 * every dropped off-diagonal into the diagonal: (A_F)_ii = A_ii + sum of the
 * dropped A_ik (ascending column).  A Dirichlet row keeps only its diagonal
 * (its off-diagonals are zero by definition).
 * 1-norm diagonal Dt_ii = sum_j |(A_F)_ij| (zero for an empty filtered row,
 * see below).  omega = omega_sym / lambda with
 * lambda from the power method on Dt^{-1} A_F.  P = P^ - omega Dt^{-1} A_F P^;
 * the pattern is the symbolic product (zeros kept).
 */
static int build_prolongator(Level *L, const OrcOptions *opt, int level)
{
    const Csr *A = &L->A;
    int n = A->n;
    Csr F = {0}, Phat = {0}, FP = {0};
    int rc = ORC_OK;
    double *dt = NULL, *v = NULL, *w = NULL;
    /* filtered matrix */
    int cnt = 0;
    for (int i = 0; i < n; ++i)
        for (int k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->col[k] == i || L->mask[k]) cnt++;
    F.n = n; F.m = n;
    F.rowptr = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    F.col = (int *)malloc(sizeof(int) * (size_t)(cnt > 0 ? cnt : 1));
    F.val = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    dt = (double *)malloc(sizeof(double) * (size_t)n);
    v = (double *)malloc(sizeof(double) * (size_t)n);
    w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!F.rowptr || !F.col || !F.val || !dt || !v || !w) { rc = ORC_OUT_OF_MEMORY; goto done; }
    cnt = 0;
    F.rowptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        double lump = 0.0;
        int diagpos = -1;
        for (int k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int j = A->col[k];
            if (j == i || L->mask[k]) {
                if (j == i) diagpos = cnt;
                F.col[cnt] = j;
                F.val[cnt] = A->val[k];
                cnt++;
            } else {
                lump += A->val[k];
            }
        }
        if (diagpos >= 0) F.val[diagpos] = F.val[diagpos] + lump;
        F.rowptr[i + 1] = cnt;
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = F.rowptr[i]; k < F.rowptr[i + 1]; ++k) s += fabs(F.val[k]);
        /* Isolated rows.  A row that keeps no off-diagonal connection has
         * (A_F)_ii = sum_k A_ik, its 1-norm diagonal is |sum_k A_ik| and the
         * formula moves its prolongator row to (1 -+ omega) P^ by the sign of
         * that sum.  The sum is zero in exact arithmetic on interior rows and
         * rounding noise in floating point, which on coarse levels (long
         * Galerkin rows) reaches any size the genuine row sums near a
         * boundary also take, so no threshold on it separates the two.  The
         * reading: a non-Dirichlet row whose kept off-diagonals weigh at most
         * 2^-46 of its 1-norm in A (none kept, or only stored zeros and
         * noise) is isolated and not smoothed -- Dt_ii = 0, its row of P is
         * its row of P^ -- which the drop mask decides, not the rounding.  A
         * Dirichlet row keeps its diagonal (its row of P^ is empty anyway). */
        double rowabs = 0.0, keptabs = 0.0;
        for (int k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            rowabs += fabs(A->val[k]);
            if (A->col[k] != i && L->mask[k]) keptabs += fabs(A->val[k]);
        }
        int isolated = !(L->dir && L->dir[i]) && !(keptabs > ROW_NOISE * rowabs);
        dt[i] = (!isolated && s > ROW_NOISE * rowabs) ? s : 0.0;
    }
    {
        double *dtinv = (double *)malloc(sizeof(double) * (size_t)n);
        if (!dtinv) { rc = ORC_OUT_OF_MEMORY; goto done; }
        for (int i = 0; i < n; ++i) dtinv[i] = dt[i] > 0.0 ? 1.0 / dt[i] : 0.0;
        L->lam_pf = power_method(&F, dtinv, opt->power_iters, stream_key(opt->seed, PURPOSE_PF, level), v, w);
        free(dtinv);
    }
    L->omega = (L->lam_pf > 0.0) ? opt->omega_sym / L->lam_pf : 0.0;
    /* tentative prolongator */
    Phat.n = n; Phat.m = L->nc;
    Phat.rowptr = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    Phat.col = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    Phat.val = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!Phat.rowptr || !Phat.col || !Phat.val) { rc = ORC_OUT_OF_MEMORY; goto done; }
    cnt = 0;
    Phat.rowptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        if (L->agg[i] >= 0) { Phat.col[cnt] = L->agg[i]; Phat.val[cnt] = 1.0; cnt++; }
        Phat.rowptr[i + 1] = cnt;
    }
    rc = spgemm(&F, &Phat, &FP);
    if (rc) goto done;
    /* P = P^ - omega Dt^{-1} (A_F P^), on the pattern of A_F P^ */
    for (int i = 0; i < n; ++i) {
        for (int k = FP.rowptr[i]; k < FP.rowptr[i + 1]; ++k) {
            double delta = (FP.col[k] == L->agg[i]) ? 1.0 : 0.0;
            double corr = (dt[i] > 0.0) ? (L->omega * FP.val[k]) / dt[i] : 0.0;
            FP.val[k] = delta - corr;
        }
    }
    L->P = FP;
    memset(&FP, 0, sizeof(FP));
done:
    csr_free(&F);
    csr_free(&Phat);
    csr_free(&FP);
    free(dt); free(v); free(w);
    return rc;
}

/* coarse coordinates and tensors: aggregate means (eq. auxiliary_transfer),
 * members summed in ascending node index, then one divide by |A_j| */
static int coarse_aux(const Level *L, Level *C)
{
    int n = L->A.n, nc = L->nc, d = L->dim, ncomp = ncomp_of(d);
    int *count = (int *)calloc((size_t)nc, sizeof(int));
    C->x = (double *)calloc((size_t)nc * d, sizeof(double));
    C->sig = (double *)calloc((size_t)nc * ncomp, sizeof(double));
    if (!count || !C->x || !C->sig) { free(count); return ORC_OUT_OF_MEMORY; }
    for (int i = 0; i < n; ++i) {
        int j = L->agg[i];
        if (j < 0) continue;
        for (int a = 0; a < d; ++a) C->x[(size_t)j * d + a] += L->x[(size_t)i * d + a];
        for (int c = 0; c < ncomp; ++c) C->sig[(size_t)j * ncomp + c] += L->sig[(size_t)i * ncomp + c];
        count[j]++;
    }
    for (int j = 0; j < nc; ++j) {
        for (int a = 0; a < d; ++a) C->x[(size_t)j * d + a] = C->x[(size_t)j * d + a] / (double)count[j];
        for (int c = 0; c < ncomp; ++c) C->sig[(size_t)j * ncomp + c] = C->sig[(size_t)j * ncomp + c] / (double)count[j];
    }
    free(count);
    return ORC_OK;
}

/* dense Cholesky A = L L^T (lower, row-major, in place, no pivoting) */
int orc_dense_cholesky(int n, double *a)
{
    for (int j = 0; j < n; ++j) {
        double d = a[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(d > 0.0) || !isfinite(d)) return ORC_NOT_SPD;
        double ljj = sqrt(d);
        a[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = a[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = s / ljj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) a[(size_t)i * n + j] = 0.0;
    return ORC_OK;
}

/* solve L L^T x = b with the factor from orc_dense_cholesky */
void orc_dense_cholesky_solve(int n, const double *l, const double *b, double *x)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= l[(size_t)i * n + k] * x[k];
        x[i] = s / l[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= l[(size_t)k * n + i] * x[k];
        x[i] = s / l[(size_t)i * n + i];
    }
}

static void level_free(Level *L)
{
    csr_free(&L->A);
    csr_free(&L->P);
    csr_free(&L->R);
    free(L->x); free(L->sig); free(L->dir); free(L->lval); free(L->ldiag);
    free(L->S); free(L->mask); free(L->agg); free(L->dinv);
    memset(L, 0, sizeof(*L));
}

void orc_free(void *hv)
{
    Hier *h = (Hier *)hv;
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) level_free(&h->lev[l]);
    free(h->chol);
    free(h->work);
    free(h);
}

void orc_default_options(OrcOptions *o)
{
    o->dim = 3;
    o->theta = 0.08;
    o->soc = SOC_MATERIAL;
    o->drop = 0;
    o->smoother = SMOOTH_CHEBYSHEV;
    o->max_coarse = 5000;
    o->max_levels = 10;
    o->cheb_degree = 2;
    o->cheb_ratio = 30.0;
    o->cheb_boost = 1.1;
    o->power_iters = 10;
    o->omega_sym = 4.0 / 3.0;
    o->jacobi_omega = 2.0 / 3.0;
    o->jacobi_sweeps = 2;
    o->seed = 0;
}

static int csr_copy(Csr *dst, int n, int m, const int32_t *rp, const int32_t *ci, const double *va)
{
    int nnz = rp[n];
    dst->n = n; dst->m = m;
    dst->rowptr = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    dst->col = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    dst->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!dst->rowptr || !dst->col || !dst->val) return ORC_OUT_OF_MEMORY;
    memcpy(dst->rowptr, rp, sizeof(int) * (size_t)(n + 1));
    memcpy(dst->col, ci, sizeof(int) * (size_t)nnz);
    memcpy(dst->val, va, sizeof(double) * (size_t)nnz);
    return ORC_OK;
}

/*
 * Hierarchy construction.  Per level (sections 2 and 3): strength of
 * connection, dropping, aggregation, smoothed prolongator, Galerkin product
 * A_c = P^T A P (with the unfiltered A), coarse coordinates and tensors;
 * the smoother's spectral estimate is taken on every level but the last.
 * Coarsening stops once n <= max_coarse or max_levels levels exist; if the
 * level cap leaves more than max_coarse unknowns, or a level fails to shrink,
 * the status is ORC_STAGNATED.  The coarsest operator is factored densely.
 */
static void *dup_bytes(const void *src, size_t bytes)
{
    void *p = malloc(bytes > 0 ? bytes : 1);
    if (p && bytes) memcpy(p, src, bytes);
    return p;
}

/*
 * With prev == NULL: the full setup.  With prev: the same construction for
 * new values of A on prev's sparsity pattern, where everything that does not
 * depend on A's values is taken from prev instead of being recomputed --
 * coordinates and nodal tensors, strength values, drop masks, aggregates and
 * the number of levels -- and everything else (diagonals, filtered matrix,
 * damping, prolongator, Galerkin products, smoother bounds, coarse factor) is
 * computed from the new values as above.  The Dirichlet rows found in the new
 * values must be prev's.
 */
static int setup_impl(int n, const int32_t *rowptr, const int32_t *col, const double *val, int nelem, int npe,
                      const int32_t *elem_nodes, const double *elem_sigma, const double *coords,
                      const OrcOptions *opt, const Hier *prev, void **out)
{
    *out = NULL;
    if (n <= 0 || !opt || opt->dim < 1 || opt->dim > 3 || opt->max_levels < 1 || opt->max_levels > 16)
        return ORC_INVALID_ARG;
    if (prev && (prev->lev[0].A.n != n || prev->lev[0].A.rowptr[n] != rowptr[n])) return ORC_INVALID_ARG;
    Hier *h = (Hier *)calloc(1, sizeof(Hier));
    if (!h) return ORC_OUT_OF_MEMORY;
    h->opt = *opt;
    int d = opt->dim, ncomp = ncomp_of(d);
    int rc;
    Level *L0 = &h->lev[0];
    h->nlev = 1;
    L0->dim = d;
    rc = csr_copy(&L0->A, n, n, rowptr, col, val);
    if (rc) goto fail;
    if (prev) {
        for (int k = 0; k <= n; ++k)
            if (rowptr[k] != prev->lev[0].A.rowptr[k]) { rc = ORC_INVALID_ARG; goto fail; }
        for (int k = 0; k < rowptr[n]; ++k)
            if (col[k] != prev->lev[0].A.col[k]) { rc = ORC_INVALID_ARG; goto fail; }
        L0->x = (double *)dup_bytes(prev->lev[0].x, sizeof(double) * (size_t)n * d);
        L0->sig = (double *)dup_bytes(prev->lev[0].sig, sizeof(double) * (size_t)n * ncomp);
        if (!L0->x || !L0->sig) { rc = ORC_OUT_OF_MEMORY; goto fail; }
    } else {
        L0->x = (double *)malloc(sizeof(double) * (size_t)n * d);
        L0->sig = (double *)malloc(sizeof(double) * (size_t)n * ncomp);
        if (!L0->x || !L0->sig) { rc = ORC_OUT_OF_MEMORY; goto fail; }
        memcpy(L0->x, coords, sizeof(double) * (size_t)n * d);
        rc = orc_clement(n, d, nelem, npe, elem_nodes, elem_sigma, L0->sig);
        if (rc) goto fail;
    }

    for (int l = 0;; ++l) {
        Level *L = &h->lev[l];
        int nl = L->A.n, nnz = L->A.rowptr[nl];
        /* smoother diagonal */
        L->dinv = (double *)malloc(sizeof(double) * (size_t)nl);
        if (!L->dinv) { rc = ORC_OUT_OF_MEMORY; goto fail; }
        for (int i = 0; i < nl; ++i) {
            double di = 0.0;
            for (int k = L->A.rowptr[i]; k < L->A.rowptr[i + 1]; ++k)
                if (L->A.col[k] == i) di = L->A.val[k];
            L->dinv[i] = (di != 0.0) ? 1.0 / di : 0.0;
        }
        if (prev ? l + 1 == prev->nlev : (nl <= opt->max_coarse || l + 1 >= opt->max_levels)) {
            if (nl > opt->max_coarse) { rc = ORC_STAGNATED; goto fail; }
            break;
        }
        L->dir = (unsigned char *)calloc((size_t)nl, 1);
        L->lval = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        L->ldiag = (double *)malloc(sizeof(double) * (size_t)nl);
        L->S = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        L->mask = (unsigned char *)malloc((size_t)(nnz > 0 ? nnz : 1));
        L->agg = (int *)malloc(sizeof(int) * (size_t)nl);
        if (!L->dir || !L->lval || !L->ldiag || !L->S || !L->mask || !L->agg) { rc = ORC_OUT_OF_MEMORY; goto fail; }
        if (l == 0) orc_detect_dirichlet(nl, L->A.rowptr, L->A.col, L->A.val, L->dir);
        if (prev) {
            const Level *Q = &prev->lev[l];
            if (Q->A.n != nl || Q->A.rowptr[nl] != nnz) { rc = ORC_INVALID_ARG; goto fail; }
            if (memcmp(L->dir, Q->dir, (size_t)nl) != 0) { rc = ORC_INVALID_ARG; goto fail; }
            memcpy(L->lval, Q->lval, sizeof(double) * (size_t)nnz);
            memcpy(L->ldiag, Q->ldiag, sizeof(double) * (size_t)nl);
            memcpy(L->S, Q->S, sizeof(double) * (size_t)nnz);
            memcpy(L->mask, Q->mask, (size_t)nnz);
            memcpy(L->agg, Q->agg, sizeof(int) * (size_t)nl);
            L->nc = Q->nc;
            L->mis_rounds = Q->mis_rounds;
        } else {
            rc = orc_strength(nl, L->A.rowptr, L->A.col, L->A.val, d, L->x, L->sig, L->dir, opt->soc, opt->drop,
                              opt->theta, L->lval, L->ldiag, L->S, L->mask);
            if (rc) goto fail;
            rc = orc_aggregate(nl, L->A.rowptr, L->A.col, L->mask, L->dir, opt->seed, l, L->agg, &L->nc,
                               &L->mis_rounds, NULL);
            if (rc) goto fail;
        }
        if (L->nc <= 0 || L->nc >= nl) { rc = ORC_STAGNATED; goto fail; }
        rc = build_prolongator(L, opt, l);
        if (rc) goto fail;
        rc = transpose(&L->P, &L->R);
        if (rc) goto fail;
        Level *C = &h->lev[l + 1];
        C->dim = d;
        {
            Csr AP = {0};
            rc = spgemm(&L->A, &L->P, &AP);
            if (rc) { csr_free(&AP); goto fail; }
            rc = spgemm(&L->R, &AP, &C->A);
            csr_free(&AP);
            if (rc) goto fail;
        }
        h->nlev = l + 2;
        rc = coarse_aux(L, C);
        if (rc) goto fail;
    }
    /* spectral estimates for the smoother on every level that smooths */
    for (int l = 0; l + 1 < h->nlev; ++l) {
        Level *L = &h->lev[l];
        int nl = L->A.n;
        double *v = (double *)malloc(sizeof(double) * (size_t)nl);
        double *w = (double *)malloc(sizeof(double) * (size_t)nl);
        if (!v || !w) { free(v); free(w); rc = ORC_OUT_OF_MEMORY; goto fail; }
        L->lam_cheb = power_method(&L->A, L->dinv, opt->power_iters, stream_key(opt->seed, PURPOSE_CHEB, l), v, w);
        free(v); free(w);
    }
    /* coarsest level: dense Cholesky */
    {
        Level *C = &h->lev[h->nlev - 1];
        int nL = C->A.n;
        h->nL = nL;
        h->chol = (double *)calloc((size_t)nL * nL, sizeof(double));
        if (!h->chol) { rc = ORC_OUT_OF_MEMORY; goto fail; }
        for (int i = 0; i < nL; ++i)
            for (int k = C->A.rowptr[i]; k < C->A.rowptr[i + 1]; ++k)
                h->chol[(size_t)i * nL + C->A.col[k]] = C->A.val[k];
        rc = orc_dense_cholesky(nL, h->chol);
        if (rc) goto fail;
    }
    *out = h;
    return ORC_OK;
fail:
    orc_free(h);
    return rc;
}

int orc_setup(int n, const int32_t *rowptr, const int32_t *col, const double *val, int nelem, int npe,
              const int32_t *elem_nodes, const double *elem_sigma, const double *coords,
              const OrcOptions *opt, void **out)
{
    return setup_impl(n, rowptr, col, val, nelem, npe, elem_nodes, elem_sigma, coords, opt, NULL, out);
}

/* Setup for new values of A reusing prev's coordinates, tensors, masks,
 * aggregates and depth (setup_impl above); prev's options apply. */
int orc_setup_reuse(const void *prev, const int32_t *rowptr, const int32_t *col, const double *val, void **out)
{
    const Hier *p = (const Hier *)prev;
    *out = NULL;
    if (!p || p->nlev < 1) return ORC_INVALID_ARG;
    return setup_impl(p->lev[0].A.n, rowptr, col, val, 0, 0, NULL, NULL, NULL, &p->opt, p, out);
}

/*
 * Jacobi-preconditioned Chebyshev smoother of degree `deg` on the interval
 * [beta/ratio, beta], beta = boost * lambda (three-term Chebyshev
 * acceleration recurrence, Saad, Iterative Methods for Sparse Linear Systems,
 * 2nd ed., ch. 12).  From a zero initial guess the first residual is b.
 */
static void chebyshev(const Level *L, const OrcOptions *opt, const double *b, double *x, int zero_init,
                      double *r, double *d)
{
    int n = L->A.n;
    double beta = opt->cheb_boost * L->lam_cheb;
    double alpha = beta / opt->cheb_ratio;
    double theta = (beta + alpha) / 2.0;
    double delta = (beta - alpha) / 2.0;
    double s1 = theta / delta;
    double rho_old = 1.0 / s1;
    if (zero_init) {
        for (int i = 0; i < n; ++i) { d[i] = (L->dinv[i] * b[i]) / theta; x[i] = d[i]; }
    } else {
        spmv(&L->A, x, r);
        for (int i = 0; i < n; ++i) {
            r[i] = b[i] - r[i];
            d[i] = (L->dinv[i] * r[i]) / theta;
            x[i] = x[i] + d[i];
        }
    }
    for (int k = 1; k < opt->cheb_degree; ++k) {
        double rho = 1.0 / (2.0 * s1 - rho_old);
        double c1 = rho * rho_old;
        double c2 = 2.0 * rho / delta;
        spmv(&L->A, x, r);
        for (int i = 0; i < n; ++i) {
            r[i] = b[i] - r[i];
            d[i] = c1 * d[i] + c2 * (L->dinv[i] * r[i]);
            x[i] = x[i] + d[i];
        }
        rho_old = rho;
    }
}

/*
 * Damped Jacobi sweeps x += w D^{-1} (b - A x), D the diagonal of A.  The
 * weight is jacobi_omega, or (scaled option) jacobi_omega * 2 / beta with
 * beta = cheb_boost * lambda the upper end of the Chebyshev interval, so that
 * w * beta = 2 * jacobi_omega whatever the level's spectrum.
 */
static void jacobi(const Level *L, const OrcOptions *opt, const double *b, double *x, int zero_init, double *r)
{
    int n = L->A.n;
    double beta = opt->cheb_boost * L->lam_cheb;
    double w = opt->jacobi_omega;
    if (opt->smoother == SMOOTH_JACOBI_SCALED && beta > 0.0) w = opt->jacobi_omega * 2.0 / beta;
    for (int s = 0; s < opt->jacobi_sweeps; ++s) {
        if (zero_init && s == 0) {
            for (int i = 0; i < n; ++i) x[i] = w * (L->dinv[i] * b[i]);
            continue;
        }
        spmv(&L->A, x, r);
        for (int i = 0; i < n; ++i) x[i] = x[i] + w * (L->dinv[i] * (b[i] - r[i]));
    }
}

static void smooth(const Level *L, const OrcOptions *opt, const double *b, double *x, int zero_init, double *r,
                   double *d)
{
    if (opt->smoother == SMOOTH_JACOBI || opt->smoother == SMOOTH_JACOBI_SCALED) jacobi(L, opt, b, x, zero_init, r);
    else chebyshev(L, opt, b, x, zero_init, r, d);
}

/* Multigrid V-cycle (Algorithm "Vcycle"), zero initial guess on every level */
static int vcycle_rec(const Hier *h, int l, const double *b, double *u)
{
    const Level *L = &h->lev[l];
    int n = L->A.n;
    if (l == h->nlev - 1) {
        orc_dense_cholesky_solve(n, h->chol, b, u);
        return ORC_OK;
    }
    const Level *C = &h->lev[l + 1];
    int nc = C->A.n;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *bc = (double *)malloc(sizeof(double) * (size_t)nc);
    double *uc = (double *)malloc(sizeof(double) * (size_t)nc);
    double *pu = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !d || !bc || !uc || !pu) {
        free(r); free(d); free(bc); free(uc); free(pu);
        return ORC_OUT_OF_MEMORY;
    }
    smooth(L, &h->opt, b, u, 1, r, d);                 /* pre-smoothing */
    spmv(&L->A, u, r);
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];    /* residual */
    spmv(&L->R, r, bc);                                /* restriction P^T r */
    int rc = vcycle_rec(h, l + 1, bc, uc);
    if (rc == ORC_OK) {
        spmv(&L->P, uc, pu);                           /* prolongation */
        for (int i = 0; i < n; ++i) u[i] = u[i] + pu[i];
        smooth(L, &h->opt, b, u, 0, r, d);             /* post-smoothing */
    }
    free(r); free(d); free(bc); free(uc); free(pu);
    return rc;
}

int orc_vcycle(void *hv, const double *r, double *z)
{
    return vcycle_rec((const Hier *)hv, 0, r, z);
}

/*
 * Preconditioned CG (the outer Krylov solver of the numerical section):
 * converged when ||b - A x||_2 / ||b||_2 <= tol.  The recurrence residual is
 * tested first; on success the true residual is recomputed and, if it fails
 * the test, replaces the recurrence residual (residual replacement) and the
 * iteration continues.  `iters` counts the preconditioned steps taken.
 */
int orc_pcg(void *hv, const double *b, double *x, double tol, int maxit, int32_t *iters, double *relres)
{
    Hier *h = (Hier *)hv;
    const Csr *A = &h->lev[0].A;
    int n = A->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = ORC_OK;
    *iters = 0;
    *relres = 0.0;
    if (!r || !z || !p || !q) { rc = ORC_OUT_OF_MEMORY; goto done; }
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        goto done;
    }
    spmv(A, x, r);
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rel = sqrt(dot(n, r, r)) / bn;
    *relres = rel;
    if (rel <= tol) goto done;
    rc = orc_vcycle(h, r, z);
    if (rc) goto done;
    for (int i = 0; i < n; ++i) p[i] = z[i];
    double rz = dot(n, r, z);
    rc = ORC_NOT_CONVERGED;
    for (int it = 1; it <= maxit; ++it) {
        spmv(A, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) { rc = ORC_BREAKDOWN; *iters = it; break; }
        double alpha = rz / pq;
        for (int i = 0; i < n; ++i) { x[i] = x[i] + alpha * p[i]; r[i] = r[i] - alpha * q[i]; }
        *iters = it;
        rel = sqrt(dot(n, r, r)) / bn;
        if (rel <= tol) {
            spmv(A, x, q);
            for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
            double relt = sqrt(dot(n, q, q)) / bn;
            *relres = relt;
            if (relt <= tol) { rc = ORC_OK; break; }
            for (int i = 0; i < n; ++i) r[i] = q[i];
        }
        *relres = rel;
        int vrc = orc_vcycle(h, r, z);
        if (vrc) { rc = vrc; break; }
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
done:
    free(r); free(z); free(p); free(q);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* accessors for the tests                                                  */
/* ------------------------------------------------------------------------ */
int orc_num_levels(void *hv) { return ((Hier *)hv)->nlev; }

/* sizes: n, nnz, nc, nnzP, mis_rounds; scalars: omega, lam_pf, lam_cheb */
int orc_level_info(void *hv, int l, int64_t *sizes, double *scalars)
{
    Hier *h = (Hier *)hv;
    if (l < 0 || l >= h->nlev) return ORC_INVALID_ARG;
    Level *L = &h->lev[l];
    sizes[0] = L->A.n;
    sizes[1] = L->A.rowptr[L->A.n];
    sizes[2] = (l + 1 < h->nlev) ? L->nc : 0;
    sizes[3] = (l + 1 < h->nlev) ? L->P.rowptr[L->P.n] : 0;
    sizes[4] = L->mis_rounds;
    scalars[0] = L->omega;
    scalars[1] = L->lam_pf;
    scalars[2] = L->lam_cheb;
    return ORC_OK;
}

/* what: 0 A.rowptr 1 A.col 2 A.val 3 P.rowptr 4 P.col 5 P.val 6 R.rowptr
 * 7 R.col 8 R.val 9 agg 10 mask 11 x 12 sig 13 ldiag 14 S 15 dir 16 dinv
 * 17 lval 18 coarse Cholesky factor (dense, coarsest level only) */
int orc_level_get(void *hv, int l, int what, void *dst)
{
    Hier *h = (Hier *)hv;
    if (l < 0 || l >= h->nlev) return ORC_INVALID_ARG;
    Level *L = &h->lev[l];
    int n = L->A.n, nnz = L->A.rowptr[n];
    int last = (l + 1 == h->nlev);
    int ncomp = ncomp_of(L->dim);
    switch (what) {
    case 0: memcpy(dst, L->A.rowptr, sizeof(int) * (size_t)(n + 1)); return 0;
    case 1: memcpy(dst, L->A.col, sizeof(int) * (size_t)nnz); return 0;
    case 2: memcpy(dst, L->A.val, sizeof(double) * (size_t)nnz); return 0;
    case 11: memcpy(dst, L->x, sizeof(double) * (size_t)n * L->dim); return 0;
    case 12: memcpy(dst, L->sig, sizeof(double) * (size_t)n * ncomp); return 0;
    case 16: memcpy(dst, L->dinv, sizeof(double) * (size_t)n); return 0;
    case 18:
        if (!last) return ORC_INVALID_ARG;
        memcpy(dst, h->chol, sizeof(double) * (size_t)n * n);
        return 0;
    default: break;
    }
    if (last) return ORC_INVALID_ARG;
    int nnzp = L->P.rowptr[n];
    switch (what) {
    case 3: memcpy(dst, L->P.rowptr, sizeof(int) * (size_t)(n + 1)); return 0;
    case 4: memcpy(dst, L->P.col, sizeof(int) * (size_t)nnzp); return 0;
    case 5: memcpy(dst, L->P.val, sizeof(double) * (size_t)nnzp); return 0;
    case 6: memcpy(dst, L->R.rowptr, sizeof(int) * (size_t)(L->nc + 1)); return 0;
    case 7: memcpy(dst, L->R.col, sizeof(int) * (size_t)nnzp); return 0;
    case 8: memcpy(dst, L->R.val, sizeof(double) * (size_t)nnzp); return 0;
    case 9: memcpy(dst, L->agg, sizeof(int) * (size_t)n); return 0;
    case 10: memcpy(dst, L->mask, (size_t)nnz); return 0;
    case 13: memcpy(dst, L->ldiag, sizeof(double) * (size_t)n); return 0;
    case 14: memcpy(dst, L->S, sizeof(double) * (size_t)nnz); return 0;
    case 15: memcpy(dst, L->dir, (size_t)n); return 0;
    case 17: memcpy(dst, L->lval, sizeof(double) * (size_t)nnz); return 0;
    default: return ORC_INVALID_ARG;
    }
}

/* standalone pieces for pin tests */
int orc_spmv(int n, const int32_t *rowptr, const int32_t *col, const double *val, const double *x, double *y)
{
    Csr a = {n, n, (int *)rowptr, (int *)col, (double *)val};
    spmv(&a, x, y);
    return ORC_OK;
}

int orc_power_method(int n, const int32_t *rowptr, const int32_t *col, const double *val, const double *dscale,
                     int iters, uint64_t seed, int purpose, int level, double *lam)
{
    Csr a = {n, n, (int *)rowptr, (int *)col, (double *)val};
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!v || !w) { free(v); free(w); return ORC_OUT_OF_MEMORY; }
    uint64_t p = purpose == 0 ? PURPOSE_PF : PURPOSE_CHEB;
    *lam = power_method(&a, dscale, iters, stream_key(seed, p, level), v, w);
    free(v); free(w);
    return ORC_OK;
}

uint64_t orc_splitmix64(uint64_t x) { return splitmix64(x); }

/* one application of the level-l smoother (pre: zero_init=1, post: 0) */
int orc_smooth(void *hv, int l, const double *b, double *x, int zero_init)
{
    Hier *h = (Hier *)hv;
    if (l < 0 || l + 1 >= h->nlev) return ORC_INVALID_ARG;
    const Level *L = &h->lev[l];
    int n = L->A.n;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !d) { free(r); free(d); return ORC_OUT_OF_MEMORY; }
    smooth(L, &h->opt, b, x, zero_init, r, d);
    free(r); free(d);
    return ORC_OK;
}
