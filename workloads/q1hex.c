/*
 * Trilinear (Q1) hexahedra of general shape on a structured index space whose
 * second direction may be periodic (input generation only: none of the
 * multigrid method's arithmetic).  Used for the annulus, whose elements are
 * mapped from a polar (r, phi, z) grid.
 *
 * Node (i, j, k) has id i + N0*(j + N1*k) with N0 = n0 + 1 and N1 = n1 + 1,
 * or N1 = n1 when direction 1 is periodic (node j = n1 is node 0).  Element
 * (e0, e1, e2) has id e0 + n0*(e1 + n1*e2) and local vertex a with bits
 * (a&1, (a>>1)&1, (a>>2)&1) at node (e0 + a0, e1 + a1 [mod n1], e2 + a2).
 *
 * Element stiffness with 2x2x2 Gauss points g on the reference cube [0,1]^3:
 *   K_ab = sum_g w_g |det J_g| (J_g^{-T} dN_a)^T sigma_e (J_g^{-T} dN_b),
 * J_pq = dx_p / dxi_q, computed for a <= b and mirrored (bitwise symmetric).
 * Element load L_a = sum_g w_g |det J_g| N_a (times the element's source).
 * 2-point Gauss integrates the stiffness of a box exactly and passes the
 * patch test on general trilinear hexes (the adjugate of J is of degree <= 2
 * per reference coordinate).  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t n0, n1, n2;   /* elements per direction */
    int32_t periodic1;    /* direction 1 wraps around */
    const double *X;      /* [nnode][3] coordinates */
    const double *sig;    /* [nelem][3][3] element tensors */
    const double *fe;     /* [nelem] element-constant source, or NULL */
    const uint8_t *dmask; /* [nnode] Dirichlet flags */
    const double *g;      /* [nnode] Dirichlet values */
} hex_input;

static void shape_fn(const double xi[3], int a, double *N, double dN[3])
{
    const int b0 = a & 1, b1 = (a >> 1) & 1, b2 = (a >> 2) & 1;
    const double f0 = b0 ? xi[0] : 1.0 - xi[0], d0 = b0 ? 1.0 : -1.0;
    const double f1 = b1 ? xi[1] : 1.0 - xi[1], d1 = b1 ? 1.0 : -1.0;
    const double f2 = b2 ? xi[2] : 1.0 - xi[2], d2 = b2 ? 1.0 : -1.0;
    *N = f0 * f1 * f2;
    dN[0] = d0 * f1 * f2;
    dN[1] = f0 * d1 * f2;
    dN[2] = f0 * f1 * d2;
}

static int64_t nodes1(const hex_input *in) { return in->periodic1 ? in->n1 : in->n1 + 1; }

static int64_t node_id(const hex_input *in, int64_t i, int64_t j, int64_t k)
{
    const int64_t N1 = nodes1(in);
    if (in->periodic1) j = ((j % N1) + N1) % N1;
    return i + (in->n0 + 1) * (j + N1 * k);
}

/* Ke [64] (row-major) and, if Le, the load weights Le [8] of element e.  0, or -1 if degenerate. */
static int element(const hex_input *in, int64_t e, double *Ke, double *Le)
{
    const int64_t e0 = e % in->n0, e1 = (e / in->n0) % in->n1, e2 = e / (in->n0 * in->n1);
    double X[8][3], S[3][3];
    for (int a = 0; a < 8; ++a) {
        const int64_t v = node_id(in, e0 + (a & 1), e1 + ((a >> 1) & 1), e2 + ((a >> 2) & 1));
        for (int p = 0; p < 3; ++p) X[a][p] = in->X[v * 3 + p];
    }
    for (int p = 0; p < 3; ++p)
        for (int r = 0; r < 3; ++r) S[p][r] = in->sig[e * 9 + p * 3 + r];
    const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    for (int t = 0; t < 64; ++t) Ke[t] = 0.0;
    if (Le)
        for (int a = 0; a < 8; ++a) Le[a] = 0.0;
    for (int q = 0; q < 8; ++q) {
        const double xi[3] = {gp[q & 1], gp[(q >> 1) & 1], gp[(q >> 2) & 1]};
        double N[8], dN[8][3], J[3][3];
        for (int a = 0; a < 8; ++a) shape_fn(xi, a, &N[a], dN[a]);
        for (int p = 0; p < 3; ++p)
            for (int r = 0; r < 3; ++r) {
                double s = 0.0;
                for (int a = 0; a < 8; ++a) s += X[a][p] * dN[a][r];
                J[p][r] = s;
            }
        /* C = cofactor matrix of J, det J = sum_r J[0][r] C[0][r]; J^{-T} = C / det */
        double C[3][3];
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        if (!(det != 0.0) || !isfinite(det)) return -1;
        const double w = 0.125 * fabs(det);
        double B[8][3], SB[8][3];
        for (int a = 0; a < 8; ++a) {
            for (int p = 0; p < 3; ++p) {
                double s = 0.0;
                for (int r = 0; r < 3; ++r) s += C[p][r] * dN[a][r];
                B[a][p] = s / det;
            }
            for (int p = 0; p < 3; ++p) {
                double s = 0.0;
                for (int r = 0; r < 3; ++r) s += S[p][r] * B[a][r];
                SB[a][p] = s;
            }
        }
        for (int a = 0; a < 8; ++a)
            for (int b = a; b < 8; ++b) {
                double s = 0.0;
                for (int p = 0; p < 3; ++p) s += B[a][p] * SB[b][p];
                Ke[a * 8 + b] += w * s;
            }
        if (Le)
            for (int a = 0; a < 8; ++a) Le[a] += w * N[a];
    }
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < a; ++b) Ke[a * 8 + b] = Ke[b * 8 + a];
    return 0;
}

/* Pass 1: Ke [nelem][64] and optionally Le [nelem][8] for elements [e_lo, e_hi).  0, or -1 (degenerate element). */
int hex_elements(const hex_input *in, int64_t e_lo, int64_t e_hi, double *Ke, double *Le)
{
    for (int64_t e = e_lo; e < e_hi; ++e)
        if (element(in, e, Ke + e * 64, Le ? Le + e * 8 : NULL) != 0) return -1;
    return 0;
}

/* columns of row (ix, iy, iz) with their offset slots (dz+1)*9 + (dy+1)*3 + (dx+1), ascending by column */
static int row_columns(const hex_input *in, int64_t ix, int64_t iy, int64_t iz, int64_t cols[27], int slots[27])
{
    const int64_t N0 = in->n0 + 1, N1 = nodes1(in), N2 = in->n2 + 1;
    int np = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int64_t jx = ix + dx, jy = iy + dy, jz = iz + dz;
                if (jx < 0 || jx >= N0 || jz < 0 || jz >= N2) continue;
                if (!in->periodic1 && (jy < 0 || jy >= N1)) continue;
                const int64_t c = node_id(in, jx, jy, jz);
                const int s = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                int p = np++;
                while (p > 0 && cols[p - 1] > c) { /* insertion sort */
                    cols[p] = cols[p - 1];
                    slots[p] = slots[p - 1];
                    --p;
                }
                cols[p] = c;
                slots[p] = s;
            }
    return np;
}

/* Pass 2: row pointer after symmetric Dirichlet elimination (Dirichlet rows keep the diagonal only).  Returns nnz. */
int64_t hex_rowptr(const hex_input *in, int64_t *rowptr)
{
    const int64_t N0 = in->n0 + 1, N1 = nodes1(in), N2 = in->n2 + 1;
    int64_t k = 0;
    rowptr[0] = 0;
    for (int64_t i = 0; i < N0 * N1 * N2; ++i) {
        if (in->dmask[i]) {
            ++k;
        } else {
            int64_t cols[27];
            int slots[27];
            const int np = row_columns(in, i % N0, (i / N0) % N1, i / (N0 * N1), cols, slots);
            for (int p = 0; p < np; ++p)
                if (cols[p] == i || !in->dmask[cols[p]]) ++k;
        }
        rowptr[i + 1] = k;
    }
    return k;
}

/*
 * Pass 3: rows [row0, row1).  Entry (i, j) is the sum over the elements that
 * hold node i, in ascending local index a of node i, of Ke[a][b(j)]; b_i is
 * the sum in the same order of fe * Le[a].  Dirichlet elimination: a free
 * row loses its Dirichlet columns (b_i -= a_ij g_j, ascending j); a Dirichlet
 * row keeps its diagonal a_ii and b_i = a_ii g_i.
 */
void hex_fill(const hex_input *in, const double *Ke, const double *Le, const int64_t *rowptr, int64_t row0,
              int64_t row1, int32_t *col, double *val, double *b)
{
    const int64_t N0 = in->n0 + 1, N1 = nodes1(in);
    for (int64_t i = row0; i < row1; ++i) {
        const int64_t ix = i % N0, iy = (i / N0) % N1, iz = i / (N0 * N1);
        double v27[27];
        for (int s = 0; s < 27; ++s) v27[s] = 0.0;
        double bi = 0.0;
        for (int a = 0; a < 8; ++a) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
            const int64_t ex = ix - ax, ez = iz - az;
            int64_t ey = iy - ay;
            if (ex < 0 || ex >= in->n0 || ez < 0 || ez >= in->n2) continue;
            if (in->periodic1) ey = (ey + in->n1) % in->n1;
            else if (ey < 0 || ey >= in->n1) continue;
            const int64_t e = ex + in->n0 * (ey + in->n1 * ez);
            if (in->fe) bi += in->fe[e] * Le[e * 8 + a];
            for (int bb = 0; bb < 8; ++bb) {
                const int dx = (bb & 1) - ax, dy = ((bb >> 1) & 1) - ay, dz = ((bb >> 2) & 1) - az;
                v27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] += Ke[e * 64 + a * 8 + bb];
            }
        }
        int64_t cols[27];
        int slots[27];
        const int np = row_columns(in, ix, iy, iz, cols, slots);
        const int di = in->dmask[i] != 0;
        int64_t k = rowptr[i];
        for (int p = 0; p < np; ++p) {
            const int64_t j = cols[p];
            const double v = v27[slots[p]];
            if (j != i && (di || in->dmask[j])) {
                if (!di) bi -= v * in->g[j];
                continue;
            }
            if (j == i && di) bi = v * in->g[i];
            col[k] = (int32_t)j;
            val[k] = v;
            ++k;
        }
        b[i] = bi;
    }
}
