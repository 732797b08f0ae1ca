/*
 * Row-streamed assembly of the structured 3D Q1 systems built by q1.py
 * (input generation only; none of the multigrid method's arithmetic).
 *
 * It reproduces q1.assemble_q1 bit for bit for dim = 3: the same node and
 * slot numbering, the same order of every floating-point operation
 * (element contributions to a stored entry and to the load vector added in
 * ascending local vertex index a, element tensors summed over (p, q) in
 * row-major order skipping zero reference integrals, Dirichlet corrections
 * in ascending slot order), so the fast path can replace the numpy loops.
 * Build with -ffp-contract=off: a fused multiply-add would change roundings.
 *
 * Conventions: node (ix, iy, iz) = ix + N0*(iy + N1*iz), N_k = n_k + 1;
 * element (ex, ey, ez) = ex + n0*(ey + n1*ez); local vertex a has bits
 * (a&1, (a>>1)&1, (a>>2)&1); slot s = (dz+1)*9 + (dy+1)*3 + (dx+1) for the
 * neighbour offset (dx, dy, dz).
 */
#include <stdint.h>

typedef struct {
    int64_t nx, ny, nz;
    int iso;              /* 1: sigma_e = kiso_e * I on every element */
    const double *kiso;   /* [nelem] (iso) */
    const double *sig;    /* [nelem][3][3] (not iso) */
    const double *G;      /* [3][3][8][8] reference gradient integrals */
    const double *Gsum;   /* [8][8] = G00 + G11 + G22 (iso) */
    const double *fg;     /* [nelem] element source times vol / 8 */
    const uint8_t *dmask; /* [n] Dirichlet nodes */
    const double *g;      /* [n] Dirichlet values (0 elsewhere) */
} q1_input;

static double entry(const q1_input *in, int64_t ix, int64_t iy, int64_t iz, int dx, int dy, int dz)
{
    double v = 0.0;
    for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        const int bx = ax + dx, by = ay + dy, bz = az + dz;
        if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
        const int64_t ex = ix - ax, ey = iy - ay, ez = iz - az;
        if (ex < 0 || ex >= in->nx || ey < 0 || ey >= in->ny || ez < 0 || ez >= in->nz) continue;
        const int64_t e = ex + in->nx * (ey + in->ny * ez);
        const int bb = bx | (by << 1) | (bz << 2);
        double ke;
        if (in->iso) {
            ke = in->kiso[e] * in->Gsum[a * 8 + bb];
        } else {
            ke = 0.0;
            const double *s = in->sig + e * 9;
            for (int pq = 0; pq < 9; ++pq) {
                const double gpq = in->G[pq * 64 + a * 8 + bb];
                if (gpq != 0.0) ke += s[pq] * gpq;
            }
        }
        v += ke;
    }
    return v;
}

/* Pass 1: rowptr[0..n] (counts after Dirichlet elimination). Returns nnz. */
int64_t q1_rowptr_3d(const q1_input *in, int64_t *rowptr)
{
    const int64_t N0 = in->nx + 1, N1 = in->ny + 1, N2 = in->nz + 1;
    int64_t k = 0;
    rowptr[0] = 0;
    for (int64_t iz = 0; iz < N2; ++iz)
        for (int64_t iy = 0; iy < N1; ++iy)
            for (int64_t ix = 0; ix < N0; ++ix) {
                const int64_t i = ix + N0 * (iy + N1 * iz);
                if (in->dmask[i]) {
                    ++k;
                } else {
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const int64_t jx = ix + dx, jy = iy + dy, jz = iz + dz;
                                if (jx < 0 || jx >= N0 || jy < 0 || jy >= N1 || jz < 0 || jz >= N2) continue;
                                const int64_t j = jx + N0 * (jy + N1 * jz);
                                if (j != i && in->dmask[j]) continue;
                                ++k;
                            }
                }
                rowptr[i + 1] = k;
            }
    return k;
}

/* Pass 2: rows [row0, row1) of col / val / b; rowptr from pass 1. */
void q1_fill_3d(const q1_input *in, const int64_t *rowptr, int64_t row0, int64_t row1, int32_t *col,
                double *val, double *b)
{
    const int64_t N0 = in->nx + 1, N1 = in->ny + 1, N2 = in->nz + 1;
    for (int64_t i = row0; i < row1; ++i) {
        const int64_t ix = i % N0, iy = (i / N0) % N1, iz = i / (N0 * N1);
        /* load vector: sum over local vertices a in ascending order */
        double bi = 0.0;
        for (int a = 0; a < 8; ++a) {
            const int64_t ex = ix - (a & 1), ey = iy - ((a >> 1) & 1), ez = iz - ((a >> 2) & 1);
            if (ex < 0 || ex >= in->nx || ey < 0 || ey >= in->ny || ez < 0 || ez >= in->nz) continue;
            bi += in->fg[ex + in->nx * (ey + in->ny * ez)];
        }
        int64_t k = rowptr[i];
        const int di = in->dmask[i] != 0;
        double diag = 0.0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int64_t jx = ix + dx, jy = iy + dy, jz = iz + dz;
                    if (jx < 0 || jx >= N0 || jy < 0 || jy >= N1 || jz < 0 || jz >= N2) continue;
                    const int64_t j = jx + N0 * (jy + N1 * jz);
                    const double v = entry(in, ix, iy, iz, dx, dy, dz);
                    if (j == i) {
                        diag = v;
                    } else if (di || in->dmask[j]) {
                        if (!di) bi -= v * in->g[j];
                        continue;
                    }
                    col[k] = (int32_t)j;
                    val[k] = v;
                    ++k;
                }
        if (di) bi = diag * in->g[i];
        b[i] = bi;
    }
}
