/*
 * cellsum.c -- CPU oracle of the truncated Gaussian kernel sums, float64,
 * with a uniform cell list so that large clouds fit in a bounded time.
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library (through oracle/cells.py).
 * The GPU library never calls, links or shares code with it.
 *
 * What it computes (paper: Cuomo, Galletti, Giunta, Starace, arXiv 1305.5179):
 *   - the operator y = A x of the interpolation system (Sec. II.B eq. RBFsys),
 *     A_ij = phi(|x_i - x_j|) when |x_i - x_j|^2 <= r_c^2 and 0 otherwise
 *     (Sec. III.A eq. matrixEntries and the finite-bandwidth remark after it);
 *   - the interpolant at evaluation points (Sec. II.B eq. matxvet),
 *     f(p) = sum_j c_j phi(|p - x_j|) with the same truncation;
 * with phi(r) = exp(-r^2 / (2 sigma^2)) and r^2 = (dx*dx + dy*dy) + dz*dz in
 * float64, the truncation test inclusive.  These are the definitions the
 * numpy oracle (rbf_oracle.py) writes as dense products; the cell list only
 * skips pairs farther apart than one cell, which the test would reject.
 *
 * Cell list: cubes of side s >= r_c over the centres' bounding box (s = r_c
 * unless that makes more than 1024 cells along an axis); the centres are
 * bucketed by cell in index order.  A query in cell q needs only the cells
 * q - 1 .. q + 1 on each axis (clipped to the box): every centre within r_c
 * of it lies there.  Without truncation (r_c = +inf) every query visits every
 * centre in index order.
 *
 * Per query the terms are added in a fixed order (cells by z, y, x, then
 * centres by index), so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t m;          /* centres */
    double *X;          /* m x 3, a copy */
    int dense;          /* no truncation */
    double rc, rc2;
    double lo[3], side;
    int64_t dims[3];
    int64_t *start;     /* ncells + 1 */
    int64_t *order;     /* centre indices bucketed by cell */
} cell_list;

static int64_t cell_coord(double v, double lo, double side) { return (int64_t)floor((v - lo) / side); }

void oracle_cells_free(cell_list *L) {
    if (!L) return;
    free(L->X);
    free(L->start);
    free(L->order);
    free(L);
}

/* Builds the cell list of the m centres X (m x 3, row-major).  rc > 0, or
 * +inf for no truncation.  Returns NULL when memory runs out. */
cell_list *oracle_cells_new(const double *X, int64_t m, double rc) {
    cell_list *L = (cell_list *)calloc(1, sizeof(cell_list));
    if (!L) return NULL;
    L->m = m;
    L->X = (double *)malloc(sizeof(double) * 3 * (size_t)(m > 0 ? m : 1));
    if (!L->X) { oracle_cells_free(L); return NULL; }
    memcpy(L->X, X, sizeof(double) * 3 * (size_t)m);
    L->rc = rc;
    L->rc2 = rc * rc;
    L->dense = !isfinite(rc);
    if (L->dense || m == 0) return L;
    double hi[3];
    for (int d = 0; d < 3; ++d) { L->lo[d] = INFINITY; hi[d] = -INFINITY; }
    for (int64_t i = 0; i < m; ++i)
        for (int d = 0; d < 3; ++d) {
            if (X[3 * i + d] < L->lo[d]) L->lo[d] = X[3 * i + d];
            if (X[3 * i + d] > hi[d]) hi[d] = X[3 * i + d];
        }
    double side = rc;
    for (int d = 0; d < 3; ++d)
        if ((hi[d] - L->lo[d]) / side > 1023.0) side = (hi[d] - L->lo[d]) / 1023.0;
    L->side = side;
    int64_t ncells = 1;
    for (int d = 0; d < 3; ++d) {
        L->dims[d] = cell_coord(hi[d], L->lo[d], side) + 1;
        ncells *= L->dims[d];
    }
    L->start = (int64_t *)calloc((size_t)ncells + 1, sizeof(int64_t));
    L->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    if (!L->start || !L->order || !cell) { free(cell); oracle_cells_free(L); return NULL; }
    for (int64_t i = 0; i < m; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            c[d] = cell_coord(X[3 * i + d], L->lo[d], side);
            if (c[d] >= L->dims[d]) c[d] = L->dims[d] - 1;
        }
        cell[i] = c[0] + L->dims[0] * (c[1] + L->dims[1] * c[2]);
        L->start[cell[i] + 1] += 1;
    }
    for (int64_t k = 0; k < ncells; ++k) L->start[k + 1] += L->start[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncells);
    if (!fill) { free(cell); oracle_cells_free(L); return NULL; }
    memcpy(fill, L->start, sizeof(int64_t) * (size_t)ncells);
    for (int64_t i = 0; i < m; ++i) L->order[fill[cell[i]]++] = i;   /* index order within a cell */
    free(fill);
    free(cell);
    return L;
}

/* sum_j w_j phi(|p - x_j|) over the centres within the truncation; adds the
 * pairs it kept and the pairs it tested to *useful / *examined. */
static double sum_at(const cell_list *L, const double *p, const double *w, double inv_two_s2, int64_t *useful,
                     int64_t *examined) {
    double acc = 0.0;
    int64_t u = 0, e = 0;
    if (L->dense) {
        for (int64_t j = 0; j < L->m; ++j) {
            const double *x = L->X + 3 * j;
            const double dx = p[0] - x[0], dy = p[1] - x[1], dz = p[2] - x[2];
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            acc += w[j] * exp(-r2 * inv_two_s2);
        }
        *useful += L->m;
        *examined += L->m;
        return acc;
    }
    int64_t q[3], a[3], b[3];
    for (int d = 0; d < 3; ++d) {
        q[d] = cell_coord(p[d], L->lo[d], L->side);
        a[d] = q[d] - 1 < 0 ? 0 : q[d] - 1;
        b[d] = q[d] + 1 > L->dims[d] - 1 ? L->dims[d] - 1 : q[d] + 1;
        if (a[d] > b[d]) return 0.0;   /* farther than one cell outside the box */
    }
    for (int64_t cz = a[2]; cz <= b[2]; ++cz)
        for (int64_t cy = a[1]; cy <= b[1]; ++cy)
            for (int64_t cx = a[0]; cx <= b[0]; ++cx) {
                const int64_t k = cx + L->dims[0] * (cy + L->dims[1] * cz);
                for (int64_t t = L->start[k]; t < L->start[k + 1]; ++t) {
                    const int64_t j = L->order[t];
                    const double *x = L->X + 3 * j;
                    const double dx = p[0] - x[0], dy = p[1] - x[1], dz = p[2] - x[2];
                    const double r2 = (dx * dx + dy * dy) + dz * dz;
                    ++e;
                    if (r2 <= L->rc2) {
                        acc += w[j] * exp(-r2 * inv_two_s2);
                        ++u;
                    }
                }
            }
    *useful += u;
    *examined += e;
    return acc;
}

/* y[k] = (A w)_{rows[k]} for k < nrows (rows NULL: every row, nrows = m),
 * on `threads` threads.  *useful / *examined (may be NULL): pairs kept and
 * tested. */
void oracle_cells_matvec(const cell_list *L, const double *w, double sigma, const int64_t *rows, int64_t nrows,
                         double *y, int threads, int64_t *useful, int64_t *examined) {
    const double inv_two_s2 = 1.0 / (2.0 * sigma * sigma);
    if (!rows) nrows = L->m;
    int64_t u = 0, e = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads) reduction(+ : u, e)
    for (int64_t k = 0; k < nrows; ++k) {
        const int64_t i = rows ? rows[k] : k;
        y[k] = sum_at(L, L->X + 3 * i, w, inv_two_s2, &u, &e);
    }
    if (useful) *useful = u;
    if (examined) *examined = e;
}

/* out[k] = f(pts[k]) = sum_j c_j phi(|pts[k] - x_j|), truncated (eq. matxvet). */
void oracle_cells_eval(const cell_list *L, const double *c, double sigma, const double *pts, int64_t npts,
                       double *out, int threads, int64_t *useful, int64_t *examined) {
    const double inv_two_s2 = 1.0 / (2.0 * sigma * sigma);
    int64_t u = 0, e = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads) reduction(+ : u, e)
    for (int64_t k = 0; k < npts; ++k) out[k] = sum_at(L, pts + 3 * k, c, inv_two_s2, &u, &e);
    if (useful) *useful = u;
    if (examined) *examined = e;
}

/* The pairs (i, j) with |x_i - x_j|^2 <= r_c^2 of the given rows (rows
 * NULL: every row): the nonzeros of those rows of A, counted with the same
 * test as the sums, without evaluating phi. */
int64_t oracle_cells_count(const cell_list *L, const int64_t *rows, int64_t nrows, int threads) {
    if (!rows) nrows = L->m;
    if (L->dense) return nrows * L->m;
    int64_t u = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads) reduction(+ : u)
    for (int64_t k = 0; k < nrows; ++k) {
        const double *p = L->X + 3 * (rows ? rows[k] : k);
        int64_t q[3], a[3], b[3];
        int empty = 0;
        for (int d = 0; d < 3; ++d) {
            q[d] = cell_coord(p[d], L->lo[d], L->side);
            a[d] = q[d] - 1 < 0 ? 0 : q[d] - 1;
            b[d] = q[d] + 1 > L->dims[d] - 1 ? L->dims[d] - 1 : q[d] + 1;
            if (a[d] > b[d]) empty = 1;
        }
        if (empty) continue;
        for (int64_t cz = a[2]; cz <= b[2]; ++cz)
            for (int64_t cy = a[1]; cy <= b[1]; ++cy)
                for (int64_t cx = a[0]; cx <= b[0]; ++cx) {
                    const int64_t c = cx + L->dims[0] * (cy + L->dims[1] * cz);
                    for (int64_t t = L->start[c]; t < L->start[c + 1]; ++t) {
                        const double *x = L->X + 3 * L->order[t];
                        const double dx = p[0] - x[0], dy = p[1] - x[1], dz = p[2] - x[2];
                        if ((dx * dx + dy * dy) + dz * dz <= L->rc2) ++u;
                    }
                }
    }
    return u;
}

/* Threads an OpenMP region gets by default on this host. */
int oracle_cells_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
