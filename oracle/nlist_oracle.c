/*
 * Neighbor-list oracle: the neighbor search problem computed by its definition.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Definition (paper, Introduction and Section 4 "Performance": the neighbors
 * of particle i are the particles within the cutoff of i under periodic
 * boundary conditions; Section 2.3, eq. (2): overlap is decided with "<=";
 * Fig. 2 caption: a particle is not its own neighbor):
 *
 *   S_i = { j != i : d_ij^2 <= r_list(t_i, t_j)^2 }
 *   d_ij^2 = (dx_0*dx_0 + dx_1*dx_1) + dx_2*dx_2
 *   dx_d   = (x_j,d - x_i,d) - L_d * round((x_j,d - x_i,d) / L_d)
 *
 * All arithmetic is IEEE fp64, in the order written above, with no
 * contraction into fused multiply-adds (build with -ffp-contract=off).
 * Positions come in as fp64: fp32 data converted exactly (the paper's fp32
 * case), or fp64 data as given (its fp64 case, Section 2.2 and Figs. 4-7).  r_list^2 is supplied by the caller per type pair;
 * a negative value means the pair of types is never listed.
 *
 * Two independent ways to evaluate S_i:
 *   - oracle_*_brute: every pair (i, j), O(N^2);
 *   - oracle_*_cells: a cell list with cells no narrower than the largest
 *     list radius and a 27-cell stencil per query (paper, Introduction,
 *     "grid" approach), usable for a chosen subset of queries.
 * Rows are returned in ascending j.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double pair_d2(const double *pi, const double *pj, const double *L)
{
    double dx[3];
    for (int d = 0; d < 3; ++d) {
        double diff = (double)pj[d] - (double)pi[d];
        dx[d] = diff - L[d] * round(diff / L[d]);
    }
    return (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
}

static int type_of(const int32_t *type, int64_t i)
{
    return type ? type[i] : 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- brute force */

/* count[q] = |S_{queries[q]}| (queries == NULL means all particles). */
int oracle_count_brute(int64_t n, const double *pos, const int32_t *type, int32_t ntypes,
                       const double *box, const double *rlist2, int64_t nq,
                       const int64_t *queries, int64_t *count, int nthreads)
{
    if (n < 0 || nq < 0 || !box || !rlist2 || !count || (n > 0 && !pos))
        return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = queries ? queries[q] : q;
        int ti = type_of(type, i);
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double r2 = rlist2[ti * ntypes + type_of(type, j)];
            if (pair_d2(pos + 3 * i, pos + 3 * j, box) <= r2)
                ++c;
        }
        count[q] = c;
    }
    return 0;
}

/* Fill rows: row q occupies cols[row_ptr[q] .. row_ptr[q+1]). */
int oracle_fill_brute(int64_t n, const double *pos, const int32_t *type, int32_t ntypes,
                      const double *box, const double *rlist2, int64_t nq,
                      const int64_t *queries, const int64_t *row_ptr, int32_t *cols,
                      int nthreads)
{
    if (n < 0 || nq < 0 || !box || !rlist2 || !row_ptr || (n > 0 && !pos))
        return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = queries ? queries[q] : q;
        int ti = type_of(type, i);
        int64_t o = row_ptr[q];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double r2 = rlist2[ti * ntypes + type_of(type, j)];
            if (pair_d2(pos + 3 * i, pos + 3 * j, box) <= r2)
                cols[o++] = (int32_t)j;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ cell list */

typedef struct {
    int64_t nc[3];
    double width[3];
    int64_t *start; /* [ncells + 1] */
    int32_t *item;  /* [n] particle indices, grouped by cell, ascending within a cell */
} cells_t;

static int64_t cell_coord(double x, double w, int64_t nc)
{
    double c = floor(x / w);
    if (!(c >= 0.0)) /* also catches NaN */
        c = 0.0;
    if (c > (double)(nc - 1))
        c = (double)(nc - 1);
    return (int64_t)c;
}

static int64_t cell_of(const cells_t *g, const double *p)
{
    int64_t c0 = cell_coord((double)p[0], g->width[0], g->nc[0]);
    int64_t c1 = cell_coord((double)p[1], g->width[1], g->nc[1]);
    int64_t c2 = cell_coord((double)p[2], g->width[2], g->nc[2]);
    return (c2 * g->nc[1] + c1) * g->nc[0] + c0;
}

/* Cells are at least rmax*(1+1e-9) wide, so two particles within rmax of each
 * other (minimum image) sit in cells whose coordinates differ by at most one,
 * modulo the cell count.  Returns 0 when fewer than 3 cells fit on an axis
 * (the 27 stencil cells would then not be distinct). */
static int cells_build(cells_t *g, int64_t n, const double *pos, const double *box, double rmax)
{
    memset(g, 0, sizeof(*g));
    for (int d = 0; d < 3; ++d) {
        double w = rmax * (1.0 + 1e-9);
        int64_t nc = (w > 0.0) ? (int64_t)floor(box[d] / w) : 3;
        if (nc > 1024)
            nc = 1024;
        if (nc < 3)
            return 0;
        g->nc[d] = nc;
        g->width[d] = box[d] / (double)nc;
    }
    int64_t ncell = g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->item = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *cid = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->start || !g->item || !cid) {
        free(g->start);
        free(g->item);
        free(cid);
        memset(g, 0, sizeof(*g));
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        cid[i] = cell_of(g, pos + 3 * i);
    for (int64_t i = 0; i < n; ++i)
        g->start[cid[i] + 1]++;
    for (int64_t c = 0; c < ncell; ++c)
        g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    if (!fill) {
        free(g->start);
        free(g->item);
        free(cid);
        memset(g, 0, sizeof(*g));
        return -1;
    }
    memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) /* ascending i within each cell */
        g->item[fill[cid[i]]++] = (int32_t)i;
    free(fill);
    free(cid);
    return 1;
}

static void cells_free(cells_t *g)
{
    free(g->start);
    free(g->item);
    memset(g, 0, sizeof(*g));
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Visit the 27 stencil cells of particle i; count or store its neighbors. */
static int64_t cells_row(const cells_t *g, int64_t i, const double *pos, const int32_t *type,
                         int32_t ntypes, const double *box, const double *rlist2, int32_t *out)
{
    int64_t c0 = cell_coord((double)pos[3 * i + 0], g->width[0], g->nc[0]);
    int64_t c1 = cell_coord((double)pos[3 * i + 1], g->width[1], g->nc[1]);
    int64_t c2 = cell_coord((double)pos[3 * i + 2], g->width[2], g->nc[2]);
    int ti = type_of(type, i);
    int64_t c = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        int64_t z = (c2 + dz + g->nc[2]) % g->nc[2];
        for (int dy = -1; dy <= 1; ++dy) {
            int64_t y = (c1 + dy + g->nc[1]) % g->nc[1];
            for (int dxc = -1; dxc <= 1; ++dxc) {
                int64_t x = (c0 + dxc + g->nc[0]) % g->nc[0];
                int64_t cell = (z * g->nc[1] + y) * g->nc[0] + x;
                for (int64_t s = g->start[cell]; s < g->start[cell + 1]; ++s) {
                    int64_t j = g->item[s];
                    if (j == i)
                        continue;
                    double r2 = rlist2[ti * ntypes + type_of(type, j)];
                    if (pair_d2(pos + 3 * i, pos + 3 * j, box) <= r2) {
                        if (out)
                            out[c] = (int32_t)j;
                        ++c;
                    }
                }
            }
        }
    }
    if (out)
        qsort(out, (size_t)c, sizeof(int32_t), cmp_i32);
    return c;
}

static double max_radius(int32_t ntypes, const double *rlist2)
{
    double m = 0.0;
    for (int32_t k = 0; k < ntypes * ntypes; ++k)
        if (rlist2[k] > m)
            m = rlist2[k];
    return sqrt(m);
}

/* Returns 0 on success, 1 when the box is too small for a 3x3x3 stencil
 * (the caller then uses the brute-force functions), -1 on error. */
int oracle_count_cells(int64_t n, const double *pos, const int32_t *type, int32_t ntypes,
                       const double *box, const double *rlist2, int64_t nq,
                       const int64_t *queries, int64_t *count, int nthreads)
{
    if (n < 0 || nq < 0 || !box || !rlist2 || !count || (n > 0 && !pos))
        return -1;
    set_threads(nthreads);
    cells_t g;
    int ok = cells_build(&g, n, pos, box, max_radius(ntypes, rlist2));
    if (ok <= 0)
        return ok == 0 ? 1 : -1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = queries ? queries[q] : q;
        count[q] = cells_row(&g, i, pos, type, ntypes, box, rlist2, NULL);
    }
    cells_free(&g);
    return 0;
}

int oracle_fill_cells(int64_t n, const double *pos, const int32_t *type, int32_t ntypes,
                      const double *box, const double *rlist2, int64_t nq,
                      const int64_t *queries, const int64_t *row_ptr, int32_t *cols,
                      int nthreads)
{
    if (n < 0 || nq < 0 || !box || !rlist2 || !row_ptr || (n > 0 && !pos))
        return -1;
    set_threads(nthreads);
    cells_t g;
    int ok = cells_build(&g, n, pos, box, max_radius(ntypes, rlist2));
    if (ok <= 0)
        return ok == 0 ? 1 : -1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = queries ? queries[q] : q;
        cells_row(&g, i, pos, type, ntypes, box, rlist2, cols + row_ptr[q]);
    }
    cells_free(&g);
    return 0;
}

/* Squared minimum-image distance of one pair, exposed for band-pair reports. */
double oracle_pair_d2(const double *pi, const double *pj, const double *box)
{
    return pair_d2(pi, pj, box);
}

/* ----------------------------------------------------------------- band pairs */

/* Pairs near the cutoff, where a floating-point evaluation of the distance in
 * another order can take the other side of eq. (2)'s inclusive test.  For each
 * query i and each j != i of a listed type pair (r = sqrt(rlist2) > 0):
 *   rel_count[q] += |d_ij - r| <= rel * r      (relative reading)
 *   abs_count[q] += |d_ij - r| <= abs_tol      (absolute reading, sigma units)
 * with d_ij = sqrt(d_ij^2) of the definition above.  Candidates come from a
 * cell list whose cells are at least max(r (1 + rel), r + abs_tol) wide, or,
 * with use_cells = 0, from every pair. */
static double band_reach(int32_t ntypes, const double *rlist2, double rel, double abs_tol)
{
    double m = 0.0;
    for (int32_t k = 0; k < ntypes * ntypes; ++k) {
        if (!(rlist2[k] > 0.0))
            continue;
        double r = sqrt(rlist2[k]);
        double a = r * (1.0 + rel), b = r + abs_tol;
        double e = a > b ? a : b;
        if (e > m)
            m = e;
    }
    return m;
}

static void band_pair(const double *pi, const double *pj, const double *box, double r2,
                      double rel, double abs_tol, int64_t *nrel, int64_t *nabs)
{
    if (!(r2 > 0.0))
        return;
    double r = sqrt(r2);
    double dev = fabs(sqrt(pair_d2(pi, pj, box)) - r);
    if (dev <= rel * r)
        ++*nrel;
    if (dev <= abs_tol)
        ++*nabs;
}

int oracle_band_count(int64_t n, const double *pos, const int32_t *type, int32_t ntypes,
                      const double *box, const double *rlist2, int64_t nq, const int64_t *queries,
                      double rel, double abs_tol, int use_cells, int64_t *rel_count,
                      int64_t *abs_count, int nthreads)
{
    if (n < 0 || nq < 0 || !box || !rlist2 || !rel_count || !abs_count || (n > 0 && !pos) ||
        !(rel >= 0.0) || !(abs_tol >= 0.0))
        return -1;
    set_threads(nthreads);
    cells_t g;
    int ok = 0;
    if (use_cells) {
        ok = cells_build(&g, n, pos, box, band_reach(ntypes, rlist2, rel, abs_tol));
        if (ok < 0)
            return -1;
        if (ok == 0)
            return 1;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = queries ? queries[q] : q;
        int ti = type_of(type, i);
        int64_t a = 0, b = 0;
        if (!use_cells) {
            for (int64_t j = 0; j < n; ++j)
                if (j != i)
                    band_pair(pos + 3 * i, pos + 3 * j, box, rlist2[ti * ntypes + type_of(type, j)],
                              rel, abs_tol, &a, &b);
        } else {
            int64_t c0 = cell_coord((double)pos[3 * i + 0], g.width[0], g.nc[0]);
            int64_t c1 = cell_coord((double)pos[3 * i + 1], g.width[1], g.nc[1]);
            int64_t c2 = cell_coord((double)pos[3 * i + 2], g.width[2], g.nc[2]);
            for (int dz = -1; dz <= 1; ++dz) {
                int64_t z = (c2 + dz + g.nc[2]) % g.nc[2];
                for (int dy = -1; dy <= 1; ++dy) {
                    int64_t y = (c1 + dy + g.nc[1]) % g.nc[1];
                    for (int dxc = -1; dxc <= 1; ++dxc) {
                        int64_t x = (c0 + dxc + g.nc[0]) % g.nc[0];
                        int64_t cell = (z * g.nc[1] + y) * g.nc[0] + x;
                        for (int64_t s = g.start[cell]; s < g.start[cell + 1]; ++s) {
                            int64_t j = g.item[s];
                            if (j != i)
                                band_pair(pos + 3 * i, pos + 3 * j, box,
                                          rlist2[ti * ntypes + type_of(type, j)], rel, abs_tol, &a, &b);
                        }
                    }
                }
            }
        }
        rel_count[q] = a;
        abs_count[q] = b;
    }
    if (use_cells)
        cells_free(&g);
    return 0;
}
