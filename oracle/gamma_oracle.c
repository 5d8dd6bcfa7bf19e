/*
 * FP64 CPU oracle for the gamma index of Gu, Jia & Jiang, "GPU-based fast gamma index
 * calculation" (arXiv:1012.1900).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with the GPU
 * library, and the GPU library never calls it.
 *
 * What it computes (Sec. 2.1, Eq. (1)): for every reference node r inside the dose
 * threshold,
 *     gamma(r) = min over points x of the evaluation surface of |r~ - x~|,
 *     r~ = (r / DTA, D_r(r) / dD),   x~ = (x / DTA, D_e(x) / dD),
 * where the evaluation surface is the graph of the piecewise-linear interpolant of D_e
 * over the Kuhn triangulation of the common grid (each cube split into d! simplices
 * along its main diagonal).  This is the "geometric method" the paper adopts: gamma is
 * the distance from the normalised reference point to the continuous surface made of
 * simplices.
 *
 * How (Algorithm A1 of Sec. 2.1, with the readings listed below):
 *   1. dose maximum, threshold mask, dD (global: DD * max D_r; local: DD * D_r(r));
 *   2. gamma0(r) = |D_e(r) - D_r(r)| / dD (step 4a, the offset-0 vertex) and the search
 *      radius R = max gamma0 over the masked nodes (step 1);
 *   3. a table of grid cells (lower-corner offsets a) with key(a) < R, sorted ascending by
 *      key (steps 2-3).  key(a) is the minimum spatial distance from the reference node to
 *      the closed cell, divided by DTA: a lower bound for every simplex of that cell;
 *   4. per reference node: gamma = gamma0; walk the table, stop at the first entry whose
 *      key >= current gamma, skip cells that are not inside the grid, and for every Kuhn
 *      simplex of the cell take the point-to-simplex distance (step 4b) computed with the
 *      normal equations w = (V^T V)^-1 V^T P of Sec. 2.1 and the recursion of Ju et al.
 *      into the facets that drop a vertex with negative weight.
 *
 * Readings of passages the paper leaves garbled or open (each also listed in the design
 * notes of the repository):
 *   - step 1 "max(D(r) - D(r))": max over masked nodes of |D_e - D_r|, normalised (=R);
 *   - step 4a: gamma0 uses |DD|;
 *   - step 4b-ii: break when the cell key >= the current gamma;
 *   - the table holds cells keyed by their minimum distance, not vertex distances, so the
 *     break is exact;
 *   - the simplices of an offset are the d! Kuhn simplices of the cell whose lower corner
 *     sits at that offset;
 *   - the mask keeps reference nodes with D_r >= fl32(fl32(thr) * fl32(max D_r)) (and
 *     D_r > 0 under local normalisation); every evaluation node forms the surface;
 *   - the surface exists over the grid box only (no extrapolation).
 *
 * Coordinates are taken relative to the reference node (a translation of the paper's P
 * and V), which keeps FP64 round-off small; the residual is formed explicitly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_PARAM (-3)
#define ORACLE_E_NOMEM (-5)

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t local;         /* 0: global dD = DD * max D_r; 1: dD = DD * D_r(r) */
    int64_t shape[3];      /* slowest axis first; 2D uses shape[0..1] */
    double spacing[3];     /* mm, same axis order */
    double dd;             /* dose criterion as a fraction, e.g. 0.03 */
    double dta;            /* distance criterion, mm */
    double thr;            /* low-dose cutoff as a fraction of max D_r, in [0, 1) */
} oracle_problem_t;

typedef struct {
    int64_t n_evaluated;   /* masked nodes among those computed */
    int64_t n_pass;        /* gamma <= 1 */
    int64_t n_borderline;  /* |gamma - 1| <= 1e-5 */
    int64_t cells_visited; /* cells whose simplices were evaluated, summed */
    int64_t cells_key0;    /* of those, cells with key 0 (the 2^d cells around the node) */
    int64_t table_len;
    int64_t n_masked;      /* masked nodes in the whole grid */
    double dose_max;
    double threshold;
    double radius;         /* R = max gamma0 over all masked nodes */
} oracle_stats_t;

#define AMB 4 /* ambient dimension of the lifted space: spatial dims + 1 (dose) */

/* ---------------------------------------------------------------------------------- */
/* Point-to-simplex distance (Sec. 2.1 projection formula + recursion of Ju et al.).   */
/* ---------------------------------------------------------------------------------- */

/* Squared distance from the origin to the m-simplex with vertices v[0..m] in R^amb.
 * With v_{m} as the base vertex (v_{k+1} of the paper): P = 0 - v_m,
 * V = [v_0 - v_m, ..., v_{m-1} - v_m]; solve (V^T V) w = V^T P by Cholesky,
 * w_m = 1 - sum w.  All w >= 0: the projection lies in the simplex and the residual
 * |P - V w| is the distance.  Otherwise the closest point lies in a facet that drops a
 * vertex with negative weight, so recurse into exactly those facets. */
static double simplex_d2(int amb, int m, const double v[][AMB], int64_t *n_proj)
{
    if (m == 0) {
        double s = 0.0;
        for (int a = 0; a < amb; ++a) s += v[0][a] * v[0][a];
        return s;
    }
    double P[AMB], V[AMB][3];
    for (int a = 0; a < amb; ++a) {
        P[a] = -v[m][a];
        for (int i = 0; i < m; ++i) V[a][i] = v[i][a] - v[m][a];
    }
    double G[3][3], b[3];
    for (int i = 0; i < m; ++i) {
        b[i] = 0.0;
        for (int a = 0; a < amb; ++a) b[i] += V[a][i] * P[a];
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int a = 0; a < amb; ++a) s += V[a][i] * V[a][j];
            G[i][j] = s;
        }
    }
    /* Cholesky G = L L^T (G is positive definite: the spatial parts of the lifted
     * vertices of a Kuhn simplex are affinely independent). */
    double L[3][3] = {{0}};
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = G[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) L[i][i] = sqrt(s);
            else L[i][j] = s / L[j][j];
        }
    }
    double y[3], w[4];
    for (int i = 0; i < m; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < m; ++k) s -= L[k][i] * w[k];
        w[i] = s / L[i][i];
    }
    double wsum = 0.0;
    for (int i = 0; i < m; ++i) wsum += w[i];
    w[m] = 1.0 - wsum;
    if (n_proj) ++*n_proj;

    int any_neg = 0;
    for (int i = 0; i <= m; ++i) any_neg |= (w[i] < 0.0);
    if (!any_neg) {
        double s = 0.0;
        for (int a = 0; a < amb; ++a) {
            double r = P[a];
            for (int i = 0; i < m; ++i) r -= V[a][i] * w[i];
            s += r * r;
        }
        return s;
    }
    double best = INFINITY;
    double f[4][AMB];
    for (int drop = 0; drop <= m; ++drop) {
        if (!(w[drop] < 0.0)) continue;
        int k = 0;
        for (int i = 0; i <= m; ++i) {
            if (i == drop) continue;
            memcpy(f[k++], v[i], sizeof(double) * AMB);
        }
        double d = simplex_d2(amb, m - 1, (const double(*)[AMB])f, n_proj);
        if (d < best) best = d;
    }
    return best;
}

/* Exposed for unit tests of the projection alone. */
double oracle_simplex_dist(int amb, int m, const double *verts /* (m+1) x amb */)
{
    double v[4][AMB];
    for (int i = 0; i <= m; ++i)
        for (int a = 0; a < AMB; ++a) v[i][a] = a < amb ? verts[i * amb + a] : 0.0;
    return sqrt(simplex_d2(amb, m, (const double(*)[AMB])v, NULL));
}

/* ---------------------------------------------------------------------------------- */
/* Radially sorted cell table (Algorithm A1 steps 2-3).                                */
/* ---------------------------------------------------------------------------------- */

typedef struct {
    double key;
    int32_t a[3];
    int64_t order; /* enumeration order, ties broken by it */
} cell_entry_t;

static int cmp_entry(const void *pa, const void *pb)
{
    const cell_entry_t *x = (const cell_entry_t *)pa, *y = (const cell_entry_t *)pb;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->order < y->order) ? -1 : (x->order > y->order);
}

/* key(a) = sqrt(sum_i (h_i * max(0, a_i, -a_i - 1))^2) / DTA: the minimum distance from
 * the reference node (offset 0) to the closed cell [a, a+1]. */
static double cell_key(int nd, const int32_t *a, const double *h, double dta)
{
    double s = 0.0;
    for (int i = 0; i < nd; ++i) {
        double g = 0.0;
        if (a[i] > 0) g = (double)a[i];
        else if (a[i] < -1) g = (double)(-a[i] - 1);
        g *= h[i];
        s += g * g;
    }
    return sqrt(s) / dta;
}

/* Cells that can lie inside the grid (lower corner q = r + a in [0, n-2] on every axis,
 * i.e. a in [-(n-1), n-2]) with key < R, ascending. */
static cell_entry_t *build_table(int nd, const int64_t *n, const double *h, double dta,
                                 double R, int64_t *len)
{
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int i = 0; i < nd; ++i) {
        double rv = R * dta / h[i];          /* radius in voxels along axis i */
        double c = ceil(rv) + 1.0;
        int64_t lim = (c > (double)n[i]) ? n[i] : (int64_t)c;
        lo[i] = -lim - 1;
        hi[i] = lim;
        if (lo[i] < -(n[i] - 1)) lo[i] = -(n[i] - 1);
        if (hi[i] > n[i] - 2) hi[i] = n[i] - 2;
    }
    int64_t cap = 1;
    for (int i = 0; i < nd; ++i) cap *= (hi[i] - lo[i] + 1);
    cell_entry_t *t = (cell_entry_t *)malloc(sizeof(cell_entry_t) * (size_t)(cap > 0 ? cap : 1));
    if (!t) return NULL;
    int64_t k = 0, ord = 0;
    int32_t a[3] = {0, 0, 0};
    int64_t z0 = nd == 3 ? lo[0] : 0, z1 = nd == 3 ? hi[0] : 0;
    for (int64_t az = z0; az <= z1; ++az)
        for (int64_t ay = lo[nd - 2]; ay <= hi[nd - 2]; ++ay)
            for (int64_t ax = lo[nd - 1]; ax <= hi[nd - 1]; ++ax) {
                if (nd == 3) { a[0] = (int32_t)az; a[1] = (int32_t)ay; a[2] = (int32_t)ax; }
                else { a[0] = (int32_t)ay; a[1] = (int32_t)ax; }
                double key = cell_key(nd, a, h, dta);
                ++ord;
                if (!(key < R)) continue;
                t[k].key = key;
                memcpy(t[k].a, a, sizeof(a));
                t[k].order = ord;
                ++k;
            }
    qsort(t, (size_t)k, sizeof(cell_entry_t), cmp_entry);
    *len = k;
    return t;
}

/* ---------------------------------------------------------------------------------- */
/* Per-node search (Algorithm A1 step 4).                                               */
/* ---------------------------------------------------------------------------------- */

static const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int PERM2[2][2] = {{0, 1}, {1, 0}};

static double search_node(const oracle_problem_t *pb, const double *ref, const double *ev,
                          int64_t r, double dD, double gamma0, const cell_entry_t *tab,
                          int64_t tlen, int32_t *cells, int32_t *cells0, int64_t *n_proj)
{
    const int nd = pb->ndim;
    const int64_t *n = pb->shape;
    int64_t rc[3];
    int64_t rem = r;
    for (int i = nd - 1; i >= 0; --i) { rc[i] = rem % n[i]; rem /= n[i]; }
    const double Dr = ref[r];
    double g = gamma0;
    int32_t visited = 0, visited0 = 0;
    for (int64_t e = 0; e < tlen; ++e) {
        if (tab[e].key >= g) break;
        int64_t q[3];
        int inside = 1;
        for (int i = 0; i < nd; ++i) {
            q[i] = rc[i] + tab[e].a[i];
            if (q[i] < 0 || q[i] > n[i] - 2) inside = 0;
        }
        if (!inside) continue;
        ++visited;
        if (tab[e].key == 0.0) ++visited0;
        /* lifted corner coordinates, relative to the reference point */
        double corner[8][AMB];
        for (int b = 0; b < (1 << nd); ++b) {
            int64_t lin = 0;
            for (int i = 0; i < nd; ++i) {
                int bit = (b >> (nd - 1 - i)) & 1;   /* bit of axis i (axis nd-1 = fastest) */
                int64_t c = q[i] + bit;
                lin = lin * n[i] + c;
                corner[b][i] = (double)(tab[e].a[i] + bit) * pb->spacing[i] / pb->dta;
            }
            corner[b][nd] = (ev[lin] - Dr) / dD;
        }
        if (nd == 3) {
            for (int p = 0; p < 6; ++p) {
                double v[4][AMB];
                int b = 0;
                memcpy(v[0], corner[0], sizeof(double) * AMB);
                for (int s = 0; s < 3; ++s) {
                    b |= 1 << (2 - PERM3[p][s]);
                    memcpy(v[s + 1], corner[b], sizeof(double) * AMB);
                }
                double d = sqrt(simplex_d2(4, 3, (const double(*)[AMB])v, n_proj));
                if (d < g) g = d;
            }
        } else {
            for (int p = 0; p < 2; ++p) {
                double v[3][AMB];
                int b = 0;
                memcpy(v[0], corner[0], sizeof(double) * AMB);
                for (int s = 0; s < 2; ++s) {
                    b |= 1 << (1 - PERM2[p][s]);
                    memcpy(v[s + 1], corner[b], sizeof(double) * AMB);
                }
                double d = sqrt(simplex_d2(3, 2, (const double(*)[AMB])v, n_proj));
                if (d < g) g = d;
            }
        }
    }
    if (cells) *cells = visited;
    if (cells0) *cells0 = visited0;
    return g;
}

static int problem_ok(const oracle_problem_t *pb)
{
    if (!pb || (pb->ndim != 2 && pb->ndim != 3)) return 0;
    for (int i = 0; i < pb->ndim; ++i)
        if (pb->shape[i] < 2 || !(pb->spacing[i] > 0.0)) return 0;
    if (!(pb->dd > 0.0) || !(pb->dta > 0.0)) return 0;
    if (!(pb->thr >= 0.0) || !(pb->thr < 1.0)) return 0;
    return 1;
}

/*
 * gamma for every masked node (subset == NULL: gamma_out has N entries, -1 where the node
 * is not evaluated) or for the listed nodes (gamma_out[k] belongs to subset[k]; -1 if that
 * node is not masked).  cells_out (optional) mirrors gamma_out with the visited-cell count.
 * nthreads <= 0 uses the OpenMP default.  Returns 0 on success.
 */
int oracle_gamma(const oracle_problem_t *pb, const double *ref, const double *ev,
                 const int64_t *subset, int64_t n_subset, double *gamma_out,
                 int32_t *cells_out, oracle_stats_t *st, int nthreads)
{
    if (!problem_ok(pb) || !ref || !ev || !gamma_out) return ORACLE_E_PARAM;
    const int nd = pb->ndim;
    int64_t N = 1;
    for (int i = 0; i < nd; ++i) N *= pb->shape[i];

    /* step: dose maximum and threshold, compared as the single-precision product */
    double dmax = -INFINITY;
    for (int64_t i = 0; i < N; ++i) if (ref[i] > dmax) dmax = ref[i];
    const float thr32 = (float)pb->thr;
    const double t = (double)(float)((double)thr32 * (double)(float)dmax);
    if (!pb->local && !(dmax > 0.0)) return ORACLE_E_PARAM;
    const double dD_global = pb->dd * dmax;

    /* step 1 (reading: radius = max over masked nodes of |DD| / dD) */
    double R = 0.0;
    int64_t n_masked = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (!(ref[i] >= t) || (pb->local && !(ref[i] > 0.0))) continue;
        ++n_masked;
        double dD = pb->local ? pb->dd * ref[i] : dD_global;
        double g0 = fabs(ev[i] - ref[i]) / dD;
        if (g0 > R) R = g0;
    }

    /* steps 2-3 */
    int64_t tlen = 0;
    cell_entry_t *tab = build_table(nd, pb->shape, pb->spacing, pb->dta, R, &tlen);
    if (!tab) return ORACLE_E_NOMEM;

    const int64_t count = subset ? n_subset : N;
    int64_t n_eval = 0, n_pass = 0, n_border = 0, cells_total = 0, cells0_total = 0, n_proj = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : n_eval, n_pass, n_border, cells_total, cells0_total, n_proj)
    for (int64_t k = 0; k < count; ++k) {
        const int64_t r = subset ? subset[k] : k;
        double gout = -1.0;
        int32_t cells = 0, cells0 = 0;
        if (r >= 0 && r < N && ref[r] >= t && !(pb->local && !(ref[r] > 0.0))) {
            double dD = pb->local ? pb->dd * ref[r] : dD_global;
            double g0 = fabs(ev[r] - ref[r]) / dD;                 /* step 4a */
            gout = search_node(pb, ref, ev, r, dD, g0, tab, tlen, &cells, &cells0, &n_proj);
            ++n_eval;
            if (gout <= 1.0) ++n_pass;
            if (fabs(gout - 1.0) <= 1e-5) ++n_border;
            cells_total += cells;
            cells0_total += cells0;
        }
        gamma_out[k] = gout;
        if (cells_out) cells_out[k] = cells;
    }
    free(tab);
    if (st) {
        st->n_evaluated = n_eval;
        st->n_pass = n_pass;
        st->n_borderline = n_border;
        st->cells_visited = cells_total;
        st->cells_key0 = cells0_total;
        st->table_len = tlen;
        st->n_masked = n_masked;
        st->dose_max = dmax;
        st->threshold = t;
        st->radius = R;
    }
    (void)n_proj;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------------- */
/* Two grids: the evaluation dose on a grid of its own (axis-aligned; its own shape,     */
/* spacing and origin).  Not in the paper; the same definition, Eq. (1), with the        */
/* surface built over the evaluation grid and the reference point at its own position.   */
/* ---------------------------------------------------------------------------------- */

/* Readings: a reference node is evaluated when it is masked (as above, on the reference
 * grid) and lies inside the closed box of the evaluation grid; others get -1.  The search
 * is a plain scan: the first bound is the nearest of the 2^d vertices of the evaluation
 * cell that holds the node, and every cell whose exact key (minimum distance from the
 * node to the closed cell, over DTA) is below that bound has all its simplices evaluated.
 * No table, no early break, no ordering: obviously complete. */
static double search_node_grids(int nd, const int64_t *ne, const double *he, const double *u,
                                double dta, const double *ev, double Dr, double dD, int64_t *n_proj)
{
    int64_t c0[3];
    for (int i = 0; i < nd; ++i) {
        c0[i] = (int64_t)floor(u[i]);
        if (c0[i] > ne[i] - 2) c0[i] = ne[i] - 2;
        if (c0[i] < 0) c0[i] = 0;
    }
    /* first bound: nearest vertex of the holding cell */
    double F = INFINITY;
    for (int b = 0; b < (1 << nd); ++b) {
        int64_t lin = 0;
        double d2 = 0.0;
        for (int i = 0; i < nd; ++i) {
            int bit = (b >> (nd - 1 - i)) & 1;
            int64_t c = c0[i] + bit;
            lin = lin * ne[i] + c;
            double x = ((double)c - u[i]) * he[i] / dta;
            d2 += x * x;
        }
        double g = (ev[lin] - Dr) / dD;
        d2 += g * g;
        if (d2 < F) F = d2;
    }
    /* every cell with key^2 < F */
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const double rad = sqrt(F);
    for (int i = 0; i < nd; ++i) {
        int64_t k = (int64_t)ceil(rad * dta / he[i]) + 1;
        lo[i] = (int64_t)floor(u[i]) - k - 1;
        hi[i] = (int64_t)floor(u[i]) + k + 1;
        if (lo[i] < 0) lo[i] = 0;
        if (hi[i] > ne[i] - 2) hi[i] = ne[i] - 2;
    }
    const double F0 = F;
    int64_t c[3] = {lo[0], lo[1], lo[2]};
    for (;;) {
        double key2 = 0.0;
        for (int i = 0; i < nd; ++i) {
            double m = 0.0;
            if ((double)c[i] > u[i]) m = (double)c[i] - u[i];
            else if (u[i] > (double)c[i] + 1.0) m = u[i] - (double)c[i] - 1.0;
            double x = m * he[i] / dta;
            key2 += x * x;
        }
        if (key2 < F0) {
            double corner[8][AMB];
            for (int b = 0; b < (1 << nd); ++b) {
                int64_t lin = 0;
                for (int i = 0; i < nd; ++i) {
                    int bit = (b >> (nd - 1 - i)) & 1;
                    int64_t cc = c[i] + bit;
                    lin = lin * ne[i] + cc;
                    corner[b][i] = ((double)cc - u[i]) * he[i] / dta;
                }
                corner[b][nd] = (ev[lin] - Dr) / dD;
            }
            if (nd == 3) {
                for (int p = 0; p < 6; ++p) {
                    double v[4][AMB];
                    int b = 0;
                    memcpy(v[0], corner[0], sizeof(double) * AMB);
                    for (int s = 0; s < 3; ++s) {
                        b |= 1 << (2 - PERM3[p][s]);
                        memcpy(v[s + 1], corner[b], sizeof(double) * AMB);
                    }
                    double d2 = simplex_d2(4, 3, (const double(*)[AMB])v, n_proj);
                    if (d2 < F) F = d2;
                }
            } else {
                for (int p = 0; p < 2; ++p) {
                    double v[3][AMB];
                    int b = 0;
                    memcpy(v[0], corner[0], sizeof(double) * AMB);
                    for (int s = 0; s < 2; ++s) {
                        b |= 1 << (1 - PERM2[p][s]);
                        memcpy(v[s + 1], corner[b], sizeof(double) * AMB);
                    }
                    double d2 = simplex_d2(3, 2, (const double(*)[AMB])v, n_proj);
                    if (d2 < F) F = d2;
                }
            }
        }
        int i = nd - 1;
        while (i >= 0) {
            if (++c[i] <= hi[i]) break;
            c[i] = lo[i];
            --i;
        }
        if (i < 0) break;
    }
    return sqrt(F);
}

/*
 * gamma of every reference node of pb (its shape and spacing describe the reference grid;
 * the node k sits at k * spacing) against an evaluation dose on the grid ev_shape x
 * ev_spacing whose node 0 sits at ev_origin (mm, same axis order).  gamma_out: N_ref
 * entries, -1 where a node is not evaluated.  st (optional): n_evaluated, n_pass,
 * n_borderline, n_masked, dose_max, threshold.
 */
int oracle_gamma_grids(const oracle_problem_t *pb, const int64_t *ev_shape, const double *ev_spacing,
                       const double *ev_origin, const double *ref, const double *ev, double *gamma_out,
                       oracle_stats_t *st, int nthreads)
{
    if (!problem_ok(pb) || !ev_shape || !ev_spacing || !ev_origin || !ref || !ev || !gamma_out)
        return ORACLE_E_PARAM;
    const int nd = pb->ndim;
    int64_t N = 1;
    for (int i = 0; i < nd; ++i) {
        N *= pb->shape[i];
        if (ev_shape[i] < 2 || !(ev_spacing[i] > 0.0) || !isfinite(ev_origin[i])) return ORACLE_E_PARAM;
    }
    double dmax = -INFINITY;
    for (int64_t i = 0; i < N; ++i) if (ref[i] > dmax) dmax = ref[i];
    const float thr32 = (float)pb->thr;
    const double t = (double)(float)((double)thr32 * (double)(float)dmax);
    if (!pb->local && !(dmax > 0.0)) return ORACLE_E_PARAM;
    const double dD_global = pb->dd * dmax;
    int64_t n_eval = 0, n_pass = 0, n_border = 0, n_masked = 0, n_proj = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_eval, n_pass, n_border, n_masked, n_proj)
    for (int64_t r = 0; r < N; ++r) {
        double gout = -1.0;
        if (ref[r] >= t && !(pb->local && !(ref[r] > 0.0))) {
            ++n_masked;
            int64_t rc[3] = {0, 0, 0};
            int64_t rem = r;
            for (int i = nd - 1; i >= 0; --i) { rc[i] = rem % pb->shape[i]; rem /= pb->shape[i]; }
            double u[3] = {0.0, 0.0, 0.0};
            int inside = 1;
            for (int i = 0; i < nd; ++i) {
                u[i] = ((double)rc[i] * pb->spacing[i] - ev_origin[i]) / ev_spacing[i];
                if (!(u[i] >= 0.0) || !(u[i] <= (double)(ev_shape[i] - 1))) inside = 0;
            }
            if (inside) {
                double dD = pb->local ? pb->dd * ref[r] : dD_global;
                gout = search_node_grids(nd, ev_shape, ev_spacing, u, pb->dta, ev, ref[r], dD, &n_proj);
                ++n_eval;
                if (gout <= 1.0) ++n_pass;
                if (fabs(gout - 1.0) <= 1e-5) ++n_border;
            }
        }
        gamma_out[r] = gout;
    }
    if (st) {
        memset(st, 0, sizeof(*st));
        st->n_evaluated = n_eval;
        st->n_pass = n_pass;
        st->n_borderline = n_border;
        st->n_masked = n_masked;
        st->dose_max = dmax;
        st->threshold = t;
    }
    (void)n_proj;
    return ORACLE_OK;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
