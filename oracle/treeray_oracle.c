/*
 * FP64 CPU oracle for the TreeRay/OnTheSpot sweep.
 *
 * TEST INFRASTRUCTURE: only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It is plain, slow and
 * written to be checked against the paper by eye: every step below names the
 * passage it follows.  It shares no code with the HIP library.
 *
 * Readings of passages that are silent, garbled or inconsistent are marked
 * "reading:" in the comments; the design notes list all of them.
 *
 * Parity status: every function here is pinned by tests against closed forms,
 * brute force or the paper's printed numbers, except the definitional choices
 * marked "parity unpinned" (the angular sub-point lattice and jitter, the
 * self-term mapping, the zeta_s / zeta_d treatment of the adjacent source).
 */
#include "treeray_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define BLK 8

/* ------------------------------------------------------------------------ */
/* Grid: leaf cells in finest-cell units                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int64_t *lo;      /* [n][3] */
    int64_t *size;    /* [n]    */
    int64_t ext[3];   /* domain extent in finest cells */
    double dx;        /* finest cell size, cm */
} grid_t;

int64_t orc_cell_count(const orc_domain *d)
{
    if (!d) return -1;
    if (!d->leaf_blocks)
        return (int64_t)d->nroot[0] * d->nroot[1] * d->nroot[2] * BLK * BLK * BLK;
    return d->n_leaf_blocks * BLK * BLK * BLK;
}

static int grid_make(const orc_domain *d, grid_t *g)
{
    memset(g, 0, sizeof(*g));
    if (d->nroot[0] <= 0 || d->nroot[1] <= 0 || d->nroot[2] <= 0 || d->max_level < 0 ||
        d->max_level > 12 || !(d->root_block_cm > 0))
        return -1;
    if (!d->leaf_blocks && d->max_level != 0) return -1;
    int64_t fine = (int64_t)BLK << d->max_level;     /* finest cells per root block */
    for (int a = 0; a < 3; ++a) g->ext[a] = d->nroot[a] * fine;
    g->dx = d->root_block_cm / (double)fine;
    g->n = orc_cell_count(d);
    g->lo = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)g->n);
    g->size = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->n);
    if (!g->lo || !g->size) return -2;
    if (!d->leaf_blocks) {
        int64_t nx = g->ext[0], ny = g->ext[1], nz = g->ext[2], c = 0;
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t k = 0; k < nz; ++k, ++c) {
                    g->lo[3 * c] = i; g->lo[3 * c + 1] = j; g->lo[3 * c + 2] = k;
                    g->size[c] = 1;
                }
        return 0;
    }
    int64_t c = 0;
    for (int64_t b = 0; b < d->n_leaf_blocks; ++b) {
        const int32_t *e = d->leaf_blocks + 4 * b;
        int lev = e[0];
        if (lev < 0 || lev > d->max_level) return -3;
        int64_t cs = (int64_t)1 << (d->max_level - lev);   /* cell size, finest units */
        int64_t nb[3];
        for (int a = 0; a < 3; ++a) {
            nb[a] = (int64_t)d->nroot[a] << lev;
            if (e[1 + a] < 0 || e[1 + a] >= nb[a]) return -3;
        }
        for (int i = 0; i < BLK; ++i)
            for (int j = 0; j < BLK; ++j)
                for (int k = 0; k < BLK; ++k, ++c) {
                    g->lo[3 * c] = ((int64_t)e[1] * BLK + i) * cs;
                    g->lo[3 * c + 1] = ((int64_t)e[2] * BLK + j) * cs;
                    g->lo[3 * c + 2] = ((int64_t)e[3] * BLK + k) * cs;
                    g->size[c] = cs;
                }
    }
    return 0;
}

static void grid_free(grid_t *g)
{
    free(g->lo);
    free(g->size);
}

int orc_cell_geometry(const orc_domain *d, int64_t *lo3, int64_t *size)
{
    grid_t g;
    int rc = grid_make(d, &g);
    if (rc) { grid_free(&g); return rc; }
    memcpy(lo3, g.lo, sizeof(int64_t) * 3 * (size_t)g.n);
    memcpy(size, g.size, sizeof(int64_t) * (size_t)g.n);
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sources onto the grid (Sec. 2.1 "Mapping sources onto the grid", Sec. 2.7)
 * reading: point sources, i.e. the limit of a vanishing source radius: the
 * rate is split equally over every leaf cell whose closed extent contains
 * the point.  A coordinate within 1e-9 finest cells of a cell face is taken
 * to lie on it.                                                             */
/* ------------------------------------------------------------------------ */

/* Finite-radius sources (Sec. 2.7: sources are mapped as uniform spheres).
 * reading: a source of radius R gives each cell the share of its rate equal
 * to the part of the sphere's volume inside the cell, normalised to the
 * volume inside the domain.  The volume of a ball cut by a box is the
 * integral over z of the area of a disk cut by a rectangle; the area is
 * exact, the integral Gauss-Legendre between the heights where the area
 * stops being smooth.                                                       */

/* area of the part of the disk of radius r (centre 0) with x >= u, y >= v */
static double quad_area(double r, double u, double v)
{
    if (u < 0) return 2.0 * quad_area(r, 0.0, v) - quad_area(r, -u, v);
    if (v < 0) return 2.0 * quad_area(r, u, 0.0) - quad_area(r, u, -v);
    if (u * u + v * v >= r * r) return 0.0;
    double x1 = sqrt(r * r - v * v);
    /* integral of sqrt(r^2 - x^2) - v over [u, x1] */
    double hu = 0.5 * (u * sqrt(fmax(r * r - u * u, 0.0)) + r * r * asin(fmin(u / r, 1.0)));
    double h1 = 0.5 * (x1 * sqrt(fmax(r * r - x1 * x1, 0.0)) + r * r * asin(fmin(x1 / r, 1.0)));
    return h1 - hu - v * (x1 - u);
}

typedef struct {
    double cz, R;              /* sphere centre height and radius */
    double x0, x1, y0, y1;     /* rectangle relative to the sphere's centre */
} slab_t;

static double slab_area(const slab_t *S, double z)
{
    double h = z - S->cz;
    double r2 = S->R * S->R - h * h;
    if (r2 <= 0) return 0.0;
    double r = sqrt(r2);
    return quad_area(r, S->x0, S->y0) - quad_area(r, S->x1, S->y0) - quad_area(r, S->x0, S->y1) +
           quad_area(r, S->x1, S->y1);
}

/* Gauss-Legendre nodes and weights on [0, 1], n points (Newton on P_n) */
#define GL_N 24
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;
static void gl_init(void)
{
    for (int i = 0; i < GL_N; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (GL_N + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= GL_N; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gl_x[i] = 0.5 * (1.0 - x);
        gl_w[i] = 1.0 / ((1.0 - x * x) * dp * dp);   /* weight on [-1, 1] is 2/(...), halved for [0, 1] */
    }
    gl_ready = 1;
}

static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* The disk area is smooth in z except where the circle meets a rectangle
 * edge line or corner; the integral is split there, and on each piece the
 * substitution z = p + (q - p)(1 - cos(pi t))/2 removes the (z - z*)^(3/2)
 * behaviour at its ends before Gauss-Legendre quadrature in t.            */
double orc_ball_box_volume(double cx, double cy, double cz, double R, const double *lo, const double *hi)
{
#pragma omp critical(orc_gl)
    {
        if (!gl_ready) gl_init();
    }
    double za = fmax(lo[2], cz - R), zb = fmin(hi[2], cz + R);
    if (!(R > 0) || za >= zb || lo[0] >= cx + R || hi[0] <= cx - R || lo[1] >= cy + R || hi[1] <= cy - R)
        return 0.0;
    slab_t S = {cz, R, lo[0] - cx, hi[0] - cx, lo[1] - cy, hi[1] - cy};
    double d[8] = {fabs(S.x0), fabs(S.x1), fabs(S.y0), fabs(S.y1), hypot(S.x0, S.y0), hypot(S.x1, S.y0),
                   hypot(S.x0, S.y1), hypot(S.x1, S.y1)};
    double cut[18];
    int nc = 0;
    cut[nc++] = za;
    cut[nc++] = zb;
    for (int k = 0; k < 8; ++k)
        if (d[k] < R) {
            double h = sqrt(R * R - d[k] * d[k]);
            if (cz - h > za && cz - h < zb) cut[nc++] = cz - h;
            if (cz + h > za && cz + h < zb) cut[nc++] = cz + h;
        }
    qsort(cut, (size_t)nc, sizeof(double), cmp_dbl);
    double v = 0.0;
    for (int k = 0; k + 1 < nc; ++k) {
        double p = cut[k], q = cut[k + 1];
        if (!(q > p)) continue;
        double sum = 0.0;
        for (int i = 0; i < GL_N; ++i) {
            double t = gl_x[i];
            double z = p + (q - p) * 0.5 * (1.0 - cos(ORC_PI * t));
            sum += gl_w[i] * slab_area(&S, z) * sin(ORC_PI * t);
        }
        v += sum * (q - p) * 0.5 * ORC_PI;
    }
    return v;
}

static int deposit_spheres(const grid_t *g, int64_t n_src, const double *xyz, const double *q, double radius,
                           double *ndot)
{
    const double R = radius / g->dx;   /* finest-cell units */
    int64_t **hit = (int64_t **)calloc((size_t)(n_src > 0 ? n_src : 1), sizeof(int64_t *));
    double **vol = (double **)calloc((size_t)(n_src > 0 ? n_src : 1), sizeof(double *));
    int64_t *nhit = (int64_t *)calloc((size_t)(n_src > 0 ? n_src : 1), sizeof(int64_t));
    if (!hit || !vol || !nhit) { free(hit); free(vol); free(nhit); return -2; }
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int64_t s = 0; s < n_src; ++s) {
        double u[3];
        for (int a = 0; a < 3; ++a) {
            u[a] = xyz[3 * s + a] / g->dx;
            if (u[a] < 0 || u[a] > (double)g->ext[a]) bad = 1;
        }
        if (!(q[s] >= 0) || !isfinite(q[s])) bad = 1;
        if (bad) continue;
        int64_t cap = 64;
        hit[s] = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        vol[s] = (double *)malloc(sizeof(double) * (size_t)cap);
        for (int64_t c = 0; c < g->n && hit[s]; ++c) {
            const int64_t *lo = g->lo + 3 * c;
            double clo[3], chi[3];
            for (int a = 0; a < 3; ++a) {
                clo[a] = (double)lo[a];
                chi[a] = (double)(lo[a] + g->size[c]);
            }
            double v = orc_ball_box_volume(u[0], u[1], u[2], R, clo, chi);
            if (v <= 0) continue;
            if (nhit[s] == cap) {
                cap *= 2;
                hit[s] = (int64_t *)realloc(hit[s], sizeof(int64_t) * (size_t)cap);
                vol[s] = (double *)realloc(vol[s], sizeof(double) * (size_t)cap);
                if (!hit[s] || !vol[s]) { bad = 1; break; }
            }
            hit[s][nhit[s]] = c;
            vol[s][nhit[s]] = v;
            nhit[s]++;
        }
        if (nhit[s] == 0) bad = 1;
    }
    memset(ndot, 0, sizeof(double) * (size_t)g->n);
    for (int64_t s = 0; s < n_src && !bad; ++s) {
        double tot = 0;
        for (int64_t m = 0; m < nhit[s]; ++m) tot += vol[s][m];
        for (int64_t m = 0; m < nhit[s]; ++m) ndot[hit[s][m]] += q[s] * (vol[s][m] / tot);
    }
    for (int64_t s = 0; s < n_src; ++s) { free(hit[s]); free(vol[s]); }
    free(hit); free(vol); free(nhit);
    return bad ? -1 : 0;
}

static int cell_contains(const grid_t *g, int64_t c, const double u[3])
{
    const int64_t *lo = g->lo + 3 * c;
    double sz = (double)g->size[c];
    return u[0] >= lo[0] && u[0] <= lo[0] + sz && u[1] >= lo[1] && u[1] <= lo[1] + sz &&
           u[2] >= lo[2] && u[2] <= lo[2] + sz;
}

static int deposit(const grid_t *g, int64_t n_src, const double *xyz, const double *q,
                   double *ndot)
{
    /* the cells holding each source are found independently per source (a
     * point of a tiling lies in at most 8 closed cells); the rates are then
     * added in source order */
    int64_t *hit = (int64_t *)malloc(sizeof(int64_t) * 9 * (size_t)(n_src > 0 ? n_src : 1));
    if (!hit) return -2;
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int64_t s = 0; s < n_src; ++s) {
        int64_t *h = hit + 9 * s;
        h[0] = 0;
        double u[3];
        for (int a = 0; a < 3; ++a) {
            u[a] = xyz[3 * s + a] / g->dx;
            double rn = floor(u[a] + 0.5);
            if (fabs(u[a] - rn) <= 1e-9) u[a] = rn;
            if (u[a] < 0 || u[a] > (double)g->ext[a]) bad = 1;
        }
        if (!(q[s] >= 0) || !isfinite(q[s])) bad = 1;
        if (bad) continue;
        for (int64_t c = 0; c < g->n; ++c)
            if (cell_contains(g, c, u)) {
                if (h[0] == 8) { bad = 1; break; }
                h[1 + h[0]++] = c;
            }
        if (h[0] == 0) bad = 1;
    }
    memset(ndot, 0, sizeof(double) * (size_t)g->n);
    if (!bad)
        for (int64_t s = 0; s < n_src; ++s) {
            const int64_t *h = hit + 9 * s;
            for (int64_t m = 0; m < h[0]; ++m) ndot[h[1 + m]] += q[s] / (double)h[0];
        }
    free(hit);
    return bad ? -1 : 0;
}

int orc_deposit(const orc_domain *d, int64_t n_src, const double *src_xyz_cm,
                const double *src_q, double *ndot_out)
{
    grid_t g;
    int rc = grid_make(d, &g);
    if (!rc) rc = deposit(&g, n_src, src_xyz_cm, src_q, ndot_out);
    grid_free(&g);
    return rc;
}

int orc_deposit_spheres(const orc_domain *d, int64_t n_src, const double *src_xyz_cm, const double *src_q,
                        double radius_cm, double *ndot_out)
{
    grid_t g;
    int rc = grid_make(d, &g);
    if (!rc) rc = deposit_spheres(&g, n_src, src_xyz_cm, src_q, radius_cm, ndot_out);
    grid_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Cell quantities (Sec. 2.1, eqs. os:ems, os:abs, os:erd)
 * reading: emission and recombination are netted inside each cell, and the
 * node values are plain sums of the netted cell values.  The energy-density
 * moment is carried as photon flux times volume: e = h nu F / c, and the
 * factor h nu / c cancels wherever e enters (zeta_d and the output).       */
/* ------------------------------------------------------------------------ */

typedef struct {
    double eps, alpha, erad, vol, mass, mion;
} cellq_t;

static void cell_quantities(const grid_t *g, const double *n_h, const double *ndot,
                            const double *f_prev, double alpha_b, cellq_t *out)
{
    for (int64_t c = 0; c < g->n; ++c) {
        double h = (double)g->size[c] * g->dx;
        double dv = h * h * h;
        double s = ndot[c] - alpha_b * n_h[c] * n_h[c] * dv;
        out[c].eps = s > 0 ? s : 0.0;
        out[c].alpha = s < 0 ? -s : 0.0;
        out[c].erad = (f_prev ? f_prev[c] : 0.0) * dv;
        out[c].vol = dv;
        out[c].mass = n_h[c] * dv;
        /* reading: a cell counts as ionised when its previous flux is
         * positive (option (i) of Sec. 2.6); its gas is then ionised mass */
        out[c].mion = (f_prev && f_prev[c] > 0) ? out[c].mass : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Octree (Sec. 2.1 "Quantities added to the tree")
 * reading: a virtual power-of-two root cube covers the root-block array;
 * octants without leaf cells are not created.  A node's position for the
 * radial kernels is its mass centre (Sec. 2.3); with zero mass, its volume
 * centroid.                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t lo[3], size;          /* cube, finest units */
    int64_t olo[3], ohi[3];       /* bounding box of the node's cells */
    int64_t child[8];             /* -1 = absent */
    int64_t cell;                 /* leaf cell, or -1 */
    int32_t level;
    double eps, alpha, erad, vol, mass, mion;
    double mx[3], vx[3];          /* sums of mass * centre and volume * centre */
    double com[3];                /* finest units */
} onode_t;

typedef struct {
    onode_t *n;
    int64_t count, cap;
    int32_t depth;
    int err;
} tree_t;

static int64_t tree_new(tree_t *t)
{
    if (t->count == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        onode_t *p = (onode_t *)realloc(t->n, sizeof(onode_t) * (size_t)nc);
        if (!p) { t->err = -2; return -1; }
        t->n = p;
        t->cap = nc;
    }
    onode_t *x = &t->n[t->count];
    memset(x, 0, sizeof(*x));
    for (int k = 0; k < 8; ++k) x->child[k] = -1;
    x->cell = -1;
    return t->count++;
}

/* builds the node covering cube (lo, size) from the cells idx[0..m) */
static int64_t tree_build(tree_t *t, const grid_t *g, const cellq_t *cq, const int64_t lo[3],
                          int64_t size, int32_t level, int64_t *idx, int64_t m, int64_t *tmp)
{
    if (m == 0 || t->err) return -1;
    int64_t id = tree_new(t);
    if (id < 0) return -1;
    if (level > t->depth) t->depth = level;
    {
        onode_t *x = &t->n[id];
        for (int a = 0; a < 3; ++a) x->lo[a] = lo[a];
        x->size = size;
        x->level = level;
    }
    if (m == 1 && g->size[idx[0]] == size) {
        int64_t c = idx[0];
        onode_t *x = &t->n[id];
        for (int a = 0; a < 3; ++a) {
            if (g->lo[3 * c + a] != lo[a]) { t->err = -3; return -1; }
            x->olo[a] = lo[a];
            x->ohi[a] = lo[a] + size;
        }
        x->cell = c;
        x->eps = cq[c].eps;
        x->alpha = cq[c].alpha;
        x->erad = cq[c].erad;
        x->vol = cq[c].vol;
        x->mass = cq[c].mass;
        x->mion = cq[c].mion;
        for (int a = 0; a < 3; ++a) {
            double ctr = (double)lo[a] + 0.5 * (double)size;
            x->mx[a] = cq[c].mass * ctr;
            x->vx[a] = cq[c].vol * ctr;
        }
    } else {
        if (size == 1) { t->err = -3; return -1; }
        int64_t half = size / 2;
        /* sort the cells into the 8 octants */
        int64_t cnt[8] = {0}, start[8];
        for (int64_t q = 0; q < m; ++q) {
            const int64_t *cl = g->lo + 3 * idx[q];
            if (g->size[idx[q]] >= size) { t->err = -3; return -1; }
            int o = ((cl[0] >= lo[0] + half) << 2) | ((cl[1] >= lo[1] + half) << 1) |
                    (cl[2] >= lo[2] + half);
            cnt[o]++;
        }
        start[0] = 0;
        for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
        int64_t pos[8];
        memcpy(pos, start, sizeof(pos));
        for (int64_t q = 0; q < m; ++q) {
            const int64_t *cl = g->lo + 3 * idx[q];
            int o = ((cl[0] >= lo[0] + half) << 2) | ((cl[1] >= lo[1] + half) << 1) |
                    (cl[2] >= lo[2] + half);
            tmp[pos[o]++] = idx[q];
        }
        memcpy(idx, tmp, sizeof(int64_t) * (size_t)m);
        for (int o = 0; o < 8; ++o) {
            int64_t clo[3] = {lo[0] + ((o >> 2) & 1) * half, lo[1] + ((o >> 1) & 1) * half,
                              lo[2] + (o & 1) * half};
            int64_t ch = tree_build(t, g, cq, clo, half, level + 1, idx + start[o], cnt[o],
                                    tmp + start[o]);
            if (t->err) return -1;
            t->n[id].child[o] = ch;
        }
        onode_t *x = &t->n[id];
        int first = 1;
        for (int o = 0; o < 8; ++o) {
            int64_t ch = x->child[o];
            if (ch < 0) continue;
            const onode_t *y = &t->n[ch];
            x->eps += y->eps;
            x->alpha += y->alpha;
            x->erad += y->erad;
            x->vol += y->vol;
            x->mass += y->mass;
            x->mion += y->mion;
            for (int a = 0; a < 3; ++a) {
                x->mx[a] += y->mx[a];
                x->vx[a] += y->vx[a];
                if (first || y->olo[a] < x->olo[a]) x->olo[a] = y->olo[a];
                if (first || y->ohi[a] > x->ohi[a]) x->ohi[a] = y->ohi[a];
            }
            first = 0;
        }
    }
    onode_t *x = &t->n[id];
    for (int a = 0; a < 3; ++a)
        x->com[a] = x->mass > 0 ? x->mx[a] / x->mass : x->vx[a] / x->vol;
    return id;
}

static int tree_make(const grid_t *g, const cellq_t *cq, tree_t *t)
{
    memset(t, 0, sizeof(*t));
    int64_t emax = g->ext[0];
    if (g->ext[1] > emax) emax = g->ext[1];
    if (g->ext[2] > emax) emax = g->ext[2];
    int64_t root = 1;
    while (root < emax) root *= 2;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->n);
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->n);
    if (!idx || !tmp) { free(idx); free(tmp); return -2; }
    for (int64_t c = 0; c < g->n; ++c) idx[c] = c;
    int64_t lo[3] = {0, 0, 0};
    tree_build(t, g, cq, lo, root, 0, idx, g->n, tmp);
    free(idx);
    free(tmp);
    if (t->err) return t->err;
    /* the leaf cells must tile the domain exactly */
    double vsum = 0;
    for (int64_t c = 0; c < g->n; ++c) vsum += (double)(g->size[c] * g->size[c] * g->size[c]);
    if (vsum != (double)g->ext[0] * (double)g->ext[1] * (double)g->ext[2]) return -3;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Evaluation points on rays (Sec. 2.2, eqs. etaR and Nr)
 * reading: when a count N_R is prescribed, the points keep the quadratic
 * spacing of eq. (etaR) and the last one sits at L_ray, the 3-D diagonal of
 * the domain: r_i = L_ray (i/(N_R-1))^2.                                    */
/* ------------------------------------------------------------------------ */

static int radial_points(const grid_t *g, const orc_params *p, int32_t max_n, double *r)
{
    double lray = g->dx * sqrt((double)g->ext[0] * g->ext[0] + (double)g->ext[1] * g->ext[1] +
                               (double)g->ext[2] * g->ext[2]);
    int32_t n;
    if (p->n_radial > 0) {
        n = p->n_radial;
        if (n < 3 || n > max_n) return -1;
        for (int i = 0; i < n; ++i) {
            double f = (double)i / (double)(n - 1);
            r[i] = lray * f * f;
        }
    } else {
        if (!(p->eta_r > 0)) return -1;
        n = (int32_t)(p->eta_r * floor(sqrt(2.0 * lray / g->dx))) + 1;
        if (n < 3 || n > max_n) return -1;
        for (int i = 0; i < n; ++i) r[i] = g->dx * (double)i * (double)i / (2.0 * p->eta_r * p->eta_r);
    }
    return n;
}

int orc_radial_points(const orc_domain *d, const orc_params *p, int32_t max_n, double *r_out)
{
    grid_t g;
    int rc = grid_make(d, &g);
    if (!rc) rc = radial_points(&g, p, max_n, r_out);
    grid_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* HEALPix pixelisation, RING numbering (Sec. 2.2; Gorski et al. 2005)
 * Equatorial zone |z| <= 2/3: the two families of pixel edges are lines of
 * constant N_side (1/2 + t -+ 3z/4), t = phi / (pi/2).  Polar caps: edges are
 * lines of constant t' sigma and (1 - t') sigma with t' the fractional part
 * of t and sigma = N_side sqrt(3 (1 - |z|)).                               */
/* ------------------------------------------------------------------------ */

static int64_t floordiv2(int64_t a) { return (a >= 0) ? a / 2 : -((-a + 1) / 2); }
static int64_t imod(int64_t a, int64_t m) { int64_t r = a % m; return r < 0 ? r + m : r; }

int64_t orc_ang2pix(int32_t nside, double x, double y, double z)
{
    int64_t ns = nside;
    double rho2 = x * x + y * y;
    double r = sqrt(rho2 + z * z);
    double zc = z / r;
    double za = fabs(zc);
    double phi = atan2(y, x);
    if (phi < 0) phi += 2.0 * ORC_PI;
    double t = phi / (0.5 * ORC_PI);                 /* [0, 4] */
    if (za <= 2.0 / 3.0) {
        double a = (double)ns * (0.5 + t - 0.75 * zc);
        double b = (double)ns * (0.5 + t + 0.75 * zc);
        int64_t jp = (int64_t)floor(a);               /* ascending edge index  */
        int64_t jm = (int64_t)floor(b);               /* descending edge index */
        int64_t ir = ns + 1 + jp - jm;                /* ring from z = 2/3, 1..2ns+1 */
        /* defensive: rounding at |z| = 2/3 may put the edges one ring outside */
        if (ir < 1) ir = 1;
        if (ir > 2 * ns + 1) ir = 2 * ns + 1;
        int64_t kshift = 1 - (ir & 1);
        int64_t ip = imod(floordiv2(jp + jm - ns + kshift + 1), 4 * ns);
        return 2 * ns * (ns - 1) + (ir - 1) * 4 * ns + ip;
    }
    double tp = t - floor(t);
    /* 1 - |z| without cancellation: rho^2 / (r (r + |z|)) */
    double omz = rho2 / (r * (r + fabs(z)));
    double sig = (double)ns * sqrt(3.0 * omz);
    int64_t jp = (int64_t)floor(tp * sig);
    int64_t jm = (int64_t)floor((1.0 - tp) * sig);
    int64_t ir = jp + jm + 1;                         /* ring from the nearer pole */
    int64_t ip = imod((int64_t)floor(t * (double)ir), 4 * ir);
    if (zc > 0) return 2 * ir * (ir - 1) + ip;
    return 12 * ns * ns - 2 * ir * (ir + 1) + ip;
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of later sweeps (n >= 1); the CPU baseline times one core and all */
void orc_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}

void orc_ang2pix_many(int32_t nside, int64_t n, const double *xyz, int64_t *out)
{
    for (int64_t q = 0; q < n; ++q) out[q] = orc_ang2pix(nside, xyz[3 * q], xyz[3 * q + 1], xyz[3 * q + 2]);
}

/* pixel centres, the inverse map; used only by the pin tests */
void orc_pix2vec(int32_t nside, int64_t pix, double *v)
{
    int64_t ns = nside, npix = 12 * ns * ns, ncap = 2 * ns * (ns - 1);
    double z, phi;
    if (pix < ncap) {
        int64_t ir = 1;
        while (2 * (ir + 1) * ir <= pix) ++ir;       /* ring ir holds pixels [2ir(ir-1), 2ir(ir+1)) */
        int64_t ip = pix - 2 * ir * (ir - 1);
        z = 1.0 - (double)(ir * ir) / (3.0 * ns * ns);
        phi = ((double)ip + 0.5) * ORC_PI / (2.0 * ir);
    } else if (pix < npix - ncap) {
        int64_t q = pix - ncap;
        int64_t ir = q / (4 * ns) + 1;               /* ring from z = 2/3 */
        int64_t ip = q % (4 * ns);
        z = (2.0 / 3.0) * (double)(ns + 1 - ir) / (double)ns;
        double shift = (ir & 1) ? 0.5 : 0.0;
        phi = ((double)ip + shift) * ORC_PI / (2.0 * ns);
    } else {
        int64_t q = npix - 1 - pix;                  /* mirror of the north cap */
        int64_t ir = 1;
        while (2 * (ir + 1) * ir <= q) ++ir;
        int64_t ipm = q - 2 * ir * (ir - 1);          /* mirrored index, counted backwards */
        int64_t ip = 4 * ir - 1 - ipm;
        z = -1.0 + (double)(ir * ir) / (3.0 * ns * ns);
        phi = ((double)ip + 0.5) * ORC_PI / (2.0 * ir);
    }
    double s = sqrt((1.0 - z) * (1.0 + z));
    v[0] = s * cos(phi);
    v[1] = s * sin(phi);
    v[2] = z;
}

/* ------------------------------------------------------------------------ */
/* Radial kernels (App. A)                                                  */
/* ------------------------------------------------------------------------ */

/* Piece-wise cubic W_p (App. A.2, eq. eKernPolynomial).
 * reading: the printed A = 4.08 is a garbled 0.408 (the kernel must fall
 * from M = 1.184 at the centre); the printed second branch does not meet its
 * own stated conditions, so it is rebuilt from them: W(1/2) = A,
 * W(sqrt3/2) = 0, W'(sqrt3/2) = 0 with leading coefficient a2.            */
double orc_wp(double x)
{
    const double a1 = 1.21, a2 = -6.35, A = 0.408, M = 1.184;
    const double xe = 0.5 * sqrt(3.0);
    x = fabs(x);
    if (x < 0.5) return a1 * x * x * x - (0.5 * a1 + 4.0 * (M - A)) * x * x + M;
    if (x < xe) {
        double q = 2.0 * A * (2.0 + sqrt(3.0)) - 0.5 * a2;
        return (x - xe) * (x - xe) * (a2 * x + q);
    }
    return 0.0;
}

/* W_p mapping weights, normalised to unit sum over the points (App. A).
 * reading: if no point lies inside the support, the node is split linearly
 * between the two points that bracket d (all of it to the last point when
 * d lies beyond it).                                                        */
void orc_wp_weights(int32_t n, const double *r, double d, double h, double *v)
{
    double sum = 0;
    for (int i = 0; i < n; ++i) {
        v[i] = orc_wp((r[i] - d) / h);
        sum += v[i];
    }
    if (sum > 0) {
        for (int i = 0; i < n; ++i) v[i] /= sum;
        return;
    }
    for (int i = 0; i < n; ++i) v[i] = 0;
    if (d >= r[n - 1]) { v[n - 1] = 1; return; }
    int i = 0;
    while (!(r[i] <= d && d < r[i + 1])) ++i;
    v[i] = (r[i + 1] - d) / (r[i + 1] - r[i]);
    v[i + 1] = 1.0 - v[i];
}

/* Two-point flux-conserving kernel W_f,3 (App. A.3, eqs. kernCond0 and the
 * third condition eps_i + eps_{i+1} = eps): the emission of a node at
 * distance d goes to the bracketing points r_i <= d < r_{i+1}, i >= 1, with
 * u_i/r_i^2 + u_{i+1}/r_{i+1}^2 = 1/d^2 and u_i + u_{i+1} = 1.
 * reading: beyond the last point everything goes to it; closer than r_1,
 * everything goes to r_1 (r_0 = 0 cannot carry emission).                  */
void orc_wf3_weights(int32_t n, const double *r, double d, double *u)
{
    for (int i = 0; i < n; ++i) u[i] = 0;
    if (d >= r[n - 1]) { u[n - 1] = 1; return; }
    if (d < r[1]) { u[1] = 1; return; }
    int i = 1;
    while (!(r[i] <= d && d < r[i + 1])) ++i;
    double ai = 1.0 / (r[i] * r[i]), an = 1.0 / (r[i + 1] * r[i + 1]), ad = 1.0 / (d * d);
    u[i] = (ad - an) / (ai - an);
    u[i + 1] = 1.0 - u[i];
}

/* Gaussian kernel W_g (App. A.1): exp(-x^2) inside |x| < sqrt(3)/2. */
double orc_wg(double x)
{
    x = fabs(x);
    return x < 0.5 * sqrt(3.0) ? exp(-x * x) : 0.0;
}

/* Normalised smoothing-kernel weights (App. A): W_p (kind ORC_K_P) or W_g
 * (ORC_K_G) of x = (r_i - d)/h, with the same linear fallback as W_p. */
void orc_mass_weights(int32_t kind, int32_t n, const double *r, double d, double h, double *v)
{
    if (kind != ORC_K_G) {
        orc_wp_weights(n, r, d, h, v);
        return;
    }
    double sum = 0;
    for (int i = 0; i < n; ++i) {
        v[i] = orc_wg((r[i] - d) / h);
        sum += v[i];
    }
    if (sum > 0) {
        for (int i = 0; i < n; ++i) v[i] /= sum;
        return;
    }
    for (int i = 0; i < n; ++i) v[i] = 0;
    if (d >= r[n - 1]) { v[n - 1] = 1; return; }
    int i = 0;
    while (!(r[i] <= d && d < r[i + 1])) ++i;
    v[i] = (r[i + 1] - d) / (r[i + 1] - r[i]);
    v[i + 1] = 1.0 - v[i];
}

/* Emission weights u_i (App. A.3 and the smoothing kernels):
 *  ORC_K_F3 (default): two-point W_f,3 (orc_wf3_weights);
 *  ORC_K_F1: the bracket points with u_i/r_i^2 + u_{i+1}/r_{i+1}^2 = 1/d^2
 *    and u_{i+1}/u_i = (d - r_i)/(r_{i+1} - d);
 *  ORC_K_F2: the bracket points with the flux also exact at r_{i-1};
 *  ORC_K_F3N: W_f,3 over the N points inside the node's extent
 *    (|r_k - d| < sqrt(3)/2 h, k >= 1), u linear in the point index, with
 *    sum u = 1 and sum u/r^2 = 1/d^2 (eqs. eKernFC1, eKernFC2);
 *  ORC_K_P, ORC_K_G: the smoothing kernels.
 * reading: F1 and F2 use the bracket and fall-backs of W_f,3; F2 needs
 * i >= 2 (at i = 1 its two conditions coincide) and F2 and F3N fall back to
 * the two-point W_f,3 when a weight would be negative or N < 2. */
void orc_eps_weights(int32_t kind, int32_t n, const double *r, double d, double h, double *u)
{
    if (kind == ORC_K_P || kind == ORC_K_G) {
        orc_mass_weights(kind, n, r, d, h, u);
        return;
    }
    orc_wf3_weights(n, r, d, u);
    if (kind == ORC_K_F3 || kind == ORC_K_DEFAULT) return;
    if (kind == ORC_K_F1 || kind == ORC_K_F2) {
        if (d >= r[n - 1] || d < r[1]) return;      /* the W_f,3 fall-backs */
        int i = 1;
        while (!(r[i] <= d && d < r[i + 1])) ++i;
        double ui, un;
        if (kind == ORC_K_F1) {
            double rho = (d - r[i]) / (r[i + 1] - d);
            ui = 1.0 / (d * d * (1.0 / (r[i] * r[i]) + rho / (r[i + 1] * r[i + 1])));
            un = rho * ui;
        } else {
            if (i < 2) return;
            /* a11 ui + a12 un = b1, a21 ui + a22 un = b2 */
            double a11 = 1.0 / (r[i] * r[i]), a12 = 1.0 / (r[i + 1] * r[i + 1]), b1 = 1.0 / (d * d);
            double p = r[i - 1];
            double a21 = 1.0 / ((r[i] - p) * (r[i] - p)), a22 = 1.0 / ((r[i + 1] - p) * (r[i + 1] - p));
            double b2 = 1.0 / ((d - p) * (d - p));
            double det = a11 * a22 - a12 * a21;
            ui = (b1 * a22 - a12 * b2) / det;
            un = (a11 * b2 - a21 * b1) / det;
            if (!(ui >= 0) || !(un >= 0)) return;
        }
        for (int k = 0; k < n; ++k) u[k] = 0;
        u[i] = ui;
        u[i + 1] = un;
        return;
    }
    /* ORC_K_F3N */
    int lo = -1, N = 0;
    for (int k = 1; k < n; ++k)
        if (fabs(r[k] - d) < 0.5 * sqrt(3.0) * h) {
            if (lo < 0) lo = k;
            ++N;
        }
    if (N < 2) return;
    /* u_k = a + b (k - lo): sum u = 1, sum u / r^2 = 1/d^2 */
    double s0 = 0, s1 = 0, t0 = 0, t1 = 0;
    for (int m = 0; m < N; ++m) {
        s0 += 1.0;
        s1 += (double)m;
        t0 += 1.0 / (r[lo + m] * r[lo + m]);
        t1 += (double)m / (r[lo + m] * r[lo + m]);
    }
    double det = s0 * t1 - s1 * t0;
    double a = (t1 - s1 / (d * d)) / det, b = (s0 / (d * d) - t0) / det;
    for (int m = 0; m < N; ++m)
        if (a + b * (double)m < 0) return;
    for (int k = 0; k < n; ++k) u[k] = 0;
    for (int m = 0; m < N; ++m) u[lo + m] = a + b * (double)m;
}

/* ------------------------------------------------------------------------ */
/* On-the-Spot integration along one ray (Sec. 2.5)
 * Phi_{j,j} = eps_j / 4pi at every point holding emission; moving inwards,
 * Phi_{i,j} = max(0, Phi_{i+1,j} - R_{i,j}) with
 * R_{i,j} = (alpha_i + alpha_{i+1})/2 dV_{i,j} zeta_d zeta_s zeta_g (eq. Rij),
 * dV_{i,j} = [(r_j - r_i)^3 - (r_j - r_{i+1})^3]/3 (eq. dV),
 * zeta_s = F_{i+1,j}/F_{i+1} (eq. Rcorr:s), zeta_d = min(2, F_{i+1}/Fbar_{i+1})
 * (eq. Rcorr:d with e c / h nu = Fbar), zeta_g = min(1, N_side (r_j - r_i)/(2 r_j))
 * (eq. Rcorr:g); finally F_0 = sum_j Phi_{0,j}/r_j^2.
 * readings: the recurrence uses the segment's own loss R_{i,j} (the printed
 * R_{i+1,j} disagrees with eq. Rij's dV_{i,j}); all sources on the ray are
 * advanced together because zeta_s needs the total flux at r_{i+1}; for the
 * source at r_{i+1} itself (F_{i+1,i+1} is singular) zeta_s = zeta_d = 1
 * [parity unpinned]; zeta_d = 2 where the previous flux is zero; per-volume
 * values at a point are the mapped totals divided by the mapped volume.    */
/* ------------------------------------------------------------------------ */

double orc_integrate_ray(int32_t n, const double *r, const double *eps, const double *A,
                         const double *E, const double *V, int32_t nside, int32_t zeta_g)
{
    double *alpha = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *fbar = alpha + n, *phi = alpha + 2 * n;
    for (int i = 0; i < n; ++i) {
        alpha[i] = V[i] > 0 ? A[i] / V[i] : 0.0;
        fbar[i] = V[i] > 0 ? E[i] / V[i] : 0.0;
        phi[i] = 0.0;
    }
    for (int i = n - 1; i >= 0; --i) {
        if (i <= n - 2) {
            double ftot = 0;                      /* F_{i+1}: sources beyond r_{i+1} */
            for (int j = i + 2; j < n; ++j)
                if (phi[j] > 0) ftot += phi[j] / ((r[j] - r[i + 1]) * (r[j] - r[i + 1]));
            for (int j = i + 1; j < n; ++j) {
                if (!(phi[j] > 0)) continue;
                double zs = 1.0, zd = 1.0, zg = 1.0;
                if (j >= i + 2) {
                    double fj = phi[j] / ((r[j] - r[i + 1]) * (r[j] - r[i + 1]));
                    zs = fj / ftot;
                    zd = fbar[i + 1] > 0 ? fmin(2.0, ftot / fbar[i + 1]) : 2.0;
                }
                if (zeta_g) zg = fmin(1.0, (double)nside * (r[j] - r[i]) / (2.0 * r[j]));
                double a = r[j] - r[i], b = r[j] - r[i + 1];
                double dv = (a * a * a - b * b * b) / 3.0;
                double R = 0.5 * (alpha[i] + alpha[i + 1]) * dv * zd * zs * zg;
                phi[j] = fmax(0.0, phi[j] - R);
            }
        }
        if (i >= 1 && eps[i] > 0) phi[i] = eps[i] / (4.0 * ORC_PI);
    }
    double f0 = 0;
    for (int j = 1; j < n; ++j) f0 += phi[j] / (r[j] * r[j]);
    free(alpha);
    return f0;
}

/* ------------------------------------------------------------------------ */
/* Tree walk for one target (Sec. 2.3 "Mapping nodes onto rays", Sec. 2.4)
 * reading: the opening-angle test uses the node's geometric centre in the
 * squared form size^2 < theta^2 d^2 (exact in finest-cell units); a node
 * containing the target is opened, every other leaf cell is accepted, and
 * the target cell itself is left to the self term.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    const tree_t *t;
    const grid_t *g;
    const orc_params *p;
    double xt[3];          /* target centre, finest units */
    int64_t t2[3];         /* twice the target centre (an integer) */
    int64_t target;        /* target cell */
    int64_t *acc;          /* accepted node ids */
    int64_t nacc, capacc;
    int64_t tested;
} walk_t;

static int walk_push(walk_t *w, int64_t id)
{
    if (w->nacc == w->capacc) {
        int64_t nc = w->capacc ? 2 * w->capacc : 1024;
        int64_t *q = (int64_t *)realloc(w->acc, sizeof(int64_t) * (size_t)nc);
        if (!q) return -2;
        w->acc = q;
        w->capacc = nc;
    }
    w->acc[w->nacc++] = id;
    return 0;
}

/* Squared limiting opening angle of a node (Sec. 2.4): theta_lim, lowered
 * to theta_IF for a node holding an ionisation front (ionised mass strictly
 * between delta_IF and 1 - delta_IF of its mass, delta_IF = 1e-8) and to
 * theta_Src for a node holding emission (eps_n > 0).  A non-positive
 * theta_IF or theta_Src switches that criterion off. */
static double opening_angle2(const orc_params *p, const onode_t *x)
{
    const double dif = 1e-8;
    double t2 = p->theta * p->theta;
    if (p->theta_if > 0 && dif * x->mass < x->mion && x->mion < (1.0 - dif) * x->mass) {
        double u = p->theta_if * p->theta_if;
        if (u < t2) t2 = u;
    }
    if (p->theta_src > 0 && x->eps > 0) {
        double u = p->theta_src * p->theta_src;
        if (u < t2) t2 = u;
    }
    return t2;
}

/* Periodic boundaries (Sec. 2.8): a node is used through its periodic copy
 * closest to the target.  The copy is chosen by the node's geometric centre:
 * per axis the shift k L (L the domain's extent) puts the centre's offset
 * from the target into (-L/2, L/2].  Isolated boundaries: no shift. */
static void nearest_copy(const walk_t *w, const onode_t *x, double shift[3])
{
    for (int a = 0; a < 3; ++a) {
        shift[a] = 0.0;
        if (!w->p->periodic) continue;
        double L = (double)w->g->ext[a];
        double off = (double)x->lo[a] + 0.5 * (double)x->size - w->xt[a];
        shift[a] = floor((0.5 * L - off) / L) * L;
    }
}

static int walk_node(walk_t *w, int64_t id)
{
    const onode_t *x = &w->t->n[id];
    w->tested++;
    int inside = 1;
    for (int a = 0; a < 3; ++a)
        if (!(w->xt[a] >= (double)x->lo[a] && w->xt[a] < (double)(x->lo[a] + x->size))) inside = 0;
    int open;
    if (inside) {
        if (x->cell >= 0) return 0;             /* the target itself */
        open = 1;
    } else if (x->cell >= 0) {
        open = 0;
    } else {
        double d2 = 0, sh[3];
        nearest_copy(w, x, sh);
        for (int a = 0; a < 3; ++a) {
            double gc = (double)x->lo[a] + 0.5 * (double)x->size + sh[a] - w->xt[a];
            d2 += gc * gc;
        }
        double h = (double)x->size;
        open = !(h * h < opening_angle2(w->p, x) * d2);
    }
    if (!open) return walk_push(w, id);
    for (int o = 0; o < 8; ++o)
        if (x->child[o] >= 0) {
            int rc = walk_node(w, x->child[o]);
            if (rc) return rc;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Node -> ray mapping and the per-target sum (Sec. 2.3, Sec. 2.5 "Sum over
 * directions")
 * reading [parity unpinned]: the node's share of ray k is the fraction of
 * s^3 sub-box midpoints of the node's cells' bounding box whose direction
 * from the target lies in pixel k; the lattice is shifted by the fixed
 * fractions (4.1e-4, 7.3e-4, 2.3e-4) of a sub-box to avoid exact ties.
 * reading [parity unpinned]: the target's own recombinations, volume and
 * previous flux are spread with W_p at d = 0, h = its size, equally over
 * all rays; its own emission adds 3 eps / (4 pi r_tp^2), the centre flux of
 * a uniformly emitting sphere of radius r_tp = half the cell size.         */
/* ------------------------------------------------------------------------ */

static const double JIT[3] = {4.1e-4, 7.3e-4, 2.3e-4};

typedef struct {
    double *eps, *A, *E, *V;   /* [npix][nr] */
    double *u, *v;             /* [nr] */
    double *wp_self;           /* [nr] */
    int64_t *pk;               /* sub-point pixels [s^3] */
    int64_t *pl;               /* distinct pixels */
    int *pc;                   /* their counts */
} tbuf_t;

/* Angular weights of one node (Sec. 2.3): the s^3 sub-box midpoints of the
 * box of extent ext whose lower corner lies rel2/2 from the target centre
 * (finest units; rel2 = twice the corner minus twice the centre, an exact
 * integer, the box already moved to the copy in use) are classified by the
 * HEALPix pixel of their direction from the target; returns the number of
 * distinct pixels, listed in pl with their sub-point counts in pc.  The
 * direction is the exact offset rel2/2 plus the sub-box fraction, one
 * rounding each, so it depends on the offset alone and not on where the
 * target lies in the domain. */
static int node_pixels(int32_t nside, int s, const int64_t rel2[3], const double ext[3], int64_t *pl, int *pc)
{
    int npl = 0;
    for (int ia = 0; ia < s; ++ia)
        for (int ib = 0; ib < s; ++ib)
            for (int ic = 0; ic < s; ++ic) {
                int ii[3] = {ia, ib, ic};
                double v[3];
                for (int a = 0; a < 3; ++a)
                    v[a] = 0.5 * (double)rel2[a] + (((double)ii[a] + 0.5) + JIT[a]) * (ext[a] / (double)s);
                int64_t pix = orc_ang2pix(nside, v[0], v[1], v[2]);
                int found = 0;
                for (int k = 0; k < npl; ++k)
                    if (pl[k] == pix) { pc[k]++; found = 1; break; }
                if (!found) { pl[npl] = pix; pc[npl] = 1; ++npl; }
            }
    return npl;
}

int32_t orc_node_pixels(int32_t nside, int32_t s, const int64_t *olo, const int64_t *ohi, const double *xt,
                        int64_t *pix_out, int32_t *count_out)
{
    if (nside < 1 || s < 1 || s > 64) return -1;
    int64_t rel2[3];
    double ext[3];
    for (int a = 0; a < 3; ++a) {
        const double t2 = 2.0 * xt[a];   /* the target centre lies on the half-integer lattice */
        if (t2 != floor(t2)) return -1;
        rel2[a] = 2 * olo[a] - (int64_t)t2;
        ext[a] = (double)(ohi[a] - olo[a]);
    }
    int *pc = (int *)malloc(sizeof(int) * (size_t)s * s * s);
    if (!pc) return -2;
    int n = node_pixels(nside, s, rel2, ext, pix_out, pc);
    for (int k = 0; k < n; ++k) count_out[k] = pc[k];
    free(pc);
    return n;
}

static void map_node(const walk_t *w, const onode_t *x, const cellq_t *q_override, int32_t nr,
                     const double *r, int64_t npix, tbuf_t *b)
{
    (void)q_override;
    (void)npix;
    const grid_t *g = w->g;
    int s = w->p->subsample;
    int ns3 = s * s * s;
    double sh[3];
    nearest_copy(w, x, sh);
    /* angular weights */
    int64_t rel2[3];
    double ext[3];
    for (int a = 0; a < 3; ++a) {
        rel2[a] = 2 * (x->olo[a] + (int64_t)sh[a]) - w->t2[a];
        ext[a] = (double)(x->ohi[a] - x->olo[a]);
    }
    int npl = node_pixels(w->p->nside, s, rel2, ext, b->pl, b->pc);
    /* radial weights */
    double d2 = 0;
    for (int a = 0; a < 3; ++a) {
        double da = x->com[a] + sh[a] - w->xt[a];
        d2 += da * da;
    }
    double d = sqrt(d2) * g->dx;
    double h = (double)x->size * g->dx;
    orc_eps_weights(w->p->eps_kernel, nr, r, d, h, b->u);
    orc_mass_weights(w->p->mass_kernel, nr, r, d, h, b->v);
    for (int k = 0; k < npl; ++k) {
        double wk = (double)b->pc[k] / (double)ns3;
        int64_t base = b->pl[k] * nr;
        for (int i = 0; i < nr; ++i) {
            if (x->eps > 0 && b->u[i] != 0) b->eps[base + i] += wk * x->eps * b->u[i];
            b->A[base + i] += wk * x->alpha * b->v[i];
            b->E[base + i] += wk * x->erad * b->v[i];
            b->V[base + i] += wk * x->vol * b->v[i];
        }
    }
}

typedef struct {
    const grid_t *g;
    const tree_t *t;
    const cellq_t *cq;
    const orc_params *p;
    const double *r;
    int32_t nr;
    const int64_t *node_of_cell;
} sweep_ctx_t;

/* walk and map one target: its ray buffers, self term included */
static int map_target(const sweep_ctx_t *S, int64_t tc, tbuf_t *b, walk_t *w, int64_t *n_acc, int64_t *n_tested)
{
    const grid_t *g = S->g;
    int32_t nr = S->nr;
    int64_t npix = 12 * (int64_t)S->p->nside * S->p->nside;
    size_t nbuf = (size_t)npix * nr;
    memset(b->eps, 0, sizeof(double) * nbuf);
    memset(b->A, 0, sizeof(double) * nbuf);
    memset(b->E, 0, sizeof(double) * nbuf);
    memset(b->V, 0, sizeof(double) * nbuf);
    w->t = S->t;
    w->g = g;
    w->p = S->p;
    w->target = tc;
    w->nacc = 0;
    w->tested = 0;
    for (int a = 0; a < 3; ++a) {
        w->xt[a] = (double)g->lo[3 * tc + a] + 0.5 * (double)g->size[tc];
        w->t2[a] = 2 * g->lo[3 * tc + a] + g->size[tc];
    }
    int rc = walk_node(w, 0);
    if (rc) return rc;
    for (int64_t q = 0; q < w->nacc; ++q) map_node(w, &S->t->n[w->acc[q]], NULL, nr, S->r, npix, b);
    /* self term */
    const cellq_t *ct = &S->cq[tc];
    double dxt = (double)g->size[tc] * g->dx;
    orc_mass_weights(S->p->mass_kernel, nr, S->r, 0.0, dxt, b->wp_self);
    for (int64_t k = 0; k < npix; ++k)
        for (int i = 0; i < nr; ++i) {
            double wv = b->wp_self[i] / (double)npix;
            b->A[k * nr + i] += ct->alpha * wv;
            b->E[k * nr + i] += ct->erad * wv;
            b->V[k * nr + i] += ct->vol * wv;
        }
    *n_acc += w->nacc;
    *n_tested += w->tested;
    return 0;
}

static int sweep_target(const sweep_ctx_t *S, int64_t tc, tbuf_t *b, walk_t *w, double *fout,
                        int64_t *n_acc, int64_t *n_tested)
{
    const grid_t *g = S->g;
    int32_t nr = S->nr;
    int64_t npix = 12 * (int64_t)S->p->nside * S->p->nside;
    int rc = map_target(S, tc, b, w, n_acc, n_tested);
    if (rc) return rc;
    const cellq_t *ct = &S->cq[tc];
    double dxt = (double)g->size[tc] * g->dx;
    double ftot = 0;
    for (int64_t k = 0; k < npix; ++k)
        ftot += orc_integrate_ray(nr, S->r, b->eps + k * nr, b->A + k * nr, b->E + k * nr,
                                  b->V + k * nr, S->p->nside, S->p->zeta_g);
    double rtp = 0.5 * dxt;
    ftot += 3.0 * ct->eps / (4.0 * ORC_PI * rtp * rtp);
    *fout = ftot;
    return 0;
}

static int tbuf_alloc(tbuf_t *b, int64_t npix, int32_t nr, int s)
{
    size_t nbuf = (size_t)npix * nr;
    b->eps = (double *)malloc(sizeof(double) * (4 * nbuf + 3 * (size_t)nr));
    b->pk = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * s * s * s));
    b->pc = (int *)malloc(sizeof(int) * (size_t)(s * s * s));
    if (!b->eps || !b->pk || !b->pc) return -2;
    b->A = b->eps + nbuf;
    b->E = b->A + nbuf;
    b->V = b->E + nbuf;
    b->u = b->V + nbuf;
    b->v = b->u + nr;
    b->wp_self = b->v + nr;
    b->pl = b->pk + s * s * s;
    return 0;
}

static void tbuf_free(tbuf_t *b)
{
    free(b->eps);
    free(b->pk);
    free(b->pc);
}

static int check_params(const orc_params *p)
{
    if (!p) return -1;
    if (p->nside < 1 || (p->nside & (p->nside - 1))) return -1;
    if (!(p->theta >= 0) || !(p->alpha_b >= 0) || p->subsample < 1) return -1;
    return 0;
}

typedef struct {
    grid_t g;
    cellq_t *cq;
    tree_t t;
    double r[1024];
    int32_t nr;
} prep_t;

static void prep_free(prep_t *P)
{
    grid_free(&P->g);
    free(P->cq);
    free(P->t.n);
}

static int prep(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
                const double *xyz, const double *q, const double *f_prev, prep_t *P)
{
    memset(P, 0, sizeof(*P));
    int rc = check_params(p);
    if (rc) return rc;
    rc = grid_make(d, &P->g);
    if (rc) return rc;
    for (int64_t c = 0; c < P->g.n; ++c)
        if (!(n_h[c] >= 0) || !isfinite(n_h[c])) return -1;
    double *ndot = (double *)malloc(sizeof(double) * (size_t)P->g.n);
    P->cq = (cellq_t *)malloc(sizeof(cellq_t) * (size_t)P->g.n);
    if (!ndot || !P->cq) { free(ndot); return -2; }
    rc = p->src_radius_cm > 0 ? deposit_spheres(&P->g, n_src, xyz, q, p->src_radius_cm, ndot)
                              : deposit(&P->g, n_src, xyz, q, ndot);
    if (rc) { free(ndot); return rc; }
    cell_quantities(&P->g, n_h, ndot, f_prev, p->alpha_b, P->cq);
    free(ndot);
    rc = tree_make(&P->g, P->cq, &P->t);
    if (rc) return rc;
    P->nr = radial_points(&P->g, p, 1024, P->r);
    if (P->nr < 0) return -1;
    return 0;
}

int orc_sweep(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
              const double *src_xyz_cm, const double *src_q, const double *f_prev,
              int64_t n_targets, const int64_t *targets, double *f_out, uint8_t *ion_out,
              orc_stats *st)
{
    return orc_sweep_timed(d, p, n_h, n_src, src_xyz_cm, src_q, f_prev, n_targets, targets, f_out, ion_out,
                           st, 0, NULL);
}

int orc_sweep_timed(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
                    const double *src_xyz_cm, const double *src_q, const double *f_prev,
                    int64_t n_targets, const int64_t *targets, double *f_out, uint8_t *ion_out,
                    orc_stats *st, int32_t threads, double *seconds)
{
    prep_t P;
    int rc = prep(d, p, n_h, n_src, src_xyz_cm, src_q, f_prev, &P);
    if (rc) { prep_free(&P); return rc; }
#ifdef _OPENMP
    const int nthr = threads > 0 ? (int)threads : omp_get_max_threads();
    const double t_start = omp_get_wtime();
#else
    (void)threads;
#endif
    int64_t nt = targets ? n_targets : P.g.n;
    for (int64_t q = 0; targets && q < nt; ++q)
        if (targets[q] < 0 || targets[q] >= P.g.n) { prep_free(&P); return -1; }
    sweep_ctx_t S = {&P.g, &P.t, P.cq, p, P.r, P.nr, NULL};
    int64_t npix = 12 * (int64_t)p->nside * p->nside;
    int64_t acc_sum = 0, tested_sum = 0;
    int err = 0;
#pragma omp parallel reduction(+ : acc_sum, tested_sum) num_threads(nthr)
    {
        tbuf_t b;
        walk_t w;
        memset(&b, 0, sizeof(b));
        memset(&w, 0, sizeof(w));
        int lrc = tbuf_alloc(&b, npix, P.nr, p->subsample);
        if (lrc) {
#pragma omp atomic write
            err = lrc;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < nt; ++q) {
            if (err) continue;
            int64_t tc = targets ? targets[q] : q;
            double f = 0;
            int e = sweep_target(&S, tc, &b, &w, &f, &acc_sum, &tested_sum);
            if (e) {
#pragma omp atomic write
                err = e;
            }
            f_out[q] = f;
            if (ion_out) ion_out[q] = f > 0 ? 1 : 0;
        }
        tbuf_free(&b);
        free(w.acc);
    }
#ifdef _OPENMP
    if (seconds) *seconds = omp_get_wtime() - t_start;
#else
    if (seconds) *seconds = 0.0;
#endif
    if (st) {
        st->nodes_accepted = acc_sum;
        st->nodes_tested = tested_sum;
        st->n_nodes = P.t.count;
        st->n_radial = P.nr;
        st->depth = P.t.depth;
    }
    prep_free(&P);
    return err;
}

int64_t orc_accepted(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
                     const double *src_xyz_cm, const double *src_q, const double *f_prev,
                     int64_t target, int64_t max_out, int64_t *lo_size_out, double *mom_out)
{
    prep_t P;
    int rc = prep(d, p, n_h, n_src, src_xyz_cm, src_q, f_prev, &P);
    if (rc) { prep_free(&P); return rc; }
    if (target < 0 || target >= P.g.n) { prep_free(&P); return -1; }
    walk_t w;
    memset(&w, 0, sizeof(w));
    w.t = &P.t;
    w.g = &P.g;
    w.p = p;
    w.target = target;
    for (int a = 0; a < 3; ++a) {
        w.xt[a] = (double)P.g.lo[3 * target + a] + 0.5 * (double)P.g.size[target];
        w.t2[a] = 2 * P.g.lo[3 * target + a] + P.g.size[target];
    }
    rc = walk_node(&w, 0);
    int64_t n = rc ? rc : w.nacc;
    for (int64_t q = 0; rc == 0 && q < w.nacc && q < max_out; ++q) {
        const onode_t *x = &P.t.n[w.acc[q]];
        for (int a = 0; a < 3; ++a) lo_size_out[4 * q + a] = x->lo[a];
        lo_size_out[4 * q + 3] = x->size;
        double *m = mom_out + 9 * q;
        m[0] = x->eps; m[1] = x->alpha; m[2] = x->erad; m[3] = x->vol; m[4] = x->mass;
        m[5] = x->com[0]; m[6] = x->com[1]; m[7] = x->com[2]; m[8] = x->mion;
    }
    free(w.acc);
    prep_free(&P);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Error control (Sec. 2.6 "Iterations and error control")
 * delta_cell = max_c |F_new - F_old| / max(F_old, median F_old) (eq.
 * delta:er:cell with its normaliser); reading: the change is taken in
 * absolute value, the median is the lower median over all cells, and a cell
 * with a zero normaliser but a non-zero new value is not converged.
 * delta_tot is eq. delta:er:tot.                                           */
/* ------------------------------------------------------------------------ */

/* The mapped ray buffers of one target (walk, node mapping and self term,
 * before the integration): eps, A, E, V as [N_PIX][N_R] each, in cgs. */
int32_t orc_target_rays(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
                        const double *src_xyz_cm, const double *src_q, const double *f_prev, int64_t target,
                        int32_t max_nr, double *eps_out, double *a_out, double *e_out, double *v_out)
{
    prep_t P;
    int rc = prep(d, p, n_h, n_src, src_xyz_cm, src_q, f_prev, &P);
    if (rc) { prep_free(&P); return rc; }
    if (target < 0 || target >= P.g.n || P.nr > max_nr) { prep_free(&P); return -1; }
    sweep_ctx_t S = {&P.g, &P.t, P.cq, p, P.r, P.nr, NULL};
    int64_t npix = 12 * (int64_t)p->nside * p->nside;
    tbuf_t b;
    walk_t w;
    memset(&b, 0, sizeof(b));
    memset(&w, 0, sizeof(w));
    rc = tbuf_alloc(&b, npix, P.nr, p->subsample);
    int64_t na = 0, nt = 0;
    if (!rc) rc = map_target(&S, target, &b, &w, &na, &nt);
    if (!rc) {
        size_t nbuf = (size_t)npix * P.nr;
        memcpy(eps_out, b.eps, sizeof(double) * nbuf);
        memcpy(a_out, b.A, sizeof(double) * nbuf);
        memcpy(e_out, b.E, sizeof(double) * nbuf);
        memcpy(v_out, b.V, sizeof(double) * nbuf);
    }
    tbuf_free(&b);
    free(w.acc);
    int32_t nr = P.nr;
    prep_free(&P);
    return rc ? rc : nr;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

double orc_delta_cell(int64_t n, const double *f_new, const double *f_old)
{
    if (n <= 0) return 0;
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(s, f_old, sizeof(double) * (size_t)n);
    qsort(s, (size_t)n, sizeof(double), cmp_double);
    double med = s[(n - 1) / 2];
    free(s);
    double dmax = 0;
    for (int64_t c = 0; c < n; ++c) {
        double norm = f_old[c] > med ? f_old[c] : med;
        double diff = fabs(f_new[c] - f_old[c]);
        double dl;
        if (norm > 0) dl = diff / norm;
        else dl = diff > 0 ? INFINITY : 0.0;
        if (dl > dmax) dmax = dl;
    }
    return dmax;
}

double orc_delta_tot(int64_t n, const double *f_new, const double *f_old, const double *dv)
{
    double a = 0, b = 0;
    for (int64_t c = 0; c < n; ++c) {
        a += f_new[c] * dv[c];
        b += f_old[c] * dv[c];
    }
    if (a + b == 0) return 0;
    return 2.0 * (a - b) / (a + b);
}

int orc_solve(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
              const double *src_xyz_cm, const double *src_q, double eps_lim, int32_t max_iter,
              double *f_out, uint8_t *ion_out, int32_t *iters, double *delta)
{
    int64_t n = orc_cell_count(d);
    if (n <= 0) return -1;
    double *fold = (double *)malloc(sizeof(double) * (size_t)n);
    if (!fold) return -2;
    orc_params thin = *p;
    thin.alpha_b = 0.0;
    int rc = orc_sweep(d, &thin, n_h, n_src, src_xyz_cm, src_q, NULL, 0, NULL, f_out, ion_out, NULL);
    int32_t it = 0;
    double dl = INFINITY;
    while (rc == 0 && it < max_iter) {
        memcpy(fold, f_out, sizeof(double) * (size_t)n);
        rc = orc_sweep(d, p, n_h, n_src, src_xyz_cm, src_q, fold, 0, NULL, f_out, ion_out, NULL);
        ++it;
        if (rc) break;
        dl = orc_delta_cell(n, f_out, fold);
        if (dl < eps_lim) break;
    }
    free(fold);
    if (iters) *iters = it;
    if (delta) *delta = dl;
    return rc;
}
