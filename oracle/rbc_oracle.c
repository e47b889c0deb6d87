/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see rbc_oracle.h).
 *
 * Model (a reading: the paper cites its two-component membrane model without
 * stating the potentials; Force Evaluation section):
 *   lipid-lipid   one-particle-thick, orientation-dependent membrane pair
 *                 potential with a = (n_i x r)(n_j x r) + sin th0 (n_j - n_i).r
 *                 - sin^2 th0, phi = 1 + mu (a - 1),
 *                 U = u_R(r) + (1 - phi) eps           r <  r_min
 *                   = u_A(r) phi                        r_min <= r < r_c
 *                 u_R = eps[(r_min/r)^4 - 2 (r_min/r)^2],
 *                 u_A = -eps cos^(2 zeta)((pi/2)(r - r_min)/(r_c - r_min)).
 *   protein pairs WCA (bonded pairs included: no exclusions).
 *   bonds         harmonic, from the bond list the paper maintains for
 *                 physically linked proteins (Force Evaluation section).
 * Neighbour set: pairs with the min-image FP64 squared distance, summed as
 * (dx*dx + dy*dy) + dz*dz with every operation rounded, strictly below
 * fl(rc*rc) of the pair's types.
 */
#include "rbc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LIPID 0

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ------------------------------------------------------------------ geometry */

static double minimg1(const orc_params *p, int a, double d) {
    if (p->periodic[a]) {
        double L = p->box[a];
        double q = d / L;
        double k = rint(q);           /* round half to even */
        double kl = k * L;
        d = d - kl;
    }
    return d;
}

double orc_dist2(const orc_params *p, const double *xi, const double *xj, double *d) {
    for (int a = 0; a < 3; ++a) d[a] = minimg1(p, a, xi[a] - xj[a]);
    double xx = d[0] * d[0];
    double yy = d[1] * d[1];
    double zz = d[2] * d[2];
    double s = xx + yy;
    return s + zz;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------ pair laws */

double orc_pair_lipid(const orc_params *p, const double *d, const double *ni, const double *nj,
                      double *Fi, double *ti, double *tj) {
    const double eps = p->eps, mu = p->mu, st0 = p->sin_theta0, rmin = p->r_min;
    const double rc = p->rc[0][0];
    double r = sqrt(dot3(d, d));
    for (int a = 0; a < 3; ++a) Fi[a] = ti[a] = tj[a] = 0.0;
    if (r >= rc) return 0.0;
    double e[3] = {d[0] / r, d[1] / r, d[2] / r};          /* unit vector from j to i */
    double s = dot3(ni, e), t = dot3(nj, e), c = dot3(ni, nj);
    double a_ = c - s * t + st0 * (t - s) - st0 * st0;
    double phi = 1.0 + mu * (a_ - 1.0);
    double U, dUdr, dUda;
    if (r < rmin) {
        double q = (rmin / r) * (rmin / r);
        double uR = eps * (q * q - 2.0 * q);
        U = uR + (1.0 - phi) * eps;
        dUdr = 4.0 * eps * (q - q * q) / r;               /* d u_R / dr */
        dUda = -mu * eps;
    } else {
        double x = 0.5 * M_PI * (r - rmin) / (rc - rmin);
        double cx = cos(x), sx = sin(x);
        double uA = -eps * pow(cx, 2.0 * p->zeta);
        U = uA * phi;
        dUdr = phi * eps * p->zeta * M_PI / (rc - rmin) * sx * pow(cx, 2.0 * p->zeta - 1.0);
        dUda = mu * uA;
    }
    /* da/de treating e as a free vector, then project onto the tangent of the unit sphere */
    double ga[3], gi[3], gj[3];
    for (int k = 0; k < 3; ++k) ga[k] = -t * ni[k] - s * nj[k] + st0 * (nj[k] - ni[k]);
    double proj = dot3(ga, e);
    for (int k = 0; k < 3; ++k) Fi[k] = -(dUdr * e[k] + dUda * (ga[k] - proj * e[k]) / r);
    /* torque = n x (-dU/dn) */
    for (int k = 0; k < 3; ++k) {
        gi[k] = -dUda * (nj[k] - t * e[k] - st0 * e[k]);
        gj[k] = -dUda * (ni[k] - s * e[k] + st0 * e[k]);
    }
    cross3(ni, gi, ti);
    cross3(nj, gj, tj);
    return U;
}

double orc_pair_wca(const orc_params *p, const double *d, double *Fi) {
    double r2 = dot3(d, d);
    double rcut = pow(2.0, 1.0 / 6.0) * p->wca_sigma;
    for (int a = 0; a < 3; ++a) Fi[a] = 0.0;
    if (r2 >= rcut * rcut) return 0.0;
    double sr2 = p->wca_sigma * p->wca_sigma / r2;
    double sr6 = sr2 * sr2 * sr2;
    double U = 4.0 * p->wca_eps * (sr6 * sr6 - sr6) + p->wca_eps;
    double f = 24.0 * p->wca_eps * (2.0 * sr6 * sr6 - sr6) / r2;   /* -dU/dr / r */
    for (int a = 0; a < 3; ++a) Fi[a] = f * d[a];
    return U;
}

double orc_bond(const orc_params *p, const double *d, double r0, double *Fi) {
    double r = sqrt(dot3(d, d));
    double ext = r - r0;
    double U = 0.5 * p->k_bond * ext * ext;
    for (int a = 0; a < 3; ++a) Fi[a] = (r > 0.0) ? -p->k_bond * ext * d[a] / r : 0.0;
    return U;
}

/* ------------------------------------------------------------------ neighbour set */

static double rc2_of(const orc_params *p, int ti, int tj) {
    double rc = p->rc[ti][tj];
    return rc * rc;
}

static double search_radius(const orc_params *p) {
    double r = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (p->rc[a][b] > r) r = p->rc[a][b];
    return r;
}

int64_t orc_pairs_brute(const orc_params *p, int64_t n, const double *x, const int32_t *type,
                        int64_t cap, int32_t *ij) {
    int64_t cnt = 0;
    double d[3];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double d2 = orc_dist2(p, x + 3 * i, x + 3 * j, d);
            if (d2 < rc2_of(p, type[i], type[j])) {
                if (cnt < cap) { ij[2 * cnt] = (int32_t)i; ij[2 * cnt + 1] = (int32_t)j; }
                ++cnt;
            }
        }
    return cnt;
}

/* Uniform grid with cell edge >= search radius, stored as particles sorted by
 * linear cell key; a cell's members are found by binary search. */
typedef struct {
    int64_t n;
    double lo[3], h[3];
    int64_t nc[3];
    int64_t *key;     /* sorted keys */
    int64_t *idx;     /* particle index per sorted slot */
} grid_t;

typedef struct { int64_t key, idx; } kv_t;
static int kv_cmp(const void *a, const void *b) {
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static double wrap_coord(const orc_params *p, int a, double v) {
    if (!p->periodic[a]) return v;
    double L = p->box[a];
    double w = v - L * floor(v / L);
    if (w >= L) w -= L;
    if (w < 0) w = 0;
    return w;
}

static void grid_cell(const grid_t *g, const orc_params *p, const double *xi, int64_t c[3]) {
    for (int a = 0; a < 3; ++a) {
        double u = wrap_coord(p, a, xi[a]) - g->lo[a];
        int64_t k = (int64_t)floor(u / g->h[a]);
        if (k < 0) k = 0;
        if (k >= g->nc[a]) k = g->nc[a] - 1;
        c[a] = k;
    }
}

static int64_t grid_key(const grid_t *g, const int64_t c[3]) {
    return (c[0] * g->nc[1] + c[1]) * g->nc[2] + c[2];
}

static void grid_build(grid_t *g, const orc_params *p, int64_t n, const double *x) {
    double rs = search_radius(p);
    g->n = n;
    for (int a = 0; a < 3; ++a) {
        if (p->periodic[a]) {
            g->lo[a] = 0.0;
            g->nc[a] = (int64_t)floor(p->box[a] / rs);
            if (g->nc[a] < 1) g->nc[a] = 1;
            g->h[a] = p->box[a] / (double)g->nc[a];
        } else {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t i = 0; i < n; ++i) {
                if (x[3 * i + a] < mn) mn = x[3 * i + a];
                if (x[3 * i + a] > mx) mx = x[3 * i + a];
            }
            if (n == 0) { mn = 0; mx = 0; }
            g->lo[a] = mn;
            g->h[a] = rs;
            g->nc[a] = (int64_t)floor((mx - mn) / rs) + 1;
        }
    }
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        grid_cell(g, p, x + 3 * i, c);
        kv[i].key = grid_key(g, c);
        kv[i].idx = i;
    }
    qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);
    g->key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    g->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { g->key[i] = kv[i].key; g->idx[i] = kv[i].idx; }
    free(kv);
}

static void grid_free(grid_t *g) { free(g->key); free(g->idx); }

static int64_t lower_bound(const int64_t *a, int64_t n, int64_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t m = (lo + hi) / 2;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

/* The distinct grid cells adjacent to (and including) particle i's cell. */
static int grid_neighbour_keys(const grid_t *g, const orc_params *p, const double *xi, int64_t *keys) {
    int64_t c[3];
    grid_cell(g, p, xi, c);
    int64_t lst[3][3];
    int cnt[3];
    for (int a = 0; a < 3; ++a) {
        cnt[a] = 0;
        for (int o = -1; o <= 1; ++o) {
            int64_t k = c[a] + o;
            if (p->periodic[a]) {
                k = ((k % g->nc[a]) + g->nc[a]) % g->nc[a];
            } else if (k < 0 || k >= g->nc[a]) {
                continue;
            }
            int dup = 0;
            for (int q = 0; q < cnt[a]; ++q) if (lst[a][q] == k) dup = 1;
            if (!dup) lst[a][cnt[a]++] = k;
        }
    }
    int m = 0;
    for (int i0 = 0; i0 < cnt[0]; ++i0)
        for (int i1 = 0; i1 < cnt[1]; ++i1)
            for (int i2 = 0; i2 < cnt[2]; ++i2) {
                int64_t cc[3] = {lst[0][i0], lst[1][i1], lst[2][i2]};
                keys[m++] = grid_key(g, cc);
            }
    return m;
}

static int ij_cmp(const void *a, const void *b) {
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return (x[1] > y[1]) - (x[1] < y[1]);
}

int64_t orc_pairs_grid(const orc_params *p, int64_t n, const double *x, const int32_t *type,
                       int64_t cap, int32_t *ij) {
    grid_t g;
    grid_build(&g, p, n, x);
    int64_t cnt = 0;
    double d[3];
    for (int64_t i = 0; i < n; ++i) {
        int64_t keys[27];
        int m = grid_neighbour_keys(&g, p, x + 3 * i, keys);
        for (int q = 0; q < m; ++q) {
            int64_t b = lower_bound(g.key, n, keys[q]);
            for (int64_t s = b; s < n && g.key[s] == keys[q]; ++s) {
                int64_t j = g.idx[s];
                if (j <= i) continue;
                double d2 = orc_dist2(p, x + 3 * i, x + 3 * j, d);
                if (d2 < rc2_of(p, type[i], type[j])) {
                    if (cnt < cap) { ij[2 * cnt] = (int32_t)i; ij[2 * cnt + 1] = (int32_t)j; }
                    ++cnt;
                }
            }
        }
    }
    grid_free(&g);
    if (cnt <= cap) qsort(ij, (size_t)cnt, 2 * sizeof(int32_t), ij_cmp);
    return cnt;
}

/* ------------------------------------------------------------------ forces */

/* Contribution of partner j to particle i (force, torque, half the pair energy
 * and half the pair virial).  Returns 1 if (i,j) is in the neighbour set. */
static int pair_on_i(const orc_params *p, const double *x, const double *nrm, const int32_t *type,
                     int64_t i, int64_t j, double *F, double *T, double *U, double *W) {
    double d[3], Fi[3] = {0, 0, 0}, ti[3] = {0, 0, 0}, tj[3];
    double d2 = orc_dist2(p, x + 3 * i, x + 3 * j, d);
    if (!(d2 < rc2_of(p, type[i], type[j]))) return 0;
    double u;
    if (type[i] == LIPID && type[j] == LIPID)
        u = orc_pair_lipid(p, d, nrm + 3 * i, nrm + 3 * j, Fi, ti, tj);
    else
        u = orc_pair_wca(p, d, Fi);
    for (int a = 0; a < 3; ++a) { F[a] += Fi[a]; T[a] += ti[a]; }
    *U += 0.5 * u;
    *W += 0.5 * dot3(d, Fi);
    return 1;
}

/* Bond terms of particle i: CSR over particle -> (partner, r0). */
typedef struct { int64_t *start; int64_t *partner; double *r0; } bond_csr_t;

static void bond_csr_build(bond_csr_t *b, int64_t n, int64_t nbond, const int32_t *bonds, const double *r0) {
    b->start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    b->partner = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * nbond + 1));
    b->r0 = (double *)malloc(sizeof(double) * (size_t)(2 * nbond + 1));
    for (int64_t e = 0; e < nbond; ++e) { b->start[bonds[2 * e] + 1]++; b->start[bonds[2 * e + 1] + 1]++; }
    for (int64_t i = 0; i < n; ++i) b->start[i + 1] += b->start[i];
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < nbond; ++e) {
        int64_t a = bonds[2 * e], c = bonds[2 * e + 1];
        int64_t pa = b->start[a] + fill[a]++, pc = b->start[c] + fill[c]++;
        b->partner[pa] = c; b->r0[pa] = r0[e];
        b->partner[pc] = a; b->r0[pc] = r0[e];
    }
    free(fill);
}

static void bond_csr_free(bond_csr_t *b) { free(b->start); free(b->partner); free(b->r0); }

static void bonds_on_i(const orc_params *p, const double *x, const bond_csr_t *b, int64_t i,
                       double *F, double *U, double *W) {
    for (int64_t q = b->start[i]; q < b->start[i + 1]; ++q) {
        double d[3], Fi[3];
        int64_t j = b->partner[q];
        (void)orc_dist2(p, x + 3 * i, x + 3 * j, d);
        double u = orc_bond(p, d, b->r0[q], Fi);
        for (int a = 0; a < 3; ++a) F[a] += Fi[a];
        *U += 0.5 * u;
        *W += 0.5 * dot3(d, Fi);
    }
}

int orc_forces(const orc_params *p, int64_t n, const double *x, const double *nrm,
               const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
               double *F, double *T, double *energy, int nthreads) {
    set_threads(nthreads);
    grid_t g;
    grid_build(&g, p, n, x);
    bond_csr_t b;
    bond_csr_build(&b, n, nbond, bonds, r0);
    double *Ui = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *Wi = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double Fa[3] = {0, 0, 0}, Ta[3] = {0, 0, 0}, U = 0, W = 0;
        int64_t keys[27];
        int m = grid_neighbour_keys(&g, p, x + 3 * i, keys);
        for (int q = 0; q < m; ++q) {
            int64_t s0 = lower_bound(g.key, n, keys[q]);
            for (int64_t s = s0; s < n && g.key[s] == keys[q]; ++s) {
                int64_t j = g.idx[s];
                if (j == i) continue;
                pair_on_i(p, x, nrm, type, i, j, Fa, Ta, &U, &W);
            }
        }
        bonds_on_i(p, x, &b, i, Fa, &U, &W);
        for (int a = 0; a < 3; ++a) { F[3 * i + a] = Fa[a]; T[3 * i + a] = Ta[a]; }
        Ui[i] = U;
        Wi[i] = W;
    }
    double U = 0, W = 0;
    for (int64_t i = 0; i < n; ++i) { U += Ui[i]; W += Wi[i]; }
    if (energy) { energy[0] = U; energy[1] = W; }
    free(Ui); free(Wi);
    bond_csr_free(&b);
    grid_free(&g);
    return 0;
}

int orc_forces_subset(const orc_params *p, int64_t n, const double *x, const double *nrm,
                      const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
                      int64_t nsub, const int64_t *idx, double *F, double *T, int nthreads) {
    set_threads(nthreads);
    bond_csr_t b;
    bond_csr_build(&b, n, nbond, bonds, r0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nsub; ++q) {
        int64_t i = idx[q];
        double Fa[3] = {0, 0, 0}, Ta[3] = {0, 0, 0}, U = 0, W = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            pair_on_i(p, x, nrm, type, i, j, Fa, Ta, &U, &W);
        }
        bonds_on_i(p, x, &b, i, Fa, &U, &W);
        for (int a = 0; a < 3; ++a) { F[3 * q + a] = Fa[a]; T[3 * q + a] = Ta[a]; }
    }
    bond_csr_free(&b);
    return 0;
}

/* ------------------------------------------------------------------ Voronoi reference */

/* E-step: nearest seed by the exact FP64 distance, ties to the lowest seed index. */
void orc_assign(const orc_params *p, int64_t n, const double *x, int64_t k, const double *seeds,
                int32_t *owner) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double best = INFINITY, d[3];
        int32_t bi = -1;
        for (int64_t s = 0; s < k; ++s) {
            double d2 = orc_dist2(p, x + 3 * i, seeds + 3 * s, d);
            if (d2 < best) { best = d2; bi = (int32_t)s; }
        }
        owner[i] = bi;
    }
}

/* M-step: each seed with lipid members moves to their (min-image) mean, summed in
 * ascending particle order; seeds without lipid members stay; wrap periodic axes. */
void orc_seed_update(const orc_params *p, int64_t n, const double *x, const int32_t *type,
                     const int32_t *owner, int64_t k, double *seeds) {
    double *sum = (double *)calloc((size_t)(3 * k + 3), sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)(k + 1), sizeof(int64_t));
    double d[3];
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != LIPID) continue;
        int64_t s = owner[i];
        (void)orc_dist2(p, x + 3 * i, seeds + 3 * s, d);
        for (int a = 0; a < 3; ++a) sum[3 * s + a] += d[a];
        cnt[s]++;
    }
    for (int64_t s = 0; s < k; ++s) {
        if (cnt[s] == 0) continue;
        for (int a = 0; a < 3; ++a) {
            double c = seeds[3 * s + a] + sum[3 * s + a] / (double)cnt[s];
            if (p->periodic[a]) c = c - p->box[a] * floor(c / p->box[a]);
            seeds[3 * s + a] = c;
        }
    }
    free(sum); free(cnt);
}

/* Morton key: 21 bits per axis, bits interleaved x (most significant), y, z. */
void orc_morton(const orc_params *p, int64_t k, const double *seeds, uint64_t *keys) {
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (p->periodic[a]) { lo[a] = 0.0; hi[a] = p->box[a]; continue; }
        lo[a] = INFINITY; hi[a] = -INFINITY;
        for (int64_t s = 0; s < k; ++s) {
            if (seeds[3 * s + a] < lo[a]) lo[a] = seeds[3 * s + a];
            if (seeds[3 * s + a] > hi[a]) hi[a] = seeds[3 * s + a];
        }
    }
    const double scale = 2097152.0;          /* 2^21 */
    for (int64_t s = 0; s < k; ++s) {
        uint64_t q[3];
        for (int a = 0; a < 3; ++a) {
            double ext = hi[a] - lo[a];
            if (!(ext > 0.0)) { q[a] = 0; continue; }
            double f = (seeds[3 * s + a] - lo[a]) / ext;
            double v = floor(f * scale);
            if (v < 0) v = 0;
            if (v > 2097151.0) v = 2097151.0;
            q[a] = (uint64_t)v;
        }
        uint64_t key = 0;
        for (int b = 20; b >= 0; --b) {
            key = (key << 3) | (((q[0] >> b) & 1u) << 2) | (((q[1] >> b) & 1u) << 1) | ((q[2] >> b) & 1u);
        }
        keys[s] = key;
    }
}

void orc_cell_bounds(const orc_params *p, int64_t n, const double *x, const int32_t *owner,
                     int64_t k, const double *seeds, double *R) {
    for (int64_t s = 0; s < k; ++s) R[s] = 0.0;
    double d[3];
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = owner[i];
        double r = sqrt(orc_dist2(p, x + 3 * i, seeds + 3 * s, d));
        if (r > R[s]) R[s] = r;
    }
}

int64_t orc_cell_pairs(const orc_params *p, int64_t k, const double *seeds, const double *R,
                       double rs, double skin, int64_t cap, int32_t *ab) {
    int64_t cnt = 0;
    double d[3];
    for (int64_t a = 0; a < k; ++a)
        for (int64_t b = a; b < k; ++b) {
            double dist = sqrt(orc_dist2(p, seeds + 3 * a, seeds + 3 * b, d));
            if (dist <= R[a] + R[b] + rs + 2.0 * skin + 1e-9) {
                if (cnt < cap) { ab[2 * cnt] = (int32_t)a; ab[2 * cnt + 1] = (int32_t)b; }
                ++cnt;
            }
        }
    return cnt;
}

/* ------------------------------------------------------------------ integrator */

static double kinetic(const orc_params *p, int64_t n, const double *v, const double *w, const int32_t *type) {
    double ke = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        ke += 0.5 * p->mass[type[i]] * dot3(v + 3 * i, v + 3 * i);
        if (type[i] == LIPID) ke += 0.5 * p->inertia * dot3(w + 3 * i, w + 3 * i);
    }
    return ke;
}

/* Rotate n about omega by |omega| dt (Rodrigues), then renormalise. */
static void rotor_drift(double *n, const double *w, double dt) {
    double wn = sqrt(dot3(w, w));
    if (wn > 0.0) {
        double k[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
        double th = wn * dt, c = cos(th), s = sin(th);
        double kxn[3];
        cross3(k, n, kxn);
        double kn = dot3(k, n);
        double out[3];
        for (int a = 0; a < 3; ++a) out[a] = n[a] * c + kxn[a] * s + k[a] * kn * (1.0 - c);
        for (int a = 0; a < 3; ++a) n[a] = out[a];
    }
    double nn = sqrt(dot3(n, n));
    if (nn > 0.0) for (int a = 0; a < 3; ++a) n[a] /= nn;
}

/* ------------------------------------------------------------------ volume and thermostat */

/* Philox4x32-10: ten rounds of two 32x32 -> 64-bit products whose halves are
 * mixed with the other counter words and the key; the key is bumped by the
 * Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The lipid sums the volume needs: sum x.n, sum x, sum n, count. */
static void lipid_sums(int64_t n, const double *x, const double *nrm, const int32_t *type,
                       double *sxn, double sx[3], double sn[3], double *cnt) {
    *sxn = 0.0; *cnt = 0.0;
    for (int a = 0; a < 3; ++a) { sx[a] = 0.0; sn[a] = 0.0; }
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != LIPID) continue;
        *sxn += dot3(x + 3 * i, nrm + 3 * i);
        for (int a = 0; a < 3; ++a) { sx[a] += x[3 * i + a]; sn[a] += nrm[3 * i + a]; }
        *cnt += 1.0;
    }
}

double orc_volume(const orc_ext *e, int64_t n, const double *x, const double *nrm, const int32_t *type) {
    double sxn, sx[3], sn[3], cnt;
    lipid_sums(n, x, nrm, type, &sxn, sx, sn, &cnt);
    if (cnt == 0.0) return 0.0;
    /* sum (x_i - xbar).n_i = sum x.n - (sum x).(sum n) / N_L */
    return e->lipid_area / 3.0 * (sxn - dot3(sx, sn) / cnt);
}

double orc_volume_forces(const orc_ext *e, int64_t n, const double *x, const double *nrm,
                         const int32_t *type, double *F, double *T) {
    if (!(e->vol_k > 0.0) || !(e->vol_target > 0.0)) return 0.0;
    double sxn, sx[3], sn[3], cnt;
    lipid_sums(n, x, nrm, type, &sxn, sx, sn, &cnt);
    if (cnt == 0.0) return 0.0;
    const double V = e->lipid_area / 3.0 * (sxn - dot3(sx, sn) / cnt);
    const double dUdV = e->vol_k * (V - e->vol_target) / e->vol_target;
    /* dV/dx_i = (a_L/3)(n_i - nbar), dV/dn_i = (a_L/3)(x_i - xbar) */
    const double kap = dUdV * e->lipid_area / 3.0;
    double xbar[3], nbar[3];
    for (int a = 0; a < 3; ++a) { xbar[a] = sx[a] / cnt; nbar[a] = sn[a] / cnt; }
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != LIPID) continue;
        const double *xi = x + 3 * i, *ni = nrm + 3 * i;
        double g[3];                          /* -dU_V/dn_i */
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] -= kap * (ni[a] - nbar[a]);
            g[a] = -kap * (xi[a] - xbar[a]);
        }
        double t[3];
        cross3(ni, g, t);
        for (int a = 0; a < 3; ++a) T[3 * i + a] += t[a];
    }
    return 0.5 * e->vol_k * (V - e->vol_target) * (V - e->vol_target) / e->vol_target;
}

int orc_forces_ext(const orc_params *p, const orc_ext *e, int64_t n, const double *x, const double *nrm,
                   const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
                   double *F, double *T, double *energy, int nthreads) {
    int r = orc_forces(p, n, x, nrm, type, nbond, bonds, r0, F, T, energy, nthreads);
    if (e) energy[0] += orc_volume_forces(e, n, x, nrm, type, F, T);
    return r;
}

/* A unit-variance uniform deviate from a 32-bit word: (r - (2^32 - 1)/2) sqrt(12) / 2^32. */
static double unit_uniform(uint32_t r) {
    return ((double)r - 2147483647.5) * (sqrt(12.0) / 4294967296.0);
}

void orc_langevin_step(const orc_params *p, const orc_ext *e, int64_t n, const int32_t *type,
                       const double *nrm, double dt, uint64_t step, double *v, double *w) {
    const uint32_t key[2] = {(uint32_t)e->seed, (uint32_t)(e->seed >> 32)};
    const double c = exp(-e->gamma * dt), cr = exp(-e->gamma_rot * dt);
    for (int64_t i = 0; i < n; ++i) {
        const int t = type[i];
        if (e->gamma > 0.0) {
            const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), 0u};
            uint32_t r[4];
            orc_philox4x32_10(ctr, key, r);
            const double amp = sqrt((1.0 - c * c) * e->kT / p->mass[t]);
            for (int a = 0; a < 3; ++a) v[3 * i + a] = c * v[3 * i + a] + amp * unit_uniform(r[a]);
        }
        if (t == LIPID && e->gamma_rot > 0.0) {
            const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), 1u};
            uint32_t r[4];
            orc_philox4x32_10(ctr, key, r);
            double xi[3] = {unit_uniform(r[0]), unit_uniform(r[1]), unit_uniform(r[2])};
            const double *ni = nrm + 3 * i;
            const double pn = dot3(xi, ni);
            const double amp = sqrt((1.0 - cr * cr) * e->kT / p->inertia);
            for (int a = 0; a < 3; ++a) w[3 * i + a] = cr * w[3 * i + a] + amp * (xi[a] - pn * ni[a]);
        }
    }
}

/* Keep the part of a along b when it points along b: a <- max(a.b, 0) b / |b|^2. */
static void project_along(double *a, const double *b) {
    const double bb = dot3(b, b);
    const double ab = dot3(a, b);
    if (bb > 0.0 && ab > 0.0) {
        const double s = ab / bb;
        for (int k = 0; k < 3; ++k) a[k] = s * b[k];
    } else {
        for (int k = 0; k < 3; ++k) a[k] = 0.0;
    }
}

void orc_quench_project(const orc_params *p, int64_t n, const int32_t *type, const double *F, const double *T,
                        double *v, double *w) {
    (void)p;
    for (int64_t i = 0; i < n; ++i) {
        project_along(v + 3 * i, F + 3 * i);
        if (type[i] == LIPID) project_along(w + 3 * i, T + 3 * i);
    }
}

/* Scale a down so that |a| dt <= m. */
static void cap_norm(double *a, double dt, double m) {
    const double s = sqrt(dot3(a, a)) * dt;
    if (s > m) {
        const double f = m / s;
        for (int k = 0; k < 3; ++k) a[k] *= f;
    }
}

void orc_quench_cap(const orc_ext *e, int64_t n, const int32_t *type, double dt, double *v, double *w) {
    for (int64_t i = 0; i < n; ++i) {
        cap_norm(v + 3 * i, dt, e->quench_max);
        if (type[i] == LIPID) cap_norm(w + 3 * i, dt, e->quench_max);
    }
}

int orc_vv_run(const orc_params *p, int64_t n, double *x, double *v, double *nrm, double *w,
               const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
               double dt, int64_t nsteps, double *energies, int nthreads) {
    return orc_vv_run_ext(p, NULL, 0, n, x, v, nrm, w, type, nbond, bonds, r0, dt, nsteps, energies, nthreads);
}

int orc_vv_run_ext(const orc_params *p, const orc_ext *e, uint64_t step0, int64_t n, double *x, double *v,
                   double *nrm, double *w, const int32_t *type, int64_t nbond, const int32_t *bonds,
                   const double *r0, double dt, int64_t nsteps, double *energies, int nthreads) {
    double *F = (double *)malloc(sizeof(double) * (size_t)(3 * n + 3));
    double *T = (double *)malloc(sizeof(double) * (size_t)(3 * n + 3));
    double en[2];
    const int quench = e && e->quench;
    const int thermo = !quench && e && (e->gamma > 0.0 || e->gamma_rot > 0.0);
    orc_forces_ext(p, e, n, x, nrm, type, nbond, bonds, r0, F, T, en, nthreads);
    if (energies) {
        double ke = kinetic(p, n, v, w, type);
        energies[0] = ke; energies[1] = en[0]; energies[2] = ke + en[0];
    }
    for (int64_t st = 1; st <= nsteps; ++st) {
        for (int64_t i = 0; i < n; ++i) {
            double m = p->mass[type[i]];
            for (int a = 0; a < 3; ++a) v[3 * i + a] += 0.5 * dt * F[3 * i + a] / m;
            if (type[i] == LIPID)
                for (int a = 0; a < 3; ++a) w[3 * i + a] += 0.5 * dt * T[3 * i + a] / p->inertia;
            if (quench) {
                cap_norm(v + 3 * i, dt, e->quench_max);
                if (type[i] == LIPID) cap_norm(w + 3 * i, dt, e->quench_max);
            }
            for (int a = 0; a < 3; ++a) x[3 * i + a] += dt * v[3 * i + a];
            if (type[i] == LIPID) rotor_drift(nrm + 3 * i, w + 3 * i, dt);
        }
        orc_forces_ext(p, e, n, x, nrm, type, nbond, bonds, r0, F, T, en, nthreads);
        for (int64_t i = 0; i < n; ++i) {
            double m = p->mass[type[i]];
            for (int a = 0; a < 3; ++a) v[3 * i + a] += 0.5 * dt * F[3 * i + a] / m;
            if (type[i] == LIPID)
                for (int a = 0; a < 3; ++a) w[3 * i + a] += 0.5 * dt * T[3 * i + a] / p->inertia;
        }
        if (thermo) orc_langevin_step(p, e, n, type, nrm, dt, step0 + (uint64_t)st, v, w);
        if (quench) orc_quench_project(p, n, type, F, T, v, w);
        if (energies) {
            double ke = kinetic(p, n, v, w, type);
            energies[3 * st] = ke; energies[3 * st + 1] = en[0]; energies[3 * st + 2] = ke + en[0];
        }
    }
    free(F); free(T);
    return 0;
}
