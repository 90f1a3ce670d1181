/*
 * fwi_oracle.c -- plain FP64 CPU oracle for the encoded-shot acoustic FWI gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the GPU
 * library is compared against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * What it computes (paper: Sec. "Forward model, data, and likelihood", Eqs. 1, 4-6, the
 * adjoint-state statement after Eq. 5, and the Langevin refinement Eqs. 8-9):
 *
 *   F_i : velocity -> shot gather, by solving the constant-density acoustic wave
 *         equation (1/v^2) u_tt - lap(u) = s.  The paper names no discretization; the
 *         one below is the reading fixed for this project:
 *           * 8th-order central second derivative per axis (weights C0..C4, Fornberg),
 *           * leapfrog in time,
 *           * a sponge of nb cells on every face, quadratic damping profile
 *             gamma = sum_a gmax_a (d_a/nb)^2, gmax_a = 3 v_ref ln(1/R) / (2 nb h_a),
 *           * model edge-replicated into the sponge, zero (Dirichlet) ghost outside.
 *         u^{n+1} = a u^n - b u^{n-1} + c (L u^n + q^n),  a = 2/(1+g dt),
 *         b = (1-g dt)/(1+g dt),  c = dt^2 v^2/(1+g dt),  u^0 = u^{-1} = 0,
 *         q^n = sum_s w_s f[n] e_{x_s} / prod_a h_a,   d[j][r] = u^{(j+1)R}[x_r].
 *   Misfit (Eq. 1 / Eq. 5): phi = (1/2 sigma^2) sum (d - d_obs)^2, rho = (d - d_obs)/sigma^2.
 *   Gradient (adjoint state, one forward + one adjoint solve): with the scaled adjoint
 *         lt = c * lambda the adjoint is the same recursion run backward,
 *         lt^k = a lt^{k+1} - b lt^{k+2} + c (L lt^{k+1} + s^k),  s^k = sum_r rho[j][r] e_r
 *         at k = (j+1)R, and dphi/dv_pad = (2/v_pad) sum_{k=1}^{nt} lt^k (L u^{k-1} + q^{k-1}).
 *         The physical-cell gradient folds each sponge cell back onto the edge cell it
 *         replicates (the adjoint of edge replication).
 *
 * Everything is FP64.  With coef_fp32 = 1 the coefficient set (a, b, c, the stencil
 * weights C_k/h^2, 1/prod h, source weights and wavelet samples) is rounded once to
 * FP32 after being computed in FP64, and all arithmetic stays FP64.  That is the
 * reference an FP32 implementation of the same scheme is measured against.
 *
 * Plain loops, no blocking or fusion: a reader can check each loop against the
 * formulas above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fwi_oracle.h"

/* Standard 8th-order central weights for the second derivative (Fornberg 1988). */
static const double C8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

static double rnd(double x, int fp32) { return fp32 ? (double)(float)x : x; }

/* ---------------------------------------------------------------- geometry */

typedef struct {
    int ndim;
    int n[3];      /* physical dims, axis order z, y, x (y = 1 in 2D) */
    int N[3];      /* padded dims */
    double h[3];   /* spacings z, y, x */
    int nb;
    int64_t ncell; /* padded cells */
    int64_t nphys; /* physical cells */
    int64_t stride[3];
} geo_t;

static int geo_init(const orc_grid *g, geo_t *o)
{
    if (g->ndim != 2 && g->ndim != 3) return -1;
    if (g->nz < 1 || g->nx < 1 || g->nb < 0) return -1;
    if (g->ndim == 3 && g->ny < 1) return -1;
    o->ndim = g->ndim;
    o->nb = g->nb;
    o->n[0] = g->nz;
    o->n[1] = g->ndim == 3 ? g->ny : 1;
    o->n[2] = g->nx;
    o->h[0] = g->dz;
    o->h[1] = g->ndim == 3 ? g->dy : 1.0;
    o->h[2] = g->dx;
    o->N[0] = g->nz + 2 * g->nb;
    o->N[1] = g->ndim == 3 ? g->ny + 2 * g->nb : 1;
    o->N[2] = g->nx + 2 * g->nb;
    o->stride[2] = 1;
    o->stride[1] = o->N[2];
    o->stride[0] = (int64_t)o->N[1] * o->N[2];
    o->ncell = (int64_t)o->N[0] * o->N[1] * o->N[2];
    o->nphys = (int64_t)o->n[0] * o->n[1] * o->n[2];
    return 0;
}

static int axis_active(const geo_t *g, int a) { return g->ndim == 3 || a != 1; }

/* padded index of physical cell index c (c = (iz*ny + iy)*nx + ix) */
static int64_t pad_of_phys(const geo_t *g, int64_t c)
{
    int64_t ix = c % g->n[2];
    int64_t iy = (c / g->n[2]) % g->n[1];
    int64_t iz = c / ((int64_t)g->n[2] * g->n[1]);
    int nby = g->ndim == 3 ? g->nb : 0;
    return (iz + g->nb) * g->stride[0] + (iy + nby) * g->stride[1] + (ix + g->nb);
}

/* physical cell that padded cell p replicates (edge replication) */
static int64_t phys_of_pad(const geo_t *g, int64_t p)
{
    int64_t i[3];
    i[2] = p % g->N[2];
    i[1] = (p / g->N[2]) % g->N[1];
    i[0] = p / ((int64_t)g->N[2] * g->N[1]);
    int64_t q[3];
    for (int a = 0; a < 3; ++a) {
        int nba = (a == 1 && g->ndim == 2) ? 0 : g->nb;
        int64_t k = i[a] - nba;
        if (k < 0) k = 0;
        if (k > g->n[a] - 1) k = g->n[a] - 1;
        q[a] = k;
    }
    return (q[0] * g->n[1] + q[1]) * g->n[2] + q[2];
}

/* ------------------------------------------------------------ coefficients */

typedef struct {
    double *a, *b, *c;  /* per padded cell */
    double w[3][5];     /* stencil weights C_k / h_a^2 per axis (0 for an inactive axis) */
    double inv_vol;     /* 1 / prod h */
} coef_t;

/* cells into the sponge along one axis: 0 inside, nb at the outer face */
static int sponge_depth(int p, int n, int nb)
{
    if (p < nb) return nb - p;
    if (p > nb + n - 1) return p - (nb + n - 1);
    return 0;
}

static int coef_build(const orc_grid *gr, const geo_t *g, const orc_time *t, const double *v, coef_t *k)
{
    int fp32 = t->coef_fp32;
    k->a = malloc(sizeof(double) * g->ncell);
    k->b = malloc(sizeof(double) * g->ncell);
    k->c = malloc(sizeof(double) * g->ncell);
    if (!k->a || !k->b || !k->c) return -1;
    double gmax[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        if (!axis_active(g, a) || g->nb == 0) continue;
        gmax[a] = 3.0 * gr->v_ref * log(1.0 / gr->refl) / (2.0 * g->nb * g->h[a]);
    }
    for (int a = 0; a < 3; ++a)
        for (int m = 0; m < 5; ++m)
            k->w[a][m] = axis_active(g, a) ? rnd(C8[m] / (g->h[a] * g->h[a]), fp32) : 0.0;
    double vol = g->h[0] * g->h[2] * (g->ndim == 3 ? g->h[1] : 1.0);
    k->inv_vol = rnd(1.0 / vol, fp32);
    double dt = t->dt;
    for (int64_t p = 0; p < g->ncell; ++p) {
        int i[3];
        i[2] = (int)(p % g->N[2]);
        i[1] = (int)((p / g->N[2]) % g->N[1]);
        i[0] = (int)(p / ((int64_t)g->N[2] * g->N[1]));
        double gam = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!axis_active(g, a) || g->nb == 0) continue;
            double d = (double)sponge_depth(i[a], g->n[a], g->nb) / g->nb;
            gam += gmax[a] * d * d;
        }
        double vp = v[phys_of_pad(g, p)];
        double gd = gam * dt;
        k->a[p] = rnd(2.0 / (1.0 + gd), fp32);
        k->b[p] = rnd((1.0 - gd) / (1.0 + gd), fp32);
        k->c[p] = rnd(dt * dt * vp * vp / (1.0 + gd), fp32);
    }
    return 0;
}

static void coef_free(coef_t *k)
{
    free(k->a);
    free(k->b);
    free(k->c);
}

/* 8th-order Laplacian at padded cell p with zero outside the padded box */
static double lap_at(const geo_t *g, const coef_t *k, const double *u, int64_t p)
{
    int i[3];
    i[2] = (int)(p % g->N[2]);
    i[1] = (int)((p / g->N[2]) % g->N[1]);
    i[0] = (int)(p / ((int64_t)g->N[2] * g->N[1]));
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!axis_active(g, a)) continue;
        s += k->w[a][0] * u[p];
        for (int m = 1; m <= 4; ++m) {
            double lo = i[a] - m >= 0 ? u[p - m * g->stride[a]] : 0.0;
            double hi = i[a] + m < g->N[a] ? u[p + m * g->stride[a]] : 0.0;
            s += k->w[a][m] * (lo + hi);
        }
    }
    return s;
}

/* ---------------------------------------------------------------- forward */

typedef struct {
    int nsrc;
    const int32_t *src_cell;
    const double *src_w;
    int nrec;
    const int32_t *rec_cell;
    const double *wavelet;
} acq_t;

static int acq_check(const geo_t *g, const acq_t *q)
{
    for (int s = 0; s < q->nsrc; ++s)
        if (q->src_cell[s] < 0 || q->src_cell[s] >= g->nphys) return -1;
    for (int r = 0; r < q->nrec; ++r)
        if (q->rec_cell[r] < 0 || q->rec_cell[r] >= g->nphys) return -1;
    return 0;
}

/* dense per-padded-cell source weight: sum of w_s of the sources at that cell */
static double *src_dense(const geo_t *g, const acq_t *q, int fp32)
{
    double *qw = calloc(g->ncell, sizeof(double));
    if (!qw) return NULL;
    for (int s = 0; s < q->nsrc; ++s) qw[pad_of_phys(g, q->src_cell[s])] += rnd(q->src_w[s], fp32);
    return qw;
}

/*
 * Forward solve.  d_out[(nt/R) * nrec] receives the recorded data.  If u_store is not
 * NULL it receives u^n for n = 0..nt-1 (ncell each), the wavefields the gradient needs.
 */
static int forward_run(const geo_t *g, const coef_t *k, const orc_time *t, const acq_t *q,
                       const double *qw, double *d_out, double *u_store)
{
    int64_t nc = g->ncell;
    double *um = calloc(nc, sizeof(double)); /* u^{n-1} */
    double *u0 = calloc(nc, sizeof(double)); /* u^n */
    double *up = calloc(nc, sizeof(double)); /* u^{n+1} */
    if (!um || !u0 || !up) return -1;
    int fp32 = t->coef_fp32;
    for (int n = 0; n < t->nt; ++n) {
        if (u_store) memcpy(u_store + (int64_t)n * nc, u0, sizeof(double) * nc);
        double f = rnd(q->wavelet[n], fp32) * k->inv_vol;
        for (int64_t p = 0; p < nc; ++p) {
            double src = qw[p] * f;
            up[p] = k->a[p] * u0[p] - k->b[p] * um[p] + k->c[p] * (lap_at(g, k, u0, p) + src);
        }
        double *tmp = um;
        um = u0;
        u0 = up;
        up = tmp;
        if ((n + 1) % t->rec_every == 0) {
            int j = (n + 1) / t->rec_every - 1;
            for (int r = 0; r < q->nrec; ++r) d_out[(int64_t)j * q->nrec + r] = u0[pad_of_phys(g, q->rec_cell[r])];
        }
    }
    free(um);
    free(u0);
    free(up);
    return 0;
}

/*
 * Adjoint solve + zero-lag imaging.  rho[(nt/R) * nrec] is the data-space residual
 * (dphi/dd).  u_store holds u^0..u^{nt-1}.  g_pad[ncell] receives
 * sum_k lt^k (L u^{k-1} + q^{k-1}) (before the 2/v factor).  If trace is not NULL,
 * trace[k-1] = lt^k at padded cell trace_cell for k = 1..nt.
 */
static int adjoint_run(const geo_t *g, const coef_t *k, const orc_time *t, const acq_t *q,
                       const double *qw, const double *rho, const double *u_store, double *g_pad,
                       double *trace, int64_t trace_cell)
{
    int64_t nc = g->ncell;
    double *l2 = calloc(nc, sizeof(double)); /* lt^{k+2} */
    double *l1 = calloc(nc, sizeof(double)); /* lt^{k+1} */
    double *l0 = calloc(nc, sizeof(double)); /* lt^k */
    double *s = calloc(nc, sizeof(double));
    if (!l2 || !l1 || !l0 || !s) return -1;
    int fp32 = t->coef_fp32;
    if (g_pad) memset(g_pad, 0, sizeof(double) * nc);
    for (int kk = t->nt; kk >= 1; --kk) {
        memset(s, 0, sizeof(double) * nc);
        if (kk % t->rec_every == 0) {
            int j = kk / t->rec_every - 1;
            for (int r = 0; r < q->nrec; ++r) s[pad_of_phys(g, q->rec_cell[r])] += rho[(int64_t)j * q->nrec + r];
        }
        for (int64_t p = 0; p < nc; ++p)
            l0[p] = k->a[p] * l1[p] - k->b[p] * l2[p] + k->c[p] * (lap_at(g, k, l1, p) + s[p]);
        if (g_pad) {
            const double *um = u_store + (int64_t)(kk - 1) * nc;
            double f = rnd(q->wavelet[kk - 1], fp32) * k->inv_vol;
            for (int64_t p = 0; p < nc; ++p) g_pad[p] += l0[p] * (lap_at(g, k, um, p) + qw[p] * f);
        }
        if (trace) trace[kk - 1] = l0[trace_cell];
        double *tmp = l2;
        l2 = l1;
        l1 = l0;
        l0 = tmp;
    }
    free(l2);
    free(l1);
    free(l0);
    free(s);
    return 0;
}

/* g_phys[c] = sum over padded cells p replicating c of (2/v[c]) g_pad[p] */
static void fold_gradient(const geo_t *g, const double *v, const double *g_pad, double *g_phys)
{
    memset(g_phys, 0, sizeof(double) * g->nphys);
    for (int64_t p = 0; p < g->ncell; ++p) {
        int64_t c = phys_of_pad(g, p);
        g_phys[c] += 2.0 / v[c] * g_pad[p];
    }
}

static void fill_acq(acq_t *q, int nsrc, const int32_t *src_cell, const double *src_w, int nrec,
                     const int32_t *rec_cell, const double *wavelet)
{
    q->nsrc = nsrc;
    q->src_cell = src_cell;
    q->src_w = src_w;
    q->nrec = nrec;
    q->rec_cell = rec_cell;
    q->wavelet = wavelet;
}

static int time_check(const orc_time *t)
{
    if (t->nt < 1 || t->rec_every < 1 || t->nt % t->rec_every != 0 || !(t->dt > 0)) return -1;
    return 0;
}

/* ------------------------------------------------------------- public API */

int orc_forward(const orc_grid *gr, const orc_time *t, const double *v, int nsrc, const int32_t *src_cell,
                const double *src_w, const double *wavelet, int nrec, const int32_t *rec_cell, double *d_out)
{
    geo_t g;
    coef_t k;
    acq_t q;
    if (geo_init(gr, &g) || time_check(t)) return -1;
    fill_acq(&q, nsrc, src_cell, src_w, nrec, rec_cell, wavelet);
    if (acq_check(&g, &q)) return -1;
    if (coef_build(gr, &g, t, v, &k)) return -2;
    double *qw = src_dense(&g, &q, t->coef_fp32);
    int rc = qw ? forward_run(&g, &k, t, &q, qw, d_out, NULL) : -2;
    free(qw);
    coef_free(&k);
    return rc;
}

int orc_adjoint(const orc_grid *gr, const orc_time *t, const double *v, int nsrc, const int32_t *src_cell,
                const double *src_w, const double *wavelet, int nrec, const int32_t *rec_cell, const double *rho,
                double *g_phys, int32_t trace_phys_cell, double *trace)
{
    geo_t g;
    coef_t k;
    acq_t q;
    if (geo_init(gr, &g) || time_check(t)) return -1;
    fill_acq(&q, nsrc, src_cell, src_w, nrec, rec_cell, wavelet);
    if (acq_check(&g, &q)) return -1;
    if (trace && (trace_phys_cell < 0 || trace_phys_cell >= g.nphys)) return -1;
    if (coef_build(gr, &g, t, v, &k)) return -2;
    double *qw = src_dense(&g, &q, t->coef_fp32);
    double *us = g_phys ? malloc(sizeof(double) * g.ncell * (int64_t)t->nt) : NULL;
    double *gp = g_phys ? malloc(sizeof(double) * g.ncell) : NULL;
    double *dtmp = malloc(sizeof(double) * (int64_t)(t->nt / t->rec_every) * (nrec > 0 ? nrec : 1));
    int rc = -2;
    if (qw && dtmp && (!g_phys || (us && gp))) {
        rc = 0;
        if (g_phys) rc = forward_run(&g, &k, t, &q, qw, dtmp, us);
        if (!rc)
            rc = adjoint_run(&g, &k, t, &q, qw, rho, us, gp, trace,
                             trace ? pad_of_phys(&g, trace_phys_cell) : 0);
        if (!rc && g_phys) fold_gradient(&g, v, gp, g_phys);
    }
    free(us);
    free(gp);
    free(dtmp);
    free(qw);
    coef_free(&k);
    return rc;
}

int orc_gradient(const orc_grid *gr, const orc_time *t, const double *v, int nsrc, const int32_t *src_cell,
                 const double *src_w, const double *wavelet, int nrec, const int32_t *rec_cell,
                 const double *d_obs, double inv_sigma2, double *d_pred, double *misfit, double *g_phys)
{
    geo_t g;
    coef_t k;
    acq_t q;
    if (geo_init(gr, &g) || time_check(t)) return -1;
    fill_acq(&q, nsrc, src_cell, src_w, nrec, rec_cell, wavelet);
    if (acq_check(&g, &q)) return -1;
    if (coef_build(gr, &g, t, v, &k)) return -2;
    int64_t nd = (int64_t)(t->nt / t->rec_every) * nrec;
    double *qw = src_dense(&g, &q, t->coef_fp32);
    double *us = malloc(sizeof(double) * g.ncell * (int64_t)t->nt);
    double *gp = malloc(sizeof(double) * g.ncell);
    double *rho = malloc(sizeof(double) * (nd > 0 ? nd : 1));
    int rc = -2;
    if (qw && us && gp && rho) {
        rc = forward_run(&g, &k, t, &q, qw, d_pred, us);
        if (!rc) {
            double is2 = rnd(inv_sigma2, t->coef_fp32);
            double phi = 0.0;
            for (int64_t i = 0; i < nd; ++i) {
                double r = d_pred[i] - d_obs[i];
                phi += r * r;
                rho[i] = r * is2;
            }
            *misfit = 0.5 * is2 * phi;
            rc = adjoint_run(&g, &k, t, &q, qw, rho, us, gp, NULL, 0);
        }
        if (!rc) fold_gradient(&g, v, gp, g_phys);
    }
    free(qw);
    free(us);
    free(gp);
    free(rho);
    coef_free(&k);
    return rc;
}

/*
 * Tangent-linear (Born) modelling: the data perturbation dd for a model perturbation dv,
 * obtained by differentiating the forward recursion:
 *   du^{n+1} = a du^n - b du^{n-1} + c L du^n + (2c/v_pad) dv_pad (L u^n + q^n).
 */
int orc_born(const orc_grid *gr, const orc_time *t, const double *v, const double *dv, int nsrc,
             const int32_t *src_cell, const double *src_w, const double *wavelet, int nrec,
             const int32_t *rec_cell, double *dd_out)
{
    geo_t g;
    coef_t k;
    acq_t q;
    if (geo_init(gr, &g) || time_check(t)) return -1;
    fill_acq(&q, nsrc, src_cell, src_w, nrec, rec_cell, wavelet);
    if (acq_check(&g, &q)) return -1;
    if (coef_build(gr, &g, t, v, &k)) return -2;
    int64_t nc = g.ncell;
    double *qw = src_dense(&g, &q, t->coef_fp32);
    double *um = calloc(nc, sizeof(double)), *u0 = calloc(nc, sizeof(double)), *up = calloc(nc, sizeof(double));
    double *bm = calloc(nc, sizeof(double)), *b0 = calloc(nc, sizeof(double)), *bp = calloc(nc, sizeof(double));
    double *sc = calloc(nc, sizeof(double));
    int rc = -2;
    if (qw && um && u0 && up && bm && b0 && bp && sc) {
        for (int64_t p = 0; p < nc; ++p) {
            int64_t c = phys_of_pad(&g, p);
            sc[p] = 2.0 * k.c[p] / v[c] * dv[c];
        }
        for (int n = 0; n < t->nt; ++n) {
            double f = rnd(wavelet[n], t->coef_fp32) * k.inv_vol;
            for (int64_t p = 0; p < nc; ++p) {
                double wv = lap_at(&g, &k, u0, p) + qw[p] * f;
                up[p] = k.a[p] * u0[p] - k.b[p] * um[p] + k.c[p] * wv;
                bp[p] = k.a[p] * b0[p] - k.b[p] * bm[p] + k.c[p] * lap_at(&g, &k, b0, p) + sc[p] * wv;
            }
            double *tmp = um; um = u0; u0 = up; up = tmp;
            tmp = bm; bm = b0; b0 = bp; bp = tmp;
            if ((n + 1) % t->rec_every == 0) {
                int j = (n + 1) / t->rec_every - 1;
                for (int r = 0; r < nrec; ++r) dd_out[(int64_t)j * nrec + r] = b0[pad_of_phys(&g, rec_cell[r])];
            }
        }
        rc = 0;
    }
    free(qw); free(um); free(u0); free(up); free(bm); free(b0); free(bp); free(sc);
    coef_free(&k);
    return rc;
}

/* Apply the 8th-order Laplacian (exact FP64 weights) to a padded field; used to pin the
 * stencil on polynomials. */
int orc_laplacian(const orc_grid *gr, const double *u_pad, double *out_pad)
{
    geo_t g;
    if (geo_init(gr, &g)) return -1;
    coef_t k;
    for (int a = 0; a < 3; ++a)
        for (int m = 0; m < 5; ++m) k.w[a][m] = axis_active(&g, a) ? C8[m] / (g.h[a] * g.h[a]) : 0.0;
    for (int64_t p = 0; p < g.ncell; ++p) out_pad[p] = lap_at(&g, &k, u_pad, p);
    return 0;
}

/* Expose the per-cell coefficients a, b, c of the padded grid (for tests). */
int orc_coefficients(const orc_grid *gr, const orc_time *t, const double *v, double *a, double *b, double *c)
{
    geo_t g;
    coef_t k;
    if (geo_init(gr, &g) || !(t->dt > 0)) return -1;
    if (coef_build(gr, &g, t, v, &k)) return -2;
    memcpy(a, k.a, sizeof(double) * g.ncell);
    memcpy(b, k.b, sizeof(double) * g.ncell);
    memcpy(c, k.c, sizeof(double) * g.ncell);
    coef_free(&k);
    return 0;
}

/* ------------------------------------------------------------ sample batch */

/*
 * Batch driver: nsim independent (sample, supergather) simulations, each with its own
 * grid, model offset, sources, receivers and observed data, run in parallel over
 * simulations with OpenMP.  Per simulation it returns d_pred, the misfit phi and the
 * physical-cell gradient (before kappa and before the sum over a sample's simulations).
 */
int orc_gradient_batch(int nsim, const orc_grid *grids, const orc_time *t, const double *const *v,
                       const int32_t *src_ptr, const int32_t *src_cell, const double *src_w,
                       const double *wavelet, const int32_t *rec_ptr, const int32_t *rec_cell,
                       const double *const *d_obs, double inv_sigma2, double *const *d_pred, double *misfit,
                       double *const *g_phys)
{
    int rc_all = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc_all)
    for (int s = 0; s < nsim; ++s) {
        int rc = orc_gradient(&grids[s], t, v[s], src_ptr[s + 1] - src_ptr[s], src_cell + src_ptr[s],
                              src_w + src_ptr[s], wavelet, rec_ptr[s + 1] - rec_ptr[s], rec_cell + rec_ptr[s],
                              d_obs[s], inv_sigma2, d_pred[s], &misfit[s], g_phys[s]);
        rc_all |= (rc != 0);
    }
    return rc_all ? -1 : 0;
}

int orc_forward_batch(int nsim, const orc_grid *grids, const orc_time *t, const double *const *v,
                      const int32_t *src_ptr, const int32_t *src_cell, const double *src_w, const double *wavelet,
                      const int32_t *rec_ptr, const int32_t *rec_cell, double *const *d_out)
{
    int rc_all = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc_all)
    for (int s = 0; s < nsim; ++s) {
        int rc = orc_forward(&grids[s], t, v[s], src_ptr[s + 1] - src_ptr[s], src_cell + src_ptr[s],
                             src_w + src_ptr[s], wavelet, rec_ptr[s + 1] - rec_ptr[s], rec_cell + rec_ptr[s],
                             d_out[s]);
        rc_all |= (rc != 0);
    }
    return rc_all ? -1 : 0;
}

/* ------------------------------------------------------- counter-based RNG */

/*
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC 2011): ten rounds of two 64x64->128 multiplies with a Weyl key schedule.
 */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *lo = (uint64_t)p;
    *hi = (uint64_t)(p >> 64);
}

void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* uniform in (0, 1) from the top 53 bits */
static double u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/*
 * Standard normals for the Langevin noise xi (Eq. 9) of one sample at one step:
 * cells 4m..4m+3 use Philox(ctr = {m, step, sample, 0}, key = {seed, 0x4C414E47}),
 * Box-Muller on the word pairs (0,1) and (2,3): r = sqrt(-2 ln u_a), th = 2 pi u_b,
 * giving r cos th, r sin th.
 */
void orc_normals_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, int64_t n, double *out);

void orc_normals(uint64_t seed, uint64_t step, uint64_t sample, int64_t n, double *out)
{
    orc_normals_key(seed, 0x4C414E47ULL, step, sample, n, out);
}

/*
 * The same construction for any stream: cells 4m..4m+3 use Philox(ctr = {m, a, b, 0},
 * key = {seed, tag}) and Box-Muller as above (the diffusion re-noising uses tag 0x44415053
 * with a = step, b = image).
 */
void orc_normals_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, int64_t n, double *out)
{
    const uint64_t key[2] = {seed, tag};
    for (int64_t m = 0; 4 * m < n; ++m) {
        uint64_t ctr[4] = {(uint64_t)m, a, b, 0}, w[4];
        orc_philox4x64(ctr, key, w);
        double z[4];
        for (int p = 0; p < 2; ++p) {
            double r = sqrt(-2.0 * log(u01(w[2 * p])));
            double th = 6.283185307179586476925 * u01(w[2 * p + 1]);
            z[2 * p] = r * cos(th);
            z[2 * p + 1] = r * sin(th);
        }
        for (int j = 0; j < 4 && 4 * m + j < n; ++j) out[4 * m + j] = z[j];
    }
}

/*
 * Unadjusted Langevin refinement (Eqs. 8-9, with the independent noise weight nu of the
 * modified refinement): z <- clamp(z - eta * g + nu * xi, lo, hi).
 */
void orc_langevin(int64_t n, double *z, const double *g, const double *xi, double eta, double nu, double lo,
                  double hi)
{
    for (int64_t i = 0; i < n; ++i) {
        double y = z[i] - eta * g[i] + nu * xi[i];
        if (y < lo) y = lo;
        if (y > hi) y = hi;
        z[i] = y;
    }
}

/*
 * Encoding draw for one sample at one Langevin step (Eq. 4): G supergathers of s shots,
 * drawn as random partitions of the N_s shots (Fisher-Yates), with Rademacher signs.
 * Word j of the stream is word (j mod 4) of Philox(ctr = {j/4, step, sample, 0},
 * key = {seed, 0x454E43}).  Partition p shuffles with words p*N_s .. p*N_s + N_s - 2
 * (i = N_s-1 down to 1: swap slots i and word mod (i+1)).  Group g uses partition
 * g / (N_s/s), slots (g mod (N_s/s))*s .. +s-1.  Signs use words P*N_s + g*s + m (P =
 * number of partitions): w = -1 if the top bit is set, else +1.  kappa = N_s/(G s).
 */
static uint64_t enc_word(uint64_t seed, uint64_t step, uint64_t sample, uint64_t j)
{
    const uint64_t key[2] = {seed, 0x454E43ULL};
    uint64_t ctr[4] = {j >> 2, step, sample, 0}, w[4];
    orc_philox4x64(ctr, key, w);
    return w[j & 3];
}

int orc_draw_encoding(uint64_t seed, uint64_t step, uint64_t sample, int nshot, int s, int G, int32_t *grp_shot,
                      double *grp_w, double *kappa)
{
    if (nshot < 1 || s < 1 || s > nshot || G < 1) return -1;
    int per = nshot / s;
    int P = (G + per - 1) / per;
    int32_t *perm = malloc(sizeof(int32_t) * nshot);
    if (!perm) return -2;
    for (int g = 0; g < G; ++g) {
        int p = g / per, slot = g % per;
        if (slot == 0) {
            for (int i = 0; i < nshot; ++i) perm[i] = i;
            for (int i = nshot - 1; i >= 1; --i) {
                uint64_t w = enc_word(seed, step, sample, (uint64_t)p * nshot + (nshot - 1 - i));
                int j = (int)(w % (uint64_t)(i + 1));
                int32_t tmp = perm[i];
                perm[i] = perm[j];
                perm[j] = tmp;
            }
        }
        for (int m = 0; m < s; ++m) {
            grp_shot[g * s + m] = perm[slot * s + m];
            uint64_t w = enc_word(seed, step, sample, (uint64_t)P * nshot + (uint64_t)g * s + m);
            grp_w[g * s + m] = (w >> 63) ? -1.0 : 1.0;
        }
    }
    *kappa = (double)nshot / ((double)G * s);
    free(perm);
    return 0;
}
