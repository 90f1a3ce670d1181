/*
 * fwi_oracle.h -- FP64 CPU oracle for the encoded-shot acoustic FWI gradient.
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  See fwi_oracle.c.
 *
 * Conventions: physical grid nz x (ny) x nx, x fastest; a physical cell index is
 * (iz*ny + iy)*nx + ix (ny = 1 in 2D).  Data are [t][receiver].  Return 0 on success,
 * -1 on a bad argument, -2 on allocation failure.
 */
#ifndef FWI_ORACLE_H
#define FWI_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t nz, ny, nx;    /* physical cells per axis (ny ignored in 2D) */
    double dz, dy, dx;     /* spacing in metres */
    int32_t nb;            /* sponge cells added on every face */
    double v_ref;          /* sponge reference velocity (m/s) */
    double refl;           /* sponge target reflection coefficient R */
} orc_grid;

typedef struct {
    double dt;             /* time step (s) */
    int32_t nt;            /* number of steps */
    int32_t rec_every;     /* record every R steps; nt % R == 0 */
    int32_t coef_fp32;     /* 1: round the coefficient set to FP32 once */
} orc_time;

int orc_forward(const orc_grid *g, const orc_time *t, const double *v, int nsrc, const int32_t *src_cell,
                const double *src_w, const double *wavelet, int nrec, const int32_t *rec_cell, double *d_out);
int orc_adjoint(const orc_grid *g, const orc_time *t, const double *v, int nsrc, const int32_t *src_cell,
                const double *src_w, const double *wavelet, int nrec, const int32_t *rec_cell, const double *rho,
                double *g_phys, int32_t trace_phys_cell, double *trace);
int orc_gradient(const orc_grid *g, const orc_time *t, const double *v, int nsrc, const int32_t *src_cell,
                 const double *src_w, const double *wavelet, int nrec, const int32_t *rec_cell,
                 const double *d_obs, double inv_sigma2, double *d_pred, double *misfit, double *g_phys);
int orc_born(const orc_grid *g, const orc_time *t, const double *v, const double *dv, int nsrc,
             const int32_t *src_cell, const double *src_w, const double *wavelet, int nrec,
             const int32_t *rec_cell, double *dd_out);
int orc_laplacian(const orc_grid *g, const double *u_pad, double *out_pad);
int orc_coefficients(const orc_grid *g, const orc_time *t, const double *v, double *a, double *b, double *c);
int orc_gradient_batch(int nsim, const orc_grid *grids, const orc_time *t, const double *const *v,
                       const int32_t *src_ptr, const int32_t *src_cell, const double *src_w,
                       const double *wavelet, const int32_t *rec_ptr, const int32_t *rec_cell,
                       const double *const *d_obs, double inv_sigma2, double *const *d_pred, double *misfit,
                       double *const *g_phys);
int orc_forward_batch(int nsim, const orc_grid *grids, const orc_time *t, const double *const *v,
                      const int32_t *src_ptr, const int32_t *src_cell, const double *src_w, const double *wavelet,
                      const int32_t *rec_ptr, const int32_t *rec_cell, double *const *d_out);
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void orc_normals(uint64_t seed, uint64_t step, uint64_t sample, int64_t n, double *out);
/* standard normals of the stream Philox(ctr = {m, a, b, 0}, key = {seed, tag}), Box-Muller */
void orc_normals_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, int64_t n, double *out);
void orc_langevin(int64_t n, double *z, const double *g, const double *xi, double eta, double nu, double lo,
                  double hi);
int orc_draw_encoding(uint64_t seed, uint64_t step, uint64_t sample, int nshot, int s, int G, int32_t *grp_shot,
                      double *grp_w, double *kappa);

#endif
