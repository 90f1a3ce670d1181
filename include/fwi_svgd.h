/*
 * fwi_svgd.h -- C ABI of the Stein variational gradient descent baseline the paper
 * compares its sampler with (the head-to-head comparison among its contributions, and the
 * 2D experiments of Sec. 3: particles moved by conventional FWI gradients, null prior, box
 * bounds).  The paper restates no formula; the step is that of the cited method (Liu and
 * Wang 2016) with the RBF kernel and the median bandwidth:
 *   k(x, y) = exp(-|x - y|^2 / h),   h = median_{i<j} |x_i - x_j|^2 / log n,
 *   phi_i = (1/n) sum_j k(x_j, x_i) [ -g_j + (2/h) (x_i - x_j) ],
 *   x_i <- clamp(x_i + eps phi_i, v_lo, v_hi),
 * g_j the misfit gradient of particle j (fwi_gradient's output: grad log p = -g).
 *
 * All arrays are device memory owned by the caller; the call is asynchronous on `stream`
 * (a hipStream_t, NULL = default stream).  Arguments are checked on the host before
 * anything is enqueued; a non-OK status comes with a text from fwi_svgd_last_error().
 */
#ifndef FWI_SVGD_H
#define FWI_SVGD_H

#include <stddef.h>
#include <stdint.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of the work buffer fwi_svgd_step needs for n particles of N cells (0 when n or N
 * is out of range). */
size_t fwi_svgd_work_size(int32_t n, int64_t N);

/*
 * One SVGD step for n particles (1 <= n <= 64) of N cells each:
 *   x, grad: device f32 [n][N] (particle j at x + j N);
 *   x_out:   device f32 [n][N], the moved particles; must not overlap x or grad;
 *   phi:     device f32 [n][N] or NULL, the direction (before eps and the clamp); must not
 *            overlap x, grad or x_out;
 *   h_out:   device f64 [1] or NULL, the bandwidth used;
 *   eps >= 0 the step (eps = 0 leaves x_out = clamp(x) and still writes phi);
 *   h > 0 fixes the bandwidth, h <= 0 selects the median heuristic (n >= 2; with n = 1,
 *     or when the median is 0 because the particles coincide, h = 1);
 *   work: device memory of fwi_svgd_work_size(n, N) bytes, 8-byte aligned.
 * Distances, bandwidth, kernel and direction are computed in FP64 (distances summed in an
 * order fixed by N alone, so results are reproducible run to run); outputs rounded once.
 * FWI_E_ARG: null x, grad or x_out, n or N out of range, eps < 0 or not finite, v_hi <=
 * v_lo, x_out or phi overlapping x, grad or each other.  FWI_E_WORKSPACE: work null,
 * misaligned or smaller than fwi_svgd_work_size.
 */
fwi_status fwi_svgd_step(int32_t n, int64_t N, const float *x, const float *grad, float eps, float h, float v_lo,
                         float v_hi, float *x_out, float *phi, double *h_out, void *work, size_t work_bytes,
                         void *stream);

const char *fwi_svgd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FWI_SVGD_H */
