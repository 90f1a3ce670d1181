/*
 * fwi_daps.h -- C ABI of the diffusion outer loop around the Langevin refinement: the
 * decoupled diffusion inference of Sec. 2 ("Decoupled diffusion inference with encoded
 * shots data"): predict a clean model from the noisy state x_t with the predict-x0
 * network (Eq. 7), refine it with the encoded-gradient Langevin steps (fwi.h), and
 * re-noise it to the next level with the DDPM posterior (Eqs. 10-12).
 *
 * Models live in two spaces: physical velocities v (m/s) and the diffusion model's
 * normalised space x = 2 (v - v_lo) / (v_hi - v_lo) - 1 (in [-1, 1] for v in [v_lo, v_hi]).
 * All arrays are device memory owned by the caller; calls are asynchronous on `stream`
 * (a hipStream_t, NULL = default stream).  Arguments are checked on the host before
 * anything is enqueued; a non-OK status comes with a text from fwi_daps_last_error().
 */
#ifndef FWI_DAPS_H
#define FWI_DAPS_H

#include <stdint.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * For nimg images of n cells each (device f32 [nimg][n] for z, x and out):
 *   out[i][j] = c0[i] * xn(z[i][j]) + c1[i] * x[i][j] + sig[i] * xi[i][j]
 * with xn(v) = 2 (v - v_lo) / (v_hi - v_lo) - 1.  z (physical models) and x (normalised
 * models) are nullable: a null one drops its term.  c0, c1, sig: device f32 [nimg].  xi are
 * standard normals drawn in the kernel: cells 4m .. 4m+3 of image i use Philox4x64-10 with
 * counter {m, step, i, 0} and key {seed, 0x44415053}, Box-Muller on the word pairs (0, 1)
 * and (2, 3) (the construction of fwi_langevin's noise, with its own key).  Evaluated in
 * FP64, rounded once.  out may alias x.
 * Uses (alpha_t = prod_{s<=t} (1 - beta_s), alpha_0 = 1):
 *   forward diffusion x_t ~ q(x_t | x_0):   c0 = sqrt(alpha_t), c1 = 0, sig = sqrt(1 - alpha_t);
 *   re-noise x_{t-1} ~ N(mu_t(x_t, z), beta~_t): c0 = sqrt(alpha_{t-1}) beta_t / (1 - alpha_t),
 *     c1 = sqrt(1 - beta_t) (1 - alpha_{t-1}) / (1 - alpha_t),
 *     sig = sqrt((1 - alpha_{t-1}) / (1 - alpha_t) beta_t);
 *   normalisation alone: c0 = 1, c1 = sig = 0.
 * FWI_E_ARG: null out or coefficient arrays, z and x both null, nimg < 1 or > 65535, n < 1,
 * or v_hi <= v_lo.
 */
fwi_status fwi_daps_mix(int32_t nimg, int64_t n, const float *z, const float *x, const float *c0, const float *c1,
                        const float *sig, float v_lo, float v_hi, uint64_t seed, uint64_t step, float *out,
                        void *stream);

/*
 * Input of the predict-x0 network for nimg normalised models x (device f32 [nimg][h][w]):
 *   x_bf16 (device bf16 [nimg][hp][w][16], 16-byte aligned): channel 0 = x, channel 1 =
 *     level[i] (device f32 [nimg]: the noise level the model carries, sqrt(1 - alpha_t)),
 *     channels 2..15 and rows h .. hp-1 zero (BF16 round to nearest even);
 *   res (device f32 [nimg][hp][w], nullable): x, rows h .. hp-1 zero -- the residual the
 *     network adds its output to, so that its channel 0 is the clean-model estimate.
 * FWI_E_ARG: null x, level or x_bf16, misaligned x_bf16, nimg < 1, h < 1, w < 1, hp < h.
 */
fwi_status fwi_daps_prep(int32_t nimg, int32_t h, int32_t w, int32_t hp, const float *x, const float *level,
                         uint16_t *x_bf16, float *res, void *stream);

/*
 * Physical models from the network's clean-model estimate: for channel 0 of pred (device
 * f32 [nimg][hp][w][c]) over the first h rows,
 *   v = v_lo + (p + 1) / 2 (v_hi - v_lo), clamped to [v_lo, v_hi]  (device f32 [nimg][h][w]),
 * in FP64, rounded once.  FWI_E_ARG: null pointers, nimg < 1, h < 1, w < 1, hp < h, c < 1,
 * v_hi <= v_lo.
 */
fwi_status fwi_daps_model(int32_t nimg, int32_t h, int32_t w, int32_t hp, int32_t c, const float *pred, float v_lo,
                          float v_hi, float *v, void *stream);

const char *fwi_daps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FWI_DAPS_H */
