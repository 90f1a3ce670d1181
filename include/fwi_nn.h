/*
 * fwi_nn.h -- C ABI of the network kernels of the learned gradient preconditioner.
 *
 * The preconditioner maps an encoded-supergather gradient (Eq. 6 estimate) and the
 * current model to an estimate of the full-shot gradient (the estimator's mean).  It is
 * a U-Net built from the operations below; every operation is a hand-written gfx950
 * kernel: 3x3 convolutions are implicit GEMMs on BF16 matrix cores (MFMA
 * 32x32x16) with FP32 accumulation.
 *
 * Layout: activations are NHWC -- element (n, y, x, c) at ((n*H + y)*W + x)*C + c -- with
 * channel counts padded to multiples of 16 (inputs of convolutions) or 32 (outputs);
 * padded channels hold zeros.  Convolution weights are BF16 [Cout][9][Cin] (tap = 3*ky +
 * kx, ky/kx = 0..2 for offsets -1..+1), zero-padded likewise.  "bf16" is the IEEE binary32
 * upper half (round to nearest even); "f32" is IEEE binary32.  All pointers are device
 * pointers unless stated; all calls are asynchronous on `stream` (hipStream_t, NULL =
 * default) and return an fwi_status (fwi.h).  Sizes are validated on the host before any
 * enqueue; pointers are not.
 */
#ifndef FWI_NN_H
#define FWI_NN_H
#include <stdint.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Shape of one NHWC activation: n images of h x w pixels, c channels (padded). */
typedef struct {
    int32_t n, h, w, c;
} fwi_nn_shape;

/*
 * 3x3 convolution, stride 1, zero padding 1 (implicit GEMM on MFMA):
 *   acc[p][co] = sum_{tap, ci} w[co][tap][ci] * x[p + offset(tap)][ci]   (FP32 accumulation)
 *   v = acc + bias[co]            (bias nullable)
 *   v = v * silu'(aux[p][co])     (aux nullable: FP32 pre-activation, used for the
 *                                  data-gradient pass: dz_in = (dL/da_in) * silu'(z_in))
 *   v = v + res[p]   for co == 0  (res nullable: FP32 [pixels] residual added to channel 0)
 *   out_f32[p][co] = v            (nullable)
 *   out_bf16[p][co] = bf16(act ? silu(v) : v)   (nullable)
 * x: bf16 [in.n][in.h][in.w][in.c], in.c % 16 == 0; w: bf16 [cout][9][in.c], cout % 32 == 0.
 * Outputs have `cout` channels.  silu(z) = z / (1 + exp(-z)).
 */
fwi_status fwi_nn_conv3x3(const uint16_t *x, fwi_nn_shape in, const uint16_t *w, int32_t cout, const float *bias,
                          const float *aux, const float *res, int32_t act, float *out_f32, uint16_t *out_bf16,
                          void *stream);

/*
 * The same convolution over the channel concatenation [up2(a), b] of a decoder level, without materialising it:
 * input channel ci < ca is a[n][y/2][x/2][ci] (a: bf16 [in.n][in.h/2][in.w/2][ca], nearest 2x upsampling), channel
 * ci >= ca is b[n][y][x][ci - ca] (b: bf16 [in.n][in.h][in.w][in.c - ca]).  in.c is the concatenated channel count;
 * ca and in.c - ca must be positive multiples of 16, in.h and in.w even.  Results equal fwi_nn_conv3x3 on the
 * materialised concatenation bit for bit.  (U-Net decoders: the skip connection of Ronneberger et al. 2015.)
 */
fwi_status fwi_nn_conv3x3_upcat(const uint16_t *a, int32_t ca, const uint16_t *b, fwi_nn_shape in, const uint16_t *w,
                                int32_t cout, const float *bias, const float *aux, const float *res, int32_t act,
                                float *out_f32, uint16_t *out_bf16, void *stream);

/*
 * Weight and bias gradients of that convolution:
 *   dw[co][tap][ci] = sum_p dz[p][co] * x[p + offset(tap)][ci]     (FP32, deterministic)
 *   db[co] = sum_p dz_f32[p][co]                                   (db nullable)
 * dz: bf16 [p][cout] (the same gradient in f32 for db: dz_f32, nullable with db),
 * x as in fwi_nn_conv3x3.  work: f32 scratch of fwi_nn_wgrad_work(in, cout) floats.
 */
int64_t fwi_nn_wgrad_work(fwi_nn_shape in, int32_t cout);
fwi_status fwi_nn_wgrad(const uint16_t *dz, const float *dz_f32, const uint16_t *x, fwi_nn_shape in, int32_t cout,
                        float *dw, float *db, float *work, void *stream);
/* The same with the input [up2(a), b] as in fwi_nn_conv3x3_upcat (work: fwi_nn_wgrad_work(in, cout) floats). */
fwi_status fwi_nn_wgrad_upcat(const uint16_t *dz, const float *dz_f32, const uint16_t *a, int32_t ca,
                              const uint16_t *b, fwi_nn_shape in, int32_t cout, float *dw, float *db, float *work,
                              void *stream);

/* 2x2 average pooling (h, w even): out[n][y][x][c] = bf16(mean of the 4 inputs).
 * Backward: dx[n][2y+i][2x+j][c] (+)= dout[n][y][x][c] / 4 (accumulate != 0 adds). */
fwi_status fwi_nn_pool2(const uint16_t *x, fwi_nn_shape in, uint16_t *out, void *stream);
fwi_status fwi_nn_pool2_bwd(const float *dout, fwi_nn_shape in, float *dx, int32_t accumulate, void *stream);

/* Nearest 2x upsampling: out[n][y][x][c] = x[n][y/2][x/2][c] (in = the small shape).
 * Backward: dx[n][y][x][c] = sum of the 4 dout values it fed. */
fwi_status fwi_nn_up2(const uint16_t *x, fwi_nn_shape in, uint16_t *out, void *stream);
fwi_status fwi_nn_up2_bwd(const float *dout, fwi_nn_shape in, float *dx, void *stream);

/* Channel concatenation out = [a (ca channels) | b (cb channels)] for every pixel, and the
 * backward split of its gradient: da (+)= d[..., :ca], db (+)= d[..., ca:]. */
fwi_status fwi_nn_concat(const uint16_t *a, int32_t ca, const uint16_t *b, int32_t cb, int64_t npix, uint16_t *out,
                         void *stream);
fwi_status fwi_nn_split_bwd(const float *d, int32_t ca, int32_t cb, int64_t npix, float *da, int32_t acc_a, float *db,
                            int32_t acc_b, void *stream);

/* Activation backward: dz = da * silu'(z); written in f32 and bf16 (either nullable). */
fwi_status fwi_nn_silu_bwd(const float *da, const float *z, int64_t n, float *dz_f32, uint16_t *dz_bf16,
                           void *stream);

/*
 * Relative squared error of channel 0 of pred (f32 [nimg][h*w][c]) against target (f32
 * [nimg][h*w]): L = (1/nimg) sum_i |pred_i - t_i|^2 / |t_i|^2.  Writes loss (f32 [1],
 * nullable) and, if dpred is not NULL, dL/dpred into dpred (f32, same layout as pred,
 * zero in channels > 0) and its bf16 copy dpred_bf16 (nullable).  work: f32 scratch of
 * 2 * nimg * 256 floats.
 */
fwi_status fwi_nn_rel_mse(const float *pred, int32_t c, const float *target, int32_t nimg, int64_t hw, float *loss,
                          float *dpred, uint16_t *dpred_bf16, float *work, void *stream);

/*
 * Adam step on n FP32 parameters (m, v moments in FP32):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
 */
fwi_status fwi_nn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, int32_t t, void *stream);

/*
 * Weight packing of one convolution from its FP32 master copy wf [cout][9][cin] (cin,
 * cout padded): w_bf16[co][tap][ci] = bf16(wf[co][tap][ci]) and the data-gradient weights
 * wt_bf16[ci][8 - tap][co] = bf16(wf[co][tap][ci]) (flipped taps, in/out swapped), both
 * nullable.
 */
fwi_status fwi_nn_pack_weights(const float *wf, int32_t cout, int32_t cin, uint16_t *w_bf16, uint16_t *wt_bf16,
                               void *stream);

/* Round f32 to bf16 (n elements). */
fwi_status fwi_nn_to_bf16(const float *x, int64_t n, uint16_t *out, void *stream);

/*
 * Network input of the gradient preconditioner (form: learned map from the encoded
 * gradient to the full-shot gradient).  For nimg images g (device f32 [nimg][h][w]) with
 * models v (device f32, same layout):
 *   scale_i = sqrt(mean over the image of g^2) (FP64, fixed order; 1 for an all-zero
 *             image), or scale_in[i] when scale_in (device f32 [nimg]) is given;
 *   x_bf16  (device bf16 [nimg][hp][w][16], 16-byte aligned, nullable): channel 0 = g/scale_i, channel 1 =
 *             (v - v_shift)/v_scale, channels 2..15 and rows h..hp-1 zero;
 *   res     (device f32 [nimg][hp][w], nullable): g/scale_i (the residual the network's
 *             output adds to), rows h..hp-1 zero.
 * scale_out (device f32 [nimg], nullable if scale_in is given) receives the scales.  With
 * scale_in and res only (v nullable), this scales training targets by the inputs' scales.
 * Rows are padded so that hp fits the network's pooling depth.
 */
fwi_status fwi_nn_prep(const float *g, const float *v, int32_t nimg, int32_t h, int32_t w, int32_t hp,
                       float v_shift, float v_scale, const float *scale_in, float *scale_out, uint16_t *x_bf16,
                       float *res, void *stream);

/*
 * Guarded use of the network's gradient: p_i = scale_i * channel 0 of pred (device f32
 * [nimg][hp][w][c]) over the first h rows is kept when its cosine with the plain gradient
 * g_i (device f32 [nimg][h][w]) is >= cos_min and |p_i|/|g_i| lies in [ratio_lo,
 * ratio_hi] (FP64 statistics, fixed order); otherwise g_i is used.  A kept image gives
 * g_i + alpha (p_i - g_i) in FP32 (alpha = 1: p_i exactly; alpha = 0: g_i), alpha in
 * [0, 1], a blend weight fitted on validation pairs.  out: device f32 [nimg][h][w]; keep:
 * device int32 [nimg] (1 = network output kept).  FWI_E_ARG for alpha outside [0, 1].
 */
fwi_status fwi_nn_guard(const float *pred, int32_t c, const float *scale, const float *g, int32_t nimg, int32_t h,
                        int32_t w, int32_t hp, float cos_min, float ratio_lo, float ratio_hi, float alpha,
                        float *out, int32_t *keep, void *stream);

/* Thread-local detail of the last non-OK status returned by an fwi_nn_* call. */
const char *fwi_nn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FWI_NN_H */
