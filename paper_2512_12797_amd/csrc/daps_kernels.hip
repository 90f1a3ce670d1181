// daps_kernels.hip -- gfx950 kernels of the diffusion outer loop around the Langevin
// refinement (include/fwi_daps.h): forward diffusion and DDPM re-noising in the
// normalised model space, the predict-x0 network's input, and the map of its clean-model
// estimate back to physical velocities.  All three are streaming elementwise passes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/fwi_daps.h"
#include "philox.h"

namespace {

constexpr uint64_t kDapsTag = 0x44415053ULL;  // key word of the re-noise stream

// f32 -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// One thread per 4 cells of one image (blockIdx.y): the normal draws of a Philox block
// cover those 4 cells.
__global__ __launch_bounds__(256) void k_daps_mix(int64_t n, const float *__restrict__ z, const float *__restrict__ x,
                                                  const float *__restrict__ c0, const float *__restrict__ c1,
                                                  const float *__restrict__ sig, double v_lo, double inv_span2,
                                                  uint64_t seed, uint64_t step, float *out)
{
    const int img = blockIdx.y;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * m >= n) return;
    const double a = c0[img], b = c1[img], s = sig[img];
    double xi[4] = {0.0, 0.0, 0.0, 0.0};
    if (s != 0.0) fwi::normals4((uint64_t)m, step, (uint64_t)img, seed, kDapsTag, xi);
    const int64_t base = (int64_t)img * n;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = 4 * m + j;
        if (i >= n) break;
        double y = s * xi[j];
        if (z) y += a * (((double)z[base + i] - v_lo) * inv_span2 - 1.0);
        if (x) y += b * (double)x[base + i];
        out[base + i] = (float)y;
    }
}

// One thread per (image, row < hp, column): 16 BF16 channels (two 16-byte stores) and the
// residual.
__global__ __launch_bounds__(256) void k_daps_prep(int32_t nimg, int32_t h, int32_t w, int32_t hp,
                                                   const float *__restrict__ x, const float *__restrict__ level,
                                                   uint4 *__restrict__ x16, float *__restrict__ res)
{
    const int64_t total = (int64_t)nimg * hp * w;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = p / ((int64_t)hp * w);
        const int64_t rc = p - img * hp * w;
        const int32_t row = (int32_t)(rc / w), col = (int32_t)(rc - (int64_t)row * w);
        const bool in = row < h;
        const float v = in ? x[(img * h + row) * w + col] : 0.0f;
        const float l = in ? level[img] : 0.0f;
        uint4 lo;
        lo.x = (uint32_t)bf16_rne(v) | ((uint32_t)bf16_rne(l) << 16);
        lo.y = lo.z = lo.w = 0u;
        x16[2 * p] = lo;
        x16[2 * p + 1] = make_uint4(0u, 0u, 0u, 0u);
        if (res) res[p] = v;
    }
}

__global__ __launch_bounds__(256) void k_daps_model(int32_t nimg, int32_t h, int32_t w, int32_t hp, int32_t c,
                                                    const float *__restrict__ pred, double v_lo, double v_hi,
                                                    float *__restrict__ v)
{
    const int64_t total = (int64_t)nimg * h * w;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = p / ((int64_t)h * w);
        const int64_t k = p - img * h * w;  // row * w + column, rows < h
        const double q = pred[(img * hp * w + k) * c];
        double y = v_lo + (q + 1.0) * 0.5 * (v_hi - v_lo);
        y = y < v_lo ? v_lo : y;
        y = y > v_hi ? v_hi : y;
        v[p] = (float)y;
    }
}

thread_local std::string g_daps_err;

fwi_status daps_fail(fwi_status s, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_daps_err = buf;
    return s;
}

fwi_status daps_check(hipError_t e, const char *what)
{
    return e == hipSuccess ? FWI_OK : daps_fail(FWI_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

}  // namespace

extern "C" {

fwi_status fwi_daps_mix(int32_t nimg, int64_t n, const float *z, const float *x, const float *c0, const float *c1,
                        const float *sig, float v_lo, float v_hi, uint64_t seed, uint64_t step, float *out,
                        void *stream)
{
    if (!out || !c0 || !c1 || !sig) return daps_fail(FWI_E_ARG, "mix: null output or coefficients");
    if (nimg < 1 || nimg > 65535 || n < 1) return daps_fail(FWI_E_ARG, "mix: need 1 <= nimg <= 65535 and n >= 1");
    if (!(v_hi > v_lo)) return daps_fail(FWI_E_ARG, "mix: need v_hi > v_lo");
    if (!z && !x) return daps_fail(FWI_E_ARG, "mix: neither z nor x given");
    const int64_t groups = (n + 3) / 4;
    if ((groups + 255) / 256 > 0x7FFFFFFF) return daps_fail(FWI_E_ARG, "mix: images too large");
    dim3 grid((unsigned)((groups + 255) / 256), (unsigned)nimg);
    k_daps_mix<<<grid, 256, 0, (hipStream_t)stream>>>(n, z, x, c0, c1, sig, (double)v_lo,
                                                      2.0 / ((double)v_hi - (double)v_lo), seed, step, out);
    return daps_check(hipGetLastError(), "mix");
}

fwi_status fwi_daps_prep(int32_t nimg, int32_t h, int32_t w, int32_t hp, const float *x, const float *level,
                         uint16_t *x_bf16, float *res, void *stream)
{
    if (!x || !level || !x_bf16) return daps_fail(FWI_E_ARG, "prep: null input, level or output");
    if (nimg < 1 || h < 1 || w < 1 || hp < h) return daps_fail(FWI_E_ARG, "prep: bad shape");
    if ((uintptr_t)x_bf16 % 16) return daps_fail(FWI_E_ARG, "prep: x_bf16 must be 16-byte aligned");
    const int64_t total = (int64_t)nimg * hp * w;
    k_daps_prep<<<grid_for(total), 256, 0, (hipStream_t)stream>>>(nimg, h, w, hp, x, level, (uint4 *)x_bf16, res);
    return daps_check(hipGetLastError(), "prep");
}

fwi_status fwi_daps_model(int32_t nimg, int32_t h, int32_t w, int32_t hp, int32_t c, const float *pred, float v_lo,
                          float v_hi, float *v, void *stream)
{
    if (!pred || !v) return daps_fail(FWI_E_ARG, "model: null pointer");
    if (nimg < 1 || h < 1 || w < 1 || hp < h || c < 1) return daps_fail(FWI_E_ARG, "model: bad shape");
    if (!(v_hi > v_lo)) return daps_fail(FWI_E_ARG, "model: need v_hi > v_lo");
    const int64_t total = (int64_t)nimg * h * w;
    k_daps_model<<<grid_for(total), 256, 0, (hipStream_t)stream>>>(nimg, h, w, hp, c, pred, (double)v_lo,
                                                                   (double)v_hi, v);
    return daps_check(hipGetLastError(), "model");
}

const char *fwi_daps_last_error(void) { return g_daps_err.c_str(); }

}  // extern "C"
