// nn_kernels.hip -- gfx950 kernels of the learned gradient preconditioner (include/fwi_nn.h).
//
// 3x3 convolutions are implicit GEMMs on the BF16 matrix cores: M = pixels, N = output
// channels, K = 9 taps x input channels, one v_mfma_f32_32x32x16_bf16 per 16-wide K step.
// Operand lane layout of that instruction (checked on the hardware): A lane l holds row
// l%32, k = 8*(l/32) .. +7; B lane l holds column l%32, the same k; accumulator register r
// holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.  With NHWC activations and [Cout][9][Cin]
// weights both operands are single 16-byte loads per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/fwi_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                            // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------------ conv3x3

// Block = 4 wavefronts in a 2 x 2 arrangement; each wavefront accumulates MT x NT tiles of
// 32 pixels x 32 output channels (each loaded fragment feeds NT or MT matrix operations)
// and fetches the fragments of the next K step while the current ones are multiplied.
template <int MT, int NT>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t *__restrict__ x, int N, int H, int W, int Cin,
                                                 const uint16_t *__restrict__ w, int Cout,
                                                 const float *__restrict__ bias, const float *__restrict__ aux,
                                                 const float *__restrict__ res, int act, float *__restrict__ of32,
                                                 uint16_t *__restrict__ obf)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t P = (int64_t)N * H * W;
    const int64_t p0 = (int64_t)blockIdx.x * (64 * MT) + (wave & 1) * (32 * MT);
    const int co0 = blockIdx.y * (64 * NT) + (wave >> 1) * (32 * NT);
    if (co0 >= Cout || p0 >= P) return;  // uniform per wavefront; no barriers below
    const int kh = (lane >> 5) * 8;
    int py[MT], px[MT], pn[MT];
    bool pin[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int64_t p = p0 + 32 * i + (lane & 31);
        pin[i] = p < P;
        px[i] = pin[i] ? (int)(p % W) : 0;
        const int64_t t = pin[i] ? p / W : 0;
        py[i] = (int)(t % H);
        pn[i] = (int)(t / H);
    }
    const uint16_t *wrow[NT];
    bool cin_[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = co0 + 32 * j + (lane & 31);
        cin_[j] = co < Cout;
        wrow[j] = w + (int64_t)(cin_[j] ? co : 0) * 9 * Cin + kh;
    }
    const int csteps = Cin / 16;
    const int ksteps = 9 * csteps;
    auto load_a = [&](int ks, uint4 (&a)[MT]) {
        const int tap = ks / csteps, c0 = (ks - tap * csteps) * 16;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int yy = py[i] + dy, xs = px[i] + dx;
            const bool v = pin[i] && yy >= 0 && yy < H && xs >= 0 && xs < W;
            a[i] = make_uint4(0u, 0u, 0u, 0u);
            if (v) a[i] = *(const uint4 *)(x + (((int64_t)pn[i] * H + yy) * W + xs) * Cin + kh + c0);
        }
    };
    auto load_b = [&](int ks, uint4 (&b)[NT]) {
        const int tap = ks / csteps, c0 = (ks - tap * csteps) * 16;
#pragma unroll
        for (int j = 0; j < NT; ++j) b[j] = *(const uint4 *)(wrow[j] + tap * Cin + c0);
    };
    f32x16 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x16{};
    uint4 a[MT], b[NT], an[MT], bn[NT];
    load_a(0, a);
    load_b(0, b);
    for (int ks = 0; ks < ksteps; ++ks) {
        if (ks + 1 < ksteps) {
            load_a(ks + 1, an);
            load_b(ks + 1, bn);
        }
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[i]),
                                                                    __builtin_bit_cast(bf16x8, b[j]), acc[i][j], 0, 0,
                                                                    0);
#pragma unroll
        for (int i = 0; i < MT; ++i) a[i] = an[i];
#pragma unroll
        for (int j = 0; j < NT; ++j) b[j] = bn[j];
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int c = co0 + 32 * j + (lane & 31);
        if (!cin_[j]) continue;
        const float bb = bias ? bias[c] : 0.0f;
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t pr = p0 + 32 * i + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
                if (pr >= P) continue;
                float val = acc[i][j][r] + bb;
                const int64_t o = pr * Cout + c;
                if (aux) val *= dsilu(aux[o]);
                if (res && c == 0) val += res[pr];
                if (of32) of32[o] = val;
                if (obf) obf[o] = f2bf(act ? silu(val) : val);
            }
    }
}

// ------------------------------------------------------------------- wgrad

// One wavefront per (32 output channels, 32 input channels, pixel chunk), all 9 taps:
// M = co, N = ci, K = pixels in steps of 16.  Each step loads the 16-pixel x 32-channel
// tiles of dz (once) and of x at the 9 shifted positions with one coalesced 16-byte load
// per lane, stages them in LDS and reads them back in the matrix-operand layout.
__global__ __launch_bounds__(64) void k_wgrad(const uint16_t *__restrict__ dz, const uint16_t *__restrict__ x,
                                              int N, int H, int W, int Cin, int Cout, int64_t per_chunk,
                                              float *__restrict__ work)
{
    __shared__ uint16_t ta[16][32];
    __shared__ uint16_t tb[16][32];
    const int lane = threadIdx.x;
    const int nci = (Cin + 31) / 32;
    const int cit = blockIdx.x % nci, cot = blockIdx.x / nci;
    const int chunk = blockIdx.y;
    const int64_t P = (int64_t)N * H * W;
    const int64_t pb = (int64_t)chunk * per_chunk;
    const int64_t pe = std::min<int64_t>(pb + per_chunk, P);
    const int lr = lane >> 2, lc = (lane & 3) * 8;  // loader role: tile row (pixel) lr, 8 channels from lc
    const int co_ld = cot * 32 + lc, ci_ld = cit * 32 + lc;
    const int kr = 8 * (lane >> 5), mc = lane & 31;  // operand role: rows kr..kr+7, column mc
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x16{};
    for (int64_t pk = pb; pk < pe; pk += 16) {
        const int64_t pp = pk + lr;
        const bool pv = pp < pe;
        uint4 av = make_uint4(0u, 0u, 0u, 0u);
        if (pv) av = *(const uint4 *)(dz + pp * Cout + co_ld);
        int y = 0, xx = 0, n = 0;
        if (pv) {
            xx = (int)(pp % W);
            const int64_t tt = pp / W;
            y = (int)(tt % H);
            n = (int)(tt / H);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        *(uint4 *)&ta[lr][lc] = av;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        bf16x8 a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_bit_cast(__bf16, ta[kr + j][mc]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int yy = y + tap / 3 - 1, xs = xx + tap % 3 - 1;
            uint4 bv = make_uint4(0u, 0u, 0u, 0u);
            if (pv && ci_ld < Cin && yy >= 0 && yy < H && xs >= 0 && xs < W)
                bv = *(const uint4 *)(x + (((int64_t)n * H + yy) * W + xs) * Cin + ci_ld);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            *(uint4 *)&tb[lr][lc] = bv;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; ++j) b[j] = __builtin_bit_cast(__bf16, tb[kr + j][mc]);
            acc[tap] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[tap], 0, 0, 0);
        }
    }
    // acc[tap][r]: row (co) 8*(r/4) + 4*(lane/32) + r%4, column (ci) lane%32
    float *wk = work + (int64_t)chunk * Cout * 9 * Cin;
    const int cic = cit * 32 + (lane & 31);
    if (cic < Cin)
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int cor = cot * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
                wk[((int64_t)cor * 9 + tap) * Cin + cic] = acc[tap][r];
            }
}

__global__ void k_sum_chunks(const float *__restrict__ work, int nchunk, int64_t n, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += work[(int64_t)c * n + i];
    out[i] = s;
}

// db partials: block = pixel chunk; the 256 threads form (256/C) pixel lanes x C channels
// (C <= 256, a power of two up to the padding) so that every load row is coalesced; the
// pixel lanes are then summed in a fixed-order LDS tree.
__global__ __launch_bounds__(256) void k_bias_partial(const float *__restrict__ dz, int64_t P, int C, int64_t per_chunk,
                                                      float *__restrict__ work)
{
    __shared__ float red[256];
    const int64_t pb = (int64_t)blockIdx.x * per_chunk, pe = std::min<int64_t>(pb + per_chunk, P);
    for (int c0 = 0; c0 < C; c0 += 256) {
        const int cw = std::min(256, C - c0);           // channels in this pass
        const int lanes = 256 / cw;                     // pixel lanes
        const int c = threadIdx.x % cw, pl = threadIdx.x / cw;
        float s = 0.0f;
        if (pl < lanes)
            for (int64_t p = pb + pl; p < pe; p += lanes) s += dz[p * C + c0 + c];
        red[threadIdx.x] = pl < lanes ? s : 0.0f;
        __syncthreads();
        if (threadIdx.x < cw) {
            float t = 0.0f;
            for (int l = 0; l < lanes; ++l) t += red[l * cw + threadIdx.x];
            work[(int64_t)blockIdx.x * C + c0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- elementwise

__global__ void k_pool2(const uint16_t *__restrict__ x, int N, int H, int W, int C, uint16_t *__restrict__ out)
{
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n_out = (int64_t)N * Ho * Wo * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int xo = (int)(t % Wo);
        t /= Wo;
        const int yo = (int)(t % Ho);
        const int n = (int)(t / Ho);
        const int64_t b = (((int64_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
        const float s = bf2f(x[b]) + bf2f(x[b + C]) + bf2f(x[b + (int64_t)W * C]) + bf2f(x[b + (int64_t)W * C + C]);
        out[i] = f2bf(0.25f * s);
    }
}

__global__ void k_pool2_bwd(const float *__restrict__ dout, int N, int H, int W, int C, float *__restrict__ dx, int accum)
{
    const int64_t n_in = (int64_t)N * H * W * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int xx = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        const int n = (int)(t / H);
        const float g = 0.25f * dout[(((int64_t)n * (H / 2) + y / 2) * (W / 2) + xx / 2) * C + c];
        dx[i] = accum ? dx[i] + g : g;
    }
}

__global__ void k_up2(const uint16_t *__restrict__ x, int N, int H, int W, int C, uint16_t *__restrict__ out)
{
    const int Ho = 2 * H, Wo = 2 * W;
    const int64_t n_out = (int64_t)N * Ho * Wo * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int xo = (int)(t % Wo);
        t /= Wo;
        const int yo = (int)(t % Ho);
        const int n = (int)(t / Ho);
        out[i] = x[(((int64_t)n * H + yo / 2) * W + xo / 2) * C + c];
    }
}

__global__ void k_up2_bwd(const float *__restrict__ dout, int N, int H, int W, int C, float *__restrict__ dx)
{
    const int64_t n_in = (int64_t)N * H * W * C;
    const int Wo = 2 * W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        int64_t t = i / C;
        const int xx = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        const int n = (int)(t / H);
        const int64_t b = (((int64_t)n * 2 * H + 2 * y) * Wo + 2 * xx) * C + c;
        dx[i] = dout[b] + dout[b + C] + dout[b + (int64_t)Wo * C] + dout[b + (int64_t)Wo * C + C];
    }
}

__global__ void k_concat(const uint16_t *__restrict__ a, int ca, const uint16_t *__restrict__ b, int cb, int64_t npix,
                         uint16_t *__restrict__ out)
{
    const int C = ca + cb;
    const int64_t n = npix * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        out[i] = c < ca ? a[p * ca + c] : b[p * cb + (c - ca)];
    }
}

__global__ void k_split_bwd(const float *__restrict__ d, int ca, int cb, int64_t npix, float *__restrict__ da, int acc_a,
                            float *__restrict__ db, int acc_b)
{
    const int C = ca + cb;
    const int64_t n = npix * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        if (c < ca) {
            if (da) da[p * ca + c] = acc_a ? da[p * ca + c] + d[i] : d[i];
        } else {
            if (db) db[p * cb + c - ca] = acc_b ? db[p * cb + c - ca] + d[i] : d[i];
        }
    }
}

__global__ void k_silu_bwd(const float *__restrict__ da, const float *__restrict__ z, int64_t n, float *__restrict__ df,
                           uint16_t *__restrict__ db)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = da[i] * dsilu(z[i]);
        if (df) df[i] = g;
        if (db) db[i] = f2bf(g);
    }
}

// relative MSE: partial sums per (chunk, image) of (pred - t)^2 and t^2
__global__ __launch_bounds__(256) void k_relmse_partial(const float *__restrict__ pred, int C, const float *__restrict__ tg,
                                                        int64_t hw, float *__restrict__ work)
{
    const int img = blockIdx.y, nch = gridDim.x;
    const int64_t per = (hw + nch - 1) / nch;
    const int64_t b = (int64_t)blockIdx.x * per, e = std::min<int64_t>(b + per, hw);
    float sn = 0.0f, sd = 0.0f;
    for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
        const float t = tg[(int64_t)img * hw + k];
        const float r = pred[((int64_t)img * hw + k) * C] - t;
        sn += r * r;
        sd += t * t;
    }
    __shared__ float rn[256], rd[256];
    rn[threadIdx.x] = sn;
    rd[threadIdx.x] = sd;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            rn[threadIdx.x] += rn[threadIdx.x + s];
            rd[threadIdx.x] += rd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        work[((int64_t)img * nch + blockIdx.x) * 2] = rn[0];
        work[((int64_t)img * nch + blockIdx.x) * 2 + 1] = rd[0];
    }
}

// one thread: per-image sums in fixed order, loss, and per-image scale 2 / (nimg |t_i|^2)
__global__ void k_relmse_final(float *__restrict__ work, int nimg, int nch, float *__restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float L = 0.0f;
    for (int i = 0; i < nimg; ++i) {
        float sn = 0.0f, sd = 0.0f;
        for (int c = 0; c < nch; ++c) {
            sn += work[((int64_t)i * nch + c) * 2];
            sd += work[((int64_t)i * nch + c) * 2 + 1];
        }
        const float den = sd > 0.0f ? sd : 1.0f;
        L += sn / den;
        work[(int64_t)nimg * nch * 2 + i] = 2.0f / ((float)nimg * den);
    }
    if (loss) loss[0] = L / (float)nimg;
}

__global__ void k_relmse_grad(const float *__restrict__ pred, int C, const float *__restrict__ tg, int nimg, int64_t hw,
                              const float *__restrict__ scale, float *__restrict__ dpred, uint16_t *__restrict__ dpb)
{
    const int64_t n = (int64_t)nimg * hw * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t pk = i / C;
        const int img = (int)(pk / hw);
        const float g = c == 0 ? scale[img] * (pred[i] - tg[pk]) : 0.0f;
        dpred[i] = g;
        if (dpb) dpb[i] = f2bf(g);
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_pack(const float *__restrict__ wf, int Cout, int Cin, uint16_t *__restrict__ wb, uint16_t *__restrict__ wt)
{
    const int64_t n = (int64_t)Cout * 9 * Cin;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % Cin);
        const int64_t t = i / Cin;
        const int tap = (int)(t % 9);
        const int co = (int)(t / 9);
        const uint16_t h = f2bf(wf[i]);
        if (wb) wb[i] = h;
        if (wt) wt[((int64_t)ci * 9 + (8 - tap)) * Cout + co] = h;
    }
}

__global__ void k_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(x[i]);
}

// ------------------------------------------------------------------- host

// --------------------------------------------------- network input and guard

// Per-image RMS of g over its h x w cells, in FP64 with a fixed reduction order (one block
// per image): scale = sqrt(mean g^2), or 1 for an all-zero image.
__global__ __launch_bounds__(256) void k_prep_scale(const float *__restrict__ g, int64_t hw, float *__restrict__ scale)
{
    const float *gi = g + (int64_t)blockIdx.x * hw;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < hw; k += 256) {
        const double x = gi[k];
        s += x * x;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rms = sqrt(red[0] / (double)hw);
        scale[blockIdx.x] = rms > 0.0 ? (float)rms : 1.0f;
    }
}

// Network input of image i, rows padded from h to hp with zeros:
//   x[i][y][x][0] = bf16(g / scale_i), x[i][y][x][1] = bf16((v - v_shift) / v_scale),
//   channels 2..15 zero;  res[i][y][x] = g / scale_i (the residual added to the output).
__global__ void k_prep_write(const float *__restrict__ g, const float *__restrict__ v, int nimg, int h, int w, int hp,
                             float v_shift, float v_scale, const float *__restrict__ scale, uint16_t *__restrict__ x,
                             float *__restrict__ res)
{
    const int64_t per = (int64_t)hp * w, total = (int64_t)nimg * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = i / per, r = i % per;
        const int y = (int)(r / w), xx = (int)(r % w);
        float gn = 0.0f, vn = 0.0f;
        if (y < h) {
            const int64_t src = (img * h + y) * w + xx;
            gn = g[src] / scale[img];
            if (v) vn = (v[src] - v_shift) / v_scale;
        }
        if (res) res[i] = gn;
        if (x) {
            uint4 lo = make_uint4((uint32_t)f2bf(gn) | ((uint32_t)f2bf(vn) << 16), 0u, 0u, 0u);
            uint4 *o = reinterpret_cast<uint4 *>(x + i * 16);
            o[0] = lo;
            o[1] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
}

// Guard statistics of image i: p = pred[i][y][x][0] * scale_i over the h physical rows
// against the plain gradient g_i, in FP64 with a fixed reduction order; keeps the network
// output when cos(p, g) >= cos_min and |p| / |g| lies in [ratio_lo, ratio_hi].
__global__ __launch_bounds__(256) void k_guard_stats(const float *__restrict__ pred, int C,
                                                     const float *__restrict__ scale, const float *__restrict__ g,
                                                     int h, int w, int hp, float cos_min, float ratio_lo,
                                                     float ratio_hi, int32_t *__restrict__ keep)
{
    const int img = blockIdx.x;
    const int64_t hw = (int64_t)h * w;
    const double sc = scale[img];
    double spg = 0.0, spp = 0.0, sgg = 0.0;
    for (int64_t k = threadIdx.x; k < hw; k += 256) {
        const double p = sc * (double)pred[((int64_t)img * hp * w + k) * C];
        const double q = g[(int64_t)img * hw + k];
        spg += p * q;
        spp += p * p;
        sgg += q * q;
    }
    __shared__ double r0[256], r1[256], r2[256];
    r0[threadIdx.x] = spg;
    r1[threadIdx.x] = spp;
    r2[threadIdx.x] = sgg;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double pn = sqrt(r1[0]), gn = sqrt(r2[0]);
        const bool ok = pn > 0.0 && gn > 0.0 && r0[0] / (pn * gn) >= (double)cos_min && pn / gn >= (double)ratio_lo &&
                        pn / gn <= (double)ratio_hi;
        keep[img] = ok ? 1 : 0;
    }
}

// out[i][y][x] = keep_i ? pred[i][y][x][0] * scale_i : g[i][y][x]  (physical rows only).
__global__ void k_guard_write(const float *__restrict__ pred, int C, const float *__restrict__ scale,
                              const float *__restrict__ g, int nimg, int h, int w, int hp,
                              const int32_t *__restrict__ keep, float *__restrict__ out)
{
    const int64_t hw = (int64_t)h * w, total = (int64_t)nimg * hw;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = i / hw, k = i % hw;
        out[i] = keep[img] ? pred[((int64_t)img * hp * w + k) * C] * scale[img] : g[i];
    }
}

thread_local std::string g_nn_err;

fwi_status nn_fail(fwi_status s, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_nn_err = buf;
    return s;
}

#define NN_TRY(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return nn_fail(FWI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

bool shape_ok(const fwi_nn_shape &s) { return s.n > 0 && s.h > 0 && s.w > 0 && s.c > 0; }

int wgrad_chunks(const fwi_nn_shape &in, int cout)
{
    const int64_t P = (int64_t)in.n * in.h * in.w;
    const int64_t per_tile = (int64_t)cout * 9 * in.c;
    int64_t ch = std::max<int64_t>(1, P / 4096);
    ch = std::min<int64_t>(ch, 128);
    ch = std::min<int64_t>(ch, std::max<int64_t>(1, ((int64_t)64 << 20) / per_tile));
    return (int)ch;
}

}  // namespace

extern "C" {

fwi_status fwi_nn_conv3x3(const uint16_t *x, fwi_nn_shape in, const uint16_t *w, int32_t cout, const float *bias,
                          const float *aux, const float *res, int32_t act, float *out_f32, uint16_t *out_bf16,
                          void *stream)
{
    if (!x || !w || !shape_ok(in) || in.c % 16 || cout <= 0 || cout % 32)
        return nn_fail(FWI_E_ARG, "conv3x3: need input channels %% 16 == 0 and output channels %% 32 == 0");
    if (!out_f32 && !out_bf16) return nn_fail(FWI_E_ARG, "conv3x3: no output");
    const int64_t P = (int64_t)in.n * in.h * in.w;
    hipStream_t st = (hipStream_t)stream;
    // 64 x 64 wavefront tiles where the output channels allow it and the grid stays large
    if (cout % 64 == 0 && P >= 64 * 1024) {
        dim3 grid((unsigned)((P + 127) / 128), (unsigned)((cout + 127) / 128));
        k_conv3x3<2, 2><<<grid, 256, 0, st>>>(x, in.n, in.h, in.w, in.c, w, cout, bias, aux, res, act, out_f32, out_bf16);
    } else if (P >= 64 * 1024) {
        dim3 grid((unsigned)((P + 127) / 128), (unsigned)((cout + 63) / 64));
        k_conv3x3<2, 1><<<grid, 256, 0, st>>>(x, in.n, in.h, in.w, in.c, w, cout, bias, aux, res, act, out_f32, out_bf16);
    } else {
        dim3 grid((unsigned)((P + 63) / 64), (unsigned)((cout + 63) / 64));
        k_conv3x3<1, 1><<<grid, 256, 0, st>>>(x, in.n, in.h, in.w, in.c, w, cout, bias, aux, res, act, out_f32, out_bf16);
    }
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

int64_t fwi_nn_wgrad_work(fwi_nn_shape in, int32_t cout)
{
    if (!shape_ok(in) || cout <= 0) return 0;
    return (int64_t)wgrad_chunks(in, cout) * cout * 9 * in.c + (int64_t)std::max<int64_t>(1, ((int64_t)in.n * in.h * in.w + 4095) / 4096) * cout;
}

fwi_status fwi_nn_wgrad(const uint16_t *dz, const float *dz_f32, const uint16_t *x, fwi_nn_shape in, int32_t cout,
                        float *dw, float *db, float *work, void *stream)
{
    if (!dz || !x || !dw || !work || !shape_ok(in) || in.c % 16 || cout % 32 || (db && !dz_f32))
        return nn_fail(FWI_E_ARG, "wgrad: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int64_t P = (int64_t)in.n * in.h * in.w;
    const int nch = wgrad_chunks(in, cout);
    const int64_t per = (P + nch - 1) / nch;
    const int nci = (in.c + 31) / 32;
    dim3 grid((unsigned)((cout / 32) * nci), (unsigned)nch);
    k_wgrad<<<grid, 64, 0, st>>>(dz, x, in.n, in.h, in.w, in.c, cout, per, work);
    NN_TRY(hipGetLastError());
    const int64_t nw = (int64_t)cout * 9 * in.c;
    k_sum_chunks<<<grid_for(nw), 256, 0, st>>>(work, nch, nw, dw);
    NN_TRY(hipGetLastError());
    if (db) {
        const int bch = (int)std::max<int64_t>(1, (P + 4095) / 4096);
        float *bw = work + (int64_t)nch * nw;
        k_bias_partial<<<bch, 256, 0, st>>>(dz_f32, P, cout, (P + bch - 1) / bch, bw);
        NN_TRY(hipGetLastError());
        k_sum_chunks<<<grid_for(cout), 256, 0, st>>>(bw, bch, cout, db);
        NN_TRY(hipGetLastError());
    }
    return FWI_OK;
}

fwi_status fwi_nn_pool2(const uint16_t *x, fwi_nn_shape in, uint16_t *out, void *stream)
{
    if (!x || !out || !shape_ok(in) || in.h % 2 || in.w % 2) return nn_fail(FWI_E_ARG, "pool2: bad shape");
    k_pool2<<<grid_for((int64_t)in.n * in.h * in.w * in.c / 4), 256, 0, (hipStream_t)stream>>>(x, in.n, in.h, in.w,
                                                                                                in.c, out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_pool2_bwd(const float *dout, fwi_nn_shape in, float *dx, int32_t accumulate, void *stream)
{
    if (!dout || !dx || !shape_ok(in) || in.h % 2 || in.w % 2) return nn_fail(FWI_E_ARG, "pool2_bwd: bad shape");
    k_pool2_bwd<<<grid_for((int64_t)in.n * in.h * in.w * in.c), 256, 0, (hipStream_t)stream>>>(dout, in.n, in.h, in.w,
                                                                                                in.c, dx, accumulate);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_up2(const uint16_t *x, fwi_nn_shape in, uint16_t *out, void *stream)
{
    if (!x || !out || !shape_ok(in)) return nn_fail(FWI_E_ARG, "up2: bad shape");
    k_up2<<<grid_for((int64_t)in.n * in.h * in.w * in.c * 4), 256, 0, (hipStream_t)stream>>>(x, in.n, in.h, in.w, in.c,
                                                                                              out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_up2_bwd(const float *dout, fwi_nn_shape in, float *dx, void *stream)
{
    if (!dout || !dx || !shape_ok(in)) return nn_fail(FWI_E_ARG, "up2_bwd: bad shape");
    k_up2_bwd<<<grid_for((int64_t)in.n * in.h * in.w * in.c), 256, 0, (hipStream_t)stream>>>(dout, in.n, in.h, in.w,
                                                                                              in.c, dx);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_concat(const uint16_t *a, int32_t ca, const uint16_t *b, int32_t cb, int64_t npix, uint16_t *out,
                         void *stream)
{
    if (!a || !b || !out || ca <= 0 || cb <= 0 || npix <= 0) return nn_fail(FWI_E_ARG, "concat: bad arguments");
    k_concat<<<grid_for(npix * (ca + cb)), 256, 0, (hipStream_t)stream>>>(a, ca, b, cb, npix, out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_split_bwd(const float *d, int32_t ca, int32_t cb, int64_t npix, float *da, int32_t acc_a, float *db,
                            int32_t acc_b, void *stream)
{
    if (!d || ca <= 0 || cb <= 0 || npix <= 0) return nn_fail(FWI_E_ARG, "split_bwd: bad arguments");
    k_split_bwd<<<grid_for(npix * (ca + cb)), 256, 0, (hipStream_t)stream>>>(d, ca, cb, npix, da, acc_a, db, acc_b);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_silu_bwd(const float *da, const float *z, int64_t n, float *dz_f32, uint16_t *dz_bf16, void *stream)
{
    if (!da || !z || n <= 0) return nn_fail(FWI_E_ARG, "silu_bwd: bad arguments");
    k_silu_bwd<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(da, z, n, dz_f32, dz_bf16);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_rel_mse(const float *pred, int32_t c, const float *target, int32_t nimg, int64_t hw, float *loss,
                          float *dpred, uint16_t *dpred_bf16, float *work, void *stream)
{
    if (!pred || !target || !work || c <= 0 || nimg <= 0 || nimg > 65535 || hw <= 0)
        return nn_fail(FWI_E_ARG, "rel_mse: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int nch = 64;
    k_relmse_partial<<<dim3(nch, nimg), 256, 0, st>>>(pred, c, target, hw, work);
    NN_TRY(hipGetLastError());
    k_relmse_final<<<1, 64, 0, st>>>(work, nimg, nch, loss);
    NN_TRY(hipGetLastError());
    if (dpred) {
        k_relmse_grad<<<grid_for((int64_t)nimg * hw * c), 256, 0, st>>>(pred, c, target, nimg, hw,
                                                                         work + (int64_t)nimg * nch * 2, dpred,
                                                                         dpred_bf16);
        NN_TRY(hipGetLastError());
    }
    return FWI_OK;
}

fwi_status fwi_nn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                       int32_t t, void *stream)
{
    if (!p || !g || !m || !v || n <= 0 || t < 1) return nn_fail(FWI_E_ARG, "adam: bad arguments");
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    k_adam<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_pack_weights(const float *wf, int32_t cout, int32_t cin, uint16_t *w_bf16, uint16_t *wt_bf16,
                               void *stream)
{
    if (!wf || cout <= 0 || cin <= 0) return nn_fail(FWI_E_ARG, "pack_weights: bad arguments");
    k_pack<<<grid_for((int64_t)cout * 9 * cin), 256, 0, (hipStream_t)stream>>>(wf, cout, cin, w_bf16, wt_bf16);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_to_bf16(const float *x, int64_t n, uint16_t *out, void *stream)
{
    if (!x || !out || n <= 0) return nn_fail(FWI_E_ARG, "to_bf16: bad arguments");
    k_to_bf16<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(x, n, out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_prep(const float *g, const float *v, int32_t nimg, int32_t h, int32_t w, int32_t hp,
                       float v_shift, float v_scale, const float *scale_in, float *scale_out, uint16_t *x_bf16,
                       float *res, void *stream)
{
    if (!g || nimg < 1 || h < 1 || w < 1 || hp < h) return nn_fail(FWI_E_ARG, "prep: bad shape");
    if (!scale_in && !scale_out) return nn_fail(FWI_E_ARG, "prep: need scale_in or scale_out");
    if (!x_bf16 && !res) return nn_fail(FWI_E_ARG, "prep: no output");
    if (x_bf16 && (!v || !(v_scale != 0.0f))) return nn_fail(FWI_E_ARG, "prep: the network input needs v and v_scale != 0");
    if ((uintptr_t)x_bf16 % 16) return nn_fail(FWI_E_ARG, "prep: x_bf16 must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const float *scale = scale_in;
    if (!scale_in) {
        k_prep_scale<<<nimg, 256, 0, st>>>(g, (int64_t)h * w, scale_out);
        NN_TRY(hipGetLastError());
        scale = scale_out;
    } else if (scale_out) {
        NN_TRY(hipMemcpyAsync(scale_out, scale_in, sizeof(float) * nimg, hipMemcpyDeviceToDevice, st));
    }
    const int64_t n = (int64_t)nimg * hp * w;
    k_prep_write<<<grid_for(n), 256, 0, st>>>(g, v, nimg, h, w, hp, v_shift, v_scale, scale, x_bf16, res);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_guard(const float *pred, int32_t c, const float *scale, const float *g, int32_t nimg, int32_t h,
                        int32_t w, int32_t hp, float cos_min, float ratio_lo, float ratio_hi, float *out,
                        int32_t *keep, void *stream)
{
    if (!pred || !scale || !g || !out || !keep || c < 1 || nimg < 1 || h < 1 || w < 1 || hp < h)
        return nn_fail(FWI_E_ARG, "guard: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    k_guard_stats<<<nimg, 256, 0, st>>>(pred, c, scale, g, h, w, hp, cos_min, ratio_lo, ratio_hi, keep);
    NN_TRY(hipGetLastError());
    const int64_t n = (int64_t)nimg * h * w;
    k_guard_write<<<grid_for(n), 256, 0, st>>>(pred, c, scale, g, nimg, h, w, hp, keep, out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

const char *fwi_nn_last_error(void) { return g_nn_err.c_str(); }

}  // extern "C"
