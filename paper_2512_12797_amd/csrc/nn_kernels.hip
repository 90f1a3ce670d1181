// nn_kernels.hip -- gfx950 kernels of the learned gradient preconditioner (include/fwi_nn.h).
//
// 3x3 convolutions are implicit GEMMs on the BF16 matrix cores (output channels x pixels,
// K = 9 taps x input channels), their weight gradients GEMMs over pixels (input x output
// channels per tap), one v_mfma_f32_32x32x16_bf16 per 16-wide K step.  Operand lane layout
// of that instruction (checked on the hardware): A lane l holds row l%32, k = 8*(l/32) ..
// +7; B lane l holds column l%32, the same k; accumulator register r holds row
// 8*(r/4) + 4*(l/32) + r%4, column l%32.  Activations are NHWC, weights [Cout][9][Cin]; the
// operand tiles are staged in LDS (see each kernel) and read as one 16-byte load per lane.
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
// The same with the hardware exponential and reciprocal (about 2 ulp), for the convolution epilogue where they run
// on every output element; exp(-z) overflowing to infinity gives sigmoid 0 as it should.
__device__ __forceinline__ float sigmoid_hw(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_hw(float z) { return z * sigmoid_hw(z); }
__device__ __forceinline__ float dsilu_hw(float z)
{
    const float s = sigmoid_hw(z);
    return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------------ conv3x3

// Hardware dispatches workgroup b to XCD b % 8 (each XCD has its own L2): give every XCD a contiguous range of tiles so
// that neighbouring tiles, which share halo rows, are fetched into the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) { return nb % 8 ? b : (b % 8) * (nb / 8) + b / 8; }

// Workgroup output tile: TY image rows x 32 columns of one image x CO_T output channels; 4 wavefronts, WM along the
// rows x 4/WM along the channels, each MT rows x NT groups of 32 channels.  The K loop runs over the input channels
// in chunks of CK (16 or 32).  Per chunk, LDS holds the (TY+2) x 34 input patch (halo included, zeros outside the
// image) as CK/8 planes of 8 channels and the chunk's weights of all 9 taps; each tap is CK/16 MFMA k-steps whose
// pixel operand is read from the patch shifted by the tap.  A = weights (rows = output channels), B = pixels (columns): accumulator
// register r of a lane then holds output channel 8(r/4) + 4(lane/32) + r%4 of pixel lane%32, so the epilogue reads
// and writes 4 consecutive channels per lane.  The next chunk's global loads are in flight during the current
// chunk's matrix operations.
// With cu > 0 the input is the channel concatenation [up(xu), x] without materialising it: channels [0, cu) come from
// xu at half resolution (nearest 2x upsampling: pixel (y, x) reads xu(y/2, x/2)), channels [cu, Cin) from x, which
// then has Cin - cu channels per pixel.
template <int TY, int CO_T, int WM, int CK>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t *__restrict__ x, int N, int H, int W, int Cin,
                                                 const uint16_t *__restrict__ w, int Cout,
                                                 const float *__restrict__ bias, const float *__restrict__ aux,
                                                 const float *__restrict__ res, int act, float *__restrict__ of32,
                                                 uint16_t *__restrict__ obf, const uint16_t *__restrict__ xu, int cu)
{
    constexpr int WN = 4 / WM, MT = TY / WM, NT = CO_T / 32 / WN;
    static_assert(WM * WN == 4 && MT * WM == TY && NT * WN * 32 == CO_T, "tile shape");
    constexpr int PC = 34, PPL = (TY + 2) * PC;            // patch columns, pixels per plane
    constexpr int NH = CK / 8, NP = NH * PPL, NWT = 9 * NH * CO_T;  // planes; 16-byte pieces: patch, weights
    constexpr int RP = (NP + 255) / 256, RW = (NWT + 255) / 256;
    __shared__ uint4 sp[NP];
    __shared__ uint4 sw[NWT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l32 = lane & 31, hl = lane >> 5;
    const int wm = wave % WM, wn = wave / WM;
    const int nseg = (W + 31) >> 5, nrt = (H + TY - 1) / TY;
    const int bt = xcd_tile(blockIdx.x, gridDim.x);
    const int seg = bt % nseg, rt = (bt / nseg) % nrt, n = bt / (nseg * nrt);
    const int y0 = rt * TY, x0 = seg * 32, cb = blockIdx.y * CO_T;

    // loader roles: patch piece q = tid + 256 i is 8-channel group q % NH of patch pixel q / NH (a pixel's groups
    // are adjacent in memory); weight piece q is group q % NH of tap (q / NH) % 9 of output channel (q / NH) / 9
    // piece offsets within this image (the host keeps an image of either input below 2^31 elements)
    const int cx = Cin - cu;  // channels per pixel of x
    const uint16_t *ximg = x + (int64_t)n * H * W * cx;
    const uint16_t *uimg = cu > 0 ? xu + (int64_t)n * (H >> 1) * (W >> 1) * cu : xu;
    int poff[RP], uoff[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) {
        const int q = tid + 256 * i, pix = q / NH, h = q % NH;
        const int pr = pix / PC, pc = pix - pr * PC;
        const int yy = y0 - 1 + pr, xx = x0 - 1 + pc;
        const bool v = q < NP && yy >= 0 && yy < H && xx >= 0 && xx < W;
        poff[i] = v ? (yy * W + xx) * cx + 8 * h : -1;
        uoff[i] = v && cu > 0 ? ((yy >> 1) * (W >> 1) + (xx >> 1)) * cu + 8 * h : -1;
    }
    uint4 rp[RP], rw[RW];
    auto gload = [&](int c0) {
        const bool up = c0 < cu;  // uniform: cu is a multiple of the chunk width CK
        const uint16_t *src = up ? uimg + c0 : ximg + (c0 - cu);
#pragma unroll
        for (int i = 0; i < RP; ++i) {
            const int o = up ? uoff[i] : poff[i];
            rp[i] = make_uint4(0u, 0u, 0u, 0u);
            if (o >= 0) rp[i] = *(const uint4 *)(src + o);
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int q = tid + 256 * i, t = q / NH;
            rw[i] = make_uint4(0u, 0u, 0u, 0u);
            if (q < NWT) rw[i] = *(const uint4 *)(w + ((int64_t)(cb + t / 9) * 9 + t % 9) * Cin + c0 + 8 * (q % NH));
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < RP; ++i) {
            const int q = tid + 256 * i;
            if (q < NP) sp[(q % NH) * PPL + q / NH] = rp[i];
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int q = tid + 256 * i, t = q / NH;
            if (q < NWT) sw[((t % 9) * NH + q % NH) * CO_T + t / 9] = rw[i];
        }
    };
    f32x16 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x16{};
    gload(0);
    const int nck = Cin / CK;
    for (int ck = 0; ck < nck; ++ck) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (ck + 1 < nck) gload(CK * (ck + 1));
        // k-steps in the order of 16-channel chunks (all taps of channels 0-15, then of 16-31): the accumulation
        // order, and so every result bit, does not depend on CK
#pragma unroll
        for (int kk = 0; kk < CK / 16; ++kk) {  // k-step: planes 2 kk (lanes 0-31) and 2 kk + 1 (lanes 32-63)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;
                const int h = 2 * kk + hl;
                bf16x8 a[NT], b[MT];
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    a[j] = __builtin_bit_cast(bf16x8, sw[(tap * NH + h) * CO_T + (wn * NT + j) * 32 + l32]);
#pragma unroll
                for (int i = 0; i < MT; ++i)
                    b[i] = __builtin_bit_cast(bf16x8, sp[h * PPL + (wm * MT + i + dy) * PC + l32 + dx]);
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], b[i], acc[i][j], 0, 0, 0);
            }
        }
    }
    const int xx = x0 + l32;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int y = y0 + wm * MT + i;
        if (y >= H || xx >= W) continue;
        const int64_t p = ((int64_t)n * H + y) * W + xx;
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int c = cb + (wn * NT + j) * 32 + 8 * g + 4 * hl;
                const int64_t o = p * Cout + c;
                float v[4] = {acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]};
                if (bias) {
                    const float4 bb = *(const float4 *)(bias + c);
                    v[0] += bb.x, v[1] += bb.y, v[2] += bb.z, v[3] += bb.w;
                }
                if (aux) {
                    const float4 z = *(const float4 *)(aux + o);
                    v[0] *= dsilu_hw(z.x), v[1] *= dsilu_hw(z.y), v[2] *= dsilu_hw(z.z), v[3] *= dsilu_hw(z.w);
                }
                if (res && c == 0) v[0] += res[p];
                if (of32) *(float4 *)(of32 + o) = make_float4(v[0], v[1], v[2], v[3]);
                if (obf) {
                    uint16_t h4[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) h4[e] = f2bf(act ? silu_hw(v[e]) : v[e]);
                    *(uint2 *)(obf + o) = make_uint2((uint32_t)h4[0] | ((uint32_t)h4[1] << 16),
                                                     (uint32_t)h4[2] | ((uint32_t)h4[3] << 16));
                }
            }
    }
}

// ------------------------------------------------------------------- wgrad

// Weight-gradient partials over a chunk of pixel tiles (TY rows x 32 columns of one image), one workgroup per
// (32 output channels, 32 input channels, chunk):  M = input channels, N = output channels, K = pixels, one
// accumulator per tap.  Per tile, LDS holds dz transposed to [co][row][32 columns] and the input patch (TY+2 rows,
// halo included) transposed to [ci][row][40 columns], so that 8 consecutive pixels of one channel are one 16-byte
// read; the transposition is done while storing (pairs of pixels packed into 32-bit words).  The column shift of a
// tap comes from one aligned 16-byte + 4-byte read per patch row: shift 0 is the 16 bytes, shift 2 drops the first
// word and appends the extra one, shift 1 is the funnel shift by 16 bits of consecutive words.  Channel pitches are
// odd multiples of 16 bytes so that the 32 rows of an operand read fall in distinct banks.  Three wavefronts, one
// per tap row dy, each with the accumulators of its 3 taps: no reduction between wavefronts, and few enough
// registers for several workgroups per compute unit to hide the tile loads.
// The input may be the concatenation [up(xu), x] as in k_conv3x3 (cu > 0).
template <int TY>
__global__ __launch_bounds__(192) void k_wgrad(const uint16_t *__restrict__ dz, const uint16_t *__restrict__ x,
                                               int N, int H, int W, int Cin, int Cout, int ntiles, int per_chunk,
                                               float *__restrict__ work, const uint16_t *__restrict__ xu, int cu)
{
    constexpr int NTH = 192, PR = TY + 2;
    constexpr int DZP = TY * 32 + 8;                                    // elements per output channel
    constexpr int XRP = 40;                                             // elements per patch row
    constexpr int XP = PR * XRP + (((PR * XRP / 8) % 2) == 0 ? 8 : 0);  // elements per input channel
    constexpr int NDZ = TY * 64;                                        // dz items: (row, pixel pair, 8 channels)
    constexpr int NX = PR * 17 * 4;                                     // patch items: (row, column pair, 8 channels)
    constexpr int RD = (NDZ + NTH - 1) / NTH, RX = (NX + NTH - 1) / NTH;
    __shared__ __align__(16) uint16_t sdz[32 * DZP];
    __shared__ __align__(16) uint16_t sx[32 * XP];
    const int tid = threadIdx.x, dy = tid >> 6, lane = tid & 63, l32 = lane & 31, hl = lane >> 5;
    const int nci = (Cin + 31) >> 5;
    const int cit = blockIdx.x % nci, cot = blockIdx.x / nci;
    const int ci0 = cit * 32, cb = cot * 32;
    const int nseg = (W + 31) >> 5, nrt = (H + TY - 1) / TY;
    const int t_beg = blockIdx.y * per_chunk, t_end = std::min(t_beg + per_chunk, ntiles);

    uint4 rd[RD][2], rx[RX][2];
    auto gload = [&](int t) {
        const int seg = t % nseg, rt = (t / nseg) % nrt, n = t / (nseg * nrt);
        const int y0 = rt * TY, x0 = seg * 32;
#pragma unroll
        for (int i = 0; i < RD; ++i) {
            const int q = tid + NTH * i, g8 = q & 3, pp = (q >> 2) & 15, r = q >> 6;
            const int y = y0 + r, xa = x0 + 2 * pp;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                rd[i][e] = make_uint4(0u, 0u, 0u, 0u);
                if (q < NDZ && y < H && xa + e < W)
                    rd[i][e] = *(const uint4 *)(dz + (((int64_t)n * H + y) * W + xa + e) * Cout + cb + 8 * g8);
            }
        }
#pragma unroll
        for (int i = 0; i < RX; ++i) {
            const int q = tid + NTH * i, g8 = q & 3, rest = q >> 2;
            const int cp = rest % 17, pr = rest / 17;
            const int y = y0 - 1 + pr, xa = x0 - 1 + 2 * cp;
            const int ci = ci0 + 8 * g8;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int xe = xa + e;
                rx[i][e] = make_uint4(0u, 0u, 0u, 0u);
                if (q < NX && y >= 0 && y < H && xe >= 0 && xe < W && ci < Cin)
                    rx[i][e] = ci < cu ? *(const uint4 *)(xu + (((int64_t)n * (H >> 1) + (y >> 1)) * (W >> 1) + (xe >> 1)) * cu + ci)
                                       : *(const uint4 *)(x + (((int64_t)n * H + y) * W + xe) * (Cin - cu) + ci - cu);
            }
        }
    };
    // 8 channels of two adjacent pixels -> 8 words (pixel pair) at the channels' rows
    auto put8 = [](uint16_t *dst, int pitch, const uint4 &a, const uint4 &b) {
        const uint32_t av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            *(uint32_t *)(dst + (2 * k) * pitch) = (av[k] & 0xffffu) | (bv[k] << 16);
            *(uint32_t *)(dst + (2 * k + 1) * pitch) = (av[k] >> 16) | (bv[k] & 0xffff0000u);
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < RD; ++i) {
            const int q = tid + NTH * i, g8 = q & 3, pp = (q >> 2) & 15, r = q >> 6;
            if (q < NDZ) put8(sdz + (8 * g8) * DZP + r * 32 + 2 * pp, DZP, rd[i][0], rd[i][1]);
        }
#pragma unroll
        for (int i = 0; i < RX; ++i) {
            const int q = tid + NTH * i, g8 = q & 3, rest = q >> 2;
            const int cp = rest % 17, pr = rest / 17;
            if (q < NX) put8(sx + (8 * g8) * XP + pr * XRP + 2 * cp, XP, rx[i][0], rx[i][1]);
        }
    };
    f32x16 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = f32x16{};
    if (t_beg < t_end) gload(t_beg);
    for (int t = t_beg; t < t_end; ++t) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (t + 1 < t_end) gload(t + 1);
#pragma unroll
        for (int ks = 0; ks < 2 * TY; ++ks) {  // k-step: row ks / 2, 16-column half ks % 2
            const int r = ks >> 1, g = 2 * (ks & 1) + hl;
            const bf16x8 b = __builtin_bit_cast(bf16x8, *(const uint4 *)(sdz + l32 * DZP + r * 32 + 8 * g));
            const uint16_t *src = sx + l32 * XP + (r + dy) * XRP + 8 * g;
            const uint4 d = *(const uint4 *)src;
            const uint32_t e4 = *(const uint32_t *)(src + 8);
            const uint4 s1 = make_uint4(__builtin_amdgcn_alignbit(d.y, d.x, 16), __builtin_amdgcn_alignbit(d.z, d.y, 16),
                                        __builtin_amdgcn_alignbit(d.w, d.z, 16), __builtin_amdgcn_alignbit(e4, d.w, 16));
            const uint4 s2 = make_uint4(d.y, d.z, d.w, e4);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, d), b, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, s1), b, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, s2), b, acc[2], 0, 0, 0);
        }
    }
    // acc[dx][r]: row (input channel) ci0 + 8(r/4) + 4(lane/32) + r%4, column (output channel) cb + lane%32
    float *wk = work + (int64_t)blockIdx.y * Cout * 9 * Cin;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int ci = ci0 + 8 * g + 4 * hl;
            if (ci < Cin)
                *(float4 *)(wk + ((int64_t)(cb + l32) * 9 + 3 * dy + dx) * Cin + ci) =
                    make_float4(acc[dx][4 * g], acc[dx][4 * g + 1], acc[dx][4 * g + 2], acc[dx][4 * g + 3]);
        }
}

// Column sums over groups of 32 rows of a [rows][n] matrix: out[g][i] = sum of m[r][i], r in [32 g, 32 g + 32)
// (rows in increasing order; deterministic).
__global__ void k_sum_rows32(const float *__restrict__ m, int rows, int64_t n, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r0 = 32 * blockIdx.y, r1 = std::min(r0 + 32, rows);
    float s = 0.0f;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) s += m[(int64_t)r * n + i];
    out[(int64_t)blockIdx.y * n + i] = s;
}

// db partials: workgroup = chunk of `per_chunk` pixels and channels [256 y, 256 y + cw), cw = min(256, C - 256 y);
// thread t sums channel t % cw over the pixels pb + t / cw, stepping by 256 / cw (coalesced rows).  Partials of the
// pixel lanes are added in a fixed order.
__global__ __launch_bounds__(256) void k_bias_partial(const float *__restrict__ dz, int64_t P, int C, int64_t per_chunk,
                                                      float *__restrict__ work)
{
    __shared__ float red[256];
    const int c0 = 256 * blockIdx.y, cw = std::min(256, C - c0), lanes = 256 / cw;
    const int c = threadIdx.x % cw, pl = threadIdx.x / cw;
    const int64_t pb = (int64_t)blockIdx.x * per_chunk, pe = std::min<int64_t>(pb + per_chunk, P);
    float s = 0.0f;
    if (pl < lanes) {
#pragma unroll 4
        for (int64_t p = pb + pl; p < pe; p += lanes) s += dz[p * C + c0 + c];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < cw) {
        float t = 0.0f;
        for (int l = 0; l < lanes; ++l) t += red[l * cw + threadIdx.x];
        work[(int64_t)blockIdx.x * C + c0 + threadIdx.x] = t;
    }
}

// db[c] = sum over the nchunk partials of channel c: one workgroup per channel, strided partial sums per thread,
// then a fixed LDS tree.
__global__ __launch_bounds__(256) void k_bias_final(const float *__restrict__ work, int nchunk, int C,
                                                    float *__restrict__ db)
{
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int k = threadIdx.x; k < nchunk; k += 256) s += work[(int64_t)k * C + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
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

// Vector forms of the elementwise kernels above for channel counts that are multiples of 4 (8 for BF16 pooling) and
// 16-byte aligned tensors: one thread per 4 channels (16-byte loads and stores), the same arithmetic per element.
__global__ void k_pool2_v8(const uint16_t *__restrict__ x, int N, int H, int W, int C, uint16_t *__restrict__ out)
{
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const int64_t n_out = (int64_t)N * Ho * Wo * C8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C8) * 8;
        int64_t t = i / C8;
        const int xo = (int)(t % Wo);
        t /= Wo;
        const int yo = (int)(t % Ho);
        const int n = (int)(t / Ho);
        const int64_t b = (((int64_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
        const uint4 q[4] = {*(const uint4 *)(x + b), *(const uint4 *)(x + b + C), *(const uint4 *)(x + b + (int64_t)W * C),
                            *(const uint4 *)(x + b + (int64_t)W * C + C)};
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t w0 = (&q[0].x)[k], w1 = (&q[1].x)[k], w2 = (&q[2].x)[k], w3 = (&q[3].x)[k];
            const float lo = bf2f(w0 & 0xffffu) + bf2f(w1 & 0xffffu) + bf2f(w2 & 0xffffu) + bf2f(w3 & 0xffffu);
            const float hi = bf2f(w0 >> 16) + bf2f(w1 >> 16) + bf2f(w2 >> 16) + bf2f(w3 >> 16);
            o[k] = (uint32_t)f2bf(0.25f * lo) | ((uint32_t)f2bf(0.25f * hi) << 16);
        }
        *(uint4 *)(out + i * 8) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

__global__ void k_pool2_bwd_v4(const float *__restrict__ dout, int N, int H, int W, int C, float *__restrict__ dx,
                               int accum)
{
    const int C4 = C / 4;
    const int64_t n_in = (int64_t)N * H * W * C4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C4) * 4;
        int64_t t = i / C4;
        const int xx = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        const int n = (int)(t / H);
        float4 g = *(const float4 *)(dout + (((int64_t)n * (H / 2) + y / 2) * (W / 2) + xx / 2) * C + c);
        g.x *= 0.25f, g.y *= 0.25f, g.z *= 0.25f, g.w *= 0.25f;
        float4 *d = (float4 *)(dx + i * 4);
        if (accum) {
            const float4 o = *d;
            g.x = o.x + g.x, g.y = o.y + g.y, g.z = o.z + g.z, g.w = o.w + g.w;
        }
        *d = g;
    }
}

__global__ void k_up2_bwd_v4(const float *__restrict__ dout, int N, int H, int W, int C, float *__restrict__ dx)
{
    const int C4 = C / 4, Wo = 2 * W;
    const int64_t n_in = (int64_t)N * H * W * C4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C4) * 4;
        int64_t t = i / C4;
        const int xx = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        const int n = (int)(t / H);
        const int64_t b = (((int64_t)n * 2 * H + 2 * y) * Wo + 2 * xx) * C + c;
        const float4 p0 = *(const float4 *)(dout + b), p1 = *(const float4 *)(dout + b + C);
        const float4 p2 = *(const float4 *)(dout + b + (int64_t)Wo * C), p3 = *(const float4 *)(dout + b + (int64_t)Wo * C + C);
        *(float4 *)(dx + i * 4) = make_float4(p0.x + p1.x + p2.x + p3.x, p0.y + p1.y + p2.y + p3.y,
                                              p0.z + p1.z + p2.z + p3.z, p0.w + p1.w + p2.w + p3.w);
    }
}

__global__ void k_split_bwd_v4(const float *__restrict__ d, int ca, int cb, int64_t npix, float *__restrict__ da,
                               int acc_a, float *__restrict__ db, int acc_b)
{
    const int C4 = (ca + cb) / 4;
    const int64_t n = npix * C4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C4) * 4;
        const int64_t p = i / C4;
        const float4 v = *(const float4 *)(d + i * 4);
        float *dst = c < ca ? (da ? da + p * ca + c : nullptr) : (db ? db + p * cb + c - ca : nullptr);
        if (!dst) continue;
        float4 r = v;
        if (c < ca ? acc_a : acc_b) {
            const float4 o = *(const float4 *)dst;
            r = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
        }
        *(float4 *)dst = r;
    }
}

__global__ void k_silu_bwd_v4(const float *__restrict__ da, const float *__restrict__ z, int64_t n4,
                              float *__restrict__ df, uint16_t *__restrict__ db)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 a = *(const float4 *)(da + i * 4), zz = *(const float4 *)(z + i * 4);
        const float4 g = make_float4(a.x * dsilu(zz.x), a.y * dsilu(zz.y), a.z * dsilu(zz.z), a.w * dsilu(zz.w));
        if (df) *(float4 *)(df + i * 4) = g;
        if (db)
            *(uint2 *)(db + i * 4) = make_uint2((uint32_t)f2bf(g.x) | ((uint32_t)f2bf(g.y) << 16),
                                                (uint32_t)f2bf(g.z) | ((uint32_t)f2bf(g.w) << 16));
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

// One workgroup: per-image sums in fixed order (a thread per image), the per-image scale 2 / (nimg |t_i|^2) and
// relative error into work, then the loss summed in image order by thread 0.
__global__ __launch_bounds__(256) void k_relmse_final(float *__restrict__ work, int nimg, int nch, float *__restrict__ loss)
{
    float *scale = work + (int64_t)nimg * nch * 2, *li = scale + nimg;
    for (int i = threadIdx.x; i < nimg; i += blockDim.x) {
        float sn = 0.0f, sd = 0.0f;
        for (int c = 0; c < nch; ++c) {
            sn += work[((int64_t)i * nch + c) * 2];
            sd += work[((int64_t)i * nch + c) * 2 + 1];
        }
        const float den = sd > 0.0f ? sd : 1.0f;
        li[i] = sn / den;
        scale[i] = 2.0f / ((float)nimg * den);
    }
    __syncthreads();
    if (threadIdx.x == 0 && loss) {
        float L = 0.0f;
        for (int i = 0; i < nimg; ++i) L += li[i];
        loss[0] = L / (float)nimg;
    }
}

// dL/dpred with 4 channels per thread (c % 4 == 0): only channel 0 is nonzero.
__global__ void k_relmse_grad_v4(const float *__restrict__ pred, int C, const float *__restrict__ tg, int nimg,
                                 int64_t hw, const float *__restrict__ scale, float *__restrict__ dpred,
                                 uint16_t *__restrict__ dpb)
{
    const int C4 = C / 4;
    const int64_t n = (int64_t)nimg * hw * C4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pk = i / C4;
        const int img = (int)(pk / hw);
        const float g = i % C4 == 0 ? scale[img] * (pred[pk * C] - tg[pk]) : 0.0f;
        *(float4 *)(dpred + i * 4) = make_float4(g, 0.0f, 0.0f, 0.0f);
        if (dpb) *(uint2 *)(dpb + i * 4) = make_uint2((uint32_t)f2bf(g), 0u);
    }
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
    // fixed-order sums: cross-lane folds within each wavefront, then the four wavefront
    // sums in wave order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        spg += __shfl_down(spg, o, 64);
        spp += __shfl_down(spp, o, 64);
        sgg += __shfl_down(sgg, o, 64);
    }
    __shared__ double part[3][4];
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = spg;
        part[1][threadIdx.x >> 6] = spp;
        part[2][threadIdx.x >> 6] = sgg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[3];
        for (int k = 0; k < 3; ++k) r[k] = ((part[k][0] + part[k][1]) + part[k][2]) + part[k][3];
        const double pn = sqrt(r[1]), gn = sqrt(r[2]);
        const bool ok = pn > 0.0 && gn > 0.0 && r[0] / (pn * gn) >= (double)cos_min && pn / gn >= (double)ratio_lo &&
                        pn / gn <= (double)ratio_hi;
        keep[img] = ok ? 1 : 0;
    }
}

// out[i][y][x] = keep_i ? g + alpha (p - g) : g, p = pred[i][y][x][0] * scale_i (physical
// rows only); alpha = 1 gives p exactly
__global__ void k_guard_write(const float *__restrict__ pred, int C, const float *__restrict__ scale,
                              const float *__restrict__ g, int nimg, int h, int w, int hp, float alpha,
                              const int32_t *__restrict__ keep, float *__restrict__ out)
{
    const int64_t hw = (int64_t)h * w, total = (int64_t)nimg * hw;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = i / hw, k = i % hw;
        const float p = pred[((int64_t)img * hp * w + k) * C] * scale[img];
        out[i] = keep[img] ? (alpha == 1.0f ? p : fmaf(alpha, p - g[i], g[i])) : g[i];
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

// null pointers count as aligned
template <typename... T> bool aligned16(const T *...p) { return (((uintptr_t)p | ...) % 16) == 0; }

// Convolution tiles (rows, output channels, wavefronts along the rows), in order of preference: larger tiles reuse
// each operand read for more matrix operations; the first whose grid has at least kConvMinBlocks workgroups (two per
// compute unit) is used, else the smallest tile.  Input channels are staged 32 at a time when the channel counts
// allow and the grid is small (half the load phases and barriers), else 16.
struct ConvCfg {
    int ty, cot, wm;
};
constexpr ConvCfg kConvCfgs[] = {{8, 128, 4}, {8, 64, 4}, {4, 128, 2}, {8, 32, 4}, {4, 64, 2}, {4, 32, 4}};
constexpr int64_t kConvMinBlocks = 512;

int64_t conv_tiles(const fwi_nn_shape &in, int ty) { return (int64_t)in.n * ((in.h + ty - 1) / ty) * ((in.w + 31) / 32); }

ConvCfg pick_conv(const fwi_nn_shape &in, int cout)
{
    ConvCfg last = kConvCfgs[0];
    for (const ConvCfg &c : kConvCfgs) {
        if (cout % c.cot) continue;
        last = c;
        if (conv_tiles(in, c.ty) * (cout / c.cot) >= kConvMinBlocks) return c;
    }
    return last;
}

// Weight-gradient partition: pixel tiles of ty rows x 32 columns, chunks of per_chunk tiles, one workgroup per
// (32 x 32 channel block, chunk); about 1024 workgroups (four per compute unit), with the partial sums capped at
// 8 M floats.  Bias partials: chunks of bias_per pixels.
struct WgradPlan {
    int ty, ntiles, per_chunk, nch;
    int64_t nw, bias_per, bias_chunks;
};

WgradPlan wgrad_plan(const fwi_nn_shape &in, int cout)
{
    WgradPlan p;
    p.ty = 4;
    p.ntiles = (int)conv_tiles(in, p.ty);
    const int64_t cc = (int64_t)(cout / 32) * ((in.c + 31) / 32);
    p.nw = (int64_t)cout * 9 * in.c;
    int64_t nch = std::max<int64_t>(1, (1024 + cc - 1) / cc);
    nch = std::min<int64_t>(nch, std::max<int64_t>(1, ((int64_t)8 << 20) / p.nw));
    nch = std::min<int64_t>(nch, p.ntiles);
    p.per_chunk = (int)((p.ntiles + nch - 1) / nch);
    p.nch = (p.ntiles + p.per_chunk - 1) / p.per_chunk;
    const int64_t P = (int64_t)in.n * in.h * in.w;
    p.bias_per = 16 * (256 / std::min(cout, 256));
    p.bias_chunks = (P + p.bias_per - 1) / p.bias_per;
    return p;
}

fwi_status conv_launch(const uint16_t *x, const uint16_t *xu, int cu, fwi_nn_shape in, const uint16_t *w, int cout,
                       const float *bias, const float *aux, const float *res, int act, float *out_f32,
                       uint16_t *out_bf16, hipStream_t st)
{
    if (!w || !shape_ok(in) || in.c % 16 || cout <= 0 || cout % 32)
        return nn_fail(FWI_E_ARG, "conv3x3: need input channels %% 16 == 0 and output channels %% 32 == 0");
    if (!out_f32 && !out_bf16) return nn_fail(FWI_E_ARG, "conv3x3: no output");
    if (((uintptr_t)x | (uintptr_t)xu | (uintptr_t)w | (uintptr_t)bias | (uintptr_t)aux | (uintptr_t)out_f32) % 16 ||
        (uintptr_t)out_bf16 % 8)
        return nn_fail(FWI_E_ARG, "conv3x3: inputs, w, bias, aux and out_f32 must be 16-byte aligned, out_bf16 8-byte");
    if ((int64_t)in.h * in.w * in.c >= ((int64_t)1 << 31))
        return nn_fail(FWI_E_ARG, "conv3x3: one image must hold fewer than 2^31 elements");
    const ConvCfg c = pick_conv(in, cout);
    const int64_t nt = conv_tiles(in, c.ty);
    if (nt >= ((int64_t)1 << 31)) return nn_fail(FWI_E_ARG, "conv3x3: too many tiles");
    const dim3 grid((unsigned)nt, (unsigned)(cout / c.cot));
    // 32-channel chunks need more registers (half the occupancy at the smallest tile): worth it when the grid is at
    // most about two workgroups per compute unit, so occupancy does not limit it
    const bool ck32 = in.c % 32 == 0 && cu % 32 == 0 && nt * (cout / c.cot) <= 1024;
#define NN_CONV(TY, COT, WM)                                                                                          \
    if (c.ty == TY && c.cot == COT && c.wm == WM) {                                                                   \
        if (ck32)                                                                                                     \
            k_conv3x3<TY, COT, WM, 32><<<grid, 256, 0, st>>>(x, in.n, in.h, in.w, in.c, w, cout, bias, aux, res, act,  \
                                                             out_f32, out_bf16, xu, cu);                              \
        else                                                                                                          \
            k_conv3x3<TY, COT, WM, 16><<<grid, 256, 0, st>>>(x, in.n, in.h, in.w, in.c, w, cout, bias, aux, res, act,  \
                                                             out_f32, out_bf16, xu, cu);                              \
    }
    NN_CONV(8, 128, 4)
    NN_CONV(8, 64, 4)
    NN_CONV(4, 128, 2)
    NN_CONV(8, 32, 4)
    NN_CONV(4, 64, 2)
    NN_CONV(4, 32, 4)
#undef NN_CONV
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

// Row groups of the two-pass chunk sum
int64_t sum_groups(int nch) { return (nch + 31) / 32; }

fwi_status wgrad_launch(const uint16_t *dz, const float *dz_f32, const uint16_t *x, const uint16_t *xu, int cu,
                        fwi_nn_shape in, int cout, float *dw, float *db, float *work, hipStream_t st)
{
    if (!dz || !dw || !work || !shape_ok(in) || in.c % 16 || cout <= 0 || cout % 32 || (db && !dz_f32))
        return nn_fail(FWI_E_ARG, "wgrad: bad arguments");
    if (((uintptr_t)dz | (uintptr_t)x | (uintptr_t)xu | (uintptr_t)dw | (uintptr_t)work) % 16)
        return nn_fail(FWI_E_ARG, "wgrad: dz, the inputs, dw and work must be 16-byte aligned");
    const WgradPlan p = wgrad_plan(in, cout);
    const dim3 grid((unsigned)((cout / 32) * ((in.c + 31) / 32)), (unsigned)p.nch);
    k_wgrad<4><<<grid, 192, 0, st>>>(dz, x, in.n, in.h, in.w, in.c, cout, p.ntiles, p.per_chunk, work, xu, cu);
    NN_TRY(hipGetLastError());
    // chunk partials -> groups of 32 -> dw (one pass when there is a single group)
    const int64_t G = sum_groups(p.nch);
    const unsigned gx = (unsigned)((p.nw + 255) / 256);
    float *tmp = work + (int64_t)p.nch * p.nw;
    k_sum_rows32<<<dim3(gx, (unsigned)G), 256, 0, st>>>(work, p.nch, p.nw, G == 1 ? dw : tmp);
    NN_TRY(hipGetLastError());
    if (G > 1) {
        k_sum_rows32<<<dim3(gx, 1), 256, 0, st>>>(tmp, (int)G, p.nw, dw);
        NN_TRY(hipGetLastError());
    }
    if (db) {
        const int64_t P = (int64_t)in.n * in.h * in.w;
        float *bw = tmp + G * p.nw;
        k_bias_partial<<<dim3((unsigned)p.bias_chunks, (unsigned)((cout + 255) / 256)), 256, 0, st>>>(dz_f32, P, cout,
                                                                                                      p.bias_per, bw);
        NN_TRY(hipGetLastError());
        k_bias_final<<<cout, 256, 0, st>>>(bw, (int)p.bias_chunks, cout, db);
        NN_TRY(hipGetLastError());
    }
    return FWI_OK;
}

bool upcat_ok(const fwi_nn_shape &in, int ca)
{
    return shape_ok(in) && ca > 0 && ca % 16 == 0 && in.c > ca && (in.c - ca) % 16 == 0 && in.h % 2 == 0 &&
           in.w % 2 == 0;
}

}  // namespace

extern "C" {

fwi_status fwi_nn_conv3x3(const uint16_t *x, fwi_nn_shape in, const uint16_t *w, int32_t cout, const float *bias,
                          const float *aux, const float *res, int32_t act, float *out_f32, uint16_t *out_bf16,
                          void *stream)
{
    if (!x) return nn_fail(FWI_E_ARG, "conv3x3: no input");
    return conv_launch(x, nullptr, 0, in, w, cout, bias, aux, res, act, out_f32, out_bf16, (hipStream_t)stream);
}

fwi_status fwi_nn_conv3x3_upcat(const uint16_t *a, int32_t ca, const uint16_t *b, fwi_nn_shape in, const uint16_t *w,
                                int32_t cout, const float *bias, const float *aux, const float *res, int32_t act,
                                float *out_f32, uint16_t *out_bf16, void *stream)
{
    if (!a || !b || !upcat_ok(in, ca))
        return nn_fail(FWI_E_ARG, "conv3x3_upcat: need ca %% 16 == 0, (c - ca) %% 16 == 0, c > ca > 0, even h and w");
    return conv_launch(b, a, ca, in, w, cout, bias, aux, res, act, out_f32, out_bf16, (hipStream_t)stream);
}

int64_t fwi_nn_wgrad_work(fwi_nn_shape in, int32_t cout)
{
    if (!shape_ok(in) || cout <= 0 || cout % 32 || in.c % 16) return 0;
    const WgradPlan p = wgrad_plan(in, cout);
    return ((int64_t)p.nch + sum_groups(p.nch)) * p.nw + p.bias_chunks * cout;
}

fwi_status fwi_nn_wgrad(const uint16_t *dz, const float *dz_f32, const uint16_t *x, fwi_nn_shape in, int32_t cout,
                        float *dw, float *db, float *work, void *stream)
{
    if (!x) return nn_fail(FWI_E_ARG, "wgrad: no input");
    return wgrad_launch(dz, dz_f32, x, nullptr, 0, in, cout, dw, db, work, (hipStream_t)stream);
}

fwi_status fwi_nn_wgrad_upcat(const uint16_t *dz, const float *dz_f32, const uint16_t *a, int32_t ca,
                              const uint16_t *b, fwi_nn_shape in, int32_t cout, float *dw, float *db, float *work,
                              void *stream)
{
    if (!a || !b || !upcat_ok(in, ca))
        return nn_fail(FWI_E_ARG, "wgrad_upcat: need ca %% 16 == 0, (c - ca) %% 16 == 0, c > ca > 0, even h and w");
    return wgrad_launch(dz, dz_f32, b, a, ca, in, cout, dw, db, work, (hipStream_t)stream);
}

fwi_status fwi_nn_pool2(const uint16_t *x, fwi_nn_shape in, uint16_t *out, void *stream)
{
    if (!x || !out || !shape_ok(in) || in.h % 2 || in.w % 2) return nn_fail(FWI_E_ARG, "pool2: bad shape");
    const int64_t n_out = (int64_t)in.n * (in.h / 2) * (in.w / 2) * in.c;
    if (in.c % 8 == 0 && aligned16(x, out))
        k_pool2_v8<<<grid_for(n_out / 8), 256, 0, (hipStream_t)stream>>>(x, in.n, in.h, in.w, in.c, out);
    else
        k_pool2<<<grid_for(n_out), 256, 0, (hipStream_t)stream>>>(x, in.n, in.h, in.w, in.c, out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_pool2_bwd(const float *dout, fwi_nn_shape in, float *dx, int32_t accumulate, void *stream)
{
    if (!dout || !dx || !shape_ok(in) || in.h % 2 || in.w % 2) return nn_fail(FWI_E_ARG, "pool2_bwd: bad shape");
    const int64_t n_in = (int64_t)in.n * in.h * in.w * in.c;
    if (in.c % 4 == 0 && aligned16(dout, dx))
        k_pool2_bwd_v4<<<grid_for(n_in / 4), 256, 0, (hipStream_t)stream>>>(dout, in.n, in.h, in.w, in.c, dx,
                                                                            accumulate);
    else
        k_pool2_bwd<<<grid_for(n_in), 256, 0, (hipStream_t)stream>>>(dout, in.n, in.h, in.w, in.c, dx, accumulate);
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
    const int64_t n_in = (int64_t)in.n * in.h * in.w * in.c;
    if (in.c % 4 == 0 && aligned16(dout, dx))
        k_up2_bwd_v4<<<grid_for(n_in / 4), 256, 0, (hipStream_t)stream>>>(dout, in.n, in.h, in.w, in.c, dx);
    else
        k_up2_bwd<<<grid_for(n_in), 256, 0, (hipStream_t)stream>>>(dout, in.n, in.h, in.w, in.c, dx);
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
    if (ca % 4 == 0 && cb % 4 == 0 && aligned16(d, da, db))
        k_split_bwd_v4<<<grid_for(npix * (ca + cb) / 4), 256, 0, (hipStream_t)stream>>>(d, ca, cb, npix, da, acc_a, db,
                                                                                         acc_b);
    else
        k_split_bwd<<<grid_for(npix * (ca + cb)), 256, 0, (hipStream_t)stream>>>(d, ca, cb, npix, da, acc_a, db, acc_b);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

fwi_status fwi_nn_silu_bwd(const float *da, const float *z, int64_t n, float *dz_f32, uint16_t *dz_bf16, void *stream)
{
    if (!da || !z || n <= 0) return nn_fail(FWI_E_ARG, "silu_bwd: bad arguments");
    if (n % 4 == 0 && aligned16(da, z, dz_f32) && (uintptr_t)dz_bf16 % 8 == 0)
        k_silu_bwd_v4<<<grid_for(n / 4), 256, 0, (hipStream_t)stream>>>(da, z, n / 4, dz_f32, dz_bf16);
    else
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
    k_relmse_final<<<1, 256, 0, st>>>(work, nimg, nch, loss);
    NN_TRY(hipGetLastError());
    if (dpred) {
        if (c % 4 == 0 && aligned16(dpred) && (uintptr_t)dpred_bf16 % 8 == 0)
            k_relmse_grad_v4<<<grid_for((int64_t)nimg * hw * c / 4), 256, 0, st>>>(
                pred, c, target, nimg, hw, work + (int64_t)nimg * nch * 2, dpred, dpred_bf16);
        else
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
                        int32_t w, int32_t hp, float cos_min, float ratio_lo, float ratio_hi, float alpha,
                        float *out, int32_t *keep, void *stream)
{
    if (!pred || !scale || !g || !out || !keep || c < 1 || nimg < 1 || h < 1 || w < 1 || hp < h)
        return nn_fail(FWI_E_ARG, "guard: bad arguments");
    if (!(alpha >= 0.0f && alpha <= 1.0f)) return nn_fail(FWI_E_ARG, "guard: alpha %g outside [0, 1]", (double)alpha);
    hipStream_t st = (hipStream_t)stream;
    k_guard_stats<<<nimg, 256, 0, st>>>(pred, c, scale, g, h, w, hp, cos_min, ratio_lo, ratio_hi, keep);
    NN_TRY(hipGetLastError());
    const int64_t n = (int64_t)nimg * h * w;
    k_guard_write<<<grid_for(n), 256, 0, st>>>(pred, c, scale, g, nimg, h, w, hp, alpha, keep, out);
    NN_TRY(hipGetLastError());
    return FWI_OK;
}

const char *fwi_nn_last_error(void) { return g_nn_err.c_str(); }

}  // extern "C"
