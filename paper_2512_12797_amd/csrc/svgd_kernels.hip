// svgd_kernels.hip -- gfx950 kernels of the SVGD baseline (include/fwi_svgd.h): pairwise
// squared distances of the particles, the median bandwidth and RBF kernel matrix, and the
// Stein direction with the clamped move.  The distance pass is a streaming reduction
// (one workgroup per pair and cell chunk, FP64 partial sums in a fixed order); the kernel
// matrix is one workgroup; the move streams the particles and gradients once per output
// particle (the re-reads of the other particles hit L2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/fwi_svgd.h"

namespace {

constexpr int kMaxParticles = 64;
constexpr int kMaxPairs = kMaxParticles * (kMaxParticles - 1) / 2;
constexpr int kThreads = 256;
constexpr int kCellsPerChunk = 4096;  // cells per distance workgroup before a second chunk is added
constexpr int kMaxChunks = 256;

// pair p of the row-major list (i < j) -> (i, j)
__device__ __forceinline__ void pair_of(int n, int p, int &i, int &j)
{
    i = 0;
    while (p >= n - 1 - i) {
        p -= n - 1 - i;
        ++i;
    }
    j = i + 1 + p;
}

__device__ __forceinline__ int pair_index(int n, int i, int j) { return i * (2 * n - i - 1) / 2 + (j - i - 1); }

__device__ double block_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    return red[0];
}

// grid (chunks, pairs): partial[p][chunk] = sum over the chunk's cells of (x_i - x_j)^2
__global__ __launch_bounds__(kThreads) void k_svgd_dist(int n, int64_t N, int chunks, const float *__restrict__ x,
                                                        double *__restrict__ partial)
{
    __shared__ double red[kThreads];
    int i, j;
    pair_of(n, (int)blockIdx.y, i, j);
    const float *xi = x + (int64_t)i * N;
    const float *xj = x + (int64_t)j * N;
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < N; c += (int64_t)chunks * kThreads) {
        const double d = (double)xi[c] - (double)xj[c];
        acc += d * d;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * chunks + blockIdx.x] = s;
}

// one workgroup: distances, bandwidth (fixed or median / log n), K[i][j] = exp(-D_ij / h)
__global__ __launch_bounds__(kThreads) void k_svgd_kernel(int n, int chunks, double h_fixed,
                                                          const double *__restrict__ partial, double *__restrict__ K,
                                                          double *__restrict__ hb, double *__restrict__ h_out)
{
    __shared__ double D[kMaxPairs > 0 ? kMaxPairs : 1];
    __shared__ double mid[2];
    const int P = n * (n - 1) / 2;
    for (int p = threadIdx.x; p < P; p += kThreads) {
        double s = 0.0;
        for (int b = 0; b < chunks; ++b) s += partial[(int64_t)p * chunks + b];
        D[p] = s;
    }
    __syncthreads();
    double h = h_fixed;
    if (!(h > 0.0)) {
        h = 1.0;
        if (P > 0) {
            // the median by rank (ties broken by index, so every rank is held once)
            const int lo = (P - 1) / 2, hi = P / 2;
            for (int p = threadIdx.x; p < P; p += kThreads) {
                const double d = D[p];
                int rank = 0;
                for (int q = 0; q < P; ++q) rank += (D[q] < d || (D[q] == d && q < p)) ? 1 : 0;
                if (rank == lo) mid[0] = d;
                if (rank == hi) mid[1] = d;
            }
            __syncthreads();
            const double m = 0.5 * (mid[0] + mid[1]);
            const double hm = m / log((double)n);
            if (hm > 0.0 && hm < INFINITY) h = hm;
        }
    }
    for (int e = threadIdx.x; e < n * n; e += kThreads) {
        const int i = e / n, j = e - (e / n) * n;
        K[e] = i == j ? 1.0 : exp(-D[i < j ? pair_index(n, i, j) : pair_index(n, j, i)] / h);
    }
    if (threadIdx.x == 0) {
        hb[0] = h;
        hb[1] = 2.0 / h;
        if (h_out) *h_out = h;
    }
}

// grid (cell blocks, particles): phi_i = (1/n) sum_j K_ij (-g_j + (2/h)(x_i - x_j)); move and clamp
__global__ __launch_bounds__(kThreads) void k_svgd_move(int n, int64_t N, const float *__restrict__ x,
                                                        const float *__restrict__ g, const double *__restrict__ K,
                                                        const double *__restrict__ hb, double eps, double v_lo,
                                                        double v_hi, float *__restrict__ x_out,
                                                        float *__restrict__ phi)
{
    const int i = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c >= N) return;
    const double two_h = hb[1];
    const double xi = x[(int64_t)i * N + c];
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
        const int64_t o = (int64_t)j * N + c;
        acc += K[i * n + j] * (-(double)g[o] + two_h * (xi - (double)x[o]));
    }
    const double ph = acc / n;
    if (phi) phi[(int64_t)i * N + c] = (float)ph;
    double y = xi + eps * ph;
    y = y < v_lo ? v_lo : y;
    y = y > v_hi ? v_hi : y;
    x_out[(int64_t)i * N + c] = (float)y;
}

thread_local std::string g_svgd_err;

fwi_status svgd_fail(fwi_status s, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_svgd_err = buf;
    return s;
}

fwi_status svgd_check(hipError_t e, const char *what)
{
    return e == hipSuccess ? FWI_OK : svgd_fail(FWI_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int chunks_for(int64_t N) { return (int)std::min<int64_t>(kMaxChunks, std::max<int64_t>(1, (N + kCellsPerChunk - 1) / kCellsPerChunk)); }

bool overlaps(const float *a, const float *b, int64_t count)
{
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b, len = (uintptr_t)count * sizeof(float);
    return pa < pb + len && pb < pa + len;
}

}  // namespace

extern "C" {

size_t fwi_svgd_work_size(int32_t n, int64_t N)
{
    if (n < 1 || n > kMaxParticles || N < 1 || (N + kThreads - 1) / kThreads > 0x7FFFFFFF) return 0;
    const int64_t P = (int64_t)n * (n - 1) / 2;
    return sizeof(double) * (size_t)(P * chunks_for(N) + (int64_t)n * n + 2);
}

fwi_status fwi_svgd_step(int32_t n, int64_t N, const float *x, const float *grad, float eps, float h, float v_lo,
                         float v_hi, float *x_out, float *phi, double *h_out, void *work, size_t work_bytes,
                         void *stream)
{
    if (!x || !grad || !x_out) return svgd_fail(FWI_E_ARG, "step: null x, grad or x_out");
    const size_t need = fwi_svgd_work_size(n, N);
    if (need == 0) return svgd_fail(FWI_E_ARG, "step: need 1 <= n <= %d and N >= 1 (N = %lld)", kMaxParticles, (long long)N);
    if (!(eps >= 0.0f) || !std::isfinite(eps)) return svgd_fail(FWI_E_ARG, "step: eps must be finite and >= 0");
    if (!(v_hi > v_lo)) return svgd_fail(FWI_E_ARG, "step: need v_hi > v_lo");
    const int64_t total = (int64_t)n * N;
    if (overlaps(x_out, x, total) || overlaps(x_out, grad, total) ||
        (phi && (overlaps(phi, x_out, total) || overlaps(phi, x, total) || overlaps(phi, grad, total))))
        return svgd_fail(FWI_E_ARG, "step: x_out and phi must not overlap x, grad or each other");
    if (!work || (uintptr_t)work % 8 || work_bytes < need)
        return svgd_fail(FWI_E_WORKSPACE, "step: work null, misaligned or under %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    const int chunks = chunks_for(N);
    const int P = n * (n - 1) / 2;
    double *partial = (double *)work;
    double *K = partial + (int64_t)P * chunks;
    double *hb = K + (int64_t)n * n;
    if (P > 0) {
        k_svgd_dist<<<dim3((unsigned)chunks, (unsigned)P), kThreads, 0, s>>>(n, N, chunks, x, partial);
        fwi_status st = svgd_check(hipGetLastError(), "distances");
        if (st != FWI_OK) return st;
    }
    k_svgd_kernel<<<1, kThreads, 0, s>>>(n, chunks, (double)h, partial, K, hb, h_out);
    fwi_status st = svgd_check(hipGetLastError(), "kernel matrix");
    if (st != FWI_OK) return st;
    k_svgd_move<<<dim3((unsigned)((N + kThreads - 1) / kThreads), (unsigned)n), kThreads, 0, s>>>(
        n, N, x, grad, K, hb, (double)eps, (double)v_lo, (double)v_hi, x_out, phi);
    return svgd_check(hipGetLastError(), "move");
}

const char *fwi_svgd_last_error(void) { return g_svgd_err.c_str(); }

}  // extern "C"
