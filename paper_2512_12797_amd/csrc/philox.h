// philox.h -- counter-based normal draws shared by the gfx950 kernels that add noise
// (the Langevin update and the diffusion re-noising).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fwi {

// Philox4x64-10 (Salmon et al., SC 2011).
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// uniform in (0, 1) from the top 53 bits
__device__ __forceinline__ double u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

// Four standard normals for cells 4m .. 4m+3 of one stream: Philox(ctr = {m, a, b, 0},
// key = {seed, tag}), Box-Muller on the word pairs (0, 1) and (2, 3).
__device__ __forceinline__ void normals4(uint64_t m, uint64_t a, uint64_t b, uint64_t seed, uint64_t tag,
                                         double z[4])
{
    uint64_t c[4] = {m, a, b, 0};
    philox4x64(c, seed, tag);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double r = sqrt(-2.0 * log(u01(c[2 * p])));
        const double th = 6.283185307179586476925 * u01(c[2 * p + 1]);
        z[2 * p] = r * cos(th);
        z[2 * p + 1] = r * sin(th);
    }
}

}  // namespace fwi
