// fwi_kernels.hip -- gfx950 (CDNA4) kernels of the encoded-shot FWI gradient.
//
// Time stepping (both dims) streams each tile along z with a 9-deep register queue for
// the z-derivative of the 8th-order Laplacian; the x (and y) neighbours come from an LDS
// row/plane.  One wavefront covers 64 consecutive x cells, so every global access of a
// row is a coalesced 256-byte segment.  One launch per time step (2D: or per two time
// steps) covers every tile of every simulation of the batch (grids may differ in size);
// the block -> tile map gives each of the 8 XCDs a contiguous chunk of tiles so
// neighbouring tiles share an L2.
//
// Scheme (per padded cell): u^{n+1} = a u^n - b u^{n-1} + c (L u^n + q^n), with
// a = 2/(1+gamma dt), b = (1-gamma dt)/(1+gamma dt) computed from the cell index in
// FP64 and rounded once, and c precomputed per sample in FP64 and rounded once.
// The scaled adjoint lt = c lambda obeys the same recursion backward in time with
// c-weighted receiver injection; the imaging term lt^k (L u^{k-1} + q^{k-1}) is summed
// in FP64 into one accumulator per sample (a workgroup covers all of a sample's sims).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fwi_internal.h"
#include "fwi_launch.h"
#include "philox.h"

namespace fwi {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int xcd_tile(int bid, int per_xcd) { return (bid & 7) * per_xcd + (bid >> 3); }

// gamma contribution of one axis: gmax * (d/nb)^2 with d the cells into the sponge.
// Evaluated with contraction off so it rounds exactly like a plain FP64 expression.
__device__ __forceinline__ double sponge_axis(int p, int n, int nb, double gmax)
{
#pragma clang fp contract(off)
    if (nb == 0) return 0.0;
    int d = p < nb ? nb - p : (p > nb + n - 1 ? p - (nb + n - 1) : 0);
    if (d == 0) return 0.0;  // interior (same value as the formula, without the division)
    double r = (double)d / (double)nb;
    return gmax * r * r;
}

__device__ __forceinline__ void sponge_ab(double gam, double dt, float &a, float &b)
{
#pragma clang fp contract(off)
    if (gam == 0.0) {
        a = 2.0f;
        b = 1.0f;
        return;
    }
    double gd = gam * dt;
    double inv = 1.0 / (1.0 + gd);
    a = (float)(2.0 * inv);           // exactly 2/(1+gd) rounded: scaling by 2 is exact
    b = (float)((1.0 - gd) * inv);
}

__device__ __forceinline__ double coef_c(double v, double gam, double dt)
{
#pragma clang fp contract(off)
    double gd = gam * dt;
    return dt * dt * v * v / (1.0 + gd);
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = val;
}

// ------------------------------------------------------------- coefficients

// c = dt^2 v_pad^2 / (1 + gamma dt) for every padded cell of every sample; flags
// non-finite, non-positive or above-v_max velocities.
__global__ void k_prep(const SampleDesc *__restrict__ smp, const float *__restrict__ v, float *__restrict__ cf,
                       int *__restrict__ status)
{
    const SampleDesc S = smp[blockIdx.y];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int Nx = S.N[2], Ny = S.N[1], P = S.px;
    const int nby = S.ndim == 3 ? S.nb : 0;
    int bad = 0;
    for (; i < S.ncell; i += stride) {
        int px = (int)(i % P);
        int64_t r = i / P;
        if (px >= Nx) {  // row pitch padding
            cf[S.c_off + i] = 0.0f;
            continue;
        }
        int py = (int)(r % Ny);
        int pz = (int)(r / Ny);
        int ix = min(max(px - S.nb, 0), S.n[2] - 1);
        int iy = min(max(py - nby, 0), S.n[1] - 1);
        int iz = min(max(pz - S.nb, 0), S.n[0] - 1);
        float vv = v[S.m_off + ((int64_t)iz * S.n[1] + iy) * S.n[2] + ix];
        if (!(vv > 0.0f) || !(vv <= (float)S.v_max) || !isfinite(vv)) bad = 1;
        double gam = 0.0;
        gam = gam + sponge_axis(pz, S.n[0], S.nb, S.gmax[0]);
        if (S.ndim == 3) gam = gam + sponge_axis(py, S.n[1], S.nb, S.gmax[1]);
        gam = gam + sponge_axis(px, S.n[2], S.nb, S.gmax[2]);
        cf[S.c_off + i] = (float)coef_c((double)vv, gam, S.dt);
    }
    if (bad) atomicOr(status, 1);
}

// ------------------------------------------------------------ 2D stepping

// Per-lane source bookkeeping for one tile: the row of the lane's source (or -1) and
// the summed weight; `multi` when a lane holds sources on more than one row.
struct LaneSrc {
    int z;
    float w;
    bool multi;
};

__device__ __forceinline__ LaneSrc scan_sources_2d(const SrcPos *__restrict__ src, int beg, int cnt, int x,
                                                   int z0, int z1)
{
    LaneSrc r{-1, 0.0f, false};
    for (int s = 0; s < cnt; ++s) {
        const SrcPos p = src[beg + s];
        if (p.x == x && p.z >= z0 && p.z < z1) {
            if (r.z < 0 || r.z == p.z) {
                r.z = p.z;
                r.w += p.w;
            } else {
                r.multi = true;
            }
        }
    }
    return r;
}

// Wave-scope ordering of LDS traffic: a wavefront executes in order, so making the
// compiler keep program order is all that is needed between a wave's own LDS write and
// its reads of neighbouring lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ buffer access
// Raw buffer loads/stores through a resource that spans one simulation's field: an
// offset outside [0, bytes) reads 0 and drops a store in hardware, so the streaming
// loops need no bounds branches (the Dirichlet ghost ring comes out as zeros).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9-family raw buffer, 32-bit data format
constexpr uint32_t kOOB = 0xFFFFFFF0u;  // an offset beyond every resource
// Lane base offsets of the sweeps: a lane that must read 0 / drop its store gets bit 31
// set, so row (plane) offset + base stays outside every buffer for all rows the sweep
// touches, with one add per access instead of an add and a select.  The host guarantees
// (padded rows or planes + 80) * row or plane bytes <= 2^30, so row offsets (and their
// doubles, for FP64 accumulators) never reach bit 31.
constexpr uint32_t kPoison = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ float bload(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
// The same with the non-temporal cache policy, for fields a launch reads once and no launch
// reads again soon (the 3D forward's u^{n-1}, the 3D adjoint's lt^{k+2} and W^{k-1}, the 2D
// two-step adjoint's imaging operands): they then displace less of what is reused from L2
// (c, halo rows, the per-sample accumulator).
__device__ __forceinline__ float bload_nt(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 2));
}
__device__ __forceinline__ double bload64(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}
// Store with the non-temporal cache policy, for what a 3D sweep writes and no workgroup of
// the same launch reads (u^{n+1}, the imaging operand and the checkpoint pair in the
// forward, lt^k in the adjoint): the next reads come in later launches, after a whole
// level has streamed through L2, so caching these lines would only displace the halo rows
// and coefficients the sweep reuses.
__device__ __forceinline__ void bstore_nt(rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 2);
}
__device__ __forceinline__ void bstore64(rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v), r,
                                          (int)off, 0, 0);
}

// 2D forward step.  A workgroup holds 4 independent wavefronts; each owns one 64 x BZ tile
// of one sim and streams it along z.  Every global load for row z+4 is issued while row z
// is computed (centre queue q 8 rows ahead, halo queue hq and the point operands 4 rows
// ahead), so the memory latency of a row overlaps four rows of work.  The row loop is
// fully unrolled: the queues shift by register renaming, so loads stay in flight across
// rows instead of being waited for by a shift.  Loads are unconditional buffer loads (rows
// outside the grid read 0, stores there are dropped, so a tile that overhangs the bottom
// of the grid needs no row guard); lanes beyond the grid's x extent keep 0.
template <int BZ>
__global__ __launch_bounds__(256) void k_fwd2d(const StepArgs A)
{
    constexpr int PF = 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the tile index is uniform per wavefront: tile and simulation descriptors are
    // fetched with scalar loads once, before the first store
    const int t = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, A.per_xcd) * 4 + wave);
    if (t >= A.ntiles) return;  // waves are independent: no workgroup barrier below
    const Tile T = A.tiles[t];
    const SimDesc &S = A.sims[T.sim];
    const int Nx = S.N[2], Nz = S.N[0];
    const int nz_phys = S.n[0], nx_phys = S.n[2], nb = S.nb;
    const double gmz = S.gmax[0], gmx = S.gmax[2];
    const int64_t u_off = S.u_off, d_off = S.d_off;
    const int nrec = S.nrec, src_beg = S.src_beg, src_cnt = S.src_cnt;
    const uint32_t fbytes = (uint32_t)Nz * (uint32_t)Nx * 4u;
    const int x = T.x0 + lane;
    const bool xin = x < Nx;
    const int z0 = T.z0;
    const int z1 = min(z0 + BZ, Nz);
    const rsrc_t rU = make_rsrc(A.cur + u_off, fbytes);
    const rsrc_t rP = make_rsrc(A.prev + u_off, fbytes);
    const rsrc_t rN = make_rsrc(A.next + u_off, fbytes);
    const rsrc_t rC = make_rsrc(A.cf + S.c_off, fbytes);
    const rsrc_t rW = make_rsrc(A.wst ? A.wst + u_off : A.next, A.wst ? fbytes : 0);
    const rsrc_t rKa = make_rsrc(A.cka ? A.cka + u_off : A.next, A.cka ? fbytes : 0);
    const rsrc_t rKb = make_rsrc(A.ckb ? A.ckb + u_off : A.next, A.ckb ? fbytes : 0);
    const int rec_j = A.rec_j;
    float *Dat = (A.dat && rec_j >= 0) ? A.dat + d_off + (int64_t)rec_j * nrec : nullptr;
    const EvRow *__restrict__ evrows = A.evrows;
    const int32_t *__restrict__ evvec = A.evvec;
    float wz[5], wx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        wz[k] = S.w[0][k];
        wx[k] = S.w[2][k];
    }
    __shared__ float rows[4][2][kTileX + 2 * kHalo];

    const double gx = sponge_axis(x, nx_phys, nb, gmx);
    const double dt = S.dt;
    float a_col, b_col;  // a, b of this column outside the z-sponge
    {
        double gam = 0.0;
        gam = gam + gx;
        sponge_ab(gam, dt, a_col, b_col);
    }
    const LaneSrc src = scan_sources_2d(A.src, src_beg, src_cnt, x, z0, z1);
    const bool multi = __any(src.multi);
    const float famp = A.fn * S.inv_vol;

    // byte offsets: lane column (clamped into the row for lanes past the edge, whose
    // values are then forced to 0), halo column for lanes 0..7
    const uint32_t xo = 4u * (uint32_t)min(x, Nx - 1);
    const int hx = lane < 4 ? T.x0 - kHalo + lane : T.x0 + kTileX - 4 + lane;
    const bool hl = lane < 8 && hx >= 0 && hx < Nx;
    const uint32_t ho = 4u * (uint32_t)min(max(hx, 0), Nx - 1);
    const uint32_t rowb = 4u * (uint32_t)Nx;
    auto roff = [&](int zz) -> uint32_t { return (uint32_t)zz * rowb; };  // zz < 0 wraps out of range
    // wavefield and point-operand reads and the stores: lanes past the x edge (or not halo
    // lanes) carry the poison bit, so they read 0 (fetching nothing) and drop their stores
    const uint32_t xb = xin ? xo : kPoison, hb = hl ? ho : kPoison;
    auto coff = [&](int zz) -> uint32_t { return roff(zz) + xb; };
    auto hoff = [&](int zz) -> uint32_t { return roff(zz) + hb; };

    float q[BZ + 12], hq[BZ + PF], cq[BZ + PF], pq[BZ + PF];
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = bload(rU, coff(z0 - kHalo + k));
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const uint32_t o = roff(z0 + k);
        hq[k] = bload(rU, hoff(z0 + k));
        cq[k] = bload(rC, o + xb);
        pq[k] = bload(rP, o + xb);
    }
    // receiver event rows of this tile, kept in scalar registers (one row per z)
    const bool rec = rec_j >= 0 && T.ev_cnt > 0;
    int ev = T.ev_beg;
    const int ev_end = T.ev_beg + T.ev_cnt;
    int ev_z = rec ? __builtin_amdgcn_readfirstlane(evrows[ev].z) : -1;
    int ev_off = rec ? __builtin_amdgcn_readfirstlane(evrows[ev].vec_off) : 0;

#pragma unroll
    for (int r = 0; r < BZ; ++r) {
        const int z = z0 + r;
        q[r + 12] = bload(rU, coff(z + 8));
        const uint32_t of = roff(z + PF);
        hq[r + PF] = bload(rU, hoff(z + PF));
        cq[r + PF] = bload(rC, of + xb);
        pq[r + PF] = bload(rP, of + xb);

        float *row = rows[wave][r & 1];
        row[lane + kHalo] = q[r + 4];
        if (lane < 4)
            row[lane] = hq[r];
        else if (lane < 8)
            row[kTileX + lane] = hq[r];
        wave_lds_sync();
        float lx = wx[0] * q[r + 4];
        lx += wx[1] * (row[lane + 3] + row[lane + 5]);
        lx += wx[2] * (row[lane + 2] + row[lane + 6]);
        lx += wx[3] * (row[lane + 1] + row[lane + 7]);
        lx += wx[4] * (row[lane + 0] + row[lane + 8]);
        float lz = wz[0] * q[r + 4];
        lz += wz[1] * (q[r + 3] + q[r + 5]);
        lz += wz[2] * (q[r + 2] + q[r + 6]);
        lz += wz[3] * (q[r + 1] + q[r + 7]);
        lz += wz[4] * (q[r + 0] + q[r + 8]);
        float wv = lz + lx;

        float a = a_col, b = b_col;
        const double gz = sponge_axis(z, nz_phys, nb, gmz);  // uniform
        if (gz != 0.0) {
            double gam = 0.0;
            gam = gam + gz;
            gam = gam + gx;
            sponge_ab(gam, dt, a, b);
        }
        if (z == src.z) wv += src.w * famp;
        if (multi) {
            float extra = 0.0f;
            if (src.multi)
                for (int s2 = 0; s2 < src_cnt; ++s2) {
                    const SrcPos p = A.src[src_beg + s2];
                    if (p.x == x && p.z == z && z != src.z) extra += p.w;
                }
            wv += extra * famp;
        }
        const uint32_t o = coff(z);
        const float un = a * q[r + 4] - b * pq[r] + cq[r] * wv;
        bstore(rN, o, un);
        // optional outputs: uniform branches skip the instructions when a buffer is absent
        if (A.wst) bstore(rW, o, wv);
        if (A.cka) bstore(rKa, o, un);
        if (A.ckb) bstore(rKb, o, q[r + 4]);
        if (z == ev_z) {  // uniform
            if (Dat) {
                const int rid = evvec[ev_off + lane];
                if (rid >= 0) Dat[rid] = un;
            }
            ++ev;
            ev_z = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].z) : -1;
            ev_off = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].vec_off) : 0;
        }
        // keep each row's loads in its own row (prefetch distance PF rows)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ------------------------------------------------------ 2D adjoint, per-sample imaging

// 2D adjoint + imaging step with the imaging sum taken per sample.  A workgroup of nw
// wavefronts owns one 64 x BZ strip of one sample's grid; wave w sweeps the strip for the
// sample's sims w, w + nw, ... with the same register queues as the per-sim step and adds
// the exact FP64 products lt^k W^{k-1} of each row into registers.  The waves' partial
// sums are then added in wave order through LDS and wave 0 applies one read-modify-write
// to the sample's FP64 accumulator, so the accumulator costs 16 B per sample cell and step
// instead of 16 B per sim cell.  The summation order depends only on nw, which makes the
// result independent of the tile heights.
//
// The row loop is fully unrolled: the queues then shift by register renaming, so loads
// stay in flight across rows instead of being waited for by the shift.  Rows of a strip
// that fall below the grid are swept too: their loads read 0, their stores fall outside
// the buffer and are dropped, and their partial sums are never written.
template <int BZ>
__global__ __launch_bounds__(1024) void k_adj2d(const StepArgs A)
{
    constexpr int PF = 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
    const int lane = threadIdx.x & 63;
    const int gt = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, A.per_xcd_g));
    if (gt >= A.ngtiles) return;  // uniform per block: nobody reaches the barriers below
    // descriptors are read before the first store so that they stay in scalar registers
    const int nw = A.nw;
    const GTile G = A.gtiles[gt];
    const SampleDesc &Sm = A.samples[G.sample];
    const int Nx = Sm.N[2], Nz = Sm.N[0];
    const int nz_phys = Sm.n[0], nx_phys = Sm.n[2], nb = Sm.nb;
    const double gmz = Sm.gmax[0], gmx = Sm.gmax[2];
    const double dt = Sm.dt;
    const int sim_beg = Sm.sim_beg, sim_cnt = Sm.sim_cnt;
    const int64_t ncell = Sm.ncell, g_off = Sm.g_off;
    const SimDesc &S0 = A.sims[sim_beg];
    const int64_t u_off0 = S0.u_off;  // sims of a sample are consecutive, ncell apart
    float wz[5], wx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        wz[k] = S0.w[0][k];
        wx[k] = S0.w[2][k];
    }
    const uint32_t fbytes = (uint32_t)Nz * (uint32_t)Nx * 4u;
    const int x = G.x0 + lane;
    const bool xin = x < Nx;
    const int z0 = G.z0;
    const int nrow = min(BZ, Nz - z0);
    const rsrc_t rC = make_rsrc(A.cf + Sm.c_off, fbytes);
    const int rec_j = A.rec_j;
    const EvRow *__restrict__ evrows = A.evrows;
    const int32_t *__restrict__ evvec = A.evvec;
    const double gx = sponge_axis(x, nx_phys, nb, gmx);

    const uint32_t xo = 4u * (uint32_t)min(x, Nx - 1);
    const int hx = lane < 4 ? G.x0 - kHalo + lane : G.x0 + kTileX - 4 + lane;
    const bool hl = lane < 8 && hx >= 0 && hx < Nx;
    const uint32_t ho = 4u * (uint32_t)min(max(hx, 0), Nx - 1);
    const uint32_t rowb = 4u * (uint32_t)Nx;
    auto roff = [&](int zz) -> uint32_t { return (uint32_t)zz * rowb; };  // zz < 0 wraps out of range

    __shared__ float rows[16][2][kTileX + 2 * kHalo];
    __shared__ double red[BZ][kTileX];
    __shared__ float2 abt[BZ][kTileX];  // leapfrog a, b of the strip's cells (shared by all sims)

    // a and b depend on the cell only: computed once per strip, not once per sim
    for (int r = wave; r < BZ; r += nw) {
        double gam = 0.0;
        gam = gam + sponge_axis(z0 + r, nz_phys, nb, gmz);
        gam = gam + gx;
        float a, b;
        sponge_ab(gam, dt, a, b);
        abt[r][lane] = make_float2(a, b);
    }
    __syncthreads();

    double acc[BZ];
#pragma unroll
    for (int r = 0; r < BZ; ++r) acc[r] = 0.0;

    for (int j = wave; j < sim_cnt; j += nw) {
        const int sim = sim_beg + j;
        const int64_t u_off = u_off0 + (int64_t)j * ncell;
        const rsrc_t rU = make_rsrc(A.cur + u_off, fbytes);
        const rsrc_t rP = make_rsrc(A.prev + u_off, fbytes);
        const rsrc_t rN = make_rsrc(A.next + u_off, fbytes);
        const rsrc_t rW = make_rsrc(A.wimg + u_off, fbytes);
        // lane offsets pass through an empty asm so that the row offsets built from them
        // are recomputed per sim next to their loads, not hoisted out of the sim loop
        // (which would keep every row's offsets live in registers)
        uint32_t xs = xo, hs = ho;  // clamped into the row
        int zs = z0;                // and the strip origin (uniform): same for the row offsets
        asm volatile("" : "+v"(xs), "+v"(hs), "+s"(zs));
        // wavefield reads and the store: lanes past the x edge (or not halo lanes) carry
        // the poison bit; point operands read the clamped column
        const uint32_t xb = xin ? xs : kPoison, hb = hl ? hs : kPoison;
        auto coff = [&](int zz) -> uint32_t { return roff(zz) + xb; };
        auto hoff = [&](int zz) -> uint32_t { return roff(zz) + hb; };
        // per-sim fields read after stores: vector loads, made uniform explicitly
        const int tile0 = __builtin_amdgcn_readfirstlane(A.sims[sim].tile0);
        const int nrec = __builtin_amdgcn_readfirstlane(A.sims[sim].nrec);
        const int64_t d_off = A.sims[sim].d_off;
        const int d_lo = __builtin_amdgcn_readfirstlane((int)(d_off & 0xFFFFFFFF));
        const int d_hi = __builtin_amdgcn_readfirstlane((int)(d_off >> 32));
        const int64_t d_off_u = (int64_t)(((uint64_t)(uint32_t)d_hi << 32) | (uint32_t)d_lo);

        // centre queue rows z-4 .. z+8, halo and point operands 4 rows ahead
        float q[BZ + 12], hq[BZ + PF], cq[BZ + PF], pq[BZ + PF], wq[BZ + PF];
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = bload(rU, coff(zs - kHalo + k));
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const uint32_t o = roff(zs + k);
            hq[k] = bload(rU, hoff(zs + k));
            cq[k] = bload(rC, o + xs);
            pq[k] = bload(rP, o + xs);
            wq[k] = bload(rW, o + xs);
        }
        const float *Rho = rec_j >= 0 ? A.rho + d_off_u + (int64_t)rec_j * nrec : nullptr;
        // receiver event rows of the sim tile that holds this strip, from row z0 on
        int ev = 0, ev_end = 0, ev_z = -1, ev_off = 0;
        if (rec_j >= 0) {
            const Tile &T = A.tiles[tile0 + G.tix];
            ev = __builtin_amdgcn_readfirstlane(T.ev_beg);
            ev_end = ev + __builtin_amdgcn_readfirstlane(T.ev_cnt);
            while (ev < ev_end) {
                ev_z = __builtin_amdgcn_readfirstlane(evrows[ev].z);
                if (ev_z >= z0) break;
                ++ev;
            }
            if (ev < ev_end)
                ev_off = __builtin_amdgcn_readfirstlane(evrows[ev].vec_off);
            else
                ev_z = -1;
        }

#pragma unroll
        for (int r = 0; r < BZ; ++r) {
            const int z = zs + r;
            q[r + 12] = bload(rU, coff(z + 8));
            const uint32_t of = roff(z + PF);
            hq[r + PF] = bload(rU, hoff(z + PF));
            cq[r + PF] = bload(rC, of + xs);
            pq[r + PF] = bload(rP, of + xs);
            wq[r + PF] = bload(rW, of + xs);

            float *row = rows[wave][r & 1];
            row[lane + kHalo] = q[r + 4];
            if (lane < 4)
                row[lane] = hq[r];
            else if (lane < 8)
                row[kTileX + lane] = hq[r];
            wave_lds_sync();
            float lx = wx[0] * q[r + 4];
            lx += wx[1] * (row[lane + 3] + row[lane + 5]);
            lx += wx[2] * (row[lane + 2] + row[lane + 6]);
            lx += wx[3] * (row[lane + 1] + row[lane + 7]);
            lx += wx[4] * (row[lane + 0] + row[lane + 8]);
            float lz = wz[0] * q[r + 4];
            lz += wz[1] * (q[r + 3] + q[r + 5]);
            lz += wz[2] * (q[r + 2] + q[r + 6]);
            lz += wz[3] * (q[r + 1] + q[r + 7]);
            lz += wz[4] * (q[r + 0] + q[r + 8]);
            float wv = lz + lx;

            const float2 ab = abt[r][lane];
            if (z == ev_z) {  // uniform
                const int rid = evvec[ev_off + lane];
                if (rid >= 0) wv += Rho[rid];
                ++ev;
                ev_z = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].z) : -1;
                ev_off = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].vec_off) : 0;
            }
            const float un = ab.x * q[r + 4] - ab.y * pq[r] + cq[r] * wv;
            bstore(rN, coff(z), un);
            acc[r] += (double)un * (double)wq[r];  // the product of two floats is exact in FP64
            // keep each row's loads in its own row: the prefetch distance stays PF rows
            // instead of the scheduler hoisting every load of the strip to the top
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // partial sums of waves 1 .. nw-1 are added to wave 0's, in wave order
    for (int w = 1; w < nw; ++w) {
        __syncthreads();
        if (wave == w)
#pragma unroll
            for (int r = 0; r < BZ; ++r) red[r][lane] = acc[r];
        __syncthreads();
        if (wave == 0)
#pragma unroll
            for (int r = 0; r < BZ; ++r) acc[r] += red[r][lane];
    }
    if (wave == 0) {
        const rsrc_t rG = make_rsrc(A.gacc + g_off, 2 * fbytes);
        double g[BZ];
#pragma unroll
        for (int r = 0; r < BZ; ++r) g[r] = bload64(rG, (xin && r < nrow) ? 2 * (roff(z0 + r) + xo) : kOOB);
#pragma unroll
        for (int r = 0; r < BZ; ++r)
            bstore64(rG, (xin && r < nrow) ? 2 * (roff(z0 + r) + xo) : kOOB, g[r] + acc[r]);
    }
}

// ------------------------------------------------ 2D, two time steps per launch
//
// One sweep advances the fields by two time steps, so u^{n-1}, u^n (or lt^{k+2}, lt^{k+1})
// are read once per two steps.  Lane l of a wavefront holds column x0 - 4 + l of a strip
// of kStrip2 columns.  The first step is evaluated on all 64 lanes and on the rows
// z0 - 4 .. z0 + BZ + 3: its values in that 4-cell margin are the neighbours the second
// step needs.  Every strip that needs them recomputes them from the same inputs with the
// same instructions, so they equal the owner's bit for bit.  The second step runs 4 rows
// behind the first, on the strip's own 56 lanes and BZ rows.  Every operand of a
// first-step cell outside the grid reads 0 (poisoned offsets), so that cell comes out
// exactly 0, the Dirichlet ghost the second step reads.  The two new levels go to
// buffers that no strip reads during the launch.

// Source term of one lane at row z: the lane's scanned source plus, when some lane of the
// wave holds sources on several rows, the others at this row.
__device__ __forceinline__ float src_term(const StepArgs &A, const LaneSrc &src, bool multi, int src_beg,
                                          int src_cnt, int x, int z, float famp, float wv)
{
    if (z == src.z) wv += src.w * famp;
    if (multi) {
        float extra = 0.0f;
        if (src.multi)
            for (int s2 = 0; s2 < src_cnt; ++s2) {
                const SrcPos p = A.src[src_beg + s2];
                if (p.x == x && p.z == z && z != src.z) extra += p.w;
            }
        wv += extra * famp;
    }
    return wv;
}

constexpr int kNoRow = -(1 << 30);  // event cursor past its last row
// Rows fetched ahead by the two-step sweeps.  The two-step forward runs at the same speed
// with 4, 6 or 8 (at its occupancy it is limited by instruction issue, not by memory
// latency), and deeper queues only cost registers.
constexpr int kPf2 = 4;

template <int BZ, int PF>
__global__ __launch_bounds__(256) void k_fwd2d2(const StepArgs A)
{
    constexpr int R1 = BZ + 2 * kHalo;  // rows of the first step
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, A.per_xcd) * 4 + wave);
    if (t >= A.ntiles) return;  // waves are independent: no workgroup barrier below
    const Tile T = A.tiles[t];
    const SimDesc &S = A.sims[T.sim];
    const int Nx = S.N[2], Nz = S.N[0];
    const int nz_phys = S.n[0], nx_phys = S.n[2], nb = S.nb;
    const double gmz = S.gmax[0], gmx = S.gmax[2];
    const int64_t u_off = S.u_off, d_off = S.d_off;
    const int nrec = S.nrec, src_beg = S.src_beg, src_cnt = S.src_cnt;
    const uint32_t fbytes = (uint32_t)Nz * (uint32_t)Nx * 4u;
    const int x = T.x0 - kHalo + lane;
    const bool xin = x >= 0 && x < Nx;
    const bool mine = lane >= kHalo && lane < kHalo + kStrip2;  // the strip's own columns
    const int z0 = T.z0;
    const rsrc_t rU = make_rsrc(A.cur + u_off, fbytes);
    const rsrc_t rP = make_rsrc(A.prev + u_off, fbytes);
    const rsrc_t rN = make_rsrc(A.next + u_off, fbytes);
    const rsrc_t rN2 = make_rsrc(A.next2 + u_off, fbytes);
    const rsrc_t rC = make_rsrc(A.cf + S.c_off, fbytes);
    const rsrc_t rW = make_rsrc(A.wst ? A.wst + u_off : A.next, A.wst ? fbytes : 0);
    const rsrc_t rW2 = make_rsrc(A.wst2 ? A.wst2 + u_off : A.next, A.wst2 ? fbytes : 0);
    float *Dat1 = (A.dat && A.rec_j >= 0) ? A.dat + d_off + (int64_t)A.rec_j * nrec : nullptr;
    float *Dat2 = (A.dat && A.rec_j2 >= 0) ? A.dat + d_off + (int64_t)A.rec_j2 * nrec : nullptr;
    const EvRow *__restrict__ evrows = A.evrows;
    const int32_t *__restrict__ evvec = A.evvec;
    float wz[5], wx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        wz[k] = S.w[0][k];
        wx[k] = S.w[2][k];
    }
    __shared__ float rows[4][2][kTileX + 2 * kHalo];   // u^n row with its x halo
    __shared__ float rows1[4][2][kTileX + 2 * kHalo];  // u^{n+1} row (entries 4 .. 67)
    if (lane < 2 * kHalo) {  // margins read only by lanes whose second step is discarded
        const int m = lane < kHalo ? lane : kTileX + lane;
        rows1[wave][0][m] = 0.0f;
        rows1[wave][1][m] = 0.0f;
    }

    const double gx = sponge_axis(x, nx_phys, nb, gmx);
    const double dt = S.dt;
    float a_col, b_col;  // a, b of this column outside the z-sponge
    {
        double gam = 0.0;
        gam = gam + gx;
        sponge_ab(gam, dt, a_col, b_col);
    }
    const LaneSrc src = scan_sources_2d(A.src, src_beg, src_cnt, x, z0 - kHalo, z0 + BZ + kHalo);
    const bool multi = __any(src.multi);
    const float famp1 = A.fn * S.inv_vol, famp2 = A.fn2 * S.inv_vol;

    const uint32_t xo = 4u * (uint32_t)min(max(x, 0), Nx - 1);
    const int hx = lane < 4 ? T.x0 - 2 * kHalo + lane : T.x0 - kHalo + kTileX - 4 + lane;
    const bool hl = lane < 8 && hx >= 0 && hx < Nx;
    const uint32_t ho = 4u * (uint32_t)min(max(hx, 0), Nx - 1);
    const uint32_t rowb = 4u * (uint32_t)Nx;
    auto roff = [&](int zz) -> uint32_t { return (uint32_t)zz * rowb; };  // zz < 0 wraps out of range
    // every read of the first step is poisoned outside the grid (it must compute 0 there);
    // stores and records are poisoned outside the strip's own columns
    const uint32_t xb = xin ? xo : kPoison, hb = hl ? ho : kPoison;
    const uint32_t sb = (xin && mine) ? xo : kPoison;
    auto coff = [&](int zz) -> uint32_t { return roff(zz) + xb; };
    auto hoff = [&](int zz) -> uint32_t { return roff(zz) + hb; };
    auto soff = [&](int zz) -> uint32_t { return roff(zz) + sb; };

    // u^n queue: q[k] holds row z0 - 8 + k; first-step queues: index k holds row z0 - 4 + k.
    // Every queue is fetched PF rows ahead of the first step that reads it.
    float q[R1 + 8 + PF], hq[R1 + PF], cq[R1 + PF], pq[R1 + PF], s1[R1], ra[R1], rb[R1];
#pragma unroll
    for (int k = 0; k < 8 + PF; ++k) q[k] = bload(rU, coff(z0 - 2 * kHalo + k));
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int zz = z0 - kHalo + k;
        hq[k] = bload(rU, hoff(zz));
        cq[k] = bload(rC, coff(zz));
        pq[k] = bload(rP, coff(zz));
    }
    // receiver event rows of the strip from row z0 on (both steps record own rows only)
    const bool rec = (Dat1 || Dat2) && T.ev_cnt > 0;
    const int ev_end = T.ev_beg + T.ev_cnt;
    int e1 = T.ev_beg;
    int ez1 = kNoRow, eo1 = 0;
    if (rec) {
        while (e1 < ev_end) {
            ez1 = __builtin_amdgcn_readfirstlane(evrows[e1].z);
            if (ez1 >= z0) break;
            ++e1;
        }
        if (e1 < ev_end)
            eo1 = __builtin_amdgcn_readfirstlane(evrows[e1].vec_off);
        else
            ez1 = kNoRow;
    }
    int e2 = e1, ez2 = ez1, eo2 = eo1;

#pragma unroll
    for (int i = 0; i < R1; ++i) {
        const int z1 = z0 - kHalo + i;
        q[i + 8 + PF] = bload(rU, coff(z1 + kHalo + PF));
        hq[i + PF] = bload(rU, hoff(z1 + PF));
        cq[i + PF] = bload(rC, coff(z1 + PF));
        pq[i + PF] = bload(rP, coff(z1 + PF));

        // both steps' x rows go to LDS before one wave-scope fence: the second step's row
        // (first-step row z1 - 4) was computed four iterations ago
        float *row = rows[wave][i & 1];
        float *row1 = rows1[wave][i & 1];
        row[lane + kHalo] = q[i + 4];
        if (lane < 4)
            row[lane] = hq[i];
        else if (lane < 8)
            row[kTileX + lane] = hq[i];
        if (i >= 2 * kHalo) row1[lane + kHalo] = s1[i - 4];
        wave_lds_sync();
        // first step, row z1 (centre q[i + 4])
        {
            float lx = wx[0] * q[i + 4];
            lx += wx[1] * (row[lane + 3] + row[lane + 5]);
            lx += wx[2] * (row[lane + 2] + row[lane + 6]);
            lx += wx[3] * (row[lane + 1] + row[lane + 7]);
            lx += wx[4] * (row[lane + 0] + row[lane + 8]);
            float lz = wz[0] * q[i + 4];
            lz += wz[1] * (q[i + 3] + q[i + 5]);
            lz += wz[2] * (q[i + 2] + q[i + 6]);
            lz += wz[3] * (q[i + 1] + q[i + 7]);
            lz += wz[4] * (q[i + 0] + q[i + 8]);
            float wv = lz + lx;
            float a = a_col, b = b_col;
            const double gz = sponge_axis(z1, nz_phys, nb, gmz);  // uniform
            if (gz != 0.0) {
                double gam = 0.0;
                gam = gam + gz;
                gam = gam + gx;
                sponge_ab(gam, dt, a, b);
            }
            ra[i] = a;
            rb[i] = b;
            wv = src_term(A, src, multi, src_beg, src_cnt, x, z1, famp1, wv);
            const float un = a * q[i + 4] - b * pq[i] + cq[i] * wv;
            s1[i] = un;
            if (i >= kHalo && i < BZ + kHalo) {  // the strip's own rows
                bstore(rN, soff(z1), un);
                if (A.wst) bstore(rW, soff(z1), wv);
                if (z1 == ez1) {  // uniform
                    if (Dat1) {
                        const int rid = evvec[eo1 + lane];
                        if (rid >= 0 && mine) Dat1[rid] = un;
                    }
                    ++e1;
                    ez1 = e1 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e1].z) : kNoRow;
                    eo1 = e1 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e1].vec_off) : 0;
                }
            }
        }
        // second step, row z2 = z1 - 4 (centre s1[i - 4]; u^n there is q[i], c is cq[i - 4])
        if (i >= 2 * kHalo) {
            const int z2 = z1 - kHalo;
            const float *row = row1;
            float lx = wx[0] * s1[i - 4];
            lx += wx[1] * (row[lane + 3] + row[lane + 5]);
            lx += wx[2] * (row[lane + 2] + row[lane + 6]);
            lx += wx[3] * (row[lane + 1] + row[lane + 7]);
            lx += wx[4] * (row[lane + 0] + row[lane + 8]);
            float lz = wz[0] * s1[i - 4];
            lz += wz[1] * (s1[i - 5] + s1[i - 3]);
            lz += wz[2] * (s1[i - 6] + s1[i - 2]);
            lz += wz[3] * (s1[i - 7] + s1[i - 1]);
            lz += wz[4] * (s1[i - 8] + s1[i - 0]);
            float wv = lz + lx;
            wv = src_term(A, src, multi, src_beg, src_cnt, x, z2, famp2, wv);
            const float un = ra[i - 4] * s1[i - 4] - rb[i - 4] * q[i] + cq[i - 4] * wv;
            bstore(rN2, soff(z2), un);
            if (A.wst2) bstore(rW2, soff(z2), wv);
            if (z2 == ez2) {  // uniform
                if (Dat2) {
                    const int rid = evvec[eo2 + lane];
                    if (rid >= 0 && mine) Dat2[rid] = un;
                }
                ++e2;
                ez2 = e2 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e2].z) : kNoRow;
                eo2 = e2 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e2].vec_off) : 0;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Adjoint steps k and k - 1 with the per-sample imaging sum, in one sweep.  A workgroup of
// nw wavefronts owns sg (1 or 2) consecutive strips of the samples' grids (lanes as in the
// forward above), nw / sg wavefronts per strip; local wave l of a strip sweeps it for the
// strip's sample's sims l, l + nw / sg, ...  (Two strips per workgroup balance the waves
// when a sample's sim count divides by nw / sg but not by nw.)  The first step (lt^k,
// residual slot of step k injected on every lane and row it computes, margins included)
// and the second (lt^{k-1}) add the exact FP64 products lt^k W^{k-1} and lt^{k-1} W^{k-2}
// of the strip's own cells into registers; each strip's wave sums are then added in wave
// order through LDS and its first wave applies one read-modify-write of the sample's
// accumulator per two steps.
template <int BZ, int PF>
__global__ __launch_bounds__(512) void k_adj2d2(const StepArgs A)
{
    constexpr int R1 = BZ + 2 * kHalo;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nw = A.nw, sg = A.sg;
    const int wps = nw / sg;                 // waves per strip
    const int sidx = wave / wps, wl = wave - sidx * wps;  // this wave's strip, its rank there
    const int gt0 = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, A.per_xcd_g) * sg);
    if (gt0 >= A.ngtiles) return;  // uniform per block: nobody reaches the barriers below
    const int gt = gt0 + sidx;
    const bool active = gt < A.ngtiles;  // uniform per wave; inactive waves only join the barriers
    const GTile G = A.gtiles[active ? gt : gt0];
    const SampleDesc &Sm = A.samples[G.sample];
    const int Nx = Sm.N[2], Nz = Sm.N[0];
    const int nz_phys = Sm.n[0], nx_phys = Sm.n[2], nb = Sm.nb;
    const double gmz = Sm.gmax[0], gmx = Sm.gmax[2];
    const double dt = Sm.dt;
    const int sim_beg = Sm.sim_beg, sim_cnt = Sm.sim_cnt;
    const int64_t ncell = Sm.ncell, g_off = Sm.g_off;
    const SimDesc &S0 = A.sims[sim_beg];
    const int64_t u_off0 = S0.u_off;  // sims of a sample are consecutive, ncell apart
    float wz[5], wx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        wz[k] = S0.w[0][k];
        wx[k] = S0.w[2][k];
    }
    const uint32_t fbytes = (uint32_t)Nz * (uint32_t)Nx * 4u;
    const int x = G.x0 - kHalo + lane;
    const bool xin = x >= 0 && x < Nx;
    const bool mine = lane >= kHalo && lane < kHalo + kStrip2;
    const int z0 = G.z0;
    const int nrow = min(BZ, Nz - z0);
    const rsrc_t rC = make_rsrc(A.cf + Sm.c_off, fbytes);
    const int rec_j1 = A.rec_j, rec_j2 = A.rec_j2;
    const EvRow *__restrict__ evrows = A.evrows;
    const int32_t *__restrict__ evvec = A.evvec;
    const double gx = sponge_axis(x, nx_phys, nb, gmx);

    const uint32_t xo = 4u * (uint32_t)min(max(x, 0), Nx - 1);
    const int hx = lane < 4 ? G.x0 - 2 * kHalo + lane : G.x0 - kHalo + kTileX - 4 + lane;
    const bool hl = lane < 8 && hx >= 0 && hx < Nx;
    const uint32_t ho = 4u * (uint32_t)min(max(hx, 0), Nx - 1);
    const uint32_t rowb = 4u * (uint32_t)Nx;
    auto roff = [&](int zz) -> uint32_t { return (uint32_t)zz * rowb; };  // zz < 0 wraps out of range

    // LDS sized by the launch (adj2d2_lds_bytes): the strips' wave sums when a strip has
    // several waves, each wave's x rows of the two steps, each strip's a, b
    extern __shared__ __align__(16) unsigned char dsm[];
    double(*red)[BZ][kTileX] = reinterpret_cast<double(*)[BZ][kTileX]>(dsm);
    float(*rows)[2][kTileX + 2 * kHalo] =
        reinterpret_cast<float(*)[2][kTileX + 2 * kHalo]>(dsm + (wps > 1 ? (size_t)sg * BZ * kTileX * sizeof(double) : 0));
    float(*rows1)[2][kTileX + 2 * kHalo] = rows + nw;
    float2(*abt)[R1][kTileX] = reinterpret_cast<float2(*)[R1][kTileX]>(rows1 + nw);  // a, b per strip

    for (int r = wl; r < R1 && active; r += wps) {
        double gam = 0.0;
        gam = gam + sponge_axis(z0 - kHalo + r, nz_phys, nb, gmz);
        gam = gam + gx;
        float a, b;
        sponge_ab(gam, dt, a, b);
        abt[sidx][r][lane] = make_float2(a, b);
    }
    if (lane < 2 * kHalo) {
        const int m = lane < kHalo ? lane : kTileX + lane;
        rows1[wave][0][m] = 0.0f;
        rows1[wave][1][m] = 0.0f;
    }
    __syncthreads();

    double acc[BZ];
#pragma unroll
    for (int r = 0; r < BZ; ++r) acc[r] = 0.0;
    // c of the strip's first-step rows, read once for all of the wave's sims
    float cr[R1];
    {
        const uint32_t cb0 = xin ? xo : kPoison;
#pragma unroll
        for (int i = 0; i < R1; ++i) cr[i] = bload(rC, roff(z0 - kHalo + i) + cb0);
    }

    for (int j = wl; j < sim_cnt && active; j += wps) {
        const int sim = sim_beg + j;
        const int64_t u_off = u_off0 + (int64_t)j * ncell;
        const rsrc_t rU = make_rsrc(A.cur + u_off, fbytes);
        const rsrc_t rP = make_rsrc(A.prev + u_off, fbytes);
        const rsrc_t rN = make_rsrc(A.next + u_off, fbytes);
        const rsrc_t rN2 = make_rsrc(A.next2 + u_off, fbytes);
        const rsrc_t rW = make_rsrc(A.wimg + u_off, fbytes);
        const rsrc_t rW2 = make_rsrc(A.wimg2 + u_off, fbytes);
        // lane offsets pass through an empty asm so that the row offsets built from them
        // are recomputed per sim next to their loads, not hoisted out of the sim loop
        uint32_t xs = xo, hs = ho;
        int zs = z0;
        asm volatile("" : "+v"(xs), "+v"(hs), "+s"(zs));
        const uint32_t xb = xin ? xs : kPoison, hb = hl ? hs : kPoison;
        const uint32_t sb = (xin && mine) ? xs : kPoison;
        auto coff = [&](int zz) -> uint32_t { return roff(zz) + xb; };
        auto hoff = [&](int zz) -> uint32_t { return roff(zz) + hb; };
        auto soff = [&](int zz) -> uint32_t { return roff(zz) + sb; };
        const int tile0b = __builtin_amdgcn_readfirstlane(A.sims[sim].tile0b);
        const int nrec = __builtin_amdgcn_readfirstlane(A.sims[sim].nrec);
        const int64_t d_off = A.sims[sim].d_off;
        const int d_lo = __builtin_amdgcn_readfirstlane((int)(d_off & 0xFFFFFFFF));
        const int d_hi = __builtin_amdgcn_readfirstlane((int)(d_off >> 32));
        const int64_t d_off_u = (int64_t)(((uint64_t)(uint32_t)d_hi << 32) | (uint32_t)d_lo);

        float q[R1 + 8 + PF], hq[R1 + PF], pq[R1 + PF], s1[R1], wq1[BZ], wq2[BZ];
#pragma unroll
        for (int k = 0; k < 8 + PF; ++k) q[k] = bload(rU, coff(zs - 2 * kHalo + k));
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int zz = zs - kHalo + k;
            hq[k] = bload(rU, hoff(zz));
            pq[k] = bload(rP, coff(zz));
        }
        const float *Rho1 = rec_j1 >= 0 ? A.rho + d_off_u + (int64_t)rec_j1 * nrec : nullptr;
        const float *Rho2 = rec_j2 >= 0 ? A.rho + d_off_u + (int64_t)rec_j2 * nrec : nullptr;
        // receiver event rows of this sim's strip: the first step injects on all of them
        // (margins included), the second from row z0 on
        int e1 = 0, ev_end = 0, ez1 = kNoRow, eo1 = 0, e2 = 0, ez2 = kNoRow, eo2 = 0;
        if (Rho1 || Rho2) {
            const Tile &T = A.tiles[tile0b + G.tix];
            e1 = __builtin_amdgcn_readfirstlane(T.ev_beg);
            ev_end = e1 + __builtin_amdgcn_readfirstlane(T.ev_cnt);
            if (e1 < ev_end) {
                ez1 = __builtin_amdgcn_readfirstlane(evrows[e1].z);
                eo1 = __builtin_amdgcn_readfirstlane(evrows[e1].vec_off);
            }
            e2 = e1;
            while (e2 < ev_end) {
                ez2 = __builtin_amdgcn_readfirstlane(evrows[e2].z);
                if (ez2 >= z0) break;
                ++e2;
            }
            if (e2 < ev_end)
                eo2 = __builtin_amdgcn_readfirstlane(evrows[e2].vec_off);
            else
                ez2 = kNoRow;
        }

#pragma unroll
        for (int i = 0; i < R1; ++i) {
            const int z1 = zs - kHalo + i;
            q[i + 8 + PF] = bload(rU, coff(z1 + kHalo + PF));
            hq[i + PF] = bload(rU, hoff(z1 + PF));
            pq[i + PF] = bload(rP, coff(z1 + PF));
            // W^{k-1} of own row z0 + r is used at i = r + 4, W^{k-2} at i = r + 8: both are
            // fetched 4 rows ahead, by the strip's own lanes only (the margin lanes' products
            // are never used, so their loads are poisoned and fetch nothing)
            if (i < BZ) wq1[i] = bload_nt(rW, roff(zs + i) + sb);
            if (i >= kHalo && i - kHalo < BZ) wq2[i - kHalo] = bload_nt(rW2, roff(zs + i - kHalo) + sb);

            // both steps' x rows go to LDS before one wave-scope fence
            float *row = rows[wave][i & 1];
            float *row1 = rows1[wave][i & 1];
            row[lane + kHalo] = q[i + 4];
            if (lane < 4)
                row[lane] = hq[i];
            else if (lane < 8)
                row[kTileX + lane] = hq[i];
            if (i >= 2 * kHalo) row1[lane + kHalo] = s1[i - 4];
            wave_lds_sync();
            {
                float lx = wx[0] * q[i + 4];
                lx += wx[1] * (row[lane + 3] + row[lane + 5]);
                lx += wx[2] * (row[lane + 2] + row[lane + 6]);
                lx += wx[3] * (row[lane + 1] + row[lane + 7]);
                lx += wx[4] * (row[lane + 0] + row[lane + 8]);
                float lz = wz[0] * q[i + 4];
                lz += wz[1] * (q[i + 3] + q[i + 5]);
                lz += wz[2] * (q[i + 2] + q[i + 6]);
                lz += wz[3] * (q[i + 1] + q[i + 7]);
                lz += wz[4] * (q[i + 0] + q[i + 8]);
                float wv = lz + lx;
                const float2 ab = abt[sidx][i][lane];
                if (z1 == ez1) {  // uniform
                    const int rid = evvec[eo1 + lane];
                    if (rid >= 0 && Rho1) wv += Rho1[rid];
                    ++e1;
                    ez1 = e1 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e1].z) : kNoRow;
                    eo1 = e1 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e1].vec_off) : 0;
                }
                const float un = ab.x * q[i + 4] - ab.y * pq[i] + cr[i] * wv;
                s1[i] = un;
                if (i >= kHalo && i < BZ + kHalo) {
                    bstore(rN, soff(z1), un);
                    acc[i - kHalo] += (double)un * (double)wq1[i - kHalo];
                }
            }
            if (i >= 2 * kHalo) {
                const int z2 = z1 - kHalo;
                const float *row = row1;
                float lx = wx[0] * s1[i - 4];
                lx += wx[1] * (row[lane + 3] + row[lane + 5]);
                lx += wx[2] * (row[lane + 2] + row[lane + 6]);
                lx += wx[3] * (row[lane + 1] + row[lane + 7]);
                lx += wx[4] * (row[lane + 0] + row[lane + 8]);
                float lz = wz[0] * s1[i - 4];
                lz += wz[1] * (s1[i - 5] + s1[i - 3]);
                lz += wz[2] * (s1[i - 6] + s1[i - 2]);
                lz += wz[3] * (s1[i - 7] + s1[i - 1]);
                lz += wz[4] * (s1[i - 8] + s1[i - 0]);
                float wv = lz + lx;
                const float2 ab = abt[sidx][i - kHalo][lane];
                if (z2 == ez2) {  // uniform
                    const int rid = evvec[eo2 + lane];
                    if (rid >= 0 && Rho2) wv += Rho2[rid];
                    ++e2;
                    ez2 = e2 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e2].z) : kNoRow;
                    eo2 = e2 < ev_end ? __builtin_amdgcn_readfirstlane(evrows[e2].vec_off) : 0;
                }
                const float un = ab.x * s1[i - 4] - ab.y * q[i] + cr[i - 4] * wv;
                bstore(rN2, soff(z2), un);
                acc[i - 2 * kHalo] += (double)un * (double)wq2[i - 2 * kHalo];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // each strip's wave sums, in wave order (every wave joins every barrier)
    for (int w = 1; w < wps; ++w) {
        __syncthreads();
        if (wl == w)
#pragma unroll
            for (int r = 0; r < BZ; ++r) red[sidx][r][lane] = acc[r];
        __syncthreads();
        if (wl == 0)
#pragma unroll
            for (int r = 0; r < BZ; ++r) acc[r] += red[sidx][r][lane];
    }
    if (wl == 0 && active) {
        const rsrc_t rG = make_rsrc(A.gacc + g_off, 2 * fbytes);
        const bool own = xin && mine;
        double g[BZ];
#pragma unroll
        for (int r = 0; r < BZ; ++r) g[r] = bload64(rG, (own && r < nrow) ? 2 * (roff(z0 + r) + xo) : kOOB);
#pragma unroll
        for (int r = 0; r < BZ; ++r)
            bstore64(rG, (own && r < nrow) ? 2 * (roff(z0 + r) + xo) : kOOB, g[r] + acc[r]);
    }
}

// ------------------------------------------------------------ 3D stepping

// 3D step.  A workgroup of kWaves3 = 8 wavefronts owns a tile of WX x-cells (WX = 64 or
// 32), TY = 8 * RW rows (RW = 64 / WX rows per wavefront) and BZ planes, and streams it
// along z.  Wavefront w holds rows w * RW .. w * RW + RW - 1, lane l the cell
// (l % WX, l / WX) of them.  The host picks the width that leaves fewer lanes idle on the
// batch's grids: a padded x extent of 220 cells runs on 224 lanes per row with 32-wide
// tiles instead of 256 with 64-wide ones.  The xy plane (tile plus a 4-cell halo in x
// and y) goes through a double-buffered LDS plane with one barrier per plane: every
// wavefront writes its own cells, the first 8 / RW wavefronts one y-halo row each per
// lane row, lanes with l % WX < 8 the x-halo cells of their row.  The z-derivative comes
// from a register queue that runs 8 planes ahead; halo and point operands are fetched 4
// planes ahead with unconditional buffer loads.
//
// The sweep is bound by instruction issue, not by HBM bandwidth: its time follows the
// number of lanes it runs, not the bytes it moves.  So it keeps instructions per cell low:
// the plane loop is fully unrolled (queues shift by register renaming), every lane offset
// carries a poison bit instead of a per-access select, the sponge coefficients a, b of
// planes outside the z-sponge are computed once per column, the optional stores are fixed
// per kernel instance (MODE) instead of tested per plane, and source terms are looked for
// only in tiles that hold sources.

constexpr int kWaves3 = 8;  // wavefronts per 3D workgroup

// Stores of a forward launch besides u^{n+1}: none, the checkpoint pair (u^{n+1}, u^n),
// or the imaging operand W^n = L u^n + q^n.
enum : int { kStorePlain = 0, kStoreCkpt = 1, kStoreImage = 2 };

// Cells into the sponge of padded index p on an axis with n physical cells (0 inside).
__device__ __forceinline__ int sponge_depth(int p, int n, int nb)
{
    return p < nb ? nb - p : (p > nb + n - 1 ? p - (nb + n - 1) : 0);
}
// gmax (d/nb)^2, rounded exactly as sponge_axis rounds it (d != 0)
__device__ __forceinline__ double sponge_of_depth(int d, int nb, double gmax)
{
#pragma clang fp contract(off)
    double r = (double)d / (double)nb;
    return gmax * r * r;
}

// Lane geometry of a 3D tile shared by the forward and adjoint sweeps.
template <int WX>
struct Lanes3 {
    static constexpr int RW = kTileX / WX;       // rows per wavefront
    static constexpr int TY = kWaves3 * RW;      // rows per tile
    static constexpr int NHW = 2 * kHalo / RW;   // wavefronts that load the 8 y-halo rows
    static constexpr int LX = WX + 2 * kHalo;    // LDS row length
    static constexpr int LY = TY + 2 * kHalo + RW;  // LDS rows (+ RW spare rows)
    int lc, ry, x, y;        // lane's column and row in the tile, cell coordinates
    bool in;                 // the cell lies in the grid
    bool row;                // the cell lies in a row of the grid (x below the row pitch)
    uint32_t col, cb, sb;    // byte offset of (y, x) in a plane; poisoned copies for loads
                             // (cells of the grid) and for stores (cells of its rows)
    uint32_t hyb, hxb;       // poisoned offsets of the lane's y- and x-halo cells
    int hrow, hcol, hxrow;   // LDS row of the y-halo cell, column and row of the x-halo cell
    __device__ __forceinline__ Lanes3(int tx0, int ty0, int Nx, int Ny, int P)
    {
        const int lane = threadIdx.x & 63;
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lr = lane / WX;
        lc = lane % WX;
        ry = w * RW + lr;
        x = tx0 + lc;
        y = ty0 + ry;
        in = x < Nx && y < Ny;
        row = x < P && y < Ny;
        col = 4u * ((uint32_t)min(y, Ny - 1) * (uint32_t)P + (uint32_t)min(x, P - 1));
        cb = in ? col : kPoison;
        sb = row ? col : kPoison;
        // y halo: rows ty0-4 .. ty0-1, then ty0+TY .. ty0+TY+3, RW per wavefront; the
        // other wavefronts load nothing and write a spare LDS row
        const int hr = w * RW + lr;
        const bool hw = w < NHW;
        const int hy = hr < kHalo ? ty0 - kHalo + hr : ty0 + TY + hr - kHalo;
        hrow = hw ? (hr < kHalo ? hr : TY + hr) : TY + 2 * kHalo + lr;
        const bool hyl = hw && x < Nx && hy >= 0 && hy < Ny;
        hyb = hyl ? 4u * ((uint32_t)min(max(hy, 0), Ny - 1) * (uint32_t)P + (uint32_t)min(x, Nx - 1)) : kPoison;
        // x halo of the lane's row: columns tx0-4 .. tx0-1 (lc 0..3), tx0+WX .. +3 (lc 4..7);
        // the other lanes load nothing and write a spare LDS row
        const int hxx = lc < kHalo ? tx0 - kHalo + lc : tx0 + WX + lc - kHalo;
        hcol = lc < kHalo ? lc : WX + lc;
        hxrow = lc < 2 * kHalo ? ry + kHalo : TY + 2 * kHalo + lr;
        if (lc >= 2 * kHalo) hcol = lc;
        const bool hxl = lc < 2 * kHalo && y < Ny && hxx >= 0 && hxx < Nx;
        hxb = hxl ? 4u * ((uint32_t)min(y, Ny - 1) * (uint32_t)P + (uint32_t)min(max(hxx, 0), Nx - 1)) : kPoison;
    }
};

// The 8th-order Laplacian of one cell from the LDS plane (x and y) and the z queue
// qq[0..8] (qq[4] = the cell), summed per axis and then z + y + x.
template <int LX>
__device__ __forceinline__ float lap3(const float (*L)[LX], int ly, int lx, const float *qq, const float *wx,
                                      const float *wy, const float *wz)
{
    float sx = wx[0] * qq[4];
    sx += wx[1] * (L[ly][lx - 1] + L[ly][lx + 1]);
    sx += wx[2] * (L[ly][lx - 2] + L[ly][lx + 2]);
    sx += wx[3] * (L[ly][lx - 3] + L[ly][lx + 3]);
    sx += wx[4] * (L[ly][lx - 4] + L[ly][lx + 4]);
    float sy = wy[0] * qq[4];
    sy += wy[1] * (L[ly - 1][lx] + L[ly + 1][lx]);
    sy += wy[2] * (L[ly - 2][lx] + L[ly + 2][lx]);
    sy += wy[3] * (L[ly - 3][lx] + L[ly + 3][lx]);
    sy += wy[4] * (L[ly - 4][lx] + L[ly + 4][lx]);
    float sz = wz[0] * qq[4];
    sz += wz[1] * (qq[3] + qq[5]);
    sz += wz[2] * (qq[2] + qq[6]);
    sz += wz[3] * (qq[1] + qq[7]);
    sz += wz[4] * (qq[0] + qq[8]);
    return sz + sy + sx;
}

// 3D forward step: one tile of one sim per workgroup.  MODE selects the extra stores.
template <int WX, int BZ, int MODE>
__global__ __launch_bounds__(64 * kWaves3) void k_fwd3d(const StepArgs A)
{
    using G = Lanes3<WX>;
    constexpr int PF = 4;
    const int slot = xcd_tile(blockIdx.x, A.per_xcd);
    if (slot >= A.ntiles) return;  // uniform per block
    // the launch order takes a sample's supergathers at one tile position in a row, so
    // that the sample's coefficient grid is read from L2 by all but the first of them
    const int t = A.order ? A.order[slot] : slot;
    const Tile T = A.tiles[t];
    const SimDesc &S = A.sims[T.sim];
    __shared__ float V[2][G::LY][G::LX];
    const int Nx = S.N[2], Ny = S.N[1], Nz = S.N[0];
    const int nz_phys = S.n[0], ny_phys = S.n[1], nx_phys = S.n[2], nb = S.nb;
    const double gmz = S.gmax[0];
    const int src_beg = S.src_beg, src_cnt = S.src_cnt;
    const uint32_t pbytes = 4u * (uint32_t)S.px * (uint32_t)Ny;
    const uint32_t fbytes = pbytes * (uint32_t)Nz;
    const int z0 = T.z0;
    const G g(T.x0, T.y0, Nx, Ny, S.px);
    const int64_t u_off = S.u_off;
    const rsrc_t rU = make_rsrc(A.cur + u_off, fbytes);
    const rsrc_t rP = make_rsrc(A.prev + u_off, fbytes);
    const rsrc_t rN = make_rsrc(A.next + u_off, fbytes);
    const rsrc_t rC = make_rsrc(A.cf + S.c_off, fbytes);
    const rsrc_t rW = make_rsrc(MODE == kStoreImage ? A.wst + u_off : A.next, MODE == kStoreImage ? fbytes : 0);
    const rsrc_t rKa = make_rsrc(MODE == kStoreCkpt ? A.cka + u_off : A.next, MODE == kStoreCkpt ? fbytes : 0);
    const rsrc_t rKb = make_rsrc(MODE == kStoreCkpt ? A.ckb + u_off : A.next, MODE == kStoreCkpt ? fbytes : 0);
    const int rec_j = A.rec_j;
    float *Dat = (A.dat && rec_j >= 0) ? A.dat + S.d_off + (int64_t)rec_j * S.nrec : nullptr;
    const EvRow *__restrict__ evrows = A.evrows;
    const int32_t *__restrict__ evvec = A.evvec;

    float wz[5], wy[5], wx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        wz[k] = S.w[0][k];
        wy[k] = S.w[1][k];
        wx[k] = S.w[2][k];
    }
    const double dt = S.dt;
    const double gx = sponge_axis(g.x, nx_phys, nb, S.gmax[2]);
    const double gy = sponge_axis(g.y, ny_phys, nb, S.gmax[1]);
    float a_col, b_col;  // a, b of this column outside the z-sponge
    {
        double gam = 0.0;
        gam = gam + gy;
        gam = gam + gx;
        sponge_ab(gam, dt, a_col, b_col);
    }
    auto poff = [&](int zz) -> uint32_t { return (uint32_t)zz * pbytes; };  // zz < 0 wraps out of range
    const uint32_t cb = g.cb, sb = g.sb, hyb = g.hyb, hxb = g.hxb;

    // sources in this thread's column
    const int z1 = min(z0 + BZ, Nz);
    int sz = -1;
    float sw = 0.0f;
    bool smulti = false;
    const float famp = A.fn * S.inv_vol;
    for (int s = 0; s < src_cnt; ++s) {
        const SrcPos p = A.src[src_beg + s];
        if (p.x != g.x || p.y != g.y || p.z < z0 || p.z >= z1) continue;
        if (sz < 0 || sz == p.z) {
            sz = p.z;
            sw += p.w;
        } else {
            smulti = true;
        }
    }
    const bool has_src = __syncthreads_or(sz >= 0);
    const bool multi = __syncthreads_or(smulti);

    // z-sponge gamma of the tile's planes, one lane per plane: a sponge plane reads it
    // instead of every lane dividing by nb again (same value, same rounding)
    __shared__ double gzs[BZ];
    if (threadIdx.x < BZ) gzs[threadIdx.x] = sponge_of_depth(sponge_depth(z0 + threadIdx.x, nz_phys, nb), nb, gmz);

    // queues indexed by plane (the plane loop is fully unrolled)
    float q[BZ + 12], cq[BZ + PF], pq[BZ + PF], hyq[BZ + PF], hxq[BZ + PF];
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = bload(rU, poff(z0 - kHalo + k) + cb);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const uint32_t pz = poff(z0 + k);
        hyq[k] = bload(rU, pz + hyb);
        hxq[k] = bload(rU, pz + hxb);
        cq[k] = bload(rC, pz + cb);
        pq[k] = bload_nt(rP, pz + cb);
    }
    int ev = T.ev_beg;
    const int ev_end = T.ev_beg + T.ev_cnt;
    int ev_z = (rec_j >= 0 && ev < ev_end) ? __builtin_amdgcn_readfirstlane(evrows[ev].z) : -1;
    int ev_off = (rec_j >= 0 && ev < ev_end) ? __builtin_amdgcn_readfirstlane(evrows[ev].vec_off) : 0;
    const int ly = g.ry + kHalo, lx = g.lc + kHalo;

    // planes below the grid are swept too: their loads read 0 and their stores fall
    // outside the buffers, so the tile needs no plane guard
#pragma unroll
    for (int r = 0; r < BZ; ++r) {
        const int z = z0 + r;
        // ---- prefetch: centre plane z+8, halos and point operands of plane z+4
        q[r + 12] = bload(rU, poff(z + 8) + cb);
        {
            const uint32_t pz = poff(z + PF);
            hyq[r + PF] = bload(rU, pz + hyb);
            hxq[r + PF] = bload(rU, pz + hxb);
            cq[r + PF] = bload(rC, pz + cb);
            pq[r + PF] = bload_nt(rP, pz + cb);
        }
        // ---- plane z into LDS
        float(*L)[G::LX] = V[r & 1];
        L[ly][lx] = q[r + 4];
        L[g.hrow][lx] = hyq[r];
        L[g.hxrow][g.hcol] = hxq[r];
        __syncthreads();

        const float *qq = &q[r];  // qq[4] is plane z
        float wv = lap3<G::LX>(L, ly, lx, qq, wx, wy, wz);
        float a = a_col, b = b_col;
        if ((unsigned)(z - nb) >= (unsigned)nz_phys) {  // uniform: a z-sponge plane
            double gam = 0.0;
            gam = gam + gzs[r];  // written before the plane loop's first barrier
            gam = gam + gy;
            gam = gam + gx;
            sponge_ab(gam, dt, a, b);
        }
        if (has_src) {  // uniform
            if (z == sz) wv += sw * famp;
            if (multi) {
                float extra = 0.0f;
                if (g.in)
                    for (int s = 0; s < src_cnt; ++s) {
                        const SrcPos p = A.src[src_beg + s];
                        if (p.x == g.x && p.y == g.y && p.z == z && z != sz) extra += p.w;
                    }
                wv += extra * famp;
            }
        }
        // stores cover the whole row pitch (zeros past the grid's rows), so that every
        // line is written whole
        const uint32_t o = poff(z) + sb;
        const float un = g.in ? a * qq[4] - b * pq[r] + cq[r] * wv : 0.0f;
        bstore_nt(rN, o, un);
        if (MODE == kStoreImage) bstore_nt(rW, o, g.in ? wv : 0.0f);
        if (MODE == kStoreCkpt) {
            bstore_nt(rKa, o, un);
            bstore_nt(rKb, o, qq[4]);  // 0 past the grid (its loads are poisoned)
        }
        if (z == ev_z) {  // uniform
            if (Dat) {
                const int rid = evvec[ev_off + threadIdx.x];
                if (rid >= 0) Dat[rid] = un;
            }
            ++ev;
            ev_z = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].z) : -1;
            ev_off = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].vec_off) : 0;
        }
        // keep each plane's loads in its own plane (prefetch distance PF planes)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// 3D adjoint + imaging step with the imaging sum taken per sample.  A workgroup (lanes as
// in the forward) owns one WX x TY x BZ tile of a sample's grid and sweeps it for each of
// the sample's sims in turn; every thread keeps the FP64 sum over sims of its cells' exact
// products lt^k W^{k-1} in LDS and applies one read-modify-write to the sample's
// accumulator at the end, so the accumulator costs 16 B per sample cell and step instead
// of 16 B per sim cell.  Per cell the sum runs over the sims in order and then into the
// accumulator step by step: the result does not depend on tile shapes or the schedule.
// Consecutive sims reuse the double-buffered plane without an extra barrier: a slot is
// rewritten only after every wave has passed the barrier of the plane that follows its
// last read.
template <int WX, int BZ>
__global__ __launch_bounds__(64 * kWaves3) void k_adj3d(const StepArgs A)
{
    using G = Lanes3<WX>;
    constexpr int PF = 4;
    const int gt = xcd_tile(blockIdx.x, A.per_xcd_g);
    if (gt >= A.ngtiles) return;  // uniform per block
    // sample-level descriptors are read before the first store (scalar loads)
    const GTile GT = A.gtiles[gt];
    const SampleDesc &Sm = A.samples[GT.sample];
    const int Nx = Sm.N[2], Ny = Sm.N[1], Nz = Sm.N[0];
    const int nz_phys = Sm.n[0], ny_phys = Sm.n[1], nx_phys = Sm.n[2], nb = Sm.nb;
    const double gmz = Sm.gmax[0];
    const double dt = Sm.dt;
    const int sim_beg = Sm.sim_beg, sim_cnt = Sm.sim_cnt;
    if (sim_cnt == 0) return;  // uniform per block: a sample without sims adds nothing
    const int64_t ncell = Sm.ncell, g_off = Sm.g_off;
    const SimDesc &S0 = A.sims[sim_beg];
    const int64_t u_off0 = S0.u_off;  // sims of a sample are consecutive, ncell apart
    float wz[5], wy[5], wx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        wz[k] = S0.w[0][k];
        wy[k] = S0.w[1][k];
        wx[k] = S0.w[2][k];
    }
    const uint32_t pbytes = 4u * (uint32_t)Sm.px * (uint32_t)Ny;
    const uint32_t fbytes = pbytes * (uint32_t)Nz;
    const int z0 = GT.z0;
    const G g(GT.x0, GT.y0, Nx, Ny, Sm.px);
    const rsrc_t rC = make_rsrc(A.cf + Sm.c_off, fbytes);
    const int rec_j = A.rec_j;
    const EvRow *__restrict__ evrows = A.evrows;
    const int32_t *__restrict__ evvec = A.evvec;

    const double gx = sponge_axis(g.x, nx_phys, nb, Sm.gmax[2]);
    const double gy = sponge_axis(g.y, ny_phys, nb, Sm.gmax[1]);
    float a_col, b_col;  // a, b of this column outside the z-sponge
    {
        double gam = 0.0;
        gam = gam + gy;
        gam = gam + gx;
        sponge_ab(gam, dt, a_col, b_col);
    }
    auto poff = [&](int zz) -> uint32_t { return (uint32_t)zz * pbytes; };  // zz < 0 wraps out of range
    const int ly = g.ry + kHalo, lx = g.lc + kHalo;

    __shared__ float V[2][G::LY][G::LX];
    __shared__ double red[BZ][G::TY][WX];
    // c of the tile's planes, read once for all of the sample's supergathers
    float cr[BZ];
#pragma unroll
    for (int r = 0; r < BZ; ++r) cr[r] = bload(rC, poff(z0 + r) + g.cb);

    for (int j = 0; j < sim_cnt; ++j) {
        const int sim = sim_beg + j;
        const int64_t u_off = u_off0 + (int64_t)j * ncell;
        const rsrc_t rU = make_rsrc(A.cur + u_off, fbytes);
        const rsrc_t rP = make_rsrc(A.prev + u_off, fbytes);
        const rsrc_t rN = make_rsrc(A.next + u_off, fbytes);
        const rsrc_t rW = make_rsrc(A.wimg + u_off, fbytes);
        // lane offsets pass through an empty asm so that the plane offsets built from them
        // are recomputed per sim next to their loads, not hoisted out of the sim loop
        uint32_t cbs = g.cb, sbs = g.sb, hybs = g.hyb, hxbs = g.hxb;
        asm volatile("" : "+v"(cbs), "+v"(sbs), "+v"(hybs), "+v"(hxbs));
        // per-sim fields read after stores: vector loads, made uniform explicitly
        const int tile0 = __builtin_amdgcn_readfirstlane(A.sims[sim].tile0);
        const int nrec = __builtin_amdgcn_readfirstlane(A.sims[sim].nrec);
        const int64_t d_off = A.sims[sim].d_off;
        const int d_lo = __builtin_amdgcn_readfirstlane((int)(d_off & 0xFFFFFFFF));
        const int d_hi = __builtin_amdgcn_readfirstlane((int)(d_off >> 32));
        const int64_t d_off_u = (int64_t)(((uint64_t)(uint32_t)d_hi << 32) | (uint32_t)d_lo);
        const float *Rho = rec_j >= 0 ? A.rho + d_off_u + (int64_t)rec_j * nrec : nullptr;
        // receiver event planes of the sim tile that holds plane z0, from plane z0 on (a
        // sim tile may be taller than BZ), then those of the next sim tile in z where this
        // tile reaches into it (event planes are in increasing z within a sim tile)
        int ev = 0, ev_end = 0, ev_z = -1, ev_off = 0, ev2 = 0, ev2_end = 0;
        if (rec_j >= 0) {
            const Tile &T = A.tiles[tile0 + GT.tix];
            ev = __builtin_amdgcn_readfirstlane(T.ev_beg);
            ev_end = ev + __builtin_amdgcn_readfirstlane(T.ev_cnt);
            if (GT.tix2 >= 0) {
                const Tile &T2 = A.tiles[tile0 + GT.tix2];
                ev2 = __builtin_amdgcn_readfirstlane(T2.ev_beg);
                ev2_end = ev2 + __builtin_amdgcn_readfirstlane(T2.ev_cnt);
            }
            while (ev < ev_end && __builtin_amdgcn_readfirstlane(evrows[ev].z) < z0) ++ev;
            if (ev == ev_end) {
                ev = ev2;
                ev_end = ev2_end;
                ev2 = ev2_end;
            }
            if (ev < ev_end) {
                ev_z = __builtin_amdgcn_readfirstlane(evrows[ev].z);
                ev_off = __builtin_amdgcn_readfirstlane(evrows[ev].vec_off);
            }
        }

        float q[BZ + 12], pq[BZ + PF], wq[BZ + PF], hyq[BZ + PF], hxq[BZ + PF];
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = bload(rU, poff(z0 - kHalo + k) + cbs);
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const uint32_t pz = poff(z0 + k);
            hyq[k] = bload(rU, pz + hybs);
            hxq[k] = bload(rU, pz + hxbs);
            pq[k] = bload_nt(rP, pz + cbs);
            wq[k] = bload_nt(rW, pz + cbs);
        }
        // planes below the grid are swept too: their loads read 0 and their stores fall
        // outside the buffers
#pragma unroll
        for (int r = 0; r < BZ; ++r) {
            const int z = z0 + r;
            q[r + 12] = bload(rU, poff(z + 8) + cbs);
            {
                const uint32_t pz = poff(z + PF);
                hyq[r + PF] = bload(rU, pz + hybs);
                hxq[r + PF] = bload(rU, pz + hxbs);
                pq[r + PF] = bload_nt(rP, pz + cbs);
                wq[r + PF] = bload_nt(rW, pz + cbs);
            }
            float(*L)[G::LX] = V[r & 1];
            L[ly][lx] = q[r + 4];
            L[g.hrow][lx] = hyq[r];
            L[g.hxrow][g.hcol] = hxq[r];
            __syncthreads();

            const float *qq = &q[r];  // qq[4] is plane z
            float wv = lap3<G::LX>(L, ly, lx, qq, wx, wy, wz);
            float a = a_col, b = b_col;
            if ((unsigned)(z - nb) >= (unsigned)nz_phys) {  // uniform: a z-sponge plane
                double gam = 0.0;
                gam = gam + sponge_of_depth(sponge_depth(z, nz_phys, nb), nb, gmz);
                gam = gam + gy;
                gam = gam + gx;
                sponge_ab(gam, dt, a, b);
            }
            if (z == ev_z) {  // uniform
                const int rid = evvec[ev_off + threadIdx.x];
                if (rid >= 0) wv += Rho[rid];
                if (++ev == ev_end) {
                    ev = ev2;
                    ev_end = ev2_end;
                    ev2 = ev2_end;
                }
                ev_z = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].z) : -1;
                ev_off = ev < ev_end ? __builtin_amdgcn_readfirstlane(evrows[ev].vec_off) : 0;
            }
            const float un = a * qq[4] - b * pq[r] + cr[r] * wv;
            bstore_nt(rN, poff(z) + sbs, g.in ? un : 0.0f);  // whole lines, as in the forward
            const double pr = (double)un * (double)wq[r];  // the product of two floats is exact in FP64
            red[r][g.ry][g.lc] = j == 0 ? pr : red[r][g.ry][g.lc] + pr;
            // keep each plane's loads in its own plane (prefetch distance PF planes)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // one read-modify-write of the sample's accumulator per cell (cells outside the grid:
    // poisoned or out-of-range offsets, so the load reads 0 and the store is dropped)
    const rsrc_t rG = make_rsrc(A.gacc + g_off, 2 * fbytes);
    const uint32_t cb2 = g.in ? 2u * g.col : kPoison, sb2 = g.row ? 2u * g.col : kPoison;
#pragma unroll
    for (int r = 0; r < BZ; ++r) {
        const uint32_t o = 2u * poff(z0 + r);
        bstore64(rG, o + sb2, bload64(rG, o + cb2) + red[r][g.ry][g.lc]);  // 0 past the grid
    }
}

// ---------------------------------------------------------- misfit/residual

// Sum of one double per thread of a 256-thread block in a fixed order: each wavefront
// folds its 64 lanes with cross-lane moves (offsets 32, 16, ..., 1), then thread 0 adds
// the four wavefront sums in wave order.  The result is valid in thread 0.
__device__ __forceinline__ double block_sum256(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    return threadIdx.x == 0 ? ((part[0] + part[1]) + part[2]) + part[3] : 0.0;
}

// Block (chunk, sim): rho = (d - d_obs) inv_sigma2 and a partial sum of (d - d_obs)^2.
__global__ __launch_bounds__(256) void k_residual(const SimDesc *__restrict__ sims, int nt_rec,
                                                  const float *d, const float *__restrict__ dobs,
                                                  float *rho, float inv_sigma2,
                                                  double *__restrict__ partial, int nchunk,
                                                  int *__restrict__ status)
{
    const SimDesc &S = sims[blockIdx.y];
    const int64_t n = (int64_t)nt_rec * S.nrec;
    const int64_t per = (n + nchunk - 1) / nchunk;
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = min(beg + per, n);
    double acc = 0.0;
    int bad = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const float r = d[S.d_off + i] - dobs[S.d_off + i];
        if (!isfinite(r)) bad = 1;
        rho[S.d_off + i] = r * inv_sigma2;
        acc += (double)r * (double)r;
    }
    const double sum = block_sum256(acc);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * nchunk + blockIdx.x] = sum;
    if (bad) atomicOr(status, 2);
}

__global__ void k_misfit_final(const double *__restrict__ partial, int nchunk, int nsim, double half_is2,
                               double *__restrict__ misfit)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsim) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += partial[(int64_t)s * nchunk + c];
    misfit[s] = half_is2 * acc;
}

// ------------------------------------------------------------- finalize

// grad[s][cell] = kappa_s (2 / v) sum_{sims of s} sum_{padded cells replicating cell} g;
// block (chunk, sample) also leaves a partial sum of grad^2.
__global__ __launch_bounds__(256) void k_finalize(const SampleDesc *__restrict__ smp, const SimDesc *__restrict__ sims,
                                                  const double *__restrict__ gacc, const float *__restrict__ v,
                                                  float *__restrict__ grad, double *__restrict__ partial,
                                                  int nchunk, int *__restrict__ status)
{
    const SampleDesc S = smp[blockIdx.y];
    const int nx = S.n[2], ny = S.n[1], nz = S.n[0];
    const int Nx = S.N[2], Ny = S.N[1];
    const int nby = S.ndim == 3 ? S.nb : 0;
    const int64_t per = (S.nphys + nchunk - 1) / nchunk;
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = min(beg + per, S.nphys);
    double acc2 = 0.0;
    int bad = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const int ix = (int)(i % nx);
        const int64_t rr = i / nx;
        const int iy = (int)(rr % ny);
        const int iz = (int)(rr / ny);
        const int xl = ix == 0 ? 0 : ix + S.nb, xh = ix == nx - 1 ? Nx - 1 : ix + S.nb;
        const int yl = iy == 0 ? 0 : iy + nby, yh = iy == ny - 1 ? Ny - 1 : iy + nby;
        const int zl = iz == 0 ? 0 : iz + S.nb, zh = iz == nz - 1 ? S.N[0] - 1 : iz + S.nb;
        double sum = 0.0;
        for (int s = 0; s < S.g_cnt; ++s) {
            const double *g = gacc + S.g_off + (int64_t)s * S.ncell;
            for (int pz = zl; pz <= zh; ++pz)
                for (int py = yl; py <= yh; ++py) {
                    const int64_t base = ((int64_t)pz * Ny + py) * S.px;
                    for (int px = xl; px <= xh; ++px) sum += g[base + px];
                }
        }
        const double val = S.kappa * (2.0 / (double)v[S.m_off + i]) * sum;
        const float gv = (float)val;
        if (!isfinite(gv)) bad = 1;
        grad[S.m_off + i] = gv;
        acc2 += (double)gv * (double)gv;
    }
    const double sum = block_sum256(acc2);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * nchunk + blockIdx.x] = sum;
    if (bad) atomicOr(status, 4);
}

__global__ void k_norm_final(const double *__restrict__ partial, int nchunk, int nsample, float *__restrict__ norm)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsample) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += partial[(int64_t)s * nchunk + c];
    norm[s] = (float)sqrt(acc);
}

// ----------------------------------------------------------------- encode

__global__ __launch_bounds__(256) void k_encode(const float *__restrict__ d, int nshot, int64_t nper,
                                                const int32_t *__restrict__ gp, const int32_t *__restrict__ gs,
                                                const float *__restrict__ gw, int n_entries, float *__restrict__ out)
{
    const int g = blockIdx.y;
    const int b = gp[g], e = gp[g + 1];
    // a malformed group table poisons the group's output instead of reading out of bounds
    bool ok = b >= 0 && e >= b && e <= n_entries;
    for (int k = b; ok && k < e; ++k) ok = gs[k] >= 0 && gs[k] < nshot;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < nper; i += stride) {
        float acc = ok ? 0.0f : __builtin_nanf("");
        if (ok)
            for (int k = b; k < e; ++k) acc += gw[k] * d[(int64_t)gs[k] * nper + i];
        out[(int64_t)g * nper + i] = acc;
    }
}

// --------------------------------------------------------------- Langevin

// One thread per group of 4 cells of one sample's model (n cells at v, g, xi).
__global__ __launch_bounds__(256) void k_langevin(int64_t n, float *__restrict__ v, const float *__restrict__ g,
                                                  const float *__restrict__ xi, uint64_t seed, uint64_t step,
                                                  uint64_t sample, double eta, double nu, double lo, double hi)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * m >= n) return;
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (xi == nullptr) normals4((uint64_t)m, step, sample, seed, 0x4C414E47ULL, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = 4 * m + j;
        if (i >= n) break;
        const double xv = xi ? (double)xi[i] : z[j];
        double y = (double)v[i] - eta * (double)g[i] + nu * xv;
        y = y < lo ? lo : y;
        y = y > hi ? hi : y;
        v[i] = (float)y;
    }
}

// ------------------------------------------------------------- copy probe

// Plain streaming copy: one 16-byte vector per thread, one short-lived workgroup per 4 KB
// (measured faster than grid-stride loops, which keep fewer requests in flight per
// wavefront).  The achievable-bandwidth reference and the byte-counter calibration kernel.
__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ s, float4 *__restrict__ d, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) d[i] = s[i];
}

// ------------------------------------------------------------ launchers

static inline int blocks_for(int64_t n, int bs, int cap)
{
    int64_t b = (n + bs - 1) / bs;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t launch_copy(const float *src, float *dst, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n / 4 + 255) / 256;
    if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    k_copy<<<(unsigned)nb, 256, 0, st>>>((const float4 *)src, (float4 *)dst, n / 4);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_fill<float><<<blocks_for(n, 256, 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_fill<double><<<blocks_for(n, 256, 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int64_t n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_fill<int><<<blocks_for(n, 256, 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_prep(const SampleDesc *smp, int nsample, int64_t max_cell, const float *v, float *cf, int *status,
                       hipStream_t st)
{
    dim3 grid(blocks_for(max_cell, 256, 4096), nsample);
    k_prep<<<grid, 256, 0, st>>>(smp, v, cf, status);
    return hipGetLastError();
}

static hipError_t fwd2d_dispatch(const StepArgs &a, int bz, hipStream_t st)
{
    // per_xcd counts workgroups of 4 tiles here
    dim3 grid(8 * a.per_xcd);
    switch (bz) {
    case 8: k_fwd2d<8><<<grid, 256, 0, st>>>(a); break;
    case 16: k_fwd2d<16><<<grid, 256, 0, st>>>(a); break;
    case 32: k_fwd2d<32><<<grid, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int WX, int BZ>
static void fwd3d_mode(const StepArgs &a, dim3 grid, hipStream_t st)
{
    if (a.cka)
        k_fwd3d<WX, BZ, kStoreCkpt><<<grid, 64 * kWaves3, 0, st>>>(a);
    else if (a.wst)
        k_fwd3d<WX, BZ, kStoreImage><<<grid, 64 * kWaves3, 0, st>>>(a);
    else
        k_fwd3d<WX, BZ, kStorePlain><<<grid, 64 * kWaves3, 0, st>>>(a);
}

static hipError_t fwd3d_dispatch(const StepArgs &a, int bz, int wx, hipStream_t st)
{
    dim3 grid(8 * a.per_xcd);
    if (a.cka && a.wst) return hipErrorInvalidValue;  // one extra store kind per launch
    // heights 24 and 40 divide depths that 16 and 32 do not (120 padded planes = 3 x 40)
    switch (wx * 100 + bz) {
    case 6416: fwd3d_mode<64, 16>(a, grid, st); break;
    case 6424: fwd3d_mode<64, 24>(a, grid, st); break;
    case 6432: fwd3d_mode<64, 32>(a, grid, st); break;
    case 6440: fwd3d_mode<64, 40>(a, grid, st); break;
    case 3216: fwd3d_mode<32, 16>(a, grid, st); break;
    case 3224: fwd3d_mode<32, 24>(a, grid, st); break;
    case 3232: fwd3d_mode<32, 32>(a, grid, st); break;
    case 3240: fwd3d_mode<32, 40>(a, grid, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t adj3d_dispatch(const StepArgs &a, int wx, hipStream_t st)
{
    dim3 grid(8 * a.per_xcd_g);  // one workgroup per tile of a sample's grid
    if (a.bzg != 16) return hipErrorInvalidValue;
    if (wx == 64)
        k_adj3d<64, 16><<<grid, 64 * kWaves3, 0, st>>>(a);
    else if (wx == 32)
        k_adj3d<32, 16><<<grid, 64 * kWaves3, 0, st>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

static hipError_t adj2d_dispatch(const StepArgs &a, hipStream_t st)
{
    if (a.nw < 1 || a.nw > 16) return hipErrorInvalidValue;
    dim3 grid(8 * a.per_xcd_g);
    switch (a.bzg) {
    case 8: k_adj2d<8><<<grid, 64 * a.nw, 0, st>>>(a); break;
    case 16: k_adj2d<16><<<grid, 64 * a.nw, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, int ndim, bool adjoint, int bz, int wx, hipStream_t st)
{
    if (a.ntiles <= 0) return hipSuccess;
    if (ndim == 2) return adjoint ? adj2d_dispatch(a, st) : fwd2d_dispatch(a, bz, st);
    return adjoint ? adj3d_dispatch(a, wx, st) : fwd3d_dispatch(a, bz, wx, st);
}

// dynamic LDS of the two-step adjoint for nw waves on sg strips: the FP64 wave sums of
// each strip (kRows2 x 64) when a strip has several waves, every wave's x rows of both
// steps (2 x 2 x (64 + 8) floats) and each strip's leapfrog a, b ((kRows2 + 8) x 64 pairs)
static size_t adj2d2_lds_bytes(int nw, int sg)
{
    const size_t red = nw / sg > 1 ? (size_t)sg * kRows2 * kTileX * sizeof(double) : 0;
    return red + (size_t)nw * 4 * (kTileX + 2 * kHalo) * sizeof(float) +
           (size_t)sg * (kRows2 + 2 * kHalo) * kTileX * 2 * sizeof(float);
}

hipError_t launch_step2(const StepArgs &a, bool adjoint, hipStream_t st)
{
    if (a.ntiles <= 0) return hipSuccess;
    if (!a.next2 || a.next2 == a.next || a.next == a.cur || a.next == a.prev || a.next2 == a.cur ||
        a.next2 == a.prev)
        return hipErrorInvalidValue;
    if (adjoint) {
        if (a.nw < 1 || a.nw > 8 || (a.sg != 1 && a.sg != 2) || a.nw % a.sg || !a.wimg || !a.wimg2)
            return hipErrorInvalidValue;
        k_adj2d2<kRows2, kPf2><<<dim3(8 * a.per_xcd_g), 64 * a.nw, adj2d2_lds_bytes(a.nw, a.sg), st>>>(a);
    } else {
        k_fwd2d2<kRows2, kPf2><<<dim3(8 * a.per_xcd), 256, 0, st>>>(a);  // 4 strips per workgroup
    }
    return hipGetLastError();
}

hipError_t launch_residual(const SimDesc *sims, int nsim, int nt_rec, const float *d, const float *dobs, float *rho,
                           float inv_sigma2, double *partial, int nchunk, int *status, hipStream_t st)
{
    dim3 grid(nchunk, nsim);
    k_residual<<<grid, 256, 0, st>>>(sims, nt_rec, d, dobs, rho, inv_sigma2, partial, nchunk, status);
    return hipGetLastError();
}

hipError_t launch_misfit_final(const double *partial, int nchunk, int nsim, double half_is2, double *misfit,
                               hipStream_t st)
{
    k_misfit_final<<<(nsim + 255) / 256, 256, 0, st>>>(partial, nchunk, nsim, half_is2, misfit);
    return hipGetLastError();
}

hipError_t launch_finalize(const SampleDesc *smp, const SimDesc *sims, int nsample, const double *gacc,
                           const float *v, float *grad, double *partial, int nchunk, int *status, hipStream_t st)
{
    dim3 grid(nchunk, nsample);
    k_finalize<<<grid, 256, 0, st>>>(smp, sims, gacc, v, grad, partial, nchunk, status);
    return hipGetLastError();
}

hipError_t launch_norm_final(const double *partial, int nchunk, int nsample, float *norm, hipStream_t st)
{
    k_norm_final<<<(nsample + 255) / 256, 256, 0, st>>>(partial, nchunk, nsample, norm);
    return hipGetLastError();
}

hipError_t launch_encode(const float *d, int nshot, int64_t nper, int ngrp, const int32_t *gp, const int32_t *gs,
                         const float *gw, int n_entries, float *out, hipStream_t st)
{
    dim3 grid(blocks_for(nper, 256, 2048), ngrp);
    k_encode<<<grid, 256, 0, st>>>(d, nshot, nper, gp, gs, gw, n_entries, out);
    return hipGetLastError();
}

hipError_t launch_langevin(int64_t n, float *v, const float *g, const float *xi, uint64_t seed, uint64_t step,
                           uint64_t sample, double eta, double nu, double lo, double hi, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_langevin<<<blocks_for((n + 3) / 4, 256, 1 << 30), 256, 0, st>>>(n, v, g, xi, seed, step, sample, eta, nu,
                                                                      lo, hi);
    return hipGetLastError();
}

}  // namespace fwi
