// fwi_internal.h -- descriptors shared by the host scheduler and the gfx950 kernels.
//
// Layout of the batch on the device: every simulation ("sim") owns one padded grid
// (physical grid plus nb sponge cells on every face) per field level, packed one after
// the other at SimDesc::u_off.  Per-sample arrays (the leapfrog coefficient c = dt^2 v^2 /
// (1 + gamma dt)) are packed at SampleDesc::c_off.  x is the fastest axis, then y, then z.
// Rows are px cells apart: in 3D the padded x extent rounded up to kRowAlign cells (128
// bytes), so that every row starts on a cache line and a 64-cell tile row covers two whole
// lines; the columns past the padded extent hold zeros, written by the step kernels so
// that they store whole lines (a partly written line costs an extra fetch).  In 2D px is
// the padded x extent.
#pragma once
#include <stdint.h>

namespace fwi {

constexpr int kTileX = 64;   // one wavefront spans 64 consecutive x cells (3D: 64 or 32 per row)
constexpr int kHalo = 4;     // 8th-order stencil radius
// Two time steps per launch (2D): a wavefront's 64 lanes hold columns x0 - 4 .. x0 + 59 of
// a strip of kStrip2 columns; strips are kRows2 rows high (forward and adjoint alike).
constexpr int kStrip2 = kTileX - 2 * kHalo;
constexpr int kRows2 = 16;
constexpr int kRowAlign = 32;  // 3D row pitch granule (cells)

struct SimDesc {
    int64_t u_off;      // element offset of this sim in every field level
    int64_t c_off;      // element offset of its sample in the coefficient array
    int64_t d_off;      // element offset of its data [nt_rec][nrec]
    int64_t m_off;      // element offset of its sample's physical model
    int32_t N[3];       // padded dims (z, y, x); y = 1 in 2D
    int32_t n[3];       // physical dims
    int32_t nb;         // sponge cells
    int32_t nrec;       // receivers of this sim
    int32_t src_beg;    // first source (index into the batch source table)
    int32_t src_cnt;    // number of sources
    int32_t sample;     // owning sample
    int32_t ndim;
    int32_t px;         // row pitch (cells)
    float w[3][5];      // stencil weights C_k / h_a^2, axes (z, y, x); zero for an unused axis
    float inv_vol;      // 1 / prod h
    int32_t tile0;      // index of this sim's first tile
    int32_t tile0b;     // 2D: index of its first two-step strip
    double gmax[3];     // sponge gmax per axis (z, y, x); zero for an unused axis
    double dt;
};

struct SampleDesc {
    int64_t m_off;      // physical model / gradient offset
    int64_t c_off;      // padded coefficient offset
    int32_t N[3];
    int32_t n[3];
    int32_t nb;
    int32_t sim_beg;    // first sim of this sample
    int32_t sim_cnt;    // its number of sims
    int32_t ndim;
    double gmax[3];
    double dt;
    double v_max;
    double kappa;
    int64_t nphys;      // physical cells
    int64_t ncell;      // padded cells
    int64_t g_off;      // element offset of its first imaging accumulator slot
    int32_t g_cnt;      // accumulator slots (padded grids of ncell cells, consecutive)
    int32_t px;         // row pitch (cells)
};

struct Tile {
    int32_t sim;
    int32_t x0, y0, z0; // padded coordinates of the tile origin
    int32_t ev_beg;     // first receiver event row of this tile
    int32_t ev_cnt;     // number of event rows
    int32_t pad0, pad1;
};

// Tile of the 2D adjoint with per-sample imaging: a 64 x bzg strip of a sample's grid,
// swept for every sim of the sample.  tix is the index, within each sim's tile list, of
// the sim tile that contains it (for its receiver event rows).
struct GTile {
    int32_t sample;
    int32_t x0, y0, z0;
    int32_t tix;   // the forward tile (of every sim of the sample) that holds plane / row z0
    int32_t tix2;  // 3D: the next forward tile in z where this tile reaches into it, else -1
    int32_t pad1, pad2;
};

// One row (2D: a grid row; 3D: an xy plane) of a tile that holds receivers.  vec_off
// points at 64 * (rows per tile / rows per wavefront) entries of receiver indices (local
// to the sim) or -1, one per lane of the workgroup: entry (y - y0) * width + (x - x0).  The event
// rows of a two-step strip cover its rows z0 - 4 .. z0 + kRows2 + 3 and, entry l, column
// x0 - 4 + l: the receivers of the margins the first step also computes.
struct EvRow {
    int32_t z;
    int32_t vec_off;
};

struct SrcPos {
    int32_t z, y, x;    // padded coordinates
    float w;            // encoding weight
};

// Arguments of one time step (forward, recompute or adjoint).
struct StepArgs {
    const SimDesc *sims;
    const Tile *tiles;
    const EvRow *evrows;
    const int32_t *evvec;
    const SrcPos *src;
    const int32_t *order;   // 3D forward: launch slot -> tile (nullable: identity)
    const float *cur;       // u^n (or lt^{k+1})
    const float *prev;      // u^{n-1} (or lt^{k+2})
    float *next;            // u^{n+1} (or lt^k); may alias prev (one step per launch)
    float *next2;           // two steps per launch: u^{n+2} (or lt^{k-1}); next and next2
                            // alias neither cur nor prev
    const float *cf;        // per-sample c
    float *wst;             // imaging operand W^n = L u^n + q^n for this step (nullable)
    float *wst2;            // two steps: W^{n+1} (nullable)
    const float *wimg;      // adjoint: W^{k-1} to image with
    const float *wimg2;     // two steps: W^{k-2}
    float *cka, *ckb;       // checkpoint slots for u^{n+1}, u^n (nullable)
    float *dat;             // forward: recorded data (nullable)
    const float *rho;       // adjoint: residual
    double *gacc;           // adjoint: imaging accumulators, one per sample
    int32_t ntiles;
    int32_t per_xcd;        // tiles per XCD chunk (grid = 8 * per_xcd)
    int32_t rec_j;          // recording slot j, or -1
    float fn;               // wavelet sample f[n] (forward)
    int32_t rec_j2;         // two steps: slot of the second step, or -1
    float fn2;              // two steps: f[n+1]
    // adjoint with per-sample imaging (2D strips; 3D tiles)
    const SampleDesc *samples;
    const GTile *gtiles;
    int32_t ngtiles;
    int32_t per_xcd_g;      // grouped tiles per XCD chunk
    int32_t nw;             // wavefronts per grouped workgroup (1..16; two steps: 1..8)
    int32_t bzg;            // rows per grouped tile (8 or 16)
    int32_t sg;             // two-step 2D adjoint: strips per workgroup (1 or 2)
};

}  // namespace fwi
