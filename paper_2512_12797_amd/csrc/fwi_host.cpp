// fwi_host.cpp -- host side of the C ABI: validation, batch tables, workspace layout and
// the time-stepping schedule (forward, residual/misfit, adjoint with checkpoint
// recomputation, finalization), all enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fwi.h"
#include "fwi_internal.h"
#include "fwi_launch.h"

namespace fwi {
// device array of the allocation-free gradient (fwi_static.hip)
hipError_t noalloc_scratch(void **ptr, size_t *bytes);
}  // namespace fwi

using namespace fwi;

namespace {

thread_local std::string g_err;

fwi_status fail(fwi_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(FWI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// 8th-order central weights of the second derivative (Fornberg 1988)
const double kC8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
// stability: largest |eigenvalue| of L8 is (2048/315) sum h^-2; leapfrog needs
// dt^2 v^2 (2048/315) sum h^-2 <= 4, i.e. v dt sqrt(sum h^-2) <= sqrt(315/512)
const double kCflLimit = 0.78436482084846;  // sqrt(315/512)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

int env_int(const char *name, int dflt)
{
    const char *s = getenv(name);
    if (!s || !*s) return dflt;
    return atoi(s);
}

// ---------------------------------------------------------------- validation

fwi_status check_grid(const fwi_grid &g, int i)
{
    if (g.ndim != 2 && g.ndim != 3) return fail(FWI_E_ARG, "grid %d: ndim must be 2 or 3", i);
    if (g.nz < 1 || g.nx < 1 || g.ny < 1) return fail(FWI_E_ARG, "grid %d: dims must be >= 1", i);
    if (g.ndim == 2 && g.ny != 1) return fail(FWI_E_ARG, "grid %d: ny must be 1 in 2D", i);
    if (!(g.dz > 0) || !(g.dx > 0) || (g.ndim == 3 && !(g.dy > 0)))
        return fail(FWI_E_ARG, "grid %d: spacings must be > 0", i);
    if (g.nb < 0) return fail(FWI_E_ARG, "grid %d: nb must be >= 0", i);
    if (g.nb > 0 && !(g.v_ref > 0)) return fail(FWI_E_ARG, "grid %d: v_ref must be > 0", i);
    if (g.nb > 0 && !(g.refl > 0 && g.refl < 1)) return fail(FWI_E_ARG, "grid %d: refl must be in (0,1)", i);
    if (!(g.v_max > 0) || !std::isfinite(g.v_max)) return fail(FWI_E_ARG, "grid %d: v_max must be > 0", i);
    // x extent with the row pitch (3D rows are padded to kRowAlign cells)
    const int64_t PX = g.ndim == 3 ? (g.nx + 2 * g.nb + kRowAlign - 1) / kRowAlign * kRowAlign : g.nx + 2 * g.nb;
    const int64_t N = (int64_t)(g.nz + 2 * g.nb) * (g.ndim == 3 ? g.ny + 2 * g.nb : 1) * PX;
    // fields are addressed through 32-bit byte offsets (FP64 accumulators: 8 bytes/cell)
    if (N >= (int64_t)1 << 28) return fail(FWI_E_UNSUPPORTED, "grid %d: more than 2^28 padded cells", i);
    // the sweeps address up to 80 rows (2D) / planes (3D) past the grid with offsets that
    // must stay below bit 31 even when doubled (out-of-grid lanes carry bit 31)
    const int64_t slice = (int64_t)4 * (g.ndim == 3 ? (int64_t)(g.ny + 2 * g.nb) * PX : PX);
    if ((int64_t)(g.nz + 2 * g.nb + 80) * slice > (int64_t)1 << 30)
        return fail(FWI_E_UNSUPPORTED, "grid %d: (padded nz + 80) x row or plane bytes exceeds 2^30", i);
    return FWI_OK;
}

double courant(const fwi_grid &g, double dt)
{
    double s = 1.0 / (g.dz * g.dz) + 1.0 / (g.dx * g.dx);
    if (g.ndim == 3) s += 1.0 / (g.dy * g.dy);
    return g.v_max * dt * std::sqrt(s);
}

fwi_status check_all(const fwi_batch *b, const fwi_time *t, double *worst)
{
    if (!b || !t) return fail(FWI_E_ARG, "null batch or time");
    if (!(t->dt > 0) || !std::isfinite(t->dt)) return fail(FWI_E_ARG, "dt must be > 0");
    if (t->nt < 1) return fail(FWI_E_ARG, "nt must be >= 1");
    if (t->rec_every < 1 || t->nt % t->rec_every != 0) return fail(FWI_E_ARG, "nt must be a multiple of rec_every >= 1");
    if (t->ckpt_every < -1) return fail(FWI_E_ARG, "ckpt_every must be >= -1");
    if (t->keep_tail < 0 || t->keep_tail > t->nt) return fail(FWI_E_ARG, "keep_tail must be in [0, nt]");
    if (t->keep_tail > 0 && t->ckpt_every < 1) return fail(FWI_E_ARG, "keep_tail needs ckpt_every >= 1");
    if (b->nsim < 1 || b->nsample < 1) return fail(FWI_E_ARG, "nsim and nsample must be >= 1");
    if (b->nsim > 65535 || b->nsample > 65535) return fail(FWI_E_UNSUPPORTED, "more than 65535 sims or samples");
    if (!b->grid || !b->model_off || !b->sample_of || !b->src_ptr || !b->rec_ptr || !b->wavelet)
        return fail(FWI_E_ARG, "null array in batch");
    int ndim = b->grid[0].ndim;
    double cmax = 0;
    for (int i = 0; i < b->nsample; ++i) {
        fwi_status s = check_grid(b->grid[i], i);
        if (s) return s;
        if (b->grid[i].ndim != ndim) return fail(FWI_E_UNSUPPORTED, "mixed 2D/3D grids in one batch");
        int64_t nphys = (int64_t)b->grid[i].nz * b->grid[i].ny * b->grid[i].nx;
        if (b->model_off[i + 1] - b->model_off[i] != nphys)
            return fail(FWI_E_ARG, "model_off[%d+1]-model_off[%d] != physical cells of its grid", i, i);
        if (b->model_off[i] < 0) return fail(FWI_E_ARG, "model_off must be >= 0");
        cmax = std::max(cmax, courant(b->grid[i], t->dt));
    }
    if (worst) *worst = cmax;
    if (cmax > kCflLimit)
        return fail(FWI_E_CFL, "Courant number %.6f exceeds the 8th-order leapfrog limit %.6f", cmax, kCflLimit);
    int prev = -1;
    std::vector<int> cnt(b->nsample, 0);
    for (int s = 0; s < b->nsim; ++s) {
        int k = b->sample_of[s];
        if (k < 0 || k >= b->nsample) return fail(FWI_E_ARG, "sample_of[%d] out of range", s);
        if (k < prev) return fail(FWI_E_ARG, "sims must be grouped by increasing sample");
        if (k != prev && prev >= 0 && cnt[k] > 0) return fail(FWI_E_ARG, "sims of a sample must be contiguous");
        prev = k;
        cnt[k]++;
    }
    for (int k = 0; k < b->nsample; ++k)
        if (cnt[k] == 0) return fail(FWI_E_ARG, "sample %d has no simulation", k);
    if (b->src_ptr[0] != 0 || b->rec_ptr[0] != 0) return fail(FWI_E_ARG, "src_ptr[0] and rec_ptr[0] must be 0");
    for (int s = 0; s < b->nsim; ++s) {
        if (b->src_ptr[s + 1] < b->src_ptr[s]) return fail(FWI_E_ARG, "src_ptr not monotonic");
        if (b->rec_ptr[s + 1] < b->rec_ptr[s]) return fail(FWI_E_ARG, "rec_ptr not monotonic");
    }
    if (b->src_ptr[b->nsim] > 0 && (!b->src_cell || !b->src_w)) return fail(FWI_E_ARG, "null source arrays");
    if (b->rec_ptr[b->nsim] > 0 && !b->rec_cell) return fail(FWI_E_ARG, "null receiver array");
    std::vector<int32_t> tmp;
    for (int s = 0; s < b->nsim; ++s) {
        const fwi_grid &g = b->grid[b->sample_of[s]];
        int64_t nphys = (int64_t)g.nz * g.ny * g.nx;
        for (int i = b->src_ptr[s]; i < b->src_ptr[s + 1]; ++i) {
            if (b->src_cell[i] < 0 || b->src_cell[i] >= nphys)
                return fail(FWI_E_ARG, "sim %d: source cell %d outside the grid", s, b->src_cell[i]);
            if (!std::isfinite(b->src_w[i])) return fail(FWI_E_ARG, "sim %d: non-finite source weight", s);
        }
        tmp.assign(b->rec_cell + b->rec_ptr[s], b->rec_cell + b->rec_ptr[s + 1]);
        for (int32_t c : tmp)
            if (c < 0 || c >= nphys) return fail(FWI_E_ARG, "sim %d: receiver cell %d outside the grid", s, c);
        std::sort(tmp.begin(), tmp.end());
        if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end())
            return fail(FWI_E_ARG, "sim %d: duplicate receiver cell", s);
    }
    for (int n = 0; n < t->nt; ++n)
        if (!std::isfinite(b->wavelet[n])) return fail(FWI_E_ARG, "non-finite wavelet sample %d", n);
    return FWI_OK;
}

// ---------------------------------------------------------------- the plan

struct Plan {
    int ndim = 2;
    int bz = 32, ty = 8;
    int wx = kTileX;  // 3D tile width: 64 or 32 cells (ty = 8 * 64 / wx rows)
    std::vector<SimDesc> sims;
    std::vector<SampleDesc> samples;
    std::vector<Tile> tiles;
    std::vector<GTile> gtiles;  // adjoint strips (2D) or tiles (3D) of the samples' grids
    // 2D, two time steps per launch: kStrip2 x kRows2 strips of every sim (forward) and of
    // every sample (adjoint); their receiver event rows cover the first step's margins
    std::vector<Tile> tiles2;
    std::vector<GTile> gtiles2;
    bool two = false;        // keep-all 2D schedule: forward with two steps per launch
    bool two_adj = false;    // and the adjoint
    int per_xcd2 = 0, per_xcd_g2 = 0, nw2 = 1, sg2 = 1;
    std::vector<EvRow> evrows;
    std::vector<int32_t> evvec;
    std::vector<SrcPos> src;
    std::vector<int32_t> order;  // 3D forward launch order (tile indices)
    int64_t cells = 0;       // one field level, all sims
    int64_t coefs = 0;       // all samples' padded cells
    int64_t data = 0;        // all sims' data
    int64_t max_cell = 0;    // largest padded sample grid
    int nt_rec = 0;
    int per_xcd = 0;
    bool grouped = false;    // adjoint images per sample (accumulator slots = samples)
    int bzg = 16, nw = 1, per_xcd_g = 0;
    int64_t gcells = 0;      // imaging accumulator cells
    // layout
    int nlev = 2, K = 0, nseg = 1;
    int head = 0, tail = 0;  // checkpoints: steps [0, head) recomputed per segment, [head, nt) kept
    int64_t ring = 0;        // imaging levels of the recomputation ring (two rings with overlap)
    int64_t tail_lev0 = 0;   // first imaging level of the kept tail (0: the ring reuses the tail's
                             // levels, which the adjoint has read before it recomputes)
    bool fwd_only = false;  // ckpt_every == -1: no adjoint state is kept
    bool overlap = false;   // checkpoints: recompute the next segment beside the current adjoint
    int64_t wst_levels = 0, ck_slots = 0;
    int nchunk_res = 1, nchunk_fin = 1;
    size_t t_sims = 0, t_samples = 0, t_tiles = 0, t_gtiles = 0, t_tiles2 = 0, t_gtiles2 = 0, t_evrows = 0,
           t_evvec = 0, t_src = 0, t_order = 0, t_bytes = 0;
    size_t t_alloc = 0;  // table region reserved in the workspace (largest over tile heights)
    size_t o_status = 0, o_tables = 0, o_cf = 0, o_fields = 0, o_wst = 0, o_ck = 0, o_gacc = 0, o_rho = 0,
           o_part = 0, o_npart = 0, o_mis = 0, total = 0;
};

void stencil_weights(const fwi_grid &g, float w[3][5], double gmax[3], float &inv_vol)
{
    const double h[3] = {g.dz, g.ndim == 3 ? g.dy : 1.0, g.dx};
    for (int a = 0; a < 3; ++a) {
        bool on = g.ndim == 3 || a != 1;
        for (int m = 0; m < 5; ++m) w[a][m] = on ? (float)(kC8[m] / (h[a] * h[a])) : 0.0f;
        gmax[a] = (on && g.nb > 0) ? 3.0 * g.v_ref * std::log(1.0 / g.refl) / (2.0 * g.nb * h[a]) : 0.0;
    }
    double vol = g.dz * g.dx * (g.ndim == 3 ? g.dy : 1.0);
    inv_vol = (float)(1.0 / vol);
}

// Tile heights the kernels are instantiated for (rows per 2D tile, planes per 3D tile).
const int kBz2[] = {8, 16, 32};
const int kBz3[] = {16, 24, 32, 40};

// Process-wide tile choices: forced per dimensionality (fwi_set_tile) or tuned per batch
// shape (fwi_tune): the tile height and, for 2D keep-all batches, the adjoint's time steps
// per launch (0: not tuned).
struct TunedShape {
    std::string sig;
    int bz;
    int adj;
};
struct TileChoices {
    std::mutex m;
    int forced[4] = {0, 0, 0, 0};
    std::vector<TunedShape> tuned;
};
TileChoices g_tiles;

void set_tuned(const std::string &sig, int bz, int adj)
{
    std::lock_guard<std::mutex> lk(g_tiles.m);
    for (auto &e : g_tiles.tuned)
        if (e.sig == sig) {
            e.bz = bz;
            e.adj = adj;
            return;
        }
    g_tiles.tuned.push_back({sig, bz, adj});
}

// 3D tile width forced process-wide (fwi_set_tile_width): 0 automatic, 32 or 64.
std::atomic<int> g_width3{0};

// Overlap of recomputation and adjoint in checkpointed schedules (fwi_set_overlap).
std::atomic<int> g_overlap{0};

// Time steps per launch of the 2D keep-all schedule, forward and adjoint, process-wide:
// 1 or 2 forced, 0 automatic (forward 1; adjoint the tuned choice for the batch shape,
// else 2).
std::atomic<int> g_blocking_fwd{0}, g_blocking_adj{0};

// Batch shape signature: dimensionality and the multiset of padded grid sizes.
std::string shape_signature(const fwi_batch *b)
{
    std::vector<std::string> v;
    for (int s = 0; s < b->nsim; ++s) {
        const fwi_grid &g = b->grid[b->sample_of[s]];
        char buf[64];
        snprintf(buf, sizeof buf, "%dx%dx%d", g.nz + 2 * g.nb, g.ndim == 3 ? g.ny + 2 * g.nb : 1, g.nx + 2 * g.nb);
        v.push_back(buf);
    }
    std::sort(v.begin(), v.end());
    std::string sig = b->grid[0].ndim == 3 ? "3d" : "2d";
    for (size_t i = 0; i < v.size();) {
        size_t j = i;
        while (j < v.size() && v[j] == v[i]) ++j;
        sig += ":" + v[i] + "*" + std::to_string(j - i);
        i = j;
    }
    return sig;
}

bool valid_bz(int ndim, int bz)
{
    if (ndim == 2) return bz == 8 || bz == 16 || bz == 32;
    return bz == 16 || bz == 24 || bz == 32 || bz == 40;
}

// 3D tile width: 32 cells (two rows per wavefront, 16 rows per tile) where that runs fewer
// lanes over the batch's grids than 64-wide tiles (8 rows per tile), else 64, unless a width
// is forced.  With rows stored at a 32-cell pitch both widths write whole lines; on the
// 220 x 220 x 120 padded grid 32-wide tiles run 12 % fewer lanes and took 649 / 902 us per
// forward / adjoint launch against 653 / 927 us (40-plane forward tiles).
int pick_width3(const fwi_batch *b)
{
    const int forced = g_width3.load();
    if (forced == 32 || forced == 64) return forced;
    int64_t lanes[2] = {0, 0};
    for (int s = 0; s < b->nsim; ++s) {
        const fwi_grid &g = b->grid[b->sample_of[s]];
        const int64_t Nx = g.nx + 2 * g.nb, Ny = g.ny + 2 * g.nb;
        for (int i = 0; i < 2; ++i) {
            const int64_t wx = i == 0 ? 64 : 32, ty = 8 * (64 / wx);
            lanes[i] += ((Nx + wx - 1) / wx) * wx * ((Ny + ty - 1) / ty) * ty;
        }
    }
    return lanes[1] < lanes[0] ? 32 : 64;
}

void pick_tiles(Plan &p, const fwi_batch *b, int bz_override, int wx_override)
{
    p.wx = p.ndim == 3 ? (wx_override == 32 || wx_override == 64 ? wx_override : pick_width3(b)) : kTileX;
    p.ty = p.ndim == 3 ? 8 * (kTileX / p.wx) : 1;
    if (valid_bz(p.ndim, bz_override)) {
        p.bz = bz_override;
        return;
    }
    {
        std::lock_guard<std::mutex> lk(g_tiles.m);
        if (valid_bz(p.ndim, g_tiles.forced[p.ndim])) {
            p.bz = g_tiles.forced[p.ndim];
            return;
        }
        const std::string sig = shape_signature(b);
        for (auto &e : g_tiles.tuned)
            if (e.sig == sig && valid_bz(p.ndim, e.bz)) {
                p.bz = e.bz;
                return;
            }
    }
    // default (3D): the tallest tile that still gives >= 4 tiles per CU (256 CUs)
    auto count = [&](int bz) {
        int64_t n = 0;
        for (int s = 0; s < b->nsim; ++s) {
            const fwi_grid &g = b->grid[b->sample_of[s]];
            int64_t Nx = g.nx + 2 * g.nb, Nz = g.nz + 2 * g.nb, Ny = p.ndim == 3 ? g.ny + 2 * g.nb : 1;
            n += ((Nx + p.wx - 1) / p.wx) * ((Nz + bz - 1) / bz) * ((Ny + p.ty - 1) / p.ty);
        }
        return n;
    };
    if (p.ndim == 2) {
        // 8 rows: the fastest forward on the 400x150 workload (the tuner's choice) and on
        // the uneven 32-sample batch (16.1 us per launch against 16.8 and 19.8 us for 16
        // and 32 rows); taller strips leave fewer wavefronts per compute unit
        p.bz = 8;
    } else {
        // the height with the fewest planes read per tile column (its planes plus the
        // 8-plane z halo, over the tiles that cover the depth) among those that still give
        // >= 4 tiles per CU (256 CUs); ties go to the taller tile
        auto planes = [&](int bz) {
            int64_t n = 0;
            for (int s = 0; s < b->nsim; ++s) {
                const fwi_grid &g = b->grid[b->sample_of[s]];
                n += (int64_t)((g.nz + 2 * g.nb + bz - 1) / bz) * (bz + 2 * kHalo);
            }
            return n;
        };
        p.bz = 16;
        int64_t best = planes(16);
        for (int c : kBz3)
            if (count(c) >= 1024 && (planes(c) < best || (planes(c) == best && c > p.bz))) {
                p.bz = c;
                best = planes(c);
            }
    }
}

size_t plan_tables_bytes(const fwi_batch *b, const fwi_time *t, int bz, int wx);

// Wavefronts per workgroup of the per-sample 2D adjoint for samples of up to g sims and
// ngt strips.  Four waves (fewer for smaller samples) pack the kernel's occupancy (six
// waves per SIMD) into whole workgroups and keep workgroups short; more waves per
// workgroup only when the launch would otherwise hold fewer than about 24 waves per CU.
// (On the 16-sample x 10-supergather 2D workload, 4 waves measured faster than 2, 5 or 10.)
int grouped_waves(int g, int64_t ngt)
{
    if (g <= 1) return 1;
    int w = std::min(g, 4);
    while (w < std::min(g, 16) && ngt * w < 256 * 24) ++w;
    return w;
}

// index one past the last tile of sim s (its tiles are contiguous, sims in order)
int s_tiles_end(const Plan &p, int s)
{
    return s + 1 < (int)p.sims.size() ? p.sims[s + 1].tile0 : (int)p.tiles.size();
}

fwi_status build_plan(const fwi_batch *b, const fwi_time *t, const double *kappa, Plan &p, int bz_override = 0,
                      bool size_for_all_tiles = true, int wx_override = 0, bool no_overlap = false)
{
    p.ndim = b->grid[0].ndim;
    pick_tiles(p, b, bz_override, wx_override);
    p.nt_rec = t->nt / t->rec_every;
    const int TYt = p.ndim == 3 ? p.ty : 1;
    const int WXt = p.ndim == 3 ? p.wx : kTileX;  // tile width
    // samples
    p.samples.resize(b->nsample);
    for (int k = 0; k < b->nsample; ++k) {
        const fwi_grid &g = b->grid[k];
        SampleDesc &S = p.samples[k];
        memset(&S, 0, sizeof S);
        S.m_off = b->model_off[k];
        S.c_off = p.coefs;
        S.N[0] = g.nz + 2 * g.nb;
        S.N[1] = g.ndim == 3 ? g.ny + 2 * g.nb : 1;
        S.N[2] = g.nx + 2 * g.nb;
        S.n[0] = g.nz;
        S.n[1] = g.ny;
        S.n[2] = g.nx;
        S.nb = g.nb;
        S.ndim = g.ndim;
        float w[3][5];
        float iv;
        stencil_weights(g, w, S.gmax, iv);
        S.dt = t->dt;
        S.v_max = g.v_max;
        S.kappa = kappa ? kappa[k] : 1.0;
        S.nphys = (int64_t)g.nz * g.ny * g.nx;
        S.px = g.ndim == 3 ? (S.N[2] + kRowAlign - 1) / kRowAlign * kRowAlign : S.N[2];
        S.ncell = (int64_t)S.N[0] * S.N[1] * S.px;
        S.sim_beg = -1;
        p.coefs += S.ncell;
        p.max_cell = std::max(p.max_cell, S.ncell);
    }
    // sims, tiles, receiver events, sources
    p.sims.resize(b->nsim);
    struct Ev {
        int32_t tile, z, slot, r;
    };
    std::vector<Ev> evs;
    for (int s = 0; s < b->nsim; ++s) {
        const int k = b->sample_of[s];
        const fwi_grid &g = b->grid[k];
        SampleDesc &Sm = p.samples[k];
        if (Sm.sim_beg < 0) Sm.sim_beg = s;
        Sm.sim_cnt++;
        SimDesc &S = p.sims[s];
        memset(&S, 0, sizeof S);
        S.u_off = p.cells;
        S.c_off = Sm.c_off;
        S.d_off = p.data;
        S.m_off = Sm.m_off;
        for (int a = 0; a < 3; ++a) {
            S.N[a] = Sm.N[a];
            S.n[a] = Sm.n[a];
        }
        S.nb = g.nb;
        S.ndim = g.ndim;
        S.px = Sm.px;
        S.nrec = b->rec_ptr[s + 1] - b->rec_ptr[s];
        S.src_beg = b->src_ptr[s];
        S.src_cnt = b->src_ptr[s + 1] - b->src_ptr[s];
        S.sample = k;
        stencil_weights(g, S.w, S.gmax, S.inv_vol);
        S.dt = t->dt;
        S.tile0 = (int32_t)p.tiles.size();
        p.cells += Sm.ncell;
        p.data += (int64_t)p.nt_rec * S.nrec;
        // tiles: z block, then y block, then x strip
        const int ntx = (S.N[2] + WXt - 1) / WXt;
        const int nty = (S.N[1] + TYt - 1) / TYt;
        const int ntz = (S.N[0] + p.bz - 1) / p.bz;
        const int tile0 = (int)p.tiles.size();
        for (int iz = 0; iz < ntz; ++iz)
            for (int iy = 0; iy < nty; ++iy)
                for (int ix = 0; ix < ntx; ++ix) {
                    Tile T;
                    memset(&T, 0, sizeof T);
                    T.sim = s;
                    T.x0 = ix * WXt;
                    T.y0 = iy * TYt;
                    T.z0 = iz * p.bz;
                    p.tiles.push_back(T);
                }
        const int nby = g.ndim == 3 ? g.nb : 0;
        for (int r = 0; r < S.nrec; ++r) {
            const int32_t c = b->rec_cell[b->rec_ptr[s] + r];
            const int ix = c % g.nx, iy = (c / g.nx) % g.ny, iz = c / (g.nx * g.ny);
            const int px = ix + g.nb, py = iy + nby, pz = iz + g.nb;
            const int tl = tile0 + ((pz / p.bz) * nty + py / TYt) * ntx + px / WXt;
            evs.push_back({tl, pz, (py % TYt) * WXt + px % WXt, r});
        }
    }
    for (int s = 0; s < b->nsim; ++s) {
        const fwi_grid &g = b->grid[b->sample_of[s]];
        const int nby = g.ndim == 3 ? g.nb : 0;
        for (int i = b->src_ptr[s]; i < b->src_ptr[s + 1]; ++i) {
            const int32_t c = b->src_cell[i];
            SrcPos sp;
            sp.x = c % g.nx + g.nb;
            sp.y = (c / g.nx) % g.ny + nby;
            sp.z = c / (g.nx * g.ny) + g.nb;
            sp.w = b->src_w[i];
            p.src.push_back(sp);
        }
    }
    std::sort(evs.begin(), evs.end(), [](const Ev &a, const Ev &b) {
        return a.tile != b.tile ? a.tile < b.tile : a.z < b.z;
    });
    const int vec = WXt * TYt;
    for (size_t i = 0; i < evs.size();) {
        size_t j = i;
        EvRow row{evs[i].z, (int32_t)p.evvec.size()};
        p.evvec.resize(p.evvec.size() + vec, -1);
        Tile &T = p.tiles[evs[i].tile];
        if (T.ev_cnt == 0) T.ev_beg = (int32_t)p.evrows.size();
        while (j < evs.size() && evs[j].tile == evs[i].tile && evs[j].z == evs[i].z) {
            p.evvec[row.vec_off + evs[j].slot] = evs[j].r;
            ++j;
        }
        p.evrows.push_back(row);
        T.ev_cnt++;
        i = j;
    }
    if (p.ndim == 2) {
        // two-step strips: sim s covers tiles2[tile0b ..], z block then x strip; a receiver
        // lands in every strip whose first-step rows and lanes (4-cell margins) hold it
        std::vector<Ev> ev2;
        for (int s = 0; s < b->nsim; ++s) {
            const fwi_grid &g = b->grid[b->sample_of[s]];
            SimDesc &S = p.sims[s];
            S.tile0b = (int32_t)p.tiles2.size();
            const int ntx = (S.N[2] + kStrip2 - 1) / kStrip2, ntz = (S.N[0] + kRows2 - 1) / kRows2;
            for (int iz = 0; iz < ntz; ++iz)
                for (int ix = 0; ix < ntx; ++ix) {
                    Tile T;
                    memset(&T, 0, sizeof T);
                    T.sim = s;
                    T.x0 = ix * kStrip2;
                    T.z0 = iz * kRows2;
                    p.tiles2.push_back(T);
                }
            for (int r = 0; r < S.nrec; ++r) {
                const int32_t c = b->rec_cell[b->rec_ptr[s] + r];
                const int px = c % g.nx + g.nb, pz = c / g.nx + g.nb;
                for (int iz = (pz + kHalo) / kRows2 - 2; iz <= (pz + kHalo) / kRows2; ++iz) {
                    if (iz < 0 || iz >= ntz || pz < iz * kRows2 - kHalo || pz >= iz * kRows2 + kRows2 + kHalo)
                        continue;
                    for (int ix = (px + kHalo) / kStrip2 - 2; ix <= (px + kHalo) / kStrip2; ++ix) {
                        const int lx = px - (ix * kStrip2 - kHalo);
                        if (ix < 0 || ix >= ntx || lx < 0 || lx >= kTileX) continue;
                        ev2.push_back({S.tile0b + iz * ntx + ix, pz, lx, r});
                    }
                }
            }
        }
        std::sort(ev2.begin(), ev2.end(), [](const Ev &a, const Ev &b) {
            return a.tile != b.tile ? a.tile < b.tile : a.z < b.z;
        });
        for (size_t i = 0; i < ev2.size();) {
            size_t j = i;
            EvRow row{ev2[i].z, (int32_t)p.evvec.size()};
            p.evvec.resize(p.evvec.size() + kTileX, -1);
            Tile &T = p.tiles2[ev2[i].tile];
            if (T.ev_cnt == 0) T.ev_beg = (int32_t)p.evrows.size();
            while (j < ev2.size() && ev2[j].tile == ev2[i].tile && ev2[j].z == ev2[i].z) {
                p.evvec[row.vec_off + ev2[j].slot] = ev2[j].r;
                ++j;
            }
            p.evrows.push_back(row);
            T.ev_cnt++;
            i = j;
        }
    }
    if (p.tiles.size() >= (size_t)1 << 30 || p.tiles2.size() >= (size_t)1 << 30)
        return fail(FWI_E_UNSUPPORTED, "too many tiles");
    if (p.ndim == 3) {
        // forward launch order: sample by sample, in groups of up to kGroup of its sims
        // (which share its geometry and coefficient grid), tile position by position with
        // the group's sims next to each other.  Small groups keep the tiles that neighbour
        // one another in y a few launch slots apart, so they run together and share their
        // halo rows in L2 as well.
        constexpr size_t kGroup = 4;
        p.order.reserve(p.tiles.size());
        for (int k = 0; k < b->nsample; ++k) {
            std::vector<int> sims_k;
            for (int s = 0; s < b->nsim; ++s)
                if (b->sample_of[s] == k) sims_k.push_back(s);
            if (sims_k.empty()) continue;
            const int per_sim = (s_tiles_end(p, sims_k[0]) - p.sims[sims_k[0]].tile0);
            for (size_t g0 = 0; g0 < sims_k.size(); g0 += kGroup) {
                const size_t g1 = std::min(sims_k.size(), g0 + kGroup);
                for (int i = 0; i < per_sim; ++i)
                    for (size_t g = g0; g < g1; ++g) p.order.push_back(p.sims[sims_k[g]].tile0 + i);
            }
        }
        if (p.order.size() != p.tiles.size()) return fail(FWI_E_ARG, "internal: tile order incomplete");
    }
    // imaging accumulators: one per sample, laid out like the coefficients (an adjoint
    // workgroup sweeps its strip or tile for every sim of the sample)
    p.grouped = true;
    int gmax = 0;
    for (auto &Sm : p.samples) {
        if (Sm.sim_beg < 0) Sm.sim_beg = 0;
        gmax = std::max(gmax, Sm.sim_cnt);
        if (p.grouped) {
            Sm.g_off = Sm.c_off;
            Sm.g_cnt = 1;
        } else {
            Sm.g_off = Sm.sim_cnt > 0 ? p.sims[Sm.sim_beg].u_off : 0;
            Sm.g_cnt = Sm.sim_cnt;
        }
    }
    p.gcells = p.grouped ? p.coefs : p.cells;
    // grouped strip / tile height: 2D 8 or 16 rows; 3D 16 planes (the LDS of the per-sample
    // sums of taller tiles would leave one workgroup per compute unit)
    p.bzg = p.ndim == 2 ? (p.bz == 8 ? 8 : 16) : 16;
    for (int k = 0; k < (p.grouped ? b->nsample : 0); ++k) {
        const SampleDesc &Sm = p.samples[k];
        const int ntx = (Sm.N[2] + WXt - 1) / WXt;
        const int nty = (Sm.N[1] + TYt - 1) / TYt;
        const int ntz = (Sm.N[0] + p.bzg - 1) / p.bzg;
        for (int iz = 0; iz < ntz; ++iz)
            for (int iy = 0; iy < nty; ++iy)
                for (int ix = 0; ix < ntx; ++ix) {
                    const int z0 = iz * p.bzg;
                    GTile G;
                    memset(&G, 0, sizeof G);
                    G.sample = k;
                    G.x0 = ix * WXt;
                    G.y0 = iy * TYt;
                    G.z0 = z0;
                    G.tix = ((z0 / p.bz) * nty + iy) * ntx + ix;
                    // a forward tile height that is not a multiple of this tile's (3D: 24, 40)
                    // splits some of these tiles between two forward tiles
                    const int iz2 = z0 / p.bz + 1;
                    G.tix2 = (z0 + p.bzg > iz2 * p.bz && iz2 < (Sm.N[0] + p.bz - 1) / p.bz)
                                 ? (iz2 * nty + iy) * ntx + ix : -1;
                    p.gtiles.push_back(G);
                }
    }
    p.nw = p.ndim == 2 ? grouped_waves(gmax, (int64_t)p.gtiles.size()) : 8;  // 3D: 8 wavefronts
    p.per_xcd_g = (int)((p.gtiles.size() + 7) / 8);
    // 2D: a workgroup runs 4 tiles (one per wavefront); 3D: one tile per workgroup
    const size_t nwg = p.ndim == 2 ? (p.tiles.size() + 3) / 4 : p.tiles.size();
    p.per_xcd = (int)((nwg + 7) / 8);
    if (p.ndim == 2) {
        for (int k = 0; k < b->nsample; ++k) {
            const SampleDesc &Sm = p.samples[k];
            const int ntx = (Sm.N[2] + kStrip2 - 1) / kStrip2, ntz = (Sm.N[0] + kRows2 - 1) / kRows2;
            for (int iz = 0; iz < ntz; ++iz)
                for (int ix = 0; ix < ntx; ++ix) {
                    GTile G;
                    memset(&G, 0, sizeof G);
                    G.sample = k;
                    G.x0 = ix * kStrip2;
                    G.z0 = iz * kRows2;
                    G.tix = iz * ntx + ix;  // the same strip in each of the sample's sims
                    G.tix2 = -1;
                    p.gtiles2.push_back(G);
                }
        }
        // (on the 16-sample x 10-supergather workload 4 waves measured faster than 2, 5 or 8:
        // 90.9 vs 108.9 / 121.6 / 125.7 us per two-step launch)
        p.nw2 = std::min(grouped_waves(gmax, (int64_t)p.gtiles2.size()), 8);
        // two strips per workgroup (half the waves on each) when that splits the largest
        // sample's sims more evenly over its waves: 10 sims on 4 waves run 3 + 3 + 2 + 2,
        // two idle waves waiting at the reduction; on 2 waves per strip, 5 + 5
        p.sg2 = 1;
        if (p.nw2 % 2 == 0) {
            auto idle = [&](int w) { return (gmax + w - 1) / w * w - gmax; };
            if (idle(p.nw2 / 2) < idle(p.nw2)) p.sg2 = 2;
        }
        // samples of one sim each: one wavefront per strip and workgroup (the LDS is sized
        // by the launch; on the uneven 32-sample batch 44.8 us per launch against 45.8 for
        // two one-wave strips per workgroup)
        if (gmax == 1) {
            p.nw2 = 1;
            p.sg2 = 1;
        }
        p.per_xcd_g2 = (int)(((p.gtiles2.size() + p.sg2 - 1) / p.sg2 + 7) / 8);
        p.per_xcd2 = (int)(((p.tiles2.size() + 3) / 4 + 7) / 8);
    }
    // table layout
    size_t o = 0;
    p.t_sims = o;
    o = align_up(o + p.sims.size() * sizeof(SimDesc));
    p.t_samples = o;
    o = align_up(o + p.samples.size() * sizeof(SampleDesc));
    p.t_tiles = o;
    o = align_up(o + p.tiles.size() * sizeof(Tile));
    p.t_gtiles = o;
    o = align_up(o + std::max<size_t>(1, p.gtiles.size()) * sizeof(GTile));
    p.t_tiles2 = o;
    o = align_up(o + std::max<size_t>(1, p.tiles2.size()) * sizeof(Tile));
    p.t_gtiles2 = o;
    o = align_up(o + std::max<size_t>(1, p.gtiles2.size()) * sizeof(GTile));
    p.t_evrows = o;
    o = align_up(o + std::max<size_t>(1, p.evrows.size()) * sizeof(EvRow));
    p.t_evvec = o;
    o = align_up(o + std::max<size_t>(1, p.evvec.size()) * sizeof(int32_t));
    p.t_src = o;
    o = align_up(o + std::max<size_t>(1, p.src.size()) * sizeof(SrcPos));
    p.t_order = o;
    o = align_up(o + std::max<size_t>(1, p.order.size()) * sizeof(int32_t));
    p.t_bytes = o;
    p.t_alloc = o;
    if (size_for_all_tiles) {
        if (p.ndim == 2)
            for (int c : kBz2) p.t_alloc = std::max(p.t_alloc, plan_tables_bytes(b, t, c, 0));
        else
            for (int c : kBz3)
                for (int w : {32, 64}) p.t_alloc = std::max(p.t_alloc, plan_tables_bytes(b, t, c, w));
    }
    // workspace layout
    p.fwd_only = t->ckpt_every < 0;
    p.K = p.fwd_only ? 0 : t->ckpt_every;
    p.tail = p.K > 0 ? t->keep_tail : 0;
    p.head = t->nt - p.tail;
    if (p.K > 0) {
        p.K = std::min(p.K, std::max(p.head, 1));
        p.nseg = (p.head + p.K - 1) / p.K;  // 0 when every step is kept
    } else {
        p.nseg = 1;
    }
    // levels: 2 (u^n, u^{n-1} updated in place), 4 with checkpoints (recomputation and
    // adjoint), and in 2D two more for the output levels of two-step launches
    p.nlev = (p.K > 0 ? 4 : 2) + (p.ndim == 2 ? 2 : 0);
    {
        int fwd = g_blocking_fwd.load(), adj = g_blocking_adj.load();
        if (p.ndim == 2 && adj == 0) {
            const std::string sig = shape_signature(b);
            std::lock_guard<std::mutex> lk(g_tiles.m);
            for (auto &e : g_tiles.tuned)
                if (e.sig == sig) adj = e.adj;
        }
        p.two = p.ndim == 2 && p.K == 0 && fwd == 2;
        p.two_adj = p.ndim == 2 && (adj == 2 || adj == 0);
    }
    // with overlap the recomputation writes one of two rings of K imaging levels while the
    // adjoint reads the other
    p.overlap = !p.fwd_only && p.K > 0 && p.nseg >= 2 && !no_overlap && g_overlap.load();
    p.ring = p.K > 0 && p.nseg > 0 ? (p.overlap ? 2 * p.K : p.K) : 0;
    // without overlap the adjoint sweeps the kept tail before its first recomputation, so a
    // tail at least as long as the ring lends it its levels
    p.tail_lev0 = (!p.overlap && p.tail >= p.ring) ? 0 : p.ring;
    p.wst_levels = p.fwd_only ? 0 : (p.K > 0 ? p.tail_lev0 + p.tail : t->nt);
    p.ck_slots = p.K > 0 && p.nseg > 0 ? 2 * (int64_t)(p.nseg - 1) : 0;
    int64_t maxdata = 0;
    for (auto &S : p.sims) maxdata = std::max(maxdata, (int64_t)p.nt_rec * S.nrec);
    p.nchunk_res = (int)std::min<int64_t>(64, std::max<int64_t>(1, maxdata / 4096));
    int64_t maxphys = 0;
    for (auto &S : p.samples) maxphys = std::max(maxphys, S.nphys);
    p.nchunk_fin = (int)std::min<int64_t>(256, std::max<int64_t>(1, maxphys / 2048));
    size_t w = 0;
    p.o_status = w;
    w = align_up(w + 64);
    p.o_tables = w;
    w = align_up(w + p.t_alloc);
    p.o_cf = w;
    w = align_up(w + (size_t)p.coefs * 4);
    p.o_fields = w;
    w = align_up(w + (size_t)p.nlev * p.cells * 4);
    p.o_wst = w;
    w = align_up(w + (size_t)p.wst_levels * p.cells * 4);
    p.o_ck = w;
    w = align_up(w + (size_t)p.ck_slots * p.cells * 4);
    p.o_gacc = w;
    w = align_up(w + (p.fwd_only ? 0 : (size_t)p.gcells * 8));
    p.o_rho = w;
    w = align_up(w + (size_t)std::max<int64_t>(1, p.data) * 4);
    p.o_part = w;
    w = align_up(w + (size_t)b->nsim * p.nchunk_res * 8);
    p.o_npart = w;
    w = align_up(w + (size_t)b->nsample * p.nchunk_fin * 8);
    p.o_mis = w;
    w = align_up(w + (size_t)b->nsim * 8);
    p.total = w;
    return FWI_OK;
}

size_t plan_tables_bytes(const fwi_batch *b, const fwi_time *t, int bz, int wx)
{
    Plan q;
    if (build_plan(b, t, nullptr, q, bz, false, wx)) return 0;
    return q.t_bytes;
}

// ----------------------------------------------------------- host staging

// The tables of a call are staged in host memory and copied to the workspace with one
// asynchronous copy.  Each thread owns two pinned staging buffers used in turn, so a call
// waits only for the upload two calls back on the same thread (its buffer is then free
// again) and calls from distinct threads never wait for each other.  Allocation-free
// calls stage in host heap memory with a pageable copy instead (the runtime consumes the
// source before the copy call returns).
struct Stager {
    struct Slot {
        void *host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Slot slot[2];
    int next = 0;
    std::vector<uint8_t> heap;  // allocation-free calls
    // no destructor: a thread's buffers stay until the process ends (releasing them at
    // thread or process exit could run after the HIP runtime has shut down)
};
thread_local Stager t_stage;

void fill_tables(const Plan &p, uint8_t *h)
{
    memset(h, 0, p.t_bytes);
    memcpy(h + p.t_sims, p.sims.data(), p.sims.size() * sizeof(SimDesc));
    memcpy(h + p.t_samples, p.samples.data(), p.samples.size() * sizeof(SampleDesc));
    memcpy(h + p.t_tiles, p.tiles.data(), p.tiles.size() * sizeof(Tile));
    if (!p.gtiles.empty()) memcpy(h + p.t_gtiles, p.gtiles.data(), p.gtiles.size() * sizeof(GTile));
    if (!p.tiles2.empty()) memcpy(h + p.t_tiles2, p.tiles2.data(), p.tiles2.size() * sizeof(Tile));
    if (!p.gtiles2.empty()) memcpy(h + p.t_gtiles2, p.gtiles2.data(), p.gtiles2.size() * sizeof(GTile));
    if (!p.evrows.empty()) memcpy(h + p.t_evrows, p.evrows.data(), p.evrows.size() * sizeof(EvRow));
    if (!p.evvec.empty()) memcpy(h + p.t_evvec, p.evvec.data(), p.evvec.size() * sizeof(int32_t));
    if (!p.src.empty()) memcpy(h + p.t_src, p.src.data(), p.src.size() * sizeof(SrcPos));
    if (!p.order.empty()) memcpy(h + p.t_order, p.order.data(), p.order.size() * sizeof(int32_t));
}

fwi_status upload_tables(const Plan &p, uint8_t *dst, hipStream_t st, bool noalloc = false)
{
    Stager &g = t_stage;
    if (noalloc) {
        g.heap.resize(p.t_bytes);
        fill_tables(p, g.heap.data());
        HIP_TRY(hipMemcpyAsync(dst, g.heap.data(), p.t_bytes, hipMemcpyHostToDevice, st));
        return FWI_OK;
    }
    Stager::Slot &sl = g.slot[g.next];
    g.next ^= 1;
    if (sl.pending) HIP_TRY(hipEventSynchronize(sl.ev));
    sl.pending = false;
    if (sl.cap < p.t_bytes) {
        if (sl.host) HIP_TRY(hipHostFree(sl.host));
        sl.host = nullptr;
        sl.cap = 0;
        HIP_TRY(hipHostMalloc(&sl.host, p.t_bytes, hipHostMallocDefault));
        sl.cap = p.t_bytes;
    }
    fill_tables(p, (uint8_t *)sl.host);
    HIP_TRY(hipMemcpyAsync(dst, sl.host, p.t_bytes, hipMemcpyHostToDevice, st));
    if (!sl.ev) HIP_TRY(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(sl.ev, st));
    sl.pending = true;
    return FWI_OK;
}

// ------------------------------------------------------------ kernel timing

// When enabled, each run of consecutive time-step launches of one kind (a forward sweep, a
// recomputation segment, an adjoint segment) is bracketed by one pair of HIP events recorded
// on the launch's stream, so the per-launch average is the run's span over its launch count
// (kernel time plus the dispatch gaps between back-to-back launches, with no event between
// them); fwi_timing_read turns the pairs into per-kind totals.
struct Timing {
    std::mutex m;
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Run {
        hipEvent_t a, b;
        int kind;
        int64_t launches;
    };
    std::vector<Run> pending;
    double total_ms[2] = {0, 0};
    int64_t count[2] = {0, 0};
};
Timing g_timing;

hipError_t pooled_event(hipEvent_t *ev)
{
    if (g_timing.pool.empty()) return hipEventCreate(ev);
    *ev = g_timing.pool.back();
    g_timing.pool.pop_back();
    return hipSuccess;
}

// Set for the duration of an allocation-free call: its launches take no timing events.
thread_local bool t_untimed = false;

// One timed run of launches; inactive when timing is off or the stream is being captured
// (the runtime gives no elapsed time for events recorded by graph replays).
struct RunTimer {
    hipEvent_t a = nullptr;
    int kind = 0;
    hipStream_t st = nullptr;

    hipError_t begin(int k, hipStream_t s)
    {
        if (t_untimed) return hipSuccess;
        {
            std::lock_guard<std::mutex> lk(g_timing.m);
            if (!g_timing.on) return hipSuccess;
        }
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess || cs == hipStreamCaptureStatusActive) return e;
        std::lock_guard<std::mutex> lk(g_timing.m);
        e = pooled_event(&a);
        if (e != hipSuccess) return e;
        kind = k;
        st = s;
        e = hipEventRecord(a, st);
        if (e != hipSuccess) {
            g_timing.pool.push_back(a);
            a = nullptr;
        }
        return e;
    }
    hipError_t end(int64_t launches)
    {
        if (!a) return hipSuccess;
        std::lock_guard<std::mutex> lk(g_timing.m);
        hipEvent_t b;
        hipError_t e = pooled_event(&b);
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e != hipSuccess) {
            g_timing.pool.push_back(a);
            a = nullptr;
            return e;
        }
        g_timing.pending.push_back({a, b, kind, launches});
        a = nullptr;
        return hipSuccess;
    }
};

// ------------------------------------------------------------------ graphs

// Replay of whole launch sequences.  When enabled, a forward / adjoint / gradient call on a
// non-default stream captures its launches (after the table upload, which stays a plain
// copy) into a HIP graph the first time a given configuration is seen and replays the
// instantiated graph on later calls.  The key covers every value that reaches a kernel
// argument: pointers, scalars, the wavelet, table offsets and launch shapes.  Table
// contents (sources, encodings, kappa) are device data and may change between replays.
struct GraphCache {
    std::mutex m;
    bool on = false;
    struct Entry {
        uint64_t key;        // hash of `full`, compared first
        std::string full;    // every byte that went into the key
        hipGraphExec_t exec;
        uint64_t used;
    };
    std::vector<Entry> entries;
    uint64_t tick = 0;
    int64_t captures = 0, replays = 0;
};
GraphCache g_graphs;
constexpr size_t kMaxGraphs = 8;

// Graph key: the bytes of every value that reaches a kernel argument, kept whole (a cached
// graph is replayed only on a byte-for-byte match) and hashed (FNV-1a) for a quick compare.
struct KeyHash {
    uint64_t h = 1469598103934665603ULL;
    std::string full;
    void bytes(const void *p, size_t n)
    {
        const uint8_t *c = (const uint8_t *)p;
        full.append((const char *)c, n);
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ULL;
        }
    }
    template <class T>
    void add(const T &v)
    {
        bytes(&v, sizeof v);
    }
};

void hash_plan(KeyHash &k, const Plan &p, const fwi_batch *b, const fwi_time *t)
{
    k.add(p.ndim); k.add(p.bz); k.add(p.ty); k.add(p.wx); k.add(p.per_xcd); k.add(p.cells); k.add(p.coefs); k.add(p.data);
    k.add(p.max_cell); k.add(p.nt_rec); k.add(p.nlev); k.add(p.K); k.add(p.nseg); k.add(p.fwd_only);
    k.add(p.head); k.add(p.tail); k.add(p.ring); k.add(p.tail_lev0); k.add(p.overlap);
    k.add(p.nchunk_res); k.add(p.nchunk_fin);
    k.add(p.grouped); k.add(p.bzg); k.add(p.nw); k.add(p.per_xcd_g); k.add(p.gcells);
    k.add(p.two); k.add(p.two_adj); k.add(p.nw2); k.add(p.sg2); k.add(p.per_xcd2); k.add(p.per_xcd_g2);
    k.add(p.tiles2.size()); k.add(p.gtiles2.size());
    const size_t ngt = p.gtiles.size();
    k.add(ngt);
    const size_t nt = p.tiles.size();
    k.add(nt);
    const size_t offs[] = {p.t_sims, p.t_samples, p.t_tiles, p.t_gtiles, p.t_tiles2, p.t_gtiles2, p.t_evrows,
                           p.t_evvec, p.t_src, p.t_order, p.t_bytes,
                           p.o_status, p.o_tables, p.o_cf, p.o_fields, p.o_wst, p.o_ck, p.o_gacc, p.o_rho,
                           p.o_part, p.o_npart, p.o_mis, p.total};
    k.bytes(offs, sizeof offs);
    k.add(b->nsim); k.add(b->nsample);
    k.add(t->dt); k.add(t->nt); k.add(t->rec_every); k.add(t->ckpt_every); k.add(t->keep_tail);
    k.bytes(b->wavelet, sizeof(float) * t->nt);
}

void destroy_entry(GraphCache::Entry &e) { (void)hipGraphExecDestroy(e.exec); }

template <class Body>
fwi_status run_maybe_graph(const KeyHash &key, hipStream_t st, Body body)
{
    bool use;
    {
        std::lock_guard<std::mutex> lk(g_graphs.m);
        use = g_graphs.on && st != nullptr;
    }
    if (!use) return body(st);
    std::lock_guard<std::mutex> lk(g_graphs.m);
    for (auto &e : g_graphs.entries)
        if (e.key == key.h && e.full == key.full) {
            e.used = ++g_graphs.tick;
            g_graphs.replays++;
            HIP_TRY(hipGraphLaunch(e.exec, st));
            return FWI_OK;
        }
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    fwi_status s = body(st);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    GraphCache::Entry ent{key.h, key.full, nullptr, 0};
    if (s || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return s ? s : fail(FWI_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&ent.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        ent.exec = nullptr;
        return fail(FWI_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    if (g_graphs.entries.size() >= kMaxGraphs) {
        auto old = std::min_element(g_graphs.entries.begin(), g_graphs.entries.end(),
                                    [](const GraphCache::Entry &a, const GraphCache::Entry &b) { return a.used < b.used; });
        destroy_entry(*old);
        g_graphs.entries.erase(old);
    }
    ent.used = ++g_graphs.tick;
    g_graphs.entries.push_back(std::move(ent));
    g_graphs.captures++;
    HIP_TRY(hipGraphLaunch(g_graphs.entries.back().exec, st));
    return FWI_OK;
}

// ------------------------------------------------------------- the schedule

// The side stream of overlapped schedules: one per device, created on first use (default
// priority, non-blocking), and the calling thread's events that order it with the caller's
// stream.
hipError_t side_stream(hipStream_t *out)
{
    static std::mutex m;
    static std::vector<hipStream_t> streams;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(m);
    if ((size_t)dev >= streams.size()) streams.resize((size_t)dev + 1, nullptr);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = streams[dev];
    return hipSuccess;
}

struct SideEvents {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // start, recomputed x2, imaged x2
};
thread_local SideEvents t_side;

hipError_t side_events(hipEvent_t **ev)
{
    for (auto &e : t_side.ev)
        if (!e) {
            hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (r != hipSuccess) return r;
        }
    *ev = t_side.ev;
    return hipSuccess;
}

struct Dev {
    uint8_t *base;
    int *status;
    const SimDesc *sims;
    const SampleDesc *samples;
    const Tile *tiles;
    const GTile *gtiles;
    const Tile *tiles2;
    const GTile *gtiles2;
    const EvRow *evrows;
    const int32_t *evvec;
    const SrcPos *src;
    const int32_t *order;
    float *cf;
    float *lev[6];
    float *wst;
    float *ck;
    double *gacc;
    float *rho;
    double *part;
    double *npart;
    double *mis;
};

Dev carve(const Plan &p, void *ws)
{
    Dev d;
    d.base = (uint8_t *)ws;
    d.status = (int *)(d.base + p.o_status);
    uint8_t *tb = d.base + p.o_tables;
    d.sims = (const SimDesc *)(tb + p.t_sims);
    d.samples = (const SampleDesc *)(tb + p.t_samples);
    d.tiles = (const Tile *)(tb + p.t_tiles);
    d.gtiles = (const GTile *)(tb + p.t_gtiles);
    d.tiles2 = (const Tile *)(tb + p.t_tiles2);
    d.gtiles2 = (const GTile *)(tb + p.t_gtiles2);
    d.evrows = (const EvRow *)(tb + p.t_evrows);
    d.evvec = (const int32_t *)(tb + p.t_evvec);
    d.src = (const SrcPos *)(tb + p.t_src);
    d.order = p.order.empty() ? nullptr : (const int32_t *)(tb + p.t_order);
    d.cf = (float *)(d.base + p.o_cf);
    for (int l = 0; l < 6; ++l) d.lev[l] = l < p.nlev ? (float *)(d.base + p.o_fields) + (size_t)l * p.cells : nullptr;
    d.wst = (float *)(d.base + p.o_wst);
    d.ck = (float *)(d.base + p.o_ck);
    d.gacc = (double *)(d.base + p.o_gacc);
    d.rho = (float *)(d.base + p.o_rho);
    d.part = (double *)(d.base + p.o_part);
    d.npart = (double *)(d.base + p.o_npart);
    d.mis = (double *)(d.base + p.o_mis);
    return d;
}

StepArgs base_args(const Plan &p, const Dev &d)
{
    StepArgs a;
    memset(&a, 0, sizeof a);
    a.sims = d.sims;
    a.tiles = d.tiles;
    a.evrows = d.evrows;
    a.evvec = d.evvec;
    a.src = d.src;
    a.order = d.order;
    a.cf = d.cf;
    a.ntiles = (int32_t)p.tiles.size();
    a.per_xcd = p.per_xcd;
    a.rec_j = -1;
    a.samples = d.samples;
    a.gtiles = d.gtiles;
    a.ngtiles = (int32_t)p.gtiles.size();
    a.per_xcd_g = p.per_xcd_g;
    a.nw = p.nw;
    a.bzg = p.bzg;
    return a;
}

// Arguments of the two-steps-per-launch kernels: the two-step strip tables in place of the
// one-step ones.
StepArgs base_args2(const Plan &p, const Dev &d)
{
    StepArgs a = base_args(p, d);
    a.tiles = d.tiles2;
    a.ntiles = (int32_t)p.tiles2.size();
    a.per_xcd = p.per_xcd2;
    a.gtiles = d.gtiles2;
    a.ngtiles = (int32_t)p.gtiles2.size();
    a.per_xcd_g = p.per_xcd_g2;
    a.nw = p.nw2;
    a.sg = p.sg2;
    a.rec_j2 = -1;
    return a;
}

fwi_status prologue(const fwi_batch *b, const fwi_time *t, const double *kappa, void *ws, size_t ws_bytes, Plan &p,
                    bool no_overlap = false)
{
    fwi_status s = check_all(b, t, nullptr);
    if (s) return s;
    s = build_plan(b, t, kappa, p, 0, true, 0, no_overlap);
    if (s) return s;
    if (!ws) return fail(FWI_E_WORKSPACE, "null workspace");
    if ((uintptr_t)ws % kAlign) return fail(FWI_E_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < p.total) return fail(FWI_E_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, p.total);
    return FWI_OK;
}

// forward sweep n = 0..nt-1; records data into `dat`; stores imaging operands (store-all)
// or checkpoints every K steps over steps [0, head) and the imaging operands of the kept
// tail [head, nt) (K >= 1)
fwi_status run_forward(const Plan &p, const Dev &d, const fwi_batch *b, const fwi_time *t, const float *v,
                       float *dat, hipStream_t st)
{
    // a forward pass starts a new evaluation: clear the device flags first (the workspace
    // is caller memory whose initial content is unknown)
    HIP_TRY(launch_fill_i32(d.status, 1, 0, st));
    HIP_TRY(launch_prep(d.samples, b->nsample, p.max_cell, v, d.cf, d.status, st));
    HIP_TRY(launch_fill_f32(d.lev[0], 2 * p.cells, 0.0f, st));
    StepArgs a = base_args(p, d);
    a.dat = dat;
    float *cur = d.lev[0], *prev = d.lev[1];
    RunTimer tm;
    HIP_TRY(tm.begin(0, st));
    auto slot = [&](int n) { return (n + 1) % t->rec_every == 0 ? (n + 1) / t->rec_every - 1 : -1; };
    int n0 = 0;
    if (p.two) {
        // steps n+1, n+2 per launch: u^{n-1}, u^n are read from two levels and u^{n+1},
        // u^{n+2} written to the other two; an odd last step runs alone below
        StepArgs a2 = base_args2(p, d);
        a2.dat = dat;
        float *other[2] = {d.lev[2], d.lev[3]};
        int64_t launches = 0;
        for (; n0 + 1 < t->nt; n0 += 2) {
            a2.cur = cur;
            a2.prev = prev;
            a2.next = other[0];
            a2.next2 = other[1];
            a2.fn = b->wavelet[n0];
            a2.fn2 = b->wavelet[n0 + 1];
            a2.rec_j = slot(n0);
            a2.rec_j2 = slot(n0 + 1);
            a2.wst = p.fwd_only ? nullptr : d.wst + (size_t)n0 * p.cells;
            a2.wst2 = p.fwd_only ? nullptr : d.wst + (size_t)(n0 + 1) * p.cells;
            HIP_TRY(launch_step2(a2, false, st));
            float *op = prev, *oc = cur;
            prev = other[0];
            cur = other[1];
            other[0] = op;
            other[1] = oc;
            ++launches;
        }
        if (n0 < t->nt) {
            HIP_TRY(tm.end(launches));
            HIP_TRY(tm.begin(0, st));
        } else {
            HIP_TRY(tm.end(launches));
            return FWI_OK;
        }
    }
    for (int n = n0; n < t->nt; ++n) {
        a.cur = cur;
        a.prev = prev;
        a.next = prev;  // in place over u^{n-1}
        a.fn = b->wavelet[n];
        a.rec_j = slot(n);
        a.wst = nullptr;
        if (!p.fwd_only && p.K == 0)
            a.wst = d.wst + (size_t)n * p.cells;
        else if (p.K > 0 && n >= p.head)  // the kept tail, after the recomputation ring(s)
            a.wst = d.wst + (size_t)(p.tail_lev0 + n - p.head) * p.cells;
        a.cka = a.ckb = nullptr;
        if (p.K > 0 && (n + 1) % p.K == 0 && (n + 1) / p.K < p.nseg) {
            const int slot = (n + 1) / p.K;
            a.cka = d.ck + (size_t)(2 * (slot - 1)) * p.cells;
            a.ckb = d.ck + (size_t)(2 * (slot - 1) + 1) * p.cells;
        }
        HIP_TRY(launch_step(a, p.ndim, false, p.bz, p.wx, st));
        std::swap(cur, prev);
    }
    HIP_TRY(tm.end(t->nt - n0));
    return FWI_OK;
}

// adjoint sweep k = nt..1 with imaging, then finalization into grad / grad_norm
fwi_status run_adjoint(const Plan &p, const Dev &d, const fwi_batch *b, const fwi_time *t, const float *v,
                       const float *rho, float *grad, float *grad_norm, hipStream_t st)
{
    HIP_TRY(launch_fill_f64(d.gacc, p.gcells, 0.0, st));
    float *L0 = p.K == 0 ? d.lev[0] : d.lev[2];
    float *L1 = p.K == 0 ? d.lev[1] : d.lev[3];
    HIP_TRY(launch_fill_f32(L0, p.cells, 0.0f, st));
    HIP_TRY(launch_fill_f32(L1, p.cells, 0.0f, st));
    StepArgs a = base_args(p, d);
    a.rho = rho;
    a.gacc = d.gacc;
    float *lcur = L0, *lprev = L1;
    auto slot = [&](int k) { return k % t->rec_every == 0 ? k / t->rec_every - 1 : -1; };
    auto adj_step = [&](int k, const float *wimg) -> fwi_status {
        a.cur = lcur;
        a.prev = lprev;
        a.next = lprev;
        a.wimg = wimg;
        a.rec_j = slot(k);
        HIP_TRY(launch_step(a, p.ndim, true, p.bz, p.wx, st));
        std::swap(lcur, lprev);
        return FWI_OK;
    };
    // two steps per launch: lt^{k+2}, lt^{k+1} in; lt^k, lt^{k-1} out to the two spare
    // levels (the last two of the 2D plan)
    StepArgs a2 = base_args2(p, d);
    a2.rho = rho;
    a2.gacc = d.gacc;
    float *spare[2] = {p.ndim == 2 ? d.lev[p.nlev - 2] : nullptr, p.ndim == 2 ? d.lev[p.nlev - 1] : nullptr};
    RunTimer tm;
    // adjoint steps k = hi .. lo + 1, imaging with W^{k-1} at wimg(k)
    auto sweep = [&](int hi, int lo, auto wimg) -> fwi_status {
        int k = hi;
        if (p.two_adj && hi - lo >= 2) {
            HIP_TRY(tm.begin(1, st));
            int64_t launches = 0;
            for (; k - 1 >= lo + 1; k -= 2) {
                a2.cur = lcur;
                a2.prev = lprev;
                a2.next = spare[0];
                a2.next2 = spare[1];
                a2.wimg = wimg(k);
                a2.wimg2 = wimg(k - 1);
                a2.rec_j = slot(k);
                a2.rec_j2 = slot(k - 1);
                HIP_TRY(launch_step2(a2, true, st));
                float *op = lprev, *oc = lcur;
                lprev = spare[0];
                lcur = spare[1];
                spare[0] = op;
                spare[1] = oc;
                ++launches;
            }
            HIP_TRY(tm.end(launches));
        }
        if (k >= lo + 1) {  // one step per launch (or an odd last step)
            const int n1 = k - lo;
            HIP_TRY(tm.begin(1, st));
            for (; k >= lo + 1; --k) {
                fwi_status s = adj_step(k, wimg(k));
                if (s) return s;
            }
            HIP_TRY(tm.end(n1));
        }
        return FWI_OK;
    };
    if (p.K == 0) {
        fwi_status s = sweep(t->nt, 0, [&](int k) { return (const float *)(d.wst + (size_t)(k - 1) * p.cells); });
        if (s) return s;
    } else {
        // the kept tail first (its imaging operands are stored), then the checkpoint segments
        // of steps [0, head), last to first: recompute the segment from its checkpoint (its
        // imaging operands into a ring of K levels), then sweep the adjoint over it.  With
        // overlap, segment sg - 1 is recomputed on the side stream into the other ring while
        // the adjoint of segment sg runs on `st`; events order each ring's writes after the
        // adjoint that last read it.
        float *P0 = d.lev[0], *P1 = d.lev[1];
        StepArgs f = base_args(p, d);
        hipStream_t rs = st;  // stream of the recomputation
        hipEvent_t *ev = nullptr;
        if (p.overlap) {
            HIP_TRY(side_stream(&rs));
            HIP_TRY(side_events(&ev));
            HIP_TRY(hipEventRecord(ev[0], st));  // the forward, residual and fills come first
            HIP_TRY(hipStreamWaitEvent(rs, ev[0], 0));
        }
        auto ring = [&](int sg) { return d.wst + (size_t)(p.overlap ? (sg & 1) * p.K : 0) * p.cells; };
        auto recompute = [&](int sg) -> fwi_status {
            const int ns = sg * p.K, ne = std::min(ns + p.K, p.head);
            float *W = ring(sg);
            const float *cur, *prev;
            if (sg == 0) {
                HIP_TRY(launch_fill_f32(P0, 2 * p.cells, 0.0f, rs));
                cur = P0;
                prev = P1;
            } else {
                cur = d.ck + (size_t)(2 * (sg - 1)) * p.cells;
                prev = d.ck + (size_t)(2 * (sg - 1) + 1) * p.cells;
            }
            RunTimer tr;
            HIP_TRY(tr.begin(0, rs));
            for (int n = ns; n < ne; ++n) {
                float *next;
                if (prev == P0 || prev == P1)
                    next = const_cast<float *>(prev);
                else
                    next = cur == P0 ? P1 : P0;
                f.cur = cur;
                f.prev = prev;
                f.next = next;
                f.fn = b->wavelet[n];
                f.wst = W + (size_t)(n - ns) * p.cells;
                HIP_TRY(launch_step(f, p.ndim, false, p.bz, p.wx, rs));
                prev = cur;
                cur = next;
            }
            HIP_TRY(tr.end(ne - ns));
            if (p.overlap) HIP_TRY(hipEventRecord(ev[1 + (sg & 1)], rs));
            return FWI_OK;
        };
        fwi_status s = FWI_OK;
        // with overlap the last segment is recomputed on the side stream while the tail is
        // swept; without, the tail goes first (the ring may reuse its levels)
        if (p.overlap && p.nseg > 0) {
            s = recompute(p.nseg - 1);
            if (s) return s;
        }
        if (p.tail > 0) {
            const float *Wt = d.wst + (size_t)p.tail_lev0 * p.cells;
            s = sweep(t->nt, p.head, [&](int k) { return Wt + (size_t)(k - 1 - p.head) * p.cells; });
            if (s) return s;
        }
        if (!p.overlap && p.nseg > 0) {
            s = recompute(p.nseg - 1);
            if (s) return s;
        }
        for (int sg = p.nseg - 1; sg >= 0; --sg) {
            const int ns = sg * p.K, ne = std::min(ns + p.K, p.head);
            if (p.overlap) {
                if (sg >= 1) {
                    // ring (sg - 1) & 1 was last read by the adjoint of segment sg + 1
                    if (sg + 1 <= p.nseg - 1) HIP_TRY(hipStreamWaitEvent(rs, ev[3 + ((sg + 1) & 1)], 0));
                    s = recompute(sg - 1);
                    if (s) return s;
                }
                HIP_TRY(hipStreamWaitEvent(st, ev[1 + (sg & 1)], 0));
            }
            float *W = ring(sg);
            s = sweep(ne, ns, [&](int k) { return (const float *)(W + (size_t)(k - 1 - ns) * p.cells); });
            if (s) return s;
            if (p.overlap) HIP_TRY(hipEventRecord(ev[3 + (sg & 1)], st));
            if (!p.overlap && sg >= 1) {
                s = recompute(sg - 1);
                if (s) return s;
            }
        }
    }
    HIP_TRY(launch_finalize(d.samples, d.sims, b->nsample, d.gacc, v, grad, d.npart, p.nchunk_fin, d.status, st));
    if (grad_norm) HIP_TRY(launch_norm_final(d.npart, p.nchunk_fin, b->nsample, grad_norm, st));
    return FWI_OK;
}

// fwi_gradient on a given workspace; `noalloc`: stage tables without pinned memory, no
// graph replay or capture, no timing (the allocation-free entry point)
fwi_status gradient_call(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_obs, float inv_sigma2,
                         const double *kappa, float *d_pred, double *misfit, float *grad, float *grad_norm, void *ws,
                         size_t ws_bytes, hipStream_t st, bool noalloc)
{
    Plan p;
    fwi_status s = prologue(b, t, kappa, ws, ws_bytes, p, noalloc);
    if (s) return s;
    if (!v || !d_obs || !grad) return fail(FWI_E_ARG, "null model, observed data or gradient");
    if (p.fwd_only) return fail(FWI_E_ARG, "ckpt_every = -1 keeps no adjoint state");
    if (!std::isfinite(inv_sigma2) || !(inv_sigma2 > 0)) return fail(FWI_E_ARG, "inv_sigma2 must be > 0");
    Dev d = carve(p, ws);
    s = upload_tables(p, d.base + p.o_tables, st, noalloc);
    if (s) return s;
    float *dat = d_pred ? d_pred : d.rho;
    auto body = [&](hipStream_t s2) -> fwi_status {
        fwi_status r = run_forward(p, d, b, t, v, dat, s2);
        if (r) return r;
        HIP_TRY(launch_residual(d.sims, b->nsim, p.nt_rec, dat, d_obs, d.rho, inv_sigma2, d.part, p.nchunk_res,
                                d.status, s2));
        HIP_TRY(launch_misfit_final(d.part, p.nchunk_res, b->nsim, 0.5 * (double)inv_sigma2,
                                    misfit ? misfit : d.mis, s2));
        return run_adjoint(p, d, b, t, v, d.rho, grad, grad_norm, s2);
    };
    if (noalloc) {
        struct Untimed {
            Untimed() { t_untimed = true; }
            ~Untimed() { t_untimed = false; }
        } untimed;
        return body(st);
    }
    KeyHash k;
    k.add(3);
    k.add(v); k.add(d_obs); k.add(inv_sigma2); k.add(d_pred); k.add(misfit); k.add(grad); k.add(grad_norm);
    k.add(ws); k.add(st);
    hash_plan(k, p, b, t);
    return run_maybe_graph(k, st, body);
}

}  // namespace

// ================================================================== C ABI

extern "C" {

const char *fwi_status_string(fwi_status s)
{
    switch (s) {
    case FWI_OK: return "ok";
    case FWI_E_ARG: return "invalid argument";
    case FWI_E_CFL: return "time step violates the stability limit";
    case FWI_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case FWI_E_HIP: return "HIP runtime error";
    case FWI_E_NONFINITE: return "non-finite value or model above v_max found on the device";
    case FWI_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

const char *fwi_last_error(void) { return g_err.c_str(); }

fwi_status fwi_check(const fwi_batch *b, const fwi_time *t, double *worst_courant)
{
    return check_all(b, t, worst_courant);
}

fwi_status fwi_workspace_size(const fwi_batch *b, const fwi_time *t, size_t *bytes)
{
    if (!bytes) return fail(FWI_E_ARG, "null bytes");
    fwi_status s = check_all(b, t, nullptr);
    if (s) return s;
    Plan p;
    s = build_plan(b, t, nullptr, p);
    if (s) return s;
    *bytes = p.total;
    return FWI_OK;
}

fwi_status fwi_schedule(const fwi_batch *b, fwi_time *t, size_t budget_bytes)
{
    if (!t) return fail(FWI_E_ARG, "null time");
    fwi_time q = *t;
    q.ckpt_every = 0;
    q.keep_tail = 0;
    fwi_status s = check_all(b, &q, nullptr);
    if (s) return s;
    Plan p;
    s = build_plan(b, &q, nullptr, p);
    if (s) return s;
    if (p.total <= budget_bytes) {  // every imaging operand kept: one forward pass
        *t = q;
        return FWI_OK;
    }
    // checkpointed layouts differ only in the imaging levels (ring + kept tail) and the
    // checkpoint slots; everything else is the same for every K and T
    const int nt = q.nt;
    q.ckpt_every = 1;
    q.keep_tail = nt;
    p = Plan();  // build_plan appends to the plan's tables
    s = build_plan(b, &q, nullptr, p);
    if (s) return s;
    const size_t lev = (size_t)p.cells * 4;
    const size_t fixed = p.total - align_up((size_t)p.wst_levels * lev) - align_up((size_t)p.ck_slots * lev);
    const bool ovl = g_overlap.load() != 0;
    auto bytes_of = [&](int K, int T) {
        const int head = nt - T;
        const int k = std::min(K, std::max(head, 1));
        const int nseg = (head + k - 1) / k;
        const bool o = ovl && nseg >= 2;
        const int64_t ring = nseg > 0 ? (o ? 2 * k : k) : 0;
        const int64_t imaging = (!o && T >= ring) ? T : ring + T;  // the ring may reuse the tail's levels
        const int64_t ck = nseg > 0 ? 2 * (int64_t)(nseg - 1) : 0;
        return fixed + align_up((size_t)imaging * lev) + align_up((size_t)ck * lev);
    };
    // fewest forward steps = longest kept tail; then the smallest workspace.  For a
    // checkpointed part of h steps with a separate ring the levels are r K + 2 ceil(h / K) - 2
    // (ring factor r = 1, or 2 with overlap), at most 4 sqrt(h) + 4 at K = ceil(sqrt(2h / r));
    // so only intervals with r K and 2 h / K below that bound can be smallest:
    // sqrt(h) / 4 - 1 <= K <= 4 sqrt(h) + 5.  A ring that reuses the tail's levels (K <= T,
    // no overlap) costs nothing, and the checkpoints are fewest at the longest such interval,
    // K = min(T, h), which is tried as well.
    for (int T = nt; T >= 0; --T) {
        const int head = nt - T;
        int best = 0;
        size_t best_bytes = 0;
        const int khi = std::min(std::max(head, 1), 3 * (int)std::sqrt(2.0 * head) + 4);
        const int klo = head > 0 ? std::max(1, head / khi - 1) : 1;
        const int kalias = std::max(1, std::min(T, head));
        auto consider = [&](int K) {
            const size_t by = bytes_of(K, T);
            if (by <= budget_bytes && (best == 0 || by < best_bytes)) {
                best = K;
                best_bytes = by;
            }
        };
        for (int K = klo; K <= khi; ++K) consider(K);
        if (kalias > khi) consider(kalias);
        if (best) {
            q.ckpt_every = best;
            q.keep_tail = T;
            p = Plan();
            s = build_plan(b, &q, nullptr, p);
            if (s) return s;
            if (p.total != best_bytes) return fail(FWI_E_UNSUPPORTED, "schedule size model disagrees with the plan");
            *t = q;
            return FWI_OK;
        }
    }
    return fail(FWI_E_WORKSPACE, "no checkpointed schedule fits in %zu bytes", budget_bytes);
}

fwi_status fwi_forward(const fwi_batch *b, const fwi_time *t, const float *v, float *d_pred, void *ws,
                       size_t ws_bytes, void *stream)
{
    Plan p;
    fwi_status s = prologue(b, t, nullptr, ws, ws_bytes, p);
    if (s) return s;
    if (!v) return fail(FWI_E_ARG, "null model");
    hipStream_t st = (hipStream_t)stream;
    Dev d = carve(p, ws);
    s = upload_tables(p, d.base + p.o_tables, st);
    if (s) return s;
    KeyHash k;
    k.add(1);
    k.add(v); k.add(d_pred); k.add(ws); k.add(st);
    hash_plan(k, p, b, t);
    return run_maybe_graph(k, st, [&](hipStream_t s2) { return run_forward(p, d, b, t, v, d_pred ? d_pred : d.rho, s2); });
}

fwi_status fwi_adjoint(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_res,
                       const double *kappa, float *grad, float *grad_norm, void *ws, size_t ws_bytes, void *stream)
{
    Plan p;
    fwi_status s = prologue(b, t, kappa, ws, ws_bytes, p);
    if (s) return s;
    if (!v || !d_res || !grad) return fail(FWI_E_ARG, "null model, residual or gradient");
    if (p.fwd_only) return fail(FWI_E_ARG, "ckpt_every = -1 keeps no adjoint state");
    hipStream_t st = (hipStream_t)stream;
    Dev d = carve(p, ws);
    s = upload_tables(p, d.base + p.o_tables, st);
    if (s) return s;
    KeyHash k;
    k.add(2);
    k.add(v); k.add(d_res); k.add(grad); k.add(grad_norm); k.add(ws); k.add(st);
    hash_plan(k, p, b, t);
    return run_maybe_graph(k, st, [&](hipStream_t s2) -> fwi_status {
        HIP_TRY(launch_prep(d.samples, b->nsample, p.max_cell, v, d.cf, d.status, s2));
        return run_adjoint(p, d, b, t, v, d_res, grad, grad_norm, s2);
    });
}

fwi_status fwi_gradient(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_obs,
                        float inv_sigma2, const double *kappa, float *d_pred, double *misfit, float *grad,
                        float *grad_norm, void *ws, size_t ws_bytes, void *stream)
{
    return gradient_call(b, t, v, d_obs, inv_sigma2, kappa, d_pred, misfit, grad, grad_norm, ws, ws_bytes,
                         (hipStream_t)stream, false);
}

fwi_status fwi_gradient_noalloc(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_obs,
                                float inv_sigma2, const double *kappa, float *d_pred, double *misfit, float *grad,
                                float *grad_norm, void *stream)
{
    if (!b || !t) return fail(FWI_E_ARG, "null batch or time axis");
    size_t need = 0;
    {
        Plan q;
        fwi_status s = check_all(b, t, nullptr);
        if (s) return s;
        s = build_plan(b, t, nullptr, q, 0, true, 0, true);
        if (s) return s;
        need = q.total;
    }
    void *ws = nullptr;
    size_t cap = 0;
    hipError_t e = noalloc_scratch(&ws, &cap);
    if (e != hipSuccess) return fail(FWI_E_HIP, "device array of the allocation-free gradient: %s", hipGetErrorString(e));
    if (need > cap)
        return fail(FWI_E_WORKSPACE, "the batch needs a %zu-byte workspace; the allocation-free gradient holds %zu",
                    need, cap);
    return gradient_call(b, t, v, d_obs, inv_sigma2, kappa, d_pred, misfit, grad, grad_norm, ws, cap,
                         (hipStream_t)stream, true);
}

fwi_status fwi_set_overlap(int32_t on)
{
    g_overlap.store(on ? 1 : 0);
    return FWI_OK;
}

fwi_status fwi_tile_shape(const fwi_batch *b, const fwi_time *t, int32_t *bz, int32_t *wx)
{
    fwi_status s = check_all(b, t, nullptr);
    if (s) return s;
    Plan p;
    s = build_plan(b, t, nullptr, p, 0, false);
    if (s) return s;
    if (bz) *bz = p.bz;
    if (wx) *wx = p.wx;
    return FWI_OK;
}

fwi_status fwi_encode(const float *d_shots, int32_t nshot, int64_t n_per_shot, int32_t ngrp, const int32_t *grp_ptr,
                      const int32_t *grp_shot, const float *grp_w, int32_t n_entries, float *d_enc, void *stream)
{
    if (!d_shots || !grp_ptr || !grp_shot || !grp_w || !d_enc) return fail(FWI_E_ARG, "null pointer");
    if (nshot < 1 || n_per_shot < 1 || ngrp < 1 || n_entries < 0) return fail(FWI_E_ARG, "sizes must be >= 1");
    if (ngrp > 65535) return fail(FWI_E_UNSUPPORTED, "more than 65535 groups");
    HIP_TRY(launch_encode(d_shots, nshot, n_per_shot, ngrp, grp_ptr, grp_shot, grp_w, n_entries, d_enc,
                          (hipStream_t)stream));
    return FWI_OK;
}

// Philox4x64-10 (Salmon et al., SC 2011), host copy for the encoding draw.
static void philox4x64_host(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
        const unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
        const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0;
        const uint64_t n2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint64_t)p1;
        c[2] = n2;
        c[3] = (uint64_t)p0;
    }
}

fwi_status fwi_draw_encoding(uint64_t seed, uint64_t step, uint64_t sample, int32_t nshot, int32_t s, int32_t G,
                             int32_t *grp_shot, float *grp_w, double *kappa)
{
    if (!grp_shot || !grp_w || !kappa) return fail(FWI_E_ARG, "null output");
    if (nshot < 1 || s < 1 || s > nshot || G < 1) return fail(FWI_E_ARG, "need 1 <= s <= nshot and G >= 1");
    // word j of the stream: word (j mod 4) of Philox({j/4, step, sample, 0}, {seed, 0x454E43})
    auto word = [&](uint64_t j) {
        uint64_t c[4] = {j >> 2, step, sample, 0};
        philox4x64_host(c, seed, 0x454E43ULL);
        return c[j & 3];
    };
    const int per = nshot / s;
    const int P = (G + per - 1) / per;
    std::vector<int32_t> perm(nshot);
    for (int g = 0; g < G; ++g) {
        const int part = g / per, slot = g % per;
        if (slot == 0) {
            for (int i = 0; i < nshot; ++i) perm[i] = i;
            for (int i = nshot - 1; i >= 1; --i) {
                const uint64_t w = word((uint64_t)part * nshot + (uint64_t)(nshot - 1 - i));
                const int j = (int)(w % (uint64_t)(i + 1));
                std::swap(perm[i], perm[j]);
            }
        }
        for (int m = 0; m < s; ++m) {
            grp_shot[g * s + m] = perm[slot * s + m];
            const uint64_t w = word((uint64_t)P * nshot + (uint64_t)g * s + m);
            grp_w[g * s + m] = (w >> 63) ? -1.0f : 1.0f;
        }
    }
    *kappa = (double)nshot / ((double)G * s);
    return FWI_OK;
}

fwi_status fwi_langevin(int32_t nsample, const int64_t *model_off, float *v, const float *grad, const float *xi,
                        uint64_t seed, uint64_t step, float eta, float nu, float v_lo, float v_hi, void *stream)
{
    if (nsample < 1 || !model_off || !v || !grad) return fail(FWI_E_ARG, "null argument or nsample < 1");
    if (!(eta >= 0) || !(nu >= 0) || !std::isfinite(eta) || !std::isfinite(nu))
        return fail(FWI_E_ARG, "eta and nu must be finite and >= 0");
    if (!(v_lo <= v_hi)) return fail(FWI_E_ARG, "v_lo must be <= v_hi");
    for (int k = 0; k < nsample; ++k)
        if (model_off[k] < 0 || model_off[k + 1] < model_off[k]) return fail(FWI_E_ARG, "model_off not monotonic");
    hipStream_t st = (hipStream_t)stream;
    for (int k = 0; k < nsample; ++k) {
        const int64_t o = model_off[k], n = model_off[k + 1] - model_off[k];
        HIP_TRY(launch_langevin(n, v + o, grad + o, xi ? xi + o : nullptr, seed, step, (uint64_t)k, (double)eta,
                                (double)nu, (double)v_lo, (double)v_hi, st));
    }
    return FWI_OK;
}

fwi_status fwi_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_timing.m);
    g_timing.on = on != 0;
    return FWI_OK;
}

fwi_status fwi_timing_read(int32_t kind, double *total_ms, int64_t *launches, int32_t reset)
{
    if (kind < 0 || kind > 1 || !total_ms || !launches) return fail(FWI_E_ARG, "bad kind or null output");
    std::lock_guard<std::mutex> lk(g_timing.m);
    for (auto &r : g_timing.pending) {
        float ms = 0.0f;
        HIP_TRY(hipEventSynchronize(r.b));
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        g_timing.total_ms[r.kind] += ms;
        g_timing.count[r.kind] += r.launches;
        g_timing.pool.push_back(r.a);
        g_timing.pool.push_back(r.b);
    }
    g_timing.pending.clear();
    *total_ms = g_timing.total_ms[kind];
    *launches = g_timing.count[kind];
    if (reset) {
        g_timing.total_ms[kind] = 0;
        g_timing.count[kind] = 0;
    }
    return FWI_OK;
}

fwi_status fwi_graphs_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_graphs.m);
    g_graphs.on = on != 0;
    if (!g_graphs.on) {
        (void)hipDeviceSynchronize();
        for (auto &e : g_graphs.entries) destroy_entry(e);
        g_graphs.entries.clear();
    }
    return FWI_OK;
}

fwi_status fwi_graphs_stats(int64_t *captures, int64_t *replays)
{
    if (!captures || !replays) return fail(FWI_E_ARG, "null output");
    std::lock_guard<std::mutex> lk(g_graphs.m);
    *captures = g_graphs.captures;
    *replays = g_graphs.replays;
    return FWI_OK;
}

fwi_status fwi_set_tile(int32_t ndim, int32_t bz)
{
    if (ndim != 2 && ndim != 3) return fail(FWI_E_ARG, "ndim must be 2 or 3");
    if (bz != 0 && !valid_bz(ndim, bz)) return fail(FWI_E_ARG, "unsupported tile height %d", bz);
    std::lock_guard<std::mutex> lk(g_tiles.m);
    g_tiles.forced[ndim] = bz;
    return FWI_OK;
}

fwi_status fwi_set_tile_width(int32_t wx)
{
    if (wx != 0 && wx != 32 && wx != 64) return fail(FWI_E_ARG, "unsupported 3D tile width %d", wx);
    g_width3.store(wx);
    return FWI_OK;
}

fwi_status fwi_set_time_blocking(int32_t fwd_steps, int32_t adj_steps)
{
    if (fwd_steps < 0 || fwd_steps > 2 || adj_steps < 0 || adj_steps > 2)
        return fail(FWI_E_ARG, "time steps per launch must be 0 (automatic), 1 or 2");
    g_blocking_fwd.store(fwd_steps);
    g_blocking_adj.store(adj_steps);
    return FWI_OK;
}

// Time one forward step and one adjoint step of every candidate tile height on the
// caller's batch and workspace, and (2D keep-all schedules) the two-step adjoint; keep the
// fastest combination for this batch shape.
fwi_status fwi_tune(const fwi_batch *b, const fwi_time *t, const float *v, void *ws, size_t ws_bytes, void *stream,
                    const char *cache_path, int32_t *bz_out, int32_t *adj_steps_out, double *ms_out)
{
    Plan p0;
    fwi_status s = prologue(b, t, nullptr, ws, ws_bytes, p0);
    if (s) return s;
    if (!v) return fail(FWI_E_ARG, "null model");
    hipStream_t st = (hipStream_t)stream;
    const std::string sig = shape_signature(b);
    // the two-step adjoint is a candidate for 2D keep-all schedules of at least two steps
    const bool try_two = p0.ndim == 2 && !p0.fwd_only && t->nt >= 2;
    // a recorded choice for this shape wins
    if (cache_path && *cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[4096];
            const std::string needle = "\"sig\": \"" + sig + "\"";
            int found = 0, adj = 0;
            double ms = 0;
            while (fgets(line, sizeof line, f)) {
                if (!strstr(line, needle.c_str())) continue;
                const char *q = strstr(line, "\"bz\": ");
                const char *a = strstr(line, "\"adj_steps\": ");
                const char *m = strstr(line, "\"ms\": ");
                if (q && valid_bz(p0.ndim, atoi(q + 6))) {
                    found = atoi(q + 6);
                    adj = a ? atoi(a + 13) : 0;
                    if (adj != 1 && adj != 2) adj = 0;
                    ms = m ? atof(m + 6) : 0.0;
                }
            }
            fclose(f);
            if (found) {
                set_tuned(sig, found, adj);
                if (bz_out) *bz_out = found;
                if (adj_steps_out) *adj_steps_out = adj;
                if (ms_out) *ms_out = ms;
                return FWI_OK;
            }
        }
    }
    std::vector<int> cand;
    if (p0.ndim == 2)
        cand.assign(std::begin(kBz2), std::end(kBz2));
    else
        cand.assign(std::begin(kBz3), std::end(kBz3));
    // the timed launches stream through distinct imaging-operand levels, as a sweep does:
    // with one level the fields stay in the 256 MB MALL and the kernels that move fewer
    // bytes gain less than they do in a real sweep
    const int reps = 16;
    auto wlev = [&](const Plan &p, const Dev &d, int r) {
        return d.wst + (size_t)(r % std::max<int64_t>(1, p.wst_levels)) * p.cells;
    };
    // every candidate's plan (the workspace layout is the same for all of them: its table
    // region holds the largest); the candidates are timed in turn, round after round, so
    // that drift of the clocks or of the caches affects them alike; round 0 warms up and
    // each candidate keeps its best later round
    std::vector<Plan> plans(cand.size());
    for (size_t c = 0; c < cand.size(); ++c) {
        s = build_plan(b, t, nullptr, plans[c], cand[c]);
        if (s) return s;
    }
    const Plan &pl = plans.back();  // its two-step tables serve every tile height
    {
        Dev d = carve(pl, ws);
        s = upload_tables(pl, d.base + pl.o_tables, st);
        if (s) return s;
        HIP_TRY(launch_prep(d.samples, b->nsample, pl.max_cell, v, d.cf, d.status, st));
        HIP_TRY(launch_fill_f32(d.lev[0], 2 * pl.cells, 0.0f, st));
        if (!pl.fwd_only) HIP_TRY(launch_fill_f64(d.gacc, pl.gcells, 0.0, st));
    }
    hipEvent_t e0, e1, e2;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventCreate(&e2));
    std::vector<double> fwd_ms(cand.size(), 1e30), adj_ms(cand.size(), 1e30);
    double adj2_ms = 1e30;  // the two-step adjoint, per time step
    const int rounds = 4;
    for (int round = 0; round < rounds && s == FWI_OK; ++round) {
        for (size_t c = 0; c < cand.size() && s == FWI_OK; ++c) {
            const Plan &p = plans[c];
            Dev d = carve(p, ws);
            s = upload_tables(p, d.base + p.o_tables, st);
            if (s) break;
            StepArgs a = base_args(p, d);
            a.fn = 0.0f;
            a.gacc = d.gacc;
            a.rho = d.rho;
            float *cur = d.lev[0], *prev = d.lev[1];
            HIP_TRY(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) {
                a.cur = cur;
                a.prev = a.next = prev;
                a.wst = p.fwd_only ? nullptr : wlev(p, d, r);
                HIP_TRY(launch_step(a, p.ndim, false, p.bz, p.wx, st));
                std::swap(cur, prev);
            }
            HIP_TRY(hipEventRecord(e1, st));
            if (!p.fwd_only)
                for (int r = 0; r < reps; ++r) {
                    a.cur = cur;
                    a.prev = a.next = prev;
                    a.wimg = wlev(p, d, reps - 1 - r);
                    HIP_TRY(launch_step(a, p.ndim, true, p.bz, p.wx, st));
                    std::swap(cur, prev);
                }
            HIP_TRY(hipEventRecord(e2, st));
            HIP_TRY(hipEventSynchronize(e2));
            float fms = 0, ams = 0;
            HIP_TRY(hipEventElapsedTime(&fms, e0, e1));
            HIP_TRY(hipEventElapsedTime(&ams, e1, e2));
            if (round > 0) {
                fwd_ms[c] = std::min(fwd_ms[c], (double)fms / reps);
                adj_ms[c] = std::min(adj_ms[c], (double)ams / reps);
            }
        }
        if (try_two && s == FWI_OK) {  // reps launches of two steps
            Dev d = carve(pl, ws);
            s = upload_tables(pl, d.base + pl.o_tables, st);
            if (s) break;
            StepArgs a = base_args2(pl, d);
            a.rho = d.rho;
            a.gacc = d.gacc;
            float *cur = d.lev[0], *prev = d.lev[1], *o0 = d.lev[2], *o1 = d.lev[3];
            HIP_TRY(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) {
                a.cur = cur;
                a.prev = prev;
                a.next = o0;
                a.next2 = o1;
                a.wimg = wlev(pl, d, 2 * reps - 1 - 2 * r);
                a.wimg2 = wlev(pl, d, 2 * reps - 2 - 2 * r);
                HIP_TRY(launch_step2(a, true, st));
                std::swap(prev, o0);
                std::swap(cur, o1);
            }
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            float ms2 = 0;
            HIP_TRY(hipEventElapsedTime(&ms2, e0, e1));
            if (round > 0) adj2_ms = std::min(adj2_ms, ms2 / (2.0 * reps));
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    if (s) return s;
    // cost of one gradient time step: forward sweeps (recomputation included: nt + head
    // forward steps per nt with checkpoints) + adjoint
    const double fwd_per_step = p0.K > 0 ? (double)(t->nt + p0.head) / t->nt : 1.0;
    int best = 0, best_adj = 0;
    double best_ms = 1e30;
    for (size_t c = 0; c < cand.size(); ++c) {
        const double f = fwd_ms[c] * fwd_per_step;
        if (f + adj_ms[c] < best_ms) {
            best_ms = f + adj_ms[c];
            best = cand[c];
            best_adj = try_two ? 1 : 0;
        }
        if (try_two && f + adj2_ms < best_ms) {
            best_ms = f + adj2_ms;
            best = cand[c];
            best_adj = 2;
        }
    }
    set_tuned(sig, best, best_adj);
    if (cache_path && *cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"sig\": \"%s\", \"bz\": %d, \"adj_steps\": %d, \"ms\": %.6f}\n", sig.c_str(), best, best_adj,
                    best_ms);
            fclose(f);
        }
    }
    if (bz_out) *bz_out = best;
    if (adj_steps_out) *adj_steps_out = best_adj;
    if (ms_out) *ms_out = best_ms;
    return FWI_OK;
}

fwi_status fwi_copy_probe(const float *src, float *dst, int64_t n, void *stream)
{
    if (!src || !dst || n < 0 || n % 4) return fail(FWI_E_ARG, "need non-null buffers and n % 4 == 0");
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(FWI_E_ARG, "buffers must be 16-byte aligned");
    HIP_TRY(launch_copy(src, dst, n, (hipStream_t)stream));
    return FWI_OK;
}

fwi_status fwi_poll_status(void *ws, size_t ws_bytes, void *stream)
{
    if (!ws || ws_bytes < 64) return fail(FWI_E_WORKSPACE, "null or too small workspace");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(st));
    int flags = 0;
    HIP_TRY(hipMemcpy(&flags, ws, sizeof flags, hipMemcpyDeviceToHost));
    if (flags) {
        const int zero = 0;
        HIP_TRY(hipMemcpy(ws, &zero, sizeof zero, hipMemcpyHostToDevice));
        return fail(FWI_E_NONFINITE, "device flags 0x%x: %s%s%s", flags,
                    (flags & 1) ? "[model non-finite, <= 0 or above v_max] " : "",
                    (flags & 2) ? "[non-finite predicted data] " : "", (flags & 4) ? "[non-finite gradient]" : "");
    }
    return FWI_OK;
}

}  // extern "C"
