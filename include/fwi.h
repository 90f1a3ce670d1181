/*
 * fwi.h -- C ABI of the MI355X (gfx950) encoded-shot acoustic FWI gradient library.
 *
 * The library computes, for a batch of simulations ("sims": one posterior sample x one
 * encoded supergather each), the quantities of the paper's encoded-shot likelihood:
 *   * the predicted supergather F~(x) = sum_{i in B} w_i F_i(x)            (Eq. 4),
 *   * the encoded misfit (1/2 sigma^2) |d~ - F~(x)|^2                      (Eq. 5),
 *   * its adjoint-state gradient (one forward + one adjoint solve, stated after Eq. 5),
 *     scaled by kappa = N_s/(G s) and summed over a sample's supergathers   (Eq. 6),
 *   * the clean-space Langevin update z <- z - eta g + nu xi               (Eqs. 8-9 and
 *     the independent noise weight of the modified refinement after Alg. 1).
 *
 * Discretization (the paper names none; this is the library's definition): constant-
 * density acoustic wave equation, 8th-order central Laplacian, leapfrog in time, a
 * sponge of nb cells on every face with damping gamma = sum_a gmax_a (d_a/nb)^2,
 * gmax_a = 3 v_ref ln(1/R)/(2 nb h_a), model edge-replicated into the sponge:
 *     u^{n+1} = a u^n - b u^{n-1} + c (L u^n + q^n),
 *     a = 2/(1+gamma dt), b = (1-gamma dt)/(1+gamma dt), c = dt^2 v^2/(1+gamma dt),
 *     q^n = sum_s w_s f[n] e_{x_s} / prod h,  recorded d[j][r] = u^{(j+1)R}[x_r].
 * The gradient is the exact derivative of the discrete misfit with respect to the
 * physical-cell velocity (sponge cells fold back onto the edge cells they replicate).
 *
 * Conventions
 *   Units SI (m, s, m/s).  Row-major, x fastest, then y, then z.  A *physical cell
 *   index* is (iz*ny + iy)*nx + ix on the physical grid (ny = 1 in 2D).  Models and
 *   gradients are FP32, packed per sample at model_off[sample] (physical cells).  Data
 *   are FP32 [sim][t][receiver], packed per sim in sim order, nt/rec_every time samples.
 *
 * Memory and streams
 *   The caller owns every buffer.  Arguments documented "host" are read before the call
 *   returns; "device" pointers must stay valid until the work enqueued on `stream`
 *   completes.  The library never allocates or frees device memory; it needs one caller
 *   workspace of fwi_workspace_size() bytes (256-byte aligned) per concurrent call.
 *   Every call is asynchronous on `stream` (a hipStream_t; NULL = default stream) except
 *   fwi_poll_status, which synchronizes it.  Calls on distinct workspaces may run from
 *   distinct threads.
 *
 * Errors
 *   Every call returns an fwi_status.  Argument, stability (CFL) and workspace errors are
 *   detected on the host before anything is enqueued.  FWI_E_HIP reports a failed HIP
 *   runtime call.  Device-side findings (non-finite model or results, a model above the
 *   declared v_max) are latched in the workspace from the start of the latest
 *   fwi_forward / fwi_gradient (which clear them) through any following fwi_adjoint, and
 *   are returned by fwi_poll_status.
 *   fwi_last_error() gives a thread-local text for the last non-OK status.
 *
 * Determinism: no floating-point atomics; reductions have a fixed order, so identical
 * inputs and launch configuration give bitwise-identical outputs.
 */
#ifndef FWI_MI355_H
#define FWI_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fwi_status;
enum {
    FWI_OK = 0,
    FWI_E_ARG = 1,          /* malformed argument (host-detected, nothing enqueued) */
    FWI_E_CFL = 2,          /* v_max * dt * sqrt(sum h^-2) exceeds sqrt(315/512)    */
    FWI_E_WORKSPACE = 3,    /* workspace missing, misaligned or too small           */
    FWI_E_HIP = 4,          /* a HIP runtime call failed                            */
    FWI_E_NONFINITE = 5,    /* device found a non-finite value or v > v_max         */
    FWI_E_UNSUPPORTED = 6   /* valid request the library does not implement        */
};

/* One grid (shared by all sims of a sample). */
typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t nz, ny, nx;    /* physical cells per axis; ny must be 1 when ndim == 2 */
    double dz, dy, dx;     /* spacing (m); dy ignored in 2D */
    int32_t nb;            /* sponge cells on every face (>= 0) */
    double v_ref;          /* sponge reference velocity (m/s), > 0 */
    double refl;           /* sponge target reflection coefficient R, 0 < R < 1 */
    double v_max;          /* upper bound of the model on this grid (m/s): CFL is
                              checked with it and the device verifies v <= v_max */
} fwi_grid;

typedef struct {
    double dt;             /* internal time step (s) */
    int32_t nt;            /* number of internal steps */
    int32_t rec_every;     /* data are recorded every rec_every steps; nt % rec_every == 0 */
    int32_t ckpt_every;    /* 0: keep every step's imaging operand (no recomputation);
                              K >= 1: checkpoint every K steps and recompute per segment;
                              -1: forward only (no adjoint state; smallest workspace) */
    int32_t keep_tail;     /* with K >= 1: the forward also keeps the imaging operands of
                              the last keep_tail steps (0 <= keep_tail <= nt), which the
                              adjoint then reads without recomputing them; checkpoints
                              cover the first nt - keep_tail steps.  A tail at least
                              as long as the recomputation ring (K levels; overlap off)
                              also holds the ring once the adjoint has read it.  Must be
                              0 when ckpt_every <= 0.  Results are identical for every
                              value. */
} fwi_time;

/* A batch of simulations.  Every array here is HOST memory. */
typedef struct {
    int32_t nsim;                /* simulations (sample x supergather) */
    int32_t nsample;             /* posterior samples */
    const fwi_grid *grid;        /* [nsample] grid of each sample */
    const int64_t *model_off;    /* [nsample+1] element offsets of each sample's model /
                                    gradient (physical cells) in the packed arrays */
    const int32_t *sample_of;    /* [nsim] sample of each sim (sims of one sample must be
                                    contiguous and in increasing sample order) */
    const int32_t *src_ptr;      /* [nsim+1] CSR into src_cell / src_w */
    const int32_t *src_cell;     /* physical cell index of each encoded source */
    const float *src_w;          /* encoding weight w_i of each source (e.g. +-1) */
    const int32_t *rec_ptr;      /* [nsim+1] CSR into rec_cell */
    const int32_t *rec_cell;     /* physical cell index of each receiver (distinct per sim) */
    const float *wavelet;        /* [nt] source time function f[n] at t = n dt */
} fwi_batch;

/* Static description of a status code. */
const char *fwi_status_string(fwi_status s);

/* Thread-local detail of the last non-OK status returned on this thread. */
const char *fwi_last_error(void);

/*
 * Host-only validation of a batch and time axis, including the stability limit of the
 * leapfrog / 8th-order scheme: v_max dt sqrt(sum_a h_a^-2) <= sqrt(315/512)
 * (the Laplacian's largest eigenvalue magnitude is (2048/315) sum_a h_a^-2).
 * worst_courant (host, nullable) receives max over grids of v_max dt sqrt(sum h^-2).
 */
fwi_status fwi_check(const fwi_batch *b, const fwi_time *t, double *worst_courant);

/* Workspace bytes needed by fwi_forward / fwi_adjoint / fwi_gradient for (b, t). */
fwi_status fwi_workspace_size(const fwi_batch *b, const fwi_time *t, size_t *bytes);

/*
 * Schedule of the adjoint state for a workspace budget (host-only).  Reads t->dt, nt and
 * rec_every and sets t->ckpt_every and t->keep_tail to the schedule whose workspace fits
 * in budget_bytes with the fewest forward time steps per gradient (nt plus the
 * recomputed ones): every imaging operand kept (ckpt_every 0) if that fits, else the
 * checkpoint interval K and kept tail T with the largest T, then the smallest workspace.
 * The checkpoint/recompute schedule is the adjoint-state method's memory/compute trade
 * (the gradient stated after Eq. 5 needs every forward state in reverse order).  Follows
 * the process-wide settings that change workspace sizes (fwi_set_overlap).
 * FWI_E_WORKSPACE if not even the smallest checkpointed schedule fits; *t is then
 * unchanged.
 */
fwi_status fwi_schedule(const fwi_batch *b, fwi_time *t, size_t budget_bytes);

/*
 * Forward solve of every sim (F~(x) of Eq. 4 for each supergather).
 *   v       device FP32 models, packed per sample at model_off (physical cells).
 *   d_pred  device FP32 [sim][nt/R][nrec_sim] recorded data (nullable).
 *   ws      device workspace; on return it holds what fwi_adjoint needs for the same
 *           (b, t, v): checkpoints or imaging operands.
 */
fwi_status fwi_forward(const fwi_batch *b, const fwi_time *t, const float *v, float *d_pred, void *ws,
                       size_t ws_bytes, void *stream);

/*
 * Adjoint solve + zero-lag imaging for a given data residual (the adjoint-state gradient
 * stated after Eq. 5), then per-sample finalization (Eq. 6):
 *   grad_s = kappa_s * sum_{sims of s} fold((2/v_pad) sum_k lt^k (L u^{k-1} + q^{k-1})).
 *   d_res     device FP32 [sim][nt/R][nrec_sim]: dPhi/dd (e.g. (d - d_obs)/sigma^2).
 *   kappa     host [nsample] scale per sample (nullable: 1).
 *   grad      device FP32 packed per sample (physical cells).
 *   grad_norm device FP32 [nsample] |grad_s|_2 (nullable).
 * Requires ws filled by fwi_forward with the same (b, t, v).  Sources may not change
 * between the two calls.
 */
fwi_status fwi_adjoint(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_res,
                       const double *kappa, float *grad, float *grad_norm, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Fused encoded misfit and gradient (Eqs. 4-6): forward, residual
 * rho = (d - d_obs) inv_sigma2, misfit phi_sim = (inv_sigma2/2) |d - d_obs|^2, adjoint,
 * imaging and finalization.
 *   d_obs     device FP32 encoded observed data d~ [sim][nt/R][nrec_sim].
 *   d_pred    device FP32, same shape (nullable).
 *   misfit    device FP64 [nsim] (nullable).
 *   grad, grad_norm, kappa as in fwi_adjoint.
 */
fwi_status fwi_gradient(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_obs,
                        float inv_sigma2, const double *kappa, float *d_pred, double *misfit, float *grad,
                        float *grad_norm, void *ws, size_t ws_bytes, void *stream);

/* Largest workspace the allocation-free gradient can use, in bytes. */
#define FWI_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/*
 * fwi_gradient_noalloc -- fwi_gradient for callers that cannot allocate memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Arguments, outputs and arithmetic are those of fwi_gradient without the workspace
 * arguments: the workspace is a device array of FWI_NOALLOC_MAX_BYTES that the library
 * holds on every GPU it runs on (from the loading of the library until the process ends),
 * taken on the current device.
 *   Size: a batch whose fwi_workspace_size exceeds FWI_NOALLOC_MAX_BYTES is rejected with
 *   FWI_E_WORKSPACE before anything is enqueued.  Other errors as fwi_gradient.
 *   The call allocates no device or pinned host memory (its tables are copied from host
 *   heap memory), never replays or records a graph (fwi_graphs_enable does not apply)
 *   and takes no kernel timings (fwi_timing_enable does not apply).
 *   Sharing: every call on one GPU uses that GPU's one array, and each call starts by
 *   clearing what must start at zero.  Calls ordered on one stream are fine; calls that
 *   overlap in time on one GPU (other streams, other threads) race and give undefined
 *   results.  fwi_forward / fwi_adjoint / fwi_gradient on caller workspaces are unaffected.
 *   Device findings (non-finite values, a model outside (0, v_max]) cannot be polled for
 *   this call (fwi_poll_status needs a caller workspace); non-finite values propagate to
 *   the outputs.
 */
fwi_status fwi_gradient_noalloc(const fwi_batch *b, const fwi_time *t, const float *v, const float *d_obs,
                                float inv_sigma2, const double *kappa, float *d_pred, double *misfit, float *grad,
                                float *grad_norm, void *stream);

/*
 * Encoded observed data (Eq. 4): d_enc[g] = sum_{k in grp_ptr[g]..grp_ptr[g+1]-1}
 * grp_w[k] d_shots[grp_shot[k]], each item n_per_shot floats.
 *   d_shots  device FP32 [nshot][n_per_shot];  d_enc device FP32 [ngrp][n_per_shot].
 *   grp_ptr [ngrp+1], grp_shot [n_entries], grp_w [n_entries]: DEVICE arrays.
 * Summation order is the group's listed order, in FP32.  The device checks the group
 * table (0 <= grp_ptr[g] <= grp_ptr[g+1] <= n_entries, 0 <= shot < nshot); a malformed
 * group's output is filled with NaN rather than read out of bounds.
 */
fwi_status fwi_encode(const float *d_shots, int32_t nshot, int64_t n_per_shot, int32_t ngrp,
                      const int32_t *grp_ptr, const int32_t *grp_shot, const float *grp_w, int32_t n_entries,
                      float *d_enc, void *stream);

/*
 * Encoding draw of one sample at one refinement step (the mini-batch B and the weights
 * of Eq. 4, redrawn every iteration): G supergathers of s shots from random partitions
 * (Fisher-Yates) of the nshot shots, Rademacher +-1 weights; kappa = nshot/(G s).
 * Counter-based (Philox4x64-10, key {seed, 0x454E43}, counter {word/4, step, sample, 0}),
 * so a draw is reproducible from (seed, step, sample).  Host-only.
 *   grp_shot [G*s], grp_w [G*s], kappa: host outputs.  Requires s <= nshot.
 */
fwi_status fwi_draw_encoding(uint64_t seed, uint64_t step, uint64_t sample, int32_t nshot, int32_t s,
                             int32_t G, int32_t *grp_shot, float *grp_w, double *kappa);

/*
 * Clean-space Langevin refinement (Eqs. 8-9; nu independent of eta in the modified
 * refinement, nu = sqrt(2 eta) for the plain unadjusted Langevin step):
 *     v <- clamp(v - eta grad + nu xi, v_lo, v_hi)   for every cell of every sample.
 *   v, grad  device FP32 packed per sample (model_off host [nsample+1]).
 *   xi       device FP32 noise (nullable).  When NULL the noise is generated in-kernel:
 *            standard normals from Philox4x64-10 (key {seed, 0x4C414E47}, counter
 *            {cell/4, step, sample, 0}) with Box-Muller on word pairs (0,1), (2,3).
 */
fwi_status fwi_langevin(int32_t nsample, const int64_t *model_off, float *v, const float *grad,
                        const float *xi, uint64_t seed, uint64_t step, float eta, float nu, float v_lo,
                        float v_hi, void *stream);

/*
 * Synchronize `stream` and report the device-side findings latched in ws since the latest
 * fwi_forward / fwi_gradient on it (FWI_E_NONFINITE), clearing them.
 */
fwi_status fwi_poll_status(void *ws, size_t ws_bytes, void *stream);

/*
 * Kernel timing for roofline measurement.  While enabled (process-wide), each run of
 * consecutive time-step launches of one kind inside fwi_forward / fwi_adjoint /
 * fwi_gradient (a forward sweep, or one checkpoint segment's recomputation or adjoint
 * sweep) is bracketed by two HIP events recorded on the launch's stream, with no event
 * between its launches; launches captured into a replay graph are not timed.
 * fwi_timing_read synchronizes the events and returns the accumulated time and launch
 * count of one kind: 0 = forward or recomputation step, 1 = adjoint + imaging step (time /
 * count = average launch duration including the dispatch gaps of back-to-back launches);
 * reset != 0 zeroes that kind afterwards.
 */
fwi_status fwi_timing_enable(int32_t on);
fwi_status fwi_timing_read(int32_t kind, double *total_ms, int64_t *launches, int32_t reset);

/*
 * Plain device copy dst[i] = src[i], i < n (n % 4 == 0, 16-byte aligned device buffers):
 * the achievable-HBM-bandwidth reference and the calibration kernel for byte counters.
 */
fwi_status fwi_copy_probe(const float *src, float *dst, int64_t n, void *stream);

/*
 * Graph replay (process-wide).  While enabled, fwi_forward / fwi_adjoint / fwi_gradient on a
 * non-default stream capture their kernel launches into a HIP graph the first time a given
 * configuration (pointers, scalars, wavelet, batch shape, time axis) is seen and replay the
 * instantiated graph on later calls; the geometry tables are still uploaded by a plain
 * copy before each replay, so encodings, sources and kappa may change between calls.  Up to
 * 8 graphs are cached (least recently used evicted).  Disabling frees them.  Calls on the
 * default (NULL) stream, and calls while kernel timing is enabled, launch directly.
 * fwi_graphs_stats returns the number of captures and replays so far.
 */
fwi_status fwi_graphs_enable(int32_t on);
fwi_status fwi_graphs_stats(int64_t *captures, int64_t *replays);

/*
 * Tile height of the step kernels: rows per 2D tile (8, 16, 32) or planes per 3D forward
 * tile (16, 24, 32, 40; the 3D adjoint's tiles are 16 planes high); the one-step 2D adjoint sweeps strips of 8 rows when the tile height is 8 and
 * of 16 rows otherwise.  fwi_set_tile forces one for every batch of that dimensionality
 * (0 returns to automatic choice).  fwi_tune times one forward and one adjoint step of
 * every candidate on the caller's batch, model v (device) and workspace (>=
 * fwi_workspace_size, whose tables are sized for any candidate); for 2D keep-all schedules
 * of at least two steps it also times the two-step adjoint (see fwi_set_time_blocking).  It
 * keeps the fastest combination for this batch shape (the multiset of padded grid sizes)
 * for later calls and returns it: bz_out, adj_steps_out (1 or 2; 0 where the two-step
 * adjoint does not apply) and the cost of one gradient time step in ms_out; all three are
 * nullable.  With cache_path (nullable) the choice is read from / appended to a JSON-lines
 * file ({"sig": ..., "bz": ..., "adj_steps": ..., "ms": ...}) so that later processes skip
 * the timing.  The workspace content is overwritten.
 */
fwi_status fwi_set_tile(int32_t ndim, int32_t bz);

/*
 * Width of the 3D step kernels' tiles, process-wide: 64 cells (8 rows per tile, one row
 * per wavefront) or 32 cells (16 rows per tile, two rows per wavefront); 0 (the default)
 * picks 32 where 32-wide tiles run fewer lanes over the batch's padded grids (x extent
 * rounded up to the width, y extent to the tile's rows) than 64-wide ones.  Results
 * are identical for both widths; only the speed differs.  The workspace size covers
 * either width.
 */
fwi_status fwi_set_tile_width(int32_t wx);

/*
 * Checkpointed schedules (ckpt_every = K >= 1): recomputation of a segment beside the
 * adjoint of the segment after it, process-wide (default off).  While the adjoint sweeps
 * segment s on the caller's stream, segment s - 1 is recomputed on a library-owned side
 * stream (one per device, default priority) into a second ring of K imaging-operand
 * levels; events order every ring write after the adjoint sweep that last read it, and
 * the caller's stream waits for the side stream before it reads a segment, so a call is
 * still complete when its stream's work is.  Results are identical with and without the
 * overlap.  The workspace then holds 2K instead of K imaging levels (fwi_workspace_size
 * follows the setting at the time it is called; change it before sizing workspaces).
 * Graph capture includes the side stream's work.  fwi_gradient_noalloc never overlaps.
 */
fwi_status fwi_set_overlap(int32_t on);

/*
 * Tile shape the step kernels would use for (b, t) under the current process-wide
 * settings (forced or tuned tile height, tile width): bz = rows per 2D tile or planes per
 * 3D tile, wx = tile width in cells (64 in 2D; 64 or 32 in 3D).  Host-only; both outputs
 * nullable.
 */
fwi_status fwi_tile_shape(const fwi_batch *b, const fwi_time *t, int32_t *bz, int32_t *wx);
fwi_status fwi_tune(const fwi_batch *b, const fwi_time *t, const float *v, void *ws, size_t ws_bytes, void *stream,
                    const char *cache_path, int32_t *bz_out, int32_t *adj_steps_out, double *ms_out);

/*
 * Time steps per launch of the 2D sweeps, process-wide: the forward sweep of the keep-all
 * schedule (fwd_steps; ckpt_every 0 or -1) and the adjoint sweep of either schedule
 * (adj_steps; with checkpoints, within each recomputed segment).  Each is 1 or 2 (forced),
 * or 0 (automatic, the default).  Automatic means one forward step per launch, and for the
 * adjoint the choice fwi_tune made for the batch shape, else two steps per launch.
 *
 * With 2, one sweep advances the wavefield (or the adjoint field) by two steps of the
 * recursion of the discretized wave equation (Sec. 2). It reads the two old levels once
 * per two steps. Each wavefront then covers a strip of 56 columns and 16 rows, and also
 * computes the first step on a 4-cell margin around it: the halo of the second step.
 *
 * The data and the imaging operands are bit-identical to those of one step per launch.
 * The per-sample gradient sums the same FP64 products in another order.
 *
 * An odd last step (of the sweep, or of a segment) is launched alone.  3D takes one step
 * per launch, and so does the recomputation of a checkpointed forward.  The setting applies
 * to calls that start after it.  A captured graph keeps
 * the setting it was captured with (the graph key includes it).  Returns FWI_E_ARG for
 * other values.
 */
fwi_status fwi_set_time_blocking(int32_t fwd_steps, int32_t adj_steps);

#ifdef __cplusplus
}
#endif
#endif /* FWI_MI355_H */
