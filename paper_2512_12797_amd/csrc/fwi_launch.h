// fwi_launch.h -- host-callable launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fwi_internal.h"

namespace fwi {

hipError_t launch_copy(const float *src, float *dst, int64_t n, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_i32(int *p, int64_t n, int v, hipStream_t st);
hipError_t launch_prep(const SampleDesc *smp, int nsample, int64_t max_cell, const float *v, float *cf, int *status,
                       hipStream_t st);
// one time step over every tile; bz = rows (2D) or planes (3D) per tile, wx = 3D tile width
// (64 or 32 cells; the tile is 8 * 64 / wx rows high)
hipError_t launch_step(const StepArgs &a, int ndim, bool adjoint, int bz, int wx, hipStream_t st);
// two 2D time steps over every two-step strip (tables and nw of the two-step plan)
hipError_t launch_step2(const StepArgs &a, bool adjoint, hipStream_t st);
hipError_t launch_residual(const SimDesc *sims, int nsim, int nt_rec, const float *d, const float *dobs, float *rho,
                           float inv_sigma2, double *partial, int nchunk, int *status, hipStream_t st);
hipError_t launch_misfit_final(const double *partial, int nchunk, int nsim, double half_is2, double *misfit,
                               hipStream_t st);
hipError_t launch_finalize(const SampleDesc *smp, const SimDesc *sims, int nsample, const double *gacc,
                           const float *v, float *grad, double *partial, int nchunk, int *status, hipStream_t st);
hipError_t launch_norm_final(const double *partial, int nchunk, int nsample, float *norm, hipStream_t st);
hipError_t launch_encode(const float *d, int nshot, int64_t nper, int ngrp, const int32_t *gp, const int32_t *gs,
                         const float *gw, int n_entries, float *out, hipStream_t st);
hipError_t launch_langevin(int64_t n, float *v, const float *g, const float *xi, uint64_t seed, uint64_t step,
                           uint64_t sample, double eta, double nu, double lo, double hi, hipStream_t st);

}  // namespace fwi
