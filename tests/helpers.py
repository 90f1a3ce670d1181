"""Shared test helpers: run the same seeded problem through the GPU library and the oracle."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W


def f32(a):
    """Round to FP32 and return as FP64 (what both sides consume)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def ogrid(g):
    """oracle.Grid from an fwi.Grid."""
    return oracle.Grid(nz=g.nz, nx=g.nx, dz=g.dz, dx=g.dx, nb=g.nb, v_ref=g.v_ref, ny=g.ny, dy=g.dy, ndim=g.ndim,
                       refl=g.refl)


def oracle_batch_gradient(batch, dt, nt, R, models, d_obs_sims, inv_sigma2, kappa):
    """Oracle per-sim (d_pred, misfit) and per-sample gradients for a fwi.Batch.

    models[k]: FP64 model of sample k (already FP32-rounded); d_obs_sims[s]: FP64 data.
    """
    grids = [ogrid(batch.grids[k]) for k in batch.sample_of]
    mods = [models[k] for k in batch.sample_of]
    dps, mis, gs = oracle.gradient_batch(grids, mods, dt, nt, R, batch.src_ptr, batch.src_cell,
                                         f32(batch.src_w), f32(batch.wavelet), batch.rec_ptr, batch.rec_cell,
                                         d_obs_sims, inv_sigma2=float(np.float32(inv_sigma2)), coef_fp32=True)
    grads = oracle.sample_gradient(gs, batch.sample_of, batch.nsample, kappa)
    return dps, mis, grads


def oracle_forward_sims(batch, dt, nt, R, models, coef_fp32=True):
    grids = [ogrid(batch.grids[k]) for k in batch.sample_of]
    mods = [models[k] for k in batch.sample_of]
    return oracle.forward_batch(grids, mods, dt, nt, R, batch.src_ptr, batch.src_cell, f32(batch.src_w),
                                f32(batch.wavelet), batch.rec_ptr, batch.rec_cell, coef_fp32=coef_fp32)


def split_data(flat, batch, nt_rec):
    off = batch.data_off(nt_rec)
    return [flat[off[s]:off[s + 1]].reshape(nt_rec, batch.nrec[s]) for s in range(batch.nsim)]


def split_model(flat, batch):
    return [flat[batch.model_off[k]:batch.model_off[k + 1]] for k in range(batch.nsample)]


def rel(a, b):
    return oracle.rel_l2(a, b)
