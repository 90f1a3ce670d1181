"""Batch builders: seeded workloads + encoding draws -> `fwi.Batch` descriptions.

Host-side arrangement only (which sources and receivers each simulation uses); no part
of the numerical method lives here.
"""
from __future__ import annotations

import numpy as np

import workloads as W

from . import fwi


def grid_of(cfg: W.Config, nz=None, nx=None, v_max=None) -> fwi.Grid:
    """Grid of a config; v_max defaults to the upper model bound + 10 % (the clamp range)."""
    vm = cfg.vmax * 1.1 if v_max is None else v_max
    if cfg.ndim == 3:
        return fwi.Grid(nz=nz or cfg.nz, nx=nx or cfg.nx, ny=cfg.ny, dz=cfg.h, dx=cfg.h, dy=cfg.h, nb=cfg.nb,
                        v_ref=cfg.v_ref, v_max=vm, ndim=3)
    return fwi.Grid(nz=nz or cfg.nz, nx=nx or cfg.nx, dz=cfg.h, dx=cfg.h, nb=cfg.nb, v_ref=cfg.v_ref, v_max=vm)


def shot_cells(cfg: W.Config, grid: fwi.Grid, nshot=None):
    nshot = nshot or cfg.nshot
    if cfg.ndim == 3:
        side = int(round(np.sqrt(nshot)))
        return W.surface_lattice_3d(grid.ny, grid.nx, side, side)
    return W.surface_shots_2d(grid.nx, nshot)


def receiver_cells(cfg: W.Config, grid: fwi.Grid):
    if cfg.ndim == 3:
        return W.receiver_lattice_3d(grid.ny, grid.nx, 4)
    return W.surface_receivers_2d(grid.nx)


def single_shot_batch(cfg: W.Config, grid: fwi.Grid, shots, wavelet, nsample=1):
    """One simulation per shot (weight 1), every sample gets all shots."""
    rec = receiver_cells(cfg, grid)
    sample_of, sources, receivers = [], [], []
    for k in range(nsample):
        for s in shots:
            sample_of.append(k)
            sources.append(([int(s)], [1.0]))
            receivers.append(rec)
    return fwi.Batch([grid] * nsample, sample_of, sources, receivers, wavelet)


def encoded_batch(cfg: W.Config, grids, wavelet, seed, step, s=None, G=None, nshot_of=None):
    """Encoded supergathers for every sample at one refinement step (Eq. 4 draw).

    grids[k] is sample k's grid; nshot_of(grid) its number of shots (default cfg.nshot).
    Returns (batch, groups) with groups[k] = (grp_shot [G*s], grp_w [G*s], kappa).
    """
    s = s or cfg.shots_per_group
    G = G or cfg.groups
    nshot_of = nshot_of or (lambda g: cfg.nshot)
    sample_of, sources, receivers, groups = [], [], [], []
    for k, g in enumerate(grids):
        shots = shot_cells(cfg, g, nshot_of(g))
        rec = receiver_cells(cfg, g)
        gs, gw, kap = fwi.fwi_draw_encoding(seed, step, k, len(shots), s, G)
        groups.append((gs, gw, kap))
        for gi in range(G):
            sample_of.append(k)
            sources.append((shots[gs[gi * s:(gi + 1) * s]], gw[gi * s:(gi + 1) * s]))
            receivers.append(rec)
    return fwi.Batch(list(grids), sample_of, sources, receivers, wavelet), groups


def encode_tables(groups, s, shot_base=None):
    """Encode tables for fwi_encode: group g of sample k sums the shots
    shot_base[k] + grp_shot of sample k's draw (shot_base defaults to 0: every sample
    encodes the same survey)."""
    ptr, shot, w = [0], [], []
    for k, (gs, gw, _) in enumerate(groups):
        base = 0 if shot_base is None else int(shot_base[k])
        for gi in range(len(gs) // s):
            shot.extend((base + gs[gi * s:(gi + 1) * s]).tolist())
            w.extend(gw[gi * s:(gi + 1) * s].tolist())
            ptr.append(len(shot))
    return (np.asarray(ptr, dtype=np.int32), np.asarray(shot, dtype=np.int32), np.asarray(w, dtype=np.float32))
