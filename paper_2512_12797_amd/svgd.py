"""Stein variational gradient descent baseline on the same solver (include/fwi_svgd.h):
particles moved by the RBF-kernel Stein direction with the median bandwidth, from the
misfit gradients of the hot path (full-shot, as in the paper's comparison, or encoded).
Python only arranges tensors and scalars and calls the library.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import fwi, nn

_bound = False


def _lib():
    global _bound
    L = fwi.lib()
    if not _bound:
        L.fwi_svgd_work_size.restype = C.c_size_t
        L.fwi_svgd_work_size.argtypes = [C.c_int32, C.c_int64]
        L.fwi_svgd_step.restype = C.c_int32
        L.fwi_svgd_step.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_float, C.c_float, C.c_float,
                                    C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p]
        L.fwi_svgd_last_error.restype = C.c_char_p
        _bound = True
    return L


def fwi_svgd_work_size(n, N):
    return int(_lib().fwi_svgd_work_size(n, N))


def fwi_svgd_step(n, N, x, grad, eps, h, v_lo, v_hi, x_out, phi=None, h_out=None, work=None, stream=None):
    nbytes = work.numel() * work.element_size() if work is not None else 0
    st = _lib().fwi_svgd_step(n, N, fwi._ptr(x), fwi._ptr(grad), eps, h, v_lo, v_hi, fwi._ptr(x_out), fwi._ptr(phi),
                              fwi._ptr(h_out), fwi._ptr(work), nbytes, fwi._stream(stream))
    if st != fwi.FWI_OK:
        raise fwi.FwiError(st, _lib().fwi_svgd_last_error().decode())


def run(sv, steps, max_update, seed, n=16, gradient="full", init_sd=20.0, h=0.0, adam_lr=None):
    """SVGD on the Survey `sv` (chains.Survey) from the smoothed start, each particle
    perturbed by seeded white noise of init_sd m/s (SVGD needs distinct particles: from
    coincident ones it moves them as one).  The step eps is set so that the largest
    first move is max_update m/s; with adam_lr the Stein direction instead drives an Adam
    ascent of that rate (m/s), moments kept over the run, then the clamp.  gradient:
    "full" (every shot, the paper's baseline) or "encoded" (Eq. 6 estimate).  Returns
    (particles, device f32 [n, nphys]; posterior-mean RMSE after each step; wall
    seconds)."""
    cfg = sv.cfg
    nphys = sv.grid.nphys
    dev = sv.dev
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    r = np.random.default_rng(seed)
    v0 = np.clip(sv.vstart.ravel()[None, :] + r.normal(0.0, init_sd, (n, nphys)), lo, hi)
    x = torch.tensor(v0, dtype=torch.float32, device=dev)
    x2 = torch.empty_like(x)
    phi = torch.empty_like(x)
    work = torch.empty((fwi_svgd_work_size(n, nphys) + 7) // 8, dtype=torch.float64, device=dev)
    vt = torch.tensor(sv.vtrue.ravel(), dtype=torch.float64, device=dev)
    rmse = []
    eps = None
    if adam_lr is not None:
        m1, m2 = torch.zeros(n * nphys, device=dev), torch.zeros(n * nphys, device=dev)
        off = np.arange(n + 1, dtype=np.int64) * nphys
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if gradient == "full":
            g = sv.full_gradient(x, n)
        else:
            g = sv.encoded_gradient(x, n, seed, k)
        g = g.reshape(n, nphys).contiguous()
        if adam_lr is not None:
            # phi only (x2 receives the clamped x and is not used); Adam with rate -adam_lr
            # on phi ascends along it; then the clamp in place
            fwi_svgd_step(n, nphys, x, g, 0.0, h, lo, hi, x2, phi, None, work)
            nn.adam(x.reshape(-1), phi.reshape(-1), m1, m2, -adam_lr, 0.9, 0.999, 1e-8, k + 1)
            fwi.fwi_langevin(off, x.reshape(-1), phi.reshape(-1), None, seed, k, 0.0, 0.0, lo, hi)
            rmse.append(float((x.double().mean(0) - vt).pow(2).mean().sqrt()))
            continue
        if eps is None:
            fwi_svgd_step(n, nphys, x, g, 0.0, h, lo, hi, x2, phi, None, work)
            eps = max_update / float(phi.abs().max())
        fwi_svgd_step(n, nphys, x, g, eps, h, lo, hi, x2, None, None, work)
        x, x2 = x2, x
        rmse.append(float((x.double().mean(0) - vt).pow(2).mean().sqrt()))
    torch.cuda.synchronize()
    return x, rmse, time.perf_counter() - t0
