"""Thin Python binding of ``libfwi_mi355.so`` (include/fwi.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; PyTorch provides device
memory (tensors) and the stream.  If the library is not built this module raises -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwi_mi355.so")

FWI_OK, FWI_E_ARG, FWI_E_CFL, FWI_E_WORKSPACE, FWI_E_HIP, FWI_E_NONFINITE, FWI_E_UNSUPPORTED = range(7)


class FwiError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__("fwi status %d: %s" % (status, detail))
        self.status = status


class FwiGrid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
                ("dz", C.c_double), ("dy", C.c_double), ("dx", C.c_double), ("nb", C.c_int32),
                ("v_ref", C.c_double), ("refl", C.c_double), ("v_max", C.c_double)]


class FwiTime(C.Structure):
    _fields_ = [("dt", C.c_double), ("nt", C.c_int32), ("rec_every", C.c_int32), ("ckpt_every", C.c_int32),
                ("keep_tail", C.c_int32)]


class FwiBatch(C.Structure):
    _fields_ = [("nsim", C.c_int32), ("nsample", C.c_int32), ("grid", C.POINTER(FwiGrid)),
                ("model_off", C.POINTER(C.c_int64)), ("sample_of", C.POINTER(C.c_int32)),
                ("src_ptr", C.POINTER(C.c_int32)), ("src_cell", C.POINTER(C.c_int32)),
                ("src_w", C.POINTER(C.c_float)), ("rec_ptr", C.POINTER(C.c_int32)),
                ("rec_cell", C.POINTER(C.c_int32)), ("wavelet", C.POINTER(C.c_float))]


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfwi_mi355.so is not built: run `python -m paper_2512_12797_amd.build` "
                              "(the HIP library is required; there is no fallback)")
        L = C.CDLL(LIB_PATH)
        L.fwi_status_string.restype = C.c_char_p
        L.fwi_last_error.restype = C.c_char_p
        for name in ("fwi_check", "fwi_workspace_size", "fwi_forward", "fwi_adjoint", "fwi_gradient",
                     "fwi_encode", "fwi_draw_encoding", "fwi_langevin", "fwi_poll_status"):
            getattr(L, name).restype = C.c_int32
        L.fwi_check.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.POINTER(C.c_double)]
        L.fwi_workspace_size.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.POINTER(C.c_size_t)]
        L.fwi_schedule.restype = C.c_int32
        L.fwi_schedule.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.c_size_t]
        L.fwi_forward.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.c_void_p]
        L.fwi_adjoint.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.fwi_gradient.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.c_void_p, C.c_void_p, C.c_float,
                                   C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_size_t, C.c_void_p]
        L.fwi_gradient_noalloc.restype = C.c_int32
        L.fwi_gradient_noalloc.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.c_void_p, C.c_void_p,
                                           C.c_float, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p]
        L.fwi_encode.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_int32, C.c_void_p, C.c_void_p]
        L.fwi_draw_encoding.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_float), C.POINTER(C.c_double)]
        L.fwi_langevin.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                   C.c_uint64, C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]
        L.fwi_poll_status.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p]
        for name in ("fwi_graphs_enable", "fwi_graphs_stats", "fwi_set_tile", "fwi_tune", "fwi_set_time_blocking"):
            getattr(L, name).restype = C.c_int32
        L.fwi_set_time_blocking.argtypes = [C.c_int32, C.c_int32]
        L.fwi_graphs_enable.argtypes = [C.c_int32]
        L.fwi_graphs_stats.argtypes = [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.fwi_set_tile.argtypes = [C.c_int32, C.c_int32]
        L.fwi_set_tile_width.restype = C.c_int32
        L.fwi_set_tile_width.argtypes = [C.c_int32]
        L.fwi_set_overlap.restype = C.c_int32
        L.fwi_set_overlap.argtypes = [C.c_int32]
        L.fwi_tile_shape.restype = C.c_int32
        L.fwi_tile_shape.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]
        L.fwi_tune.argtypes = [C.POINTER(FwiBatch), C.POINTER(FwiTime), C.c_void_p, C.c_void_p, C.c_size_t,
                               C.c_void_p, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]
        for name in ("fwi_timing_enable", "fwi_timing_read", "fwi_copy_probe"):
            getattr(L, name).restype = C.c_int32
        L.fwi_timing_enable.argtypes = [C.c_int32]
        L.fwi_timing_read.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
        L.fwi_copy_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        _lib = L
    return _lib


def _ok(status):
    if status != FWI_OK:
        raise FwiError(status, lib().fwi_last_error().decode())


# ---------------------------------------------------------------- batches

@dataclass
class Grid:
    """A sample's grid: physical cells nz x ny x nx (ny = 1 in 2D), spacings, sponge."""
    nz: int
    nx: int
    dz: float
    dx: float
    nb: int
    v_ref: float
    v_max: float
    ny: int = 1
    dy: float = 1.0
    ndim: int = 2
    refl: float = 1e-3

    @property
    def nphys(self):
        return self.nz * self.ny * self.nx

    def c(self):
        return FwiGrid(self.ndim, self.nz, self.ny, self.nx, self.dz, self.dy, self.dx, self.nb, self.v_ref,
                       self.refl, self.v_max)


class Batch:
    """Host description of a batch of simulations.

    grids[k] is sample k's grid; sample_of[s] the sample of sim s; sources[s] = (cells,
    weights) and receivers[s] = cells (physical cell indices).  Keeps the host arrays
    alive for as long as the ctypes struct is used.
    """

    def __init__(self, grids, sample_of, sources, receivers, wavelet):
        self.grids = list(grids)
        self.nsample = len(self.grids)
        self.sample_of = np.ascontiguousarray(sample_of, dtype=np.int32)
        self.nsim = len(self.sample_of)
        self.model_off = np.zeros(self.nsample + 1, dtype=np.int64)
        self.model_off[1:] = np.cumsum([g.nphys for g in self.grids])
        self.src_ptr = np.zeros(self.nsim + 1, dtype=np.int32)
        self.src_ptr[1:] = np.cumsum([len(s[0]) for s in sources])
        def cat(parts, dtype):
            return np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=dtype) for x in parts])
                                        if len(parts) else np.zeros(0), dtype=dtype)

        self.src_cell = cat([s[0] for s in sources], np.int32)
        self.src_w = cat([s[1] for s in sources], np.float32)
        self.rec_ptr = np.zeros(self.nsim + 1, dtype=np.int32)
        self.rec_ptr[1:] = np.cumsum([len(r) for r in receivers])
        self.rec_cell = cat(receivers, np.int32)
        self.wavelet = np.ascontiguousarray(wavelet, dtype=np.float32)
        self.nrec = np.diff(self.rec_ptr)
        self._grid_arr = (FwiGrid * self.nsample)(*[g.c() for g in self.grids])
        self._c = FwiBatch(self.nsim, self.nsample, self._grid_arr,
                           self.model_off.ctypes.data_as(C.POINTER(C.c_int64)),
                           self.sample_of.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.src_ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.src_cell.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.src_w.ctypes.data_as(C.POINTER(C.c_float)),
                           self.rec_ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.rec_cell.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.wavelet.ctypes.data_as(C.POINTER(C.c_float)))

    @property
    def c(self):
        return C.byref(self._c)

    def data_size(self, nt_rec):
        return int(nt_rec * self.rec_ptr[-1])

    def data_off(self, nt_rec):
        return np.concatenate([[0], np.cumsum(self.nrec.astype(np.int64) * nt_rec)])

    @property
    def model_size(self):
        return int(self.model_off[-1])


def time_axis(dt, nt, rec_every=1, ckpt_every=0, keep_tail=0):
    return FwiTime(float(dt), int(nt), int(rec_every), int(ckpt_every), int(keep_tail))


# ----------------------------------------------------------- device helpers

def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check_f32(t, n, name):
    import torch
    if t.dtype != torch.float32 or t.numel() < n:
        raise ValueError("%s: need a float32 device tensor with >= %d elements" % (name, n))


def _kappa(kappa, nsample):
    if kappa is None:
        return None
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nsample,)))
    return k, k.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------------ the C ABI

def fwi_check(batch: Batch, time: FwiTime) -> float:
    """Host validation; returns the worst Courant number v_max dt sqrt(sum h^-2)."""
    w = C.c_double(0.0)
    _ok(lib().fwi_check(batch.c, C.byref(time), C.byref(w)))
    return w.value


def fwi_workspace_size(batch: Batch, time: FwiTime) -> int:
    n = C.c_size_t(0)
    _ok(lib().fwi_workspace_size(batch.c, C.byref(time), C.byref(n)))
    return n.value


def fwi_schedule(batch: Batch, time: FwiTime, budget_bytes: int) -> FwiTime:
    """A copy of ``time`` with ckpt_every and keep_tail chosen for the budget."""
    t = FwiTime(time.dt, time.nt, time.rec_every, time.ckpt_every, time.keep_tail)
    _ok(lib().fwi_schedule(batch.c, C.byref(t), C.c_size_t(int(budget_bytes))))
    return t


def alloc_workspace(batch: Batch, time: FwiTime, device="cuda"):
    import torch
    n = fwi_workspace_size(batch, time)
    ws = torch.empty(n, dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace not 256-byte aligned")
    return ws


def fwi_forward(batch, time, v, d_pred, ws, stream=None):
    _check_f32(v, batch.model_size, "v")
    if d_pred is not None:
        _check_f32(d_pred, batch.data_size(time.nt // time.rec_every), "d_pred")
    _ok(lib().fwi_forward(batch.c, C.byref(time), _ptr(v), _ptr(d_pred), _ptr(ws), ws.numel(), _stream(stream)))


def fwi_adjoint(batch, time, v, d_res, kappa, grad, grad_norm, ws, stream=None):
    _check_f32(v, batch.model_size, "v")
    _check_f32(d_res, batch.data_size(time.nt // time.rec_every), "d_res")
    _check_f32(grad, batch.model_size, "grad")
    k = _kappa(kappa, batch.nsample)
    _ok(lib().fwi_adjoint(batch.c, C.byref(time), _ptr(v), _ptr(d_res), k[1] if k else None, _ptr(grad),
                          _ptr(grad_norm), _ptr(ws), ws.numel(), _stream(stream)))


def fwi_gradient(batch, time, v, d_obs, inv_sigma2, kappa, d_pred, misfit, grad, grad_norm, ws, stream=None):
    import torch
    _check_f32(v, batch.model_size, "v")
    nd = batch.data_size(time.nt // time.rec_every)
    _check_f32(d_obs, nd, "d_obs")
    if d_pred is not None:
        _check_f32(d_pred, nd, "d_pred")
    if misfit is not None and (misfit.dtype != torch.float64 or misfit.numel() < batch.nsim):
        raise ValueError("misfit: need a float64 device tensor with nsim elements")
    _check_f32(grad, batch.model_size, "grad")
    k = _kappa(kappa, batch.nsample)
    _ok(lib().fwi_gradient(batch.c, C.byref(time), _ptr(v), _ptr(d_obs), C.c_float(inv_sigma2),
                           k[1] if k else None, _ptr(d_pred), _ptr(misfit), _ptr(grad), _ptr(grad_norm),
                           _ptr(ws), ws.numel(), _stream(stream)))


def fwi_gradient_noalloc(batch, time, v, d_obs, inv_sigma2, kappa, d_pred, misfit, grad, grad_norm,
                         stream=None):
    """fwi_gradient on the library's own device array (FWI_NOALLOC_MAX_BYTES): no workspace."""
    import torch
    _check_f32(v, batch.model_size, "v")
    nd = batch.data_size(time.nt // time.rec_every)
    _check_f32(d_obs, nd, "d_obs")
    if d_pred is not None:
        _check_f32(d_pred, nd, "d_pred")
    if misfit is not None and (misfit.dtype != torch.float64 or misfit.numel() < batch.nsim):
        raise ValueError("misfit: need a float64 device tensor with nsim elements")
    _check_f32(grad, batch.model_size, "grad")
    k = _kappa(kappa, batch.nsample)
    _ok(lib().fwi_gradient_noalloc(batch.c, C.byref(time), _ptr(v), _ptr(d_obs), C.c_float(inv_sigma2),
                                   k[1] if k else None, _ptr(d_pred), _ptr(misfit), _ptr(grad), _ptr(grad_norm),
                                   _stream(stream)))


NOALLOC_MAX_BYTES = 64 << 20  # FWI_NOALLOC_MAX_BYTES


def fwi_encode(d_shots, grp_ptr, grp_shot, grp_w, d_enc, stream=None):
    """grp_* are device tensors (int32, int32, float32); d_shots [nshot, ...] float32."""
    nshot = d_shots.shape[0]
    nper = d_shots.numel() // nshot
    ngrp = grp_ptr.numel() - 1
    _ok(lib().fwi_encode(_ptr(d_shots), nshot, nper, ngrp, _ptr(grp_ptr), _ptr(grp_shot), _ptr(grp_w),
                         grp_shot.numel(), _ptr(d_enc), _stream(stream)))


def fwi_draw_encoding(seed, step, sample, nshot, s, G):
    shots = np.zeros(G * s, dtype=np.int32)
    w = np.zeros(G * s, dtype=np.float32)
    kap = C.c_double(0.0)
    _ok(lib().fwi_draw_encoding(C.c_uint64(seed), C.c_uint64(step), C.c_uint64(sample), nshot, s, G,
                                shots.ctypes.data_as(C.POINTER(C.c_int32)), w.ctypes.data_as(C.POINTER(C.c_float)),
                                C.byref(kap)))
    return shots, w, kap.value


def fwi_langevin(model_off, v, grad, xi, seed, step, eta, nu, v_lo, v_hi, stream=None):
    off = np.ascontiguousarray(model_off, dtype=np.int64)
    _ok(lib().fwi_langevin(len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(v), _ptr(grad), _ptr(xi),
                           C.c_uint64(seed), C.c_uint64(step), C.c_float(eta), C.c_float(nu), C.c_float(v_lo),
                           C.c_float(v_hi), _stream(stream)))


def fwi_poll_status(ws, stream=None):
    _ok(lib().fwi_poll_status(_ptr(ws), ws.numel(), _stream(stream)))


def fwi_timing_enable(on: bool):
    _ok(lib().fwi_timing_enable(1 if on else 0))


def fwi_timing_read(kind: int, reset: bool = True):
    """(total kernel ms, launches) of kind 0 (forward/recompute step) or 1 (adjoint step)."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _ok(lib().fwi_timing_read(kind, C.byref(ms), C.byref(n), 1 if reset else 0))
    return ms.value, n.value


def fwi_copy_probe(src, dst, stream=None):
    _ok(lib().fwi_copy_probe(_ptr(src), _ptr(dst), src.numel(), _stream(stream)))


def fwi_graphs_enable(on: bool):
    _ok(lib().fwi_graphs_enable(1 if on else 0))


def fwi_graphs_stats():
    c, r = C.c_int64(0), C.c_int64(0)
    _ok(lib().fwi_graphs_stats(C.byref(c), C.byref(r)))
    return c.value, r.value


def fwi_set_tile(ndim: int, bz: int):
    _ok(lib().fwi_set_tile(ndim, bz))


def fwi_set_tile_width(wx: int):
    """3D tile width: 64, 32, or 0 for the automatic choice."""
    _ok(lib().fwi_set_tile_width(wx))


def fwi_tile_shape(batch, time):
    """(tile height or planes, tile width) the step kernels would use for this batch."""
    bz, wx = C.c_int32(0), C.c_int32(0)
    _ok(lib().fwi_tile_shape(batch.c, C.byref(time), C.byref(bz), C.byref(wx)))
    return bz.value, wx.value


def fwi_set_overlap(on: bool):
    """Checkpointed schedules: recompute the next segment beside the current adjoint."""
    _ok(lib().fwi_set_overlap(1 if on else 0))


def fwi_set_time_blocking(fwd_steps: int, adj_steps: int):
    """Time steps per launch of the 2D keep-all forward and adjoint sweeps: 1 or 2 forced,
    0 automatic (the default: forward 1, adjoint the tuned choice, else 2); process-wide."""
    _ok(lib().fwi_set_time_blocking(fwd_steps, adj_steps))


def fwi_tune(batch, time, v, ws, cache_path=None, stream=None):
    """Returns (tile height, adjoint time steps per launch (0: not applicable),
    ms per gradient time step)."""
    bz = C.c_int32(0)
    adj = C.c_int32(0)
    ms = C.c_double(0.0)
    _ok(lib().fwi_tune(batch.c, C.byref(time), _ptr(v), _ptr(ws), ws.numel(), _stream(stream),
                       cache_path.encode() if cache_path else None, C.byref(bz), C.byref(adj), C.byref(ms)))
    return bz.value, adj.value, ms.value
