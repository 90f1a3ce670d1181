"""FP64 CPU oracle for the encoded-shot acoustic FWI gradient -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and this package
shares no code with it: the numerics live in ``fwi_oracle.c`` (plain C, FP64) and the
few steps done here (encoding of observed data, per-sample sums, kappa) are written out
in NumPy FP64.

Paper passages followed (cited by section / equation, see fwi_oracle.c for the scheme):
  * Eq. 1 (full-shot misfit), Eq. 4 (encoded data / operator), Eq. 5 (encoded misfit),
    Eq. 6 (unbiased estimator N_s/m * grad), the adjoint-state statement after Eq. 5,
  * Eqs. 8-9 (unadjusted Langevin refinement) and the modified refinement with an
    independent noise weight (text after Alg. 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fwi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O3, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcGrid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
                ("dz", C.c_double), ("dy", C.c_double), ("dx", C.c_double), ("nb", C.c_int32),
                ("v_ref", C.c_double), ("refl", C.c_double)]


class OrcTime(C.Structure):
    _fields_ = [("dt", C.c_double), ("nt", C.c_int32), ("rec_every", C.c_int32), ("coef_fp32", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.orc_philox4x64.restype = None
        _lib.orc_normals.restype = None
        _lib.orc_normals_key.restype = None
        _lib.orc_langevin.restype = None
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


@dataclass
class Grid:
    """Physical grid + sponge.  nz, ny, nx physical cells (ny = 1 in 2D), spacings in m."""
    nz: int
    nx: int
    dz: float
    dx: float
    nb: int
    v_ref: float
    ny: int = 1
    dy: float = 1.0
    ndim: int = 2
    refl: float = 1e-3

    def c(self) -> OrcGrid:
        return OrcGrid(self.ndim, self.nz, self.ny, self.nx, self.dz, self.dy, self.dx, self.nb,
                       self.v_ref, self.refl)

    @property
    def nphys(self) -> int:
        return self.nz * self.ny * self.nx

    @property
    def padded_shape(self):
        if self.ndim == 3:
            return (self.nz + 2 * self.nb, self.ny + 2 * self.nb, self.nx + 2 * self.nb)
        return (self.nz + 2 * self.nb, self.nx + 2 * self.nb)


def _time(dt, nt, rec_every, coef_fp32):
    return OrcTime(float(dt), int(nt), int(rec_every), int(bool(coef_fp32)))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def forward(grid: Grid, v, dt, nt, rec_every, src_cell, src_w, wavelet, rec_cell, coef_fp32=True):
    """Data d[nt/R][nrec] of one simulation (all listed sources fire together)."""
    v, src_w, wavelet = _f64(v).ravel(), _f64(src_w), _f64(wavelet)
    src_cell, rec_cell = _i32(src_cell), _i32(rec_cell)
    d = np.zeros((nt // rec_every, len(rec_cell)))
    g, t = grid.c(), _time(dt, nt, rec_every, coef_fp32)
    rc = lib().orc_forward(C.byref(g), C.byref(t), _dp(v), len(src_cell), _ip(src_cell), _dp(src_w),
                           _dp(wavelet), len(rec_cell), _ip(rec_cell), _dp(d))
    if rc:
        raise ValueError("orc_forward failed (%d)" % rc)
    return d


def gradient(grid: Grid, v, dt, nt, rec_every, src_cell, src_w, wavelet, rec_cell, d_obs, inv_sigma2=1.0,
             coef_fp32=True):
    """One simulation: (d_pred, misfit phi, physical gradient dphi/dv before kappa)."""
    v, src_w, wavelet, d_obs = _f64(v).ravel(), _f64(src_w), _f64(wavelet), _f64(d_obs)
    src_cell, rec_cell = _i32(src_cell), _i32(rec_cell)
    d = np.zeros((nt // rec_every, len(rec_cell)))
    gph = np.zeros(grid.nphys)
    phi = C.c_double(0.0)
    g, t = grid.c(), _time(dt, nt, rec_every, coef_fp32)
    rc = lib().orc_gradient(C.byref(g), C.byref(t), _dp(v), len(src_cell), _ip(src_cell), _dp(src_w),
                            _dp(wavelet), len(rec_cell), _ip(rec_cell), _dp(d_obs), C.c_double(inv_sigma2),
                            _dp(d), C.byref(phi), _dp(gph))
    if rc:
        raise ValueError("orc_gradient failed (%d)" % rc)
    return d, phi.value, gph


def adjoint(grid: Grid, v, dt, nt, rec_every, src_cell, src_w, wavelet, rec_cell, rho, coef_fp32=True,
            want_gradient=True, trace_cell=None):
    """Adjoint solve for a given residual rho[nt/R][nrec].

    Returns (gradient or None, trace or None); trace[k-1] is the scaled adjoint
    c*lambda at step k (k = 1..nt) at physical cell ``trace_cell``.
    """
    v, src_w, wavelet, rho = _f64(v).ravel(), _f64(src_w), _f64(wavelet), _f64(rho)
    src_cell, rec_cell = _i32(src_cell), _i32(rec_cell)
    gph = np.zeros(grid.nphys) if want_gradient else None
    tr = np.zeros(nt) if trace_cell is not None else None
    g, t = grid.c(), _time(dt, nt, rec_every, coef_fp32)
    rc = lib().orc_adjoint(C.byref(g), C.byref(t), _dp(v), len(src_cell), _ip(src_cell), _dp(src_w),
                           _dp(wavelet), len(rec_cell), _ip(rec_cell), _dp(rho),
                           _dp(gph) if gph is not None else None,
                           C.c_int32(-1 if trace_cell is None else int(trace_cell)),
                           _dp(tr) if tr is not None else None)
    if rc:
        raise ValueError("orc_adjoint failed (%d)" % rc)
    return gph, tr


def born(grid: Grid, v, dv, dt, nt, rec_every, src_cell, src_w, wavelet, rec_cell, coef_fp32=False):
    """Tangent-linear data perturbation dd for model perturbation dv."""
    v, dv, src_w, wavelet = _f64(v).ravel(), _f64(dv).ravel(), _f64(src_w), _f64(wavelet)
    src_cell, rec_cell = _i32(src_cell), _i32(rec_cell)
    dd = np.zeros((nt // rec_every, len(rec_cell)))
    g, t = grid.c(), _time(dt, nt, rec_every, coef_fp32)
    rc = lib().orc_born(C.byref(g), C.byref(t), _dp(v), _dp(dv), len(src_cell), _ip(src_cell), _dp(src_w),
                        _dp(wavelet), len(rec_cell), _ip(rec_cell), _dp(dd))
    if rc:
        raise ValueError("orc_born failed (%d)" % rc)
    return dd


def laplacian(grid: Grid, u_pad):
    """8th-order Laplacian (exact weights, zero outside) of a padded field."""
    u = _f64(u_pad)
    out = np.zeros_like(u)
    g = grid.c()
    if lib().orc_laplacian(C.byref(g), _dp(u), _dp(out)):
        raise ValueError("orc_laplacian failed")
    return out


def coefficients(grid: Grid, v, dt, coef_fp32=False):
    """Per padded cell (a, b, c) of the leapfrog/sponge recursion."""
    v = _f64(v).ravel()
    shape = grid.padded_shape
    a, b, c = (np.zeros(shape) for _ in range(3))
    g, t = grid.c(), _time(dt, 1, 1, coef_fp32)
    if lib().orc_coefficients(C.byref(g), C.byref(t), _dp(v), _dp(a), _dp(b), _dp(c)):
        raise ValueError("orc_coefficients failed")
    return a, b, c


# ----------------------------------------------------------------- batches

def forward_batch(grids, models, dt, nt, rec_every, src_ptr, src_cell, src_w, wavelet, rec_ptr, rec_cell,
                  coef_fp32=True):
    """Forward of nsim simulations in parallel (OpenMP).  Returns a list of d[nt/R][nrec_s]."""
    nsim = len(grids)
    garr = (OrcGrid * nsim)(*[g.c() for g in grids])
    vs = [_f64(m).ravel() for m in models]
    vptr = (C.POINTER(C.c_double) * nsim)(*[_dp(m) for m in vs])
    src_ptr, src_cell, rec_ptr, rec_cell = _i32(src_ptr), _i32(src_cell), _i32(rec_ptr), _i32(rec_cell)
    src_w, wavelet = _f64(src_w), _f64(wavelet)
    outs = [np.zeros((nt // rec_every, rec_ptr[s + 1] - rec_ptr[s])) for s in range(nsim)]
    optr = (C.POINTER(C.c_double) * nsim)(*[_dp(o) for o in outs])
    t = _time(dt, nt, rec_every, coef_fp32)
    rc = lib().orc_forward_batch(nsim, garr, C.byref(t), vptr, _ip(src_ptr), _ip(src_cell), _dp(src_w),
                                 _dp(wavelet), _ip(rec_ptr), _ip(rec_cell), optr)
    if rc:
        raise ValueError("orc_forward_batch failed")
    return outs


def gradient_batch(grids, models, dt, nt, rec_every, src_ptr, src_cell, src_w, wavelet, rec_ptr, rec_cell,
                   d_obs, inv_sigma2=1.0, coef_fp32=True):
    """Per-simulation (d_pred list, misfit array, physical gradient list), OpenMP over sims."""
    nsim = len(grids)
    garr = (OrcGrid * nsim)(*[g.c() for g in grids])
    vs = [_f64(m).ravel() for m in models]
    vptr = (C.POINTER(C.c_double) * nsim)(*[_dp(m) for m in vs])
    src_ptr, src_cell, rec_ptr, rec_cell = _i32(src_ptr), _i32(src_cell), _i32(rec_ptr), _i32(rec_cell)
    src_w, wavelet = _f64(src_w), _f64(wavelet)
    dob = [_f64(d) for d in d_obs]
    dptr = (C.POINTER(C.c_double) * nsim)(*[_dp(d) for d in dob])
    dps = [np.zeros((nt // rec_every, rec_ptr[s + 1] - rec_ptr[s])) for s in range(nsim)]
    pptr = (C.POINTER(C.c_double) * nsim)(*[_dp(o) for o in dps])
    gs = [np.zeros(g.nphys) for g in grids]
    gptr = (C.POINTER(C.c_double) * nsim)(*[_dp(o) for o in gs])
    mis = np.zeros(nsim)
    t = _time(dt, nt, rec_every, coef_fp32)
    rc = lib().orc_gradient_batch(nsim, garr, C.byref(t), vptr, _ip(src_ptr), _ip(src_cell), _dp(src_w),
                                  _dp(wavelet), _ip(rec_ptr), _ip(rec_cell), dptr, C.c_double(inv_sigma2), pptr,
                                  _dp(mis), gptr)
    if rc:
        raise ValueError("orc_gradient_batch failed")
    return dps, mis, gs


def encode(d_shots, grp_ptr, grp_shot, grp_w):
    """Eq. 4: encoded observed data d~_g = sum_{i in B_g} w_i d_i, FP64."""
    d_shots = np.asarray(d_shots, dtype=np.float64)
    out = np.zeros((len(grp_ptr) - 1,) + d_shots.shape[1:])
    for g in range(len(grp_ptr) - 1):
        for k in range(grp_ptr[g], grp_ptr[g + 1]):
            out[g] += grp_w[k] * d_shots[grp_shot[k]]
    return out


def sample_gradient(g_sims, sample_of, nsample, kappa):
    """Eq. 6: g_hat_s = kappa_s * sum over the sample's supergathers of grad Phi~."""
    kappa = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nsample,))
    out = [None] * nsample
    for s, g in enumerate(g_sims):
        k = sample_of[s]
        out[k] = g.copy() if out[k] is None else out[k] + g
    return [kappa[k] * out[k] for k in range(nsample)]


# -------------------------------------------------------------------- RNG

def philox4x64(ctr, key):
    """Philox4x64-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(c.ctypes.data_as(C.POINTER(C.c_uint64)), k.ctypes.data_as(C.POINTER(C.c_uint64)),
                         o.ctypes.data_as(C.POINTER(C.c_uint64)))
    return o


def normals(seed, step, sample, n):
    """Langevin noise xi ~ N(0, I) for one sample at one step (counter-based, reproducible)."""
    out = np.zeros(int(n))
    lib().orc_normals(C.c_uint64(seed), C.c_uint64(step), C.c_uint64(sample), C.c_int64(n), _dp(out))
    return out


def normals_key(seed, tag, a, b, n):
    """Standard normals of any counter-based stream: cells 4m..4m+3 from Philox(ctr = {m, a,
    b, 0}, key = {seed, tag}) with Box-Muller (normals() is tag 0x4C414E47)."""
    out = np.zeros(int(n))
    lib().orc_normals_key(C.c_uint64(seed), C.c_uint64(tag), C.c_uint64(a), C.c_uint64(b), C.c_int64(n), _dp(out))
    return out


def langevin(z, g, xi, eta, nu, lo, hi):
    """Eqs. 8-9: z <- clamp(z - eta g + nu xi, lo, hi) (returns a new array)."""
    z = _f64(z).copy().ravel()
    g, xi = _f64(g).ravel(), _f64(xi).ravel()
    lib().orc_langevin(C.c_int64(z.size), _dp(z), _dp(g), _dp(xi), C.c_double(eta), C.c_double(nu),
                       C.c_double(lo), C.c_double(hi))
    return z


def draw_encoding(seed, step, sample, nshot, s, G):
    """Eq. 4 draw: (grp_shot[G*s], grp_w[G*s], kappa) for one sample at one step."""
    shots = np.zeros(G * s, dtype=np.int32)
    w = np.zeros(G * s)
    kap = C.c_double(0.0)
    rc = lib().orc_draw_encoding(C.c_uint64(seed), C.c_uint64(step), C.c_uint64(sample), int(nshot), int(s),
                                 int(G), _ip(shots), _dp(w), C.byref(kap))
    if rc:
        raise ValueError("orc_draw_encoding failed")
    return shots, w, kap.value


def rel_l2(x, ref):
    """||x - ref||_2 / ||ref||_2 accumulated in FP64."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
