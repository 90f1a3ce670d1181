"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test checks the oracle against mathematics the paper and the discretization fix:
exactness of the stencil on polynomials, the closed-form stability limit, analytic
Green's functions of the acoustic wave equation, the adjoint identity, reciprocity,
finite differences of the misfit, linearity of encoding and exact unbiasedness of the
+-1 estimator (Eq. 6) over sign patterns and (with kappa) over random shot subsets, the
sponge against a domain too large to reflect, an independent Philox implementation
(NumPy's) and the stationary law of the Langevin chain (Eqs. 8-9) on a linear-Gaussian
problem.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel2
from scipy.stats import kstest

import oracle
import workloads as W


def rel(a, b):
    return oracle.rel_l2(a, b)


# ----------------------------------------------------------------- stencil

def test_stencil_exact_on_polynomials_and_order_8():
    # Interior of a padded 2D field (nb = 0 so the field is the whole box); x spacing 7,
    # z spacing 11 so that a swapped axis or weight shows.
    g = oracle.Grid(nz=40, nx=36, dz=11.0, dx=7.0, nb=0, v_ref=1.0)
    zz, xx = np.mgrid[0:40, 0:36].astype(np.float64)
    z, x = zz * 11.0 / 100.0, xx * 7.0 / 100.0  # coordinates in units of 100 m
    inner = (slice(6, -6), slice(6, -6))
    for p in range(0, 10):
        u = x ** p
        ref = p * (p - 1) * x ** max(p - 2, 0) / 100.0 ** 2 if p >= 2 else np.zeros_like(x)
        got = oracle.laplacian(g, u)
        assert np.allclose(got[inner], ref[inner], rtol=1e-9, atol=1e-9 * np.abs(ref).max() + 1e-12), p
        u = z ** p
        ref = p * (p - 1) * z ** max(p - 2, 0) / 100.0 ** 2 if p >= 2 else np.zeros_like(z)
        got = oracle.laplacian(g, u)
        assert np.allclose(got[inner], ref[inner], rtol=1e-9, atol=1e-9 * np.abs(ref).max() + 1e-12), p
    # degree 10 leaves exactly the leading truncation term of the 8th-order scheme,
    # D u - u'' = -(h^8 / 3150) u^(10) = -1152 h^8 for u = x^10 (h in units of 100 m)
    u = x ** 10
    ref = 90 * x ** 8 / 100.0 ** 2
    err = oracle.laplacian(g, u)[inner] - ref[inner]
    h = 0.07
    assert np.allclose(err, -1152.0 * h ** 8 / 100.0 ** 2, rtol=1e-3)
    # mixed polynomial: the two axes add
    u = x ** 3 * z ** 2
    ref = (6 * x * z ** 2 + 2 * x ** 3) / 100.0 ** 2
    assert np.allclose(oracle.laplacian(g, u)[inner], ref[inner], rtol=1e-9, atol=1e-12)


def test_stencil_nyquist_symbol():
    # The checkerboard (-1)^ix is an eigenvector in the interior with eigenvalue
    # -(2048/315)/h^2 (symbol of the 8th-order weights at kh = pi).
    g = oracle.Grid(nz=20, nx=40, dz=1.0, dx=3.0, nb=0, v_ref=1.0)
    u = np.tile((-1.0) ** np.arange(40), (20, 1))
    got = oracle.laplacian(g, u)[4:-4, 4:-4]
    assert np.allclose(got, -(2048.0 / 315.0) / 9.0 * u[4:-4, 4:-4], rtol=1e-12)


def test_stencil_3d_axes():
    g = oracle.Grid(nz=20, ny=22, nx=24, dz=3.0, dy=5.0, dx=7.0, nb=0, v_ref=1.0, ndim=3)
    zz, yy, xx = np.mgrid[0:20, 0:22, 0:24].astype(np.float64)
    z, y, x = zz * 3.0, yy * 5.0, xx * 7.0
    u = x ** 2 + 2 * y ** 4 + 3 * z ** 6 * 1e-6
    ref = 2 + 24 * y ** 2 + 90 * z ** 4 * 1e-6
    got = oracle.laplacian(g, u)
    s = (slice(6, -6),) * 3
    assert np.allclose(got[s], ref[s], rtol=1e-8)


# --------------------------------------------------------------------- CFL

@pytest.mark.parametrize("ndim", [2, 3])
def test_cfl_closed_form(ndim):
    # exact limit v dt sqrt(D)/h <= sqrt(315/(512 D)) * sqrt(D) ... i.e. Courant
    # v dt / h <= sqrt(315 / (512 D)) for equal spacing.
    h, v0 = 10.0, 2000.0
    lim = math.sqrt(315.0 / (512.0 * ndim))
    if ndim == 2:
        g = oracle.Grid(nz=48, nx=48, dz=h, dx=h, nb=0, v_ref=v0)
        src = [24 * 48 + 24]
        rec = [10 * 48 + 30]
    else:
        g = oracle.Grid(nz=20, ny=20, nx=20, dz=h, dy=h, dx=h, nb=0, v_ref=v0, ndim=3)
        src = [(10 * 20 + 10) * 20 + 10]
        rec = [(5 * 20 + 12) * 20 + 7]
    v = np.full(g.nphys, v0)
    nt = 1500 if ndim == 2 else 800
    out = {}
    for fac in (0.95, 1.05):
        dt = fac * lim * h / v0
        wav = W.ricker(25.0, dt, nt)
        d = oracle.forward(g, v, dt, nt, 1, src, [1.0], wav, rec, coef_fp32=False)
        out[fac] = np.abs(d).max()
    assert np.isfinite(out[0.95]) and out[0.95] < 1.0
    assert not np.isfinite(out[1.05]) or out[1.05] > 1e6


# --------------------------------------------------------- Green's functions

def green_2d(wavelet, dt, r, v, nt_out):
    """u(r, t) for u_tt = v^2 (lap u + delta(x) f(t)), 2D: F(w) * (-i/4) H0^(2)(w r / v)
    in NumPy's e^{+i w t} convention (outgoing)."""
    n = 8 * len(wavelet)
    F = np.fft.rfft(wavelet, n)
    w = 2 * math.pi * np.fft.rfftfreq(n, dt)
    G = np.zeros_like(F)
    G[1:] = -0.25j * hankel2(0, w[1:] * r / v)
    u = np.fft.irfft(F * G, n)
    return u[:nt_out]


def _green2d_error(h, dt, nt):
    v0, f = 2500.0, 10.0
    n = int(round(2000.0 / h))
    g = oracle.Grid(nz=n, nx=n, dz=h * 1.25, dx=h, nb=20, v_ref=v0)
    v = np.full(g.nphys, v0)
    iz0, ix0 = n // 2, n // 2
    src = [iz0 * n + ix0]
    offs = [(0, int(round(300 / h))), (int(round(240 / (1.25 * h))), 0),
            (int(round(160 / (1.25 * h))), int(round(200 / h)))]
    rec = [(iz0 + a) * n + ix0 + b for a, b in offs]
    wav = W.ricker(f, dt, nt)
    d = oracle.forward(g, v, dt, nt, 1, src, [1.0], wav, rec, coef_fp32=False)
    errs = []
    for k, (a, b) in enumerate(offs):
        r = math.hypot(a * 1.25 * h, b * h)
        # d[j] = u^{j+1} ~ u(t = (j+1) dt)
        ref = green_2d(wav, dt, r, v0, nt + 1)[1:]
        errs.append(rel(d[:, k], ref))
    return max(errs)


def test_green_2d_accuracy_and_convergence():
    # 10 Hz Ricker at 2500 m/s: >= 10 points per wavelength at 2.5 f for h = 10 m.
    # dz = 1.25 dx so that an exchanged axis would move the arrivals.
    e1 = _green2d_error(10.0, 1e-3, 500)
    e2 = _green2d_error(5.0, 0.5e-3, 1000)
    assert e1 < 0.02, e1
    assert e2 < e1 / 3.0, (e1, e2)


def test_green_3d_accuracy():
    # u = f(t - r/v) / (4 pi r) for u_tt = v^2 (lap u + delta(x) f(t)).
    v0, f, h = 2500.0, 20.0, 5.0
    n = 64
    g = oracle.Grid(nz=n, ny=n, nx=n, dz=h, dy=h, dx=h, nb=10, v_ref=v0, ndim=3)
    v = np.full(g.nphys, v0)
    dt, nt = 0.4e-3, 300
    c0 = n // 2
    src = [(c0 * n + c0) * n + c0]
    offs = [(0, 0, 12), (9, 0, 0), (0, 8, 6)]
    rec = [((c0 + a) * n + c0 + b) * n + c0 + cc for a, b, cc in offs]
    wav = W.ricker(f, dt, nt)
    d = oracle.forward(g, v, dt, nt, 1, src, [1.0], wav, rec, coef_fp32=False)
    t = (np.arange(nt) + 1) * dt
    for k, (a, b, cc) in enumerate(offs):
        r = h * math.sqrt(a * a + b * b + cc * cc)
        ref = W.ricker(f, dt, nt, t0=1.5 / f + r / v0 - 0.0)
        ref = np.interp(t - r / v0, np.arange(nt) * dt, wav, left=0.0) / (4 * math.pi * r)
        # window before the earliest sponge return (boundary 160 m from the source)
        win = t < 1.5 / f + (2 * 160.0 - r) / v0 - 1.2 / f
        assert rel(d[win, k], ref[win]) < 0.02


# ----------------------------------------------------------- adjoint pins

def _hetero_2d(seed=3, nz=30, nx=34, nb=8):
    g = oracle.Grid(nz=nz, nx=nx, dz=10.0, dx=12.0, nb=nb, v_ref=3500.0)
    r = np.random.default_rng(seed)
    v = W.layered_1d(nz, nx, seed, 1500.0, 3500.0, 3, 5, nz - 2) + r.uniform(-100, 100, (nz, nx))
    return g, v.ravel()


def test_adjoint_dot_product_2d():
    g, v = _hetero_2d()
    dt, nt, R = 1e-3, 300, 2
    r = np.random.default_rng(1)
    s_cell = 1 * g.nx + 7
    rec = np.arange(g.nx, dtype=np.int32)[::3] + g.nx * 2
    s = r.standard_normal(nt)
    d = oracle.forward(g, v, dt, nt, R, [s_cell], [1.0], s, rec, coef_fp32=False)
    rho = r.standard_normal(d.shape)
    _, tr = oracle.adjoint(g, v, dt, nt, R, [s_cell], [1.0], s, rec, rho, coef_fp32=False,
                           want_gradient=False, trace_cell=s_cell)
    lhs = float(np.sum(d * rho))
    rhs = float(np.sum(s * tr)) / (g.dz * g.dx)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_dot_product_3d():
    g = oracle.Grid(nz=10, ny=12, nx=14, dz=10.0, dy=11.0, dx=12.0, nb=4, v_ref=3000.0, ndim=3)
    r = np.random.default_rng(2)
    v = r.uniform(1800, 3000, g.nphys)
    dt, nt, R = 1e-3, 120, 3
    s_cell = (1 * 12 + 5) * 14 + 6
    rec = np.array([(2 * 12 + a) * 14 + b for a in (1, 6, 10) for b in (2, 7, 12)], dtype=np.int32)
    s = r.standard_normal(nt)
    d = oracle.forward(g, v, dt, nt, R, [s_cell], [1.0], s, rec, coef_fp32=False)
    rho = r.standard_normal(d.shape)
    _, tr = oracle.adjoint(g, v, dt, nt, R, [s_cell], [1.0], s, rec, rho, coef_fp32=False,
                           want_gradient=False, trace_cell=s_cell)
    lhs = float(np.sum(d * rho))
    rhs = float(np.sum(s * tr)) / (g.dz * g.dy * g.dx)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_exact_reciprocity():
    g, v = _hetero_2d(seed=5)
    dt, nt = 1e-3, 250
    wav = W.ricker(20.0, dt, nt)
    a, b = 1 * g.nx + 4, 20 * g.nx + 29
    dab = oracle.forward(g, v, dt, nt, 1, [a], [1.0], wav, [b], coef_fp32=False)
    dba = oracle.forward(g, v, dt, nt, 1, [b], [1.0], wav, [a], coef_fp32=False)
    assert np.abs(dab - dba).max() <= 1e-12 * np.abs(dab).max()


def _fd_setup(seed=7):
    g, v = _hetero_2d(seed, nz=24, nx=32, nb=6)
    dt, nt, R = 1e-3, 300, 2
    srcs = np.array([1 * g.nx + 5, 1 * g.nx + 26], dtype=np.int32)
    w = np.array([1.0, -1.0])
    rec = (np.arange(g.nx) + g.nx).astype(np.int32)
    wav = W.ricker(20.0, dt, nt)
    vtrue = v + 150.0 * np.exp(-((np.arange(g.nphys) // g.nx - 14) ** 2) / 8.0)
    dobs = oracle.forward(g, vtrue, dt, nt, R, srcs, w, wav, rec, coef_fp32=False)
    return g, v, dt, nt, R, srcs, w, rec, wav, dobs


def test_gradient_matches_central_differences():
    g, v, dt, nt, R, srcs, w, rec, wav, dobs = _fd_setup()
    is2 = 0.37
    _, phi, grad = oracle.gradient(g, v, dt, nt, R, srcs, w, wav, rec, dobs, is2, coef_fp32=False)
    r = np.random.default_rng(11)
    for _ in range(2):
        dv = r.standard_normal(g.nphys)
        eps = 1e-2
        pp = oracle.gradient(g, v + eps * dv, dt, nt, R, srcs, w, wav, rec, dobs, is2, coef_fp32=False)[1]
        pm = oracle.gradient(g, v - eps * dv, dt, nt, R, srcs, w, wav, rec, dobs, is2, coef_fp32=False)[1]
        fd = (pp - pm) / (2 * eps)
        an = float(grad @ dv)
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)
    # the misfit is the closed form of Eq. 1 on the returned prediction
    dpred = oracle.forward(g, v, dt, nt, R, srcs, w, wav, rec, coef_fp32=False)
    assert abs(phi - 0.5 * is2 * np.sum((dpred - dobs) ** 2)) <= 1e-12 * phi


def test_gradient_edge_cells_fold():
    # a perturbation concentrated on edge cells (those replicated into the sponge) --
    # the fold must account for every replicated copy
    g, v, dt, nt, R, srcs, w, rec, wav, dobs = _fd_setup(seed=8)
    _, _, grad = oracle.gradient(g, v, dt, nt, R, srcs, w, wav, rec, dobs, 1.0, coef_fp32=False)
    dv = np.zeros((g.nz, g.nx))
    dv[0, :] = 1.0
    dv[:, 0] = 1.0
    dv[-1, -1] = 3.0
    dv = dv.ravel()
    eps = 1e-2
    pp = oracle.gradient(g, v + eps * dv, dt, nt, R, srcs, w, wav, rec, dobs, 1.0, coef_fp32=False)[1]
    pm = oracle.gradient(g, v - eps * dv, dt, nt, R, srcs, w, wav, rec, dobs, 1.0, coef_fp32=False)[1]
    fd = (pp - pm) / (2 * eps)
    assert abs(fd - grad @ dv) <= 1e-7 * abs(fd)


def test_born_dot_product():
    g, v, dt, nt, R, srcs, w, rec, wav, dobs = _fd_setup(seed=9)
    r = np.random.default_rng(3)
    dv = r.standard_normal(g.nphys)
    dd = oracle.born(g, v, dv, dt, nt, R, srcs, w, wav, rec, coef_fp32=False)
    rho = r.standard_normal(dd.shape)
    gr, _ = oracle.adjoint(g, v, dt, nt, R, srcs, w, wav, rec, rho, coef_fp32=False)
    lhs, rhs = float(np.sum(dd * rho)), float(gr @ dv)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


# ------------------------------------------------------------- encoding

def test_encoding_linearity():
    g, v = _hetero_2d(seed=12)
    dt, nt = 1e-3, 200
    wav = W.ricker(15.0, dt, nt)
    srcs = np.array([g.nx + 3, g.nx + 11, g.nx + 30], dtype=np.int32)
    w = np.array([1.0, -1.0, 1.0])
    rec = (np.arange(g.nx) + g.nx).astype(np.int32)
    enc = oracle.forward(g, v, dt, nt, 1, srcs, w, wav, rec, coef_fp32=False)
    ind = sum(wi * oracle.forward(g, v, dt, nt, 1, [s], [1.0], wav, rec, coef_fp32=False)
              for s, wi in zip(srcs, w))
    assert np.abs(enc - ind).max() <= 1e-12 * np.abs(ind).max()


def test_exact_unbiasedness_over_all_sign_patterns():
    # Eq. 6: with w_i = +-1 (zero mean, unit variance) the mean of the encoded gradient
    # over all 2^s patterns equals the full-shot gradient, exactly.
    g, v, dt, nt, R, _, _, rec, wav, _ = _fd_setup(seed=13)
    shots = np.array([g.nx + 4, g.nx + 15, g.nx + 27], dtype=np.int32)
    vtrue = v * (1 + 0.05 * np.sin(np.arange(g.nphys) / 37.0))
    d_i = [oracle.forward(g, vtrue, dt, nt, R, [s], [1.0], wav, rec, coef_fp32=False) for s in shots]
    full = sum(oracle.gradient(g, v, dt, nt, R, [s], [1.0], wav, rec, d_i[k], 1.0, coef_fp32=False)[2]
               for k, s in enumerate(shots))
    acc = np.zeros(g.nphys)
    for bits in range(8):
        w = np.array([1.0 if (bits >> k) & 1 == 0 else -1.0 for k in range(3)])
        dt_enc = oracle.encode(d_i, [0, 3], [0, 1, 2], w)[0]
        acc += oracle.gradient(g, v, dt, nt, R, shots, w, wav, rec, dt_enc, 1.0, coef_fp32=False)[2]
    acc /= 8.0
    assert rel(acc, full) < 1e-12


def test_draw_encoding_properties():
    nshot, s, G = 80, 16, 10
    shots, w, kappa = oracle.draw_encoding(1234, 7, 3, nshot, s, G)
    assert kappa == nshot / (G * s)
    groups = shots.reshape(G, s)
    per = nshot // s
    for p in range(G // per):
        part = groups[p * per:(p + 1) * per].ravel()
        assert sorted(part.tolist()) == list(range(nshot))  # a partition
    assert set(np.unique(w).tolist()) <= {-1.0, 1.0}
    again = oracle.draw_encoding(1234, 7, 3, nshot, s, G)
    assert np.array_equal(again[0], shots) and np.array_equal(again[1], w)
    other = oracle.draw_encoding(1234, 8, 3, nshot, s, G)
    assert not np.array_equal(other[0], shots)
    # uniformity of membership and sign balance over many draws
    cnt = np.zeros(nshot)
    sg = 0.0
    n = 400
    for step in range(n):
        sh, ww, _ = oracle.draw_encoding(99, step, 0, 40, 8, 1)
        cnt[sh] += 1
        sg += ww.sum()
    p = 8 / 40
    expect = n * p
    assert np.all(np.abs(cnt[:40] - expect) < 5 * math.sqrt(n * p * (1 - p)))
    assert abs(sg) < 5 * math.sqrt(n * 8)


# ----------------------------------------------------------- RNG pins

@pytest.mark.parametrize("ctr,key", [
    ([1, 0, 0, 0], [0, 0]),
    ([5, 17, 3, 0], [1234, 0x4C414E47]),
    ([2 ** 63 + 12345, 2 ** 64 - 1, 77, 2 ** 40], [2 ** 64 - 2, 31337]),
])
def test_philox_matches_numpy(ctr, key):
    # NumPy's Philox is Philox4x64-10 and increments its counter before each block.
    prev = list(ctr)
    prev[0] = (prev[0] - 1) % 2 ** 64
    if ctr[0] == 0:
        pytest.skip("borrow case not needed")
    bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    ref = bg.random_raw(4)
    got = oracle.philox4x64(ctr, key)
    assert np.array_equal(got, ref)


def test_normals_distribution():
    z = oracle.normals(42, 3, 1, 400_000)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert kstest(z, "norm").pvalue > 1e-4
    # independent streams per (step, sample)
    z2 = oracle.normals(42, 4, 1, 1000)
    assert abs(np.corrcoef(z[:1000], z2)[0, 1]) < 0.15


# ---------------------------------------------------------- Langevin pin

def test_langevin_linear_gaussian_stationary_law():
    # Phi(z) = |A z - y|^2 / (2 s^2): the posterior is N(mu, s^2 (A^T A)^-1).  Unadjusted
    # Langevin with nu = sqrt(2 eta) targets it up to O(eta).
    A = np.array([[1.0, 0.3], [0.2, 0.8], [0.5, -0.4]])
    y = np.array([0.7, -0.2, 1.1])
    s2 = 0.25
    P = A.T @ A / s2
    cov = np.linalg.inv(P)
    mu = cov @ (A.T @ y / s2)
    nch, eta, nsteps = 20000, 0.01, 600
    z = np.zeros((nch, 2))
    for k in range(nsteps):
        grad = (z @ A.T - y) @ A / s2
        xi = oracle.normals(7, k, 0, 2 * nch).reshape(nch, 2)
        z = oracle.langevin(z, grad, xi, eta, math.sqrt(2 * eta), -1e9, 1e9).reshape(nch, 2)
    m = z.mean(0)
    c = np.cov(z.T)
    assert np.abs(m - mu).max() < 0.02
    assert np.abs(c - cov).max() < 0.1 * np.abs(cov).max()
    # the clamp is applied after the update
    out = oracle.langevin(np.array([1.0, 2.0]), np.array([0.0, 0.0]), np.array([10.0, -10.0]), 0.1, 1.0, 0.0, 5.0)
    assert np.array_equal(out, [5.0, 0.0])


# ------------------------------------------------------------------ sponge

def _box_field(nb, n=80, N=None, v0=2000.0, h=10.0, dt=1e-3, nt=600, R=10):
    """u over an n x n box (every cell recorded every R steps) from a centred 15 Hz source,
    computed on an n x n grid with nb sponge cells, or, with N, inside an N x N grid
    (whose boundaries are too far to be heard within nt steps)."""
    wav = W.ricker(15.0, dt, nt)
    M = N or n
    g = oracle.Grid(nz=M, nx=M, dz=h, dx=h, nb=nb, v_ref=v0)
    o = (M - n) // 2
    rec = np.array([(o + i) * M + o + j for i in range(n) for j in range(n)], dtype=np.int32)
    src = [(o + n // 2) * M + o + n // 2]
    return oracle.forward(g, np.full(M * M, v0), dt, nt, R, src, [1.0], wav, rec, coef_fp32=False)


def test_sponge_absorbs_outgoing_waves():
    # A point source in a homogeneous 800 m box with a 20-cell sponge against the same
    # box inside a 4 km domain (no reflection back within 0.6 s): after the wave has left
    # the box its energy is <= 1 % of the peak, and the reflected field (box
    # minus reference) stays below 10 % of the direct wave's peak norm.  Rigid walls
    # (no sponge) fail both bounds.
    ref = _box_field(20, N=400)
    peak_e = (ref ** 2).sum(1).max()
    peak_n = np.linalg.norm(ref, axis=1).max()
    late = slice(45, None)  # t >= 0.45 s (the 2D wave leaves a slowly decaying tail behind its front)
    assert (ref[late] ** 2).sum(1).max() < 1e-3 * peak_e  # the reference box is empty by then
    box = _box_field(20)
    assert (box[late] ** 2).sum(1).max() < 1e-2 * peak_e
    assert np.linalg.norm(box - ref, axis=1).max() < 0.10 * peak_n
    walls = _box_field(0)
    assert (walls[late] ** 2).sum(1).max() > 0.1 * peak_e
    assert np.linalg.norm(walls - ref, axis=1).max() > 0.5 * peak_n


# ------------------------------------------------------- kappa, random subsets

def test_kappa_makes_random_subsets_exactly_unbiased():
    # Eq. 6 with B a uniformly random subset of s of the N_s shots and kappa = N_s/s: the
    # mean over every subset and every +-1 pattern of kappa x (encoded gradient) is the
    # full-shot gradient, exactly (sign averaging removes cross terms, subset averaging
    # gives each shot weight s/N_s).
    g, v, dt, nt, R, _, _, rec, wav, _ = _fd_setup(seed=21)
    shots = np.array([g.nx + 3, g.nx + 11, g.nx + 19, g.nx + 28], dtype=np.int32)
    vtrue = v * (1 + 0.04 * np.cos(np.arange(g.nphys) / 29.0))
    d_i = [oracle.forward(g, vtrue, dt, nt, R, [s], [1.0], wav, rec, coef_fp32=False) for s in shots]
    full = sum(oracle.gradient(g, v, dt, nt, R, [s], [1.0], wav, rec, d_i[k], 1.0, coef_fp32=False)[2]
               for k, s in enumerate(shots))
    ns, s = len(shots), 2
    kappa = ns / s
    acc, count = np.zeros(g.nphys), 0
    for a in range(ns):
        for b in range(a + 1, ns):
            for bits in range(4):
                w = np.array([1.0 if bits & 1 else -1.0, 1.0 if bits & 2 else -1.0])
                d_enc = oracle.encode(d_i, [0, 2], [a, b], w)[0]
                acc += kappa * oracle.gradient(g, v, dt, nt, R, shots[[a, b]], w, wav, rec, d_enc, 1.0,
                                               coef_fp32=False)[2]
                count += 1
    assert rel(acc / count, full) < 1e-12
    # a wrong scale (kappa = 1) is off by N_s/s
    assert rel(acc / count / kappa, full) > 0.4
