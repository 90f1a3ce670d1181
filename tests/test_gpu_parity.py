"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerance: relative L2 <= 1e-5 for FP32 wavefield results (data, misfit, gradient), with
the oracle evaluating the FP32-rounded coefficient set in FP64 arithmetic.  Gradient
parity is asserted where the residual ratio |d - d_obs| / |d_obs| >= 0.3 (below that
the difference d - d_obs amplifies FP32 rounding of the data); a shared-residual test
checks the adjoint and imaging alone at any model.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import workloads as W
from helpers import f32, ogrid, oracle_batch_gradient, oracle_forward_sims, rel, split_data, split_model

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import fwi
    fwi.lib()
    return fwi


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run_gradient(F, batch, time, models, d_obs_flat, inv_sigma2, kappa):
    nt_rec = time.nt // time.rec_every
    v = dev(np.concatenate([m.ravel() for m in models]))
    dobs = dev(d_obs_flat)
    dpred = torch.zeros(batch.data_size(nt_rec), device="cuda")
    mis = torch.zeros(batch.nsim, dtype=torch.float64, device="cuda")
    grad = torch.zeros(batch.model_size, device="cuda")
    gn = torch.zeros(batch.nsample, device="cuda")
    ws = F.alloc_workspace(batch, time)
    F.fwi_gradient(batch, time, v, dobs, inv_sigma2, kappa, dpred, mis, grad, gn, ws)
    F.fwi_poll_status(ws)
    return dpred.cpu().numpy().astype(np.float64), mis.cpu().numpy(), grad.cpu().numpy().astype(np.float64), \
        gn.cpu().numpy().astype(np.float64)


# ------------------------------------------------------------ C1 full size

def c1_problem():
    from paper_2512_12797_amd import problems
    cfg = W.C1
    grid = problems.grid_of(cfg)
    wav = W.ricker(cfg.freq, cfg.dt, cfg.nt)
    shots = problems.shot_cells(cfg, grid)
    batch = problems.single_shot_batch(cfg, grid, shots, wav)
    vtrue = f32(W.layered_1d(cfg.nz, cfg.nx, seed=0))
    vstart = f32(W.linear_gradient(cfg.nz, cfg.nx, 1500.0, 4000.0))
    return cfg, grid, batch, vtrue, vstart


@pytest.mark.parametrize("ckpt", [0, 10])
def test_c1_gradient_parity(F, ckpt):
    cfg, grid, batch, vtrue, vstart = c1_problem()
    say("case c1 gradient ckpt_every=%d" % ckpt)
    time = F.time_axis(cfg.dt, cfg.nt, cfg.rec_every, ckpt)
    nt_rec = cfg.nt_rec
    # observed data: oracle forward on the true model (exact coefficients), rounded to FP32
    dobs = [f32(d) for d in oracle_forward_sims(batch, cfg.dt, cfg.nt, 1, [vtrue.ravel()], coef_fp32=False)]
    dobs_flat = np.concatenate([d.ravel() for d in dobs])
    dp, mis, gr, gn = run_gradient(F, batch, time, [vstart], dobs_flat, 1.0, [1.0])
    odp, omis, ogr = oracle_batch_gradient(batch, cfg.dt, cfg.nt, 1, [vstart.ravel()], dobs, 1.0, [1.0])
    gdp = split_data(dp, batch, nt_rec)
    for s in range(batch.nsim):
        e = rel(gdp[s], odp[s])
        ratio = np.linalg.norm(odp[s] - dobs[s]) / np.linalg.norm(dobs[s])
        say("  sim %d data rel %.2e residual ratio %.2f misfit rel %.2e" % (s, e, ratio, abs(mis[s] / omis[s] - 1)))
        assert e < TOL
        assert abs(mis[s] / omis[s] - 1) < TOL
    eg = rel(gr, ogr[0])
    say("  gradient rel %.2e  norm rel %.2e" % (eg, abs(gn[0] / np.linalg.norm(ogr[0]) - 1)))
    assert eg < TOL
    assert abs(gn[0] / np.linalg.norm(gr) - 1) < 1e-6


def test_c1_shared_residual_adjoint(F):
    # adjoint + imaging alone, with the same FP32 residual on both sides, kappa != 1
    cfg, grid, batch, vtrue, vstart = c1_problem()
    say("case c1 shared-residual adjoint")
    time = F.time_axis(cfg.dt, cfg.nt, cfg.rec_every, 0)
    r = np.random.default_rng(5)
    vmix = f32(0.5 * (vtrue + vstart))
    rho = [f32(r.standard_normal((cfg.nt_rec, batch.nrec[s])) * 1e-3) for s in range(batch.nsim)]
    v = dev(vmix.ravel())
    ws = F.alloc_workspace(batch, time)
    F.fwi_forward(batch, time, v, None, ws)
    grad = torch.zeros(batch.model_size, device="cuda")
    F.fwi_adjoint(batch, time, v, dev(np.concatenate([x.ravel() for x in rho])), [2.5], grad, None, ws)
    F.fwi_poll_status(ws)
    g = grad.cpu().numpy().astype(np.float64)
    ref = np.zeros(grid.nphys)
    for s in range(batch.nsim):
        gs, _ = oracle.adjoint(ogrid(grid), vmix.ravel(), cfg.dt, cfg.nt, 1, batch.src_cell[s:s + 1], [1.0],
                               f32(batch.wavelet), batch.rec_cell[batch.rec_ptr[s]:batch.rec_ptr[s + 1]], rho[s],
                               coef_fp32=True)
        ref += gs
    e = rel(g, 2.5 * ref)
    say("  shared-residual gradient rel %.2e" % e)
    assert e < TOL


# ---------------------------------------------- ragged / uneven edge cases

def edge_problem(F, ckpt, R=3, nt=240):
    """Two samples with different odd-sized grids and spacings, several sims each;
    sources stacked in one column on different rows, two sources on one cell, sources
    and receivers on ragged tile edges and inside the sponge-adjacent edge cells."""
    g0 = F.Grid(nz=37, nx=83, dz=9.0, dx=11.0, nb=7, v_ref=3200.0, v_max=3300.0)
    g1 = F.Grid(nz=70, nx=130, dz=10.0, dx=10.0, nb=5, v_ref=3000.0, v_max=3300.0)
    r = np.random.default_rng(17)
    m0 = f32(r.uniform(1600, 3200, g0.nphys))
    m1 = f32(W.salt_2d(70, 130, seed=3, vtop=1500, vbot=2800, vsalt=3200).ravel())

    def cell(g, z, x):
        return z * g.nx + x

    s0 = [([cell(g0, 3, 10), cell(g0, 20, 10), cell(g0, 36, 82)], [1.0, -1.0, 1.0]),
          ([cell(g0, 0, 0), cell(g0, 5, 63), cell(g0, 5, 64)], [-1.0, 1.0, 1.0])]
    s1 = [([cell(g1, 1, 65), cell(g1, 1, 65), cell(g1, 40, 127)], [1.0, 1.0, -1.0]),
          ([cell(g1, 60, 2)], [1.0]),
          ([cell(g1, 2, 9), cell(g1, 30, 9), cell(g1, 31, 9), cell(g1, 69, 129)], [1.0, -1.0, -1.0, 1.0])]
    rec0 = np.array([cell(g0, 1, x) for x in range(0, 83, 2)] + [cell(g0, 30, 10), cell(g0, 36, 0)], dtype=np.int32)
    rec1 = np.array([cell(g1, 2, x) for x in range(130)] + [cell(g1, 50, 64), cell(g1, 69, 63), cell(g1, 33, 9)],
                    dtype=np.int32)
    wav = W.ricker(18.0, 1e-3, nt)
    batch = F.Batch([g0, g1], [0, 0, 1, 1, 1], s0 + s1, [rec0, rec0, rec1, rec1, rec1], wav)
    time = F.time_axis(1e-3, nt, R, ckpt)
    return batch, time, [m0, m1]


@pytest.mark.parametrize("ckpt", [0, 7])
def test_edge_cases_uneven_batch(F, ckpt):
    batch, time, models = edge_problem(F, ckpt)
    say("case edge uneven batch ckpt_every=%d" % ckpt)
    nt_rec = time.nt // time.rec_every
    r = np.random.default_rng(23)
    # observed data: oracle forward on perturbed models
    truth = [f32(m * (1 + 0.05 * r.standard_normal(m.shape))) for m in models]
    dobs = [f32(d) for d in oracle_forward_sims(batch, 1e-3, time.nt, time.rec_every, truth, coef_fp32=False)]
    kappa = [1.5, 0.75]
    is2 = 3.0
    dp, mis, gr, gn = run_gradient(F, batch, time, models, np.concatenate([d.ravel() for d in dobs]), is2, kappa)
    odp, omis, ogr = oracle_batch_gradient(batch, 1e-3, time.nt, time.rec_every, [m.ravel() for m in models], dobs,
                                           is2, kappa)
    gdp = split_data(dp, batch, nt_rec)
    for s in range(batch.nsim):
        e = rel(gdp[s], odp[s])
        say("  sim %d data rel %.2e misfit rel %.2e" % (s, e, abs(mis[s] / omis[s] - 1)))
        assert e < TOL and abs(mis[s] / omis[s] - 1) < TOL
    gg = split_model(gr, batch)
    for k in range(batch.nsample):
        e = rel(gg[k], ogr[k])
        say("  sample %d gradient rel %.2e" % (k, e))
        assert e < TOL
        assert abs(gn[k] / np.linalg.norm(gg[k]) - 1) < 1e-6


def test_store_all_equals_checkpointed(F):
    # with one time step per launch both schedules run identical arithmetic in identical
    # order: bitwise equal (two steps per launch sum the gradient in another order)
    outs = []
    F.fwi_set_time_blocking(1, 1)
    try:
        for ckpt in (0, 5):
            batch, time, models = edge_problem(F, ckpt, R=2, nt=100)
            nd = batch.data_size(time.nt // 2)
            dobs = np.random.default_rng(1).standard_normal(nd) * 1e-6
            outs.append(run_gradient(F, batch, time, models, dobs, 1.0, [1.0, 1.0]))
    finally:
        F.fwi_set_time_blocking(0, 0)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_determinism(F):
    batch, time, models = edge_problem(F, 0, R=2, nt=120)
    nd = batch.data_size(60)
    dobs = np.random.default_rng(2).standard_normal(nd) * 1e-6
    a = run_gradient(F, batch, time, models, dobs, 1.0, [1.0, 1.0])
    b = run_gradient(F, batch, time, models, dobs, 1.0, [1.0, 1.0])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# --------------------------------------------------------------------- 3D

@pytest.mark.parametrize("ckpt,wx", [(0, 32), (6, 32), (0, 64), (6, 64)])
def test_3d_parity(F, ckpt, wx):
    say("case 3d ckpt_every=%d tile width %d" % (ckpt, wx))
    g = F.Grid(nz=18, ny=21, nx=70, dz=20.0, dy=22.0, dx=25.0, nb=5, v_ref=3500.0, v_max=3600.0, ndim=3)
    cfg = W.C5
    m = f32(W.layered_salt_3d(18, 21, 70, seed=4, vmin=1500, vmax=3500).ravel())
    truth = f32(m * 0.9)  # 10 % slower: traveltimes move by many samples (residual ratio ~1)
    nt, R = 150, 2

    def cell(z, y, x):
        return (z * 21 + y) * 70 + x

    srcs = [([cell(1, 10, 35), cell(1, 2, 3), cell(9, 10, 35)], [1.0, -1.0, 1.0]),
            ([cell(1, 20, 69), cell(1, 7, 64), cell(1, 8, 64)], [1.0, 1.0, -1.0])]
    rec = np.array([cell(1, y, x) for y in range(0, 21, 2) for x in range(0, 70, 3)] + [cell(17, 20, 69)],
                   dtype=np.int32)
    wav = W.ricker(6.0, 2e-3, nt)
    batch = F.Batch([g], [0, 0], srcs, [rec, rec], wav)
    time = F.time_axis(2e-3, nt, R, ckpt)
    # half-amplitude observed data keeps the residual ratio near 1 (well-conditioned
    # d - d_obs) despite the short record being dominated by direct arrivals
    dobs = [f32(0.5 * d) for d in oracle_forward_sims(batch, 2e-3, nt, R, [truth], coef_fp32=False)]
    try:
        F.fwi_set_tile_width(wx)
        dp, mis, gr, gn = run_gradient(F, batch, time, [m], np.concatenate([d.ravel() for d in dobs]), 1.0, [1.0])
    finally:
        F.fwi_set_tile_width(0)
    odp, omis, ogr = oracle_batch_gradient(batch, 2e-3, nt, R, [m], dobs, 1.0, [1.0])
    gdp = split_data(dp, batch, nt // R)
    for s in range(2):
        e = rel(gdp[s], odp[s])
        ratio = np.linalg.norm(odp[s] - dobs[s]) / np.linalg.norm(dobs[s])
        say("  sim %d data rel %.2e (residual ratio %.2f) misfit rel %.2e" % (s, e, ratio, abs(mis[s] / omis[s] - 1)))
        assert e < TOL and abs(mis[s] / omis[s] - 1) < TOL
        assert ratio >= 0.3
    e = rel(gr, ogr[0])
    say("  gradient rel %.2e" % e)
    assert e < TOL


def test_3d_uneven_batch_per_sample_imaging(F):
    """Two 3D samples of different grid sizes with 3 and 1 supergathers, receivers on planes
    through the whole depth, against the oracle, with 16-, 24-, 32- and 40-plane forward
    tiles (the adjoint sweeps 16-plane tiles of each sample's grid for all of its
    supergathers; under taller forward tiles it skips the receiver events above its first
    plane, and a 40-plane tile is taller than either grid) and tiles 64 and 32 cells wide
    (one and two rows per wavefront) -- and all eight tile shapes bit-identical."""
    say("case 3d uneven batch")
    grids = [F.Grid(nz=30, ny=9, nx=40, dz=20.0, dy=22.0, dx=25.0, nb=4, v_ref=3500.0, v_max=3600.0, ndim=3),
             F.Grid(nz=20, ny=12, nx=70, dz=20.0, dy=22.0, dx=25.0, nb=3, v_ref=3500.0, v_max=3600.0, ndim=3)]
    r = np.random.default_rng(11)

    def cell(g, z, y, x):
        return (z * g.ny + y) * g.nx + x

    g0, g1 = grids
    srcs = [([cell(g0, 1, 4, 20), cell(g0, 1, 1, 5)], [1.0, -1.0]),
            ([cell(g0, 15, 8, 39), cell(g0, 2, 0, 0), cell(g0, 29, 4, 10)], [-1.0, 1.0, 1.0]),
            ([cell(g0, 1, 6, 33)], [1.0]),
            ([cell(g1, 1, 6, 35), cell(g1, 10, 2, 3)], [1.0, -1.0])]
    rec0 = np.array([cell(g0, z, y, x) for z in (1, 10, 20, 29) for y in range(0, 9, 4) for x in range(0, 40, 7)],
                    dtype=np.int32)
    rec1 = np.array([cell(g1, z, y, x) for z in (1, 12, 19) for y in range(0, 12, 5) for x in range(0, 70, 9)],
                    dtype=np.int32)
    nt, R = 120, 2
    wav = W.ricker(7.0, 2e-3, nt)
    batch = F.Batch(grids, [0, 0, 0, 1], srcs, [rec0, rec0, rec0, rec1], wav)
    time = F.time_axis(2e-3, nt, R, 0)
    models = [f32(r.uniform(1800, 3400, g.nphys)) for g in grids]
    truths = [f32(m * 0.9) for m in models]
    dobs = [f32(0.5 * d) for d in oracle_forward_sims(batch, 2e-3, nt, R, truths, coef_fp32=False)]
    flat = np.concatenate([d.ravel() for d in dobs])
    kappa = [1.5, 1.0]
    outs = []
    try:
        for bz in (16, 24, 32, 40):
            for wx in (64, 32):
                F.fwi_set_tile(3, bz)
                F.fwi_set_tile_width(wx)
                outs.append(run_gradient(F, batch, time, models, flat, 1.0, kappa))
    finally:
        F.fwi_set_tile(3, 0)
        F.fwi_set_tile_width(0)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    dp, mis, gr, _ = outs[0]
    odp, omis, ogr = oracle_batch_gradient(batch, 2e-3, nt, R, models, dobs, 1.0, kappa)
    gdp = split_data(dp, batch, nt // R)
    for s in range(batch.nsim):
        e = rel(gdp[s], odp[s])
        ratio = np.linalg.norm(odp[s] - dobs[s]) / np.linalg.norm(dobs[s])
        say("  sim %d data rel %.2e (residual ratio %.2f)" % (s, e, ratio))
        assert e < TOL and abs(mis[s] / omis[s] - 1) < TOL and ratio >= 0.3
    gs = split_model(gr, batch)
    for k in range(2):
        e = rel(gs[k], ogr[k])
        say("  sample %d gradient rel %.2e" % (k, e))
        assert e < TOL


@pytest.mark.parametrize("nx", [56, 57])
def test_3d_row_pitch(F, nx):
    """Rows of the padded 3D grid are stored 32 cells apart: nx = 56 with a 4-cell sponge
    pads to exactly 64 cells (no pitch columns), nx = 57 to 65 (31 pitch columns, a second
    row of 64-wide tiles that holds one grid column).  Sources and receivers sit on the
    last grid column; data, misfits and the gradient against the oracle."""
    say("case 3d row pitch, nx %d" % nx)
    ny, nz = 10, 12
    g = F.Grid(nz=nz, ny=ny, nx=nx, dz=20.0, dy=20.0, dx=20.0, nb=4, v_ref=3500.0, v_max=3600.0, ndim=3)
    r = np.random.default_rng(nx)
    m = f32(r.uniform(1800, 3400, g.nphys))
    truth = f32(m * 0.9)

    def cell(z, y, x):
        return (z * ny + y) * nx + x

    srcs = [([cell(1, 5, nx - 1), cell(6, 0, 0)], [1.0, -1.0]), ([cell(1, 9, nx // 2)], [1.0])]
    rec = np.array([cell(1, y, x) for y in range(0, ny, 3) for x in sorted(set(range(0, nx, 5)) | {nx - 1})],
                   dtype=np.int32)
    nt, R = 80, 1
    batch = F.Batch([g], [0, 0], srcs, [rec, rec], W.ricker(8.0, 2e-3, nt))
    time = F.time_axis(2e-3, nt, R, 7)
    dobs = [f32(0.5 * d) for d in oracle_forward_sims(batch, 2e-3, nt, R, [truth], coef_fp32=False)]
    dp, mis, gr, _ = run_gradient(F, batch, time, [m], np.concatenate([d.ravel() for d in dobs]), 1.0, [1.0])
    odp, omis, ogr = oracle_batch_gradient(batch, 2e-3, nt, R, [m], dobs, 1.0, [1.0])
    gdp = split_data(dp, batch, nt // R)
    for s in range(batch.nsim):
        e = rel(gdp[s], odp[s])
        say("  sim %d data rel %.2e misfit rel %.2e" % (s, e, abs(mis[s] / omis[s] - 1)))
        assert e < TOL and abs(mis[s] / omis[s] - 1) < TOL
    e = rel(gr, ogr[0])
    say("  gradient rel %.2e" % e)
    assert e < TOL


@pytest.mark.parametrize("wx", [32, 64])
def test_3d_launch_order_groups(F, wx):
    """3D batch of two samples with 5 and 2 supergathers on different grids: the forward's
    launch order takes at most 4 of a sample's supergathers at a tile position (groups of
    4 + 1, then 2), and every result matches the oracle."""
    say("case 3d launch-order groups, tile width %d" % wx)
    grids = [F.Grid(nz=22, ny=10, nx=37, dz=20.0, dy=20.0, dx=20.0, nb=4, v_ref=3500.0, v_max=3600.0, ndim=3),
             F.Grid(nz=18, ny=13, nx=30, dz=20.0, dy=20.0, dx=20.0, nb=3, v_ref=3500.0, v_max=3600.0, ndim=3)]
    r = np.random.default_rng(21)
    sample_of = [0, 0, 0, 0, 0, 1, 1]
    srcs, recs = [], []
    for k in sample_of:
        g = grids[k]
        srcs.append((r.integers(0, g.nphys, 2).astype(np.int32), r.choice([-1.0, 1.0], 2)))
        recs.append(np.array([(z * g.ny + y) * g.nx + x for z in (1, g.nz - 1) for y in range(0, g.ny, 4)
                              for x in range(0, g.nx, 6)], dtype=np.int32))
    nt, R = 80, 2
    batch = F.Batch(grids, sample_of, srcs, recs, W.ricker(7.0, 2e-3, nt))
    time = F.time_axis(2e-3, nt, R, 0)
    models = [f32(r.uniform(1800, 3400, g.nphys)) for g in grids]
    truths = [f32(m * 0.9) for m in models]
    dobs = [f32(0.5 * d) for d in oracle_forward_sims(batch, 2e-3, nt, R, truths, coef_fp32=False)]
    kappa = [0.7, 1.3]
    try:
        F.fwi_set_tile_width(wx)
        dp, mis, gr, _ = run_gradient(F, batch, time, models, np.concatenate([d.ravel() for d in dobs]), 1.0, kappa)
    finally:
        F.fwi_set_tile_width(0)
    odp, omis, ogr = oracle_batch_gradient(batch, 2e-3, nt, R, models, dobs, 1.0, kappa)
    gdp = split_data(dp, batch, nt // R)
    for s in range(batch.nsim):
        e = rel(gdp[s], odp[s])
        say("  sim %d (sample %d) data rel %.2e" % (s, sample_of[s], e))
        assert e < TOL and abs(mis[s] / omis[s] - 1) < TOL
    gs = split_model(gr, batch)
    for k in range(2):
        e = rel(gs[k], ogr[k])
        say("  sample %d gradient rel %.2e" % (k, e))
        assert e < TOL


# ------------------------------------------------------ stored oracle golden

def test_stored_oracle_golden(F):
    """The HIP path against the oracle's stored values for the tiny encoded 2D problem of
    tests/golden/oracle_tiny_2d.json (written by tests/golden/make_oracle_golden.py from the
    oracle alone): per-supergather misfits, data norms and sampled data, and the sample's
    gradient, all within 1e-5 relative."""
    import importlib.util
    import json
    import os
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_oracle_golden", os.path.join(gdir, "make_oracle_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    ref = json.load(open(os.path.join(gdir, "oracle_tiny_2d.json")))
    p = mk.PROBLEM
    say("case stored oracle golden")
    og, v, truth, wav, sims, rec = mk.build_problem(p)
    g = F.Grid(nz=og.nz, nx=og.nx, dz=og.dz, dx=og.dx, nb=og.nb, v_ref=og.v_ref, v_max=3000.0)
    batch = F.Batch([g], [0] * len(sims), [(c, w) for c, w in sims], [rec] * len(sims), wav)
    time = F.time_axis(p["dt"], p["nt"], p["rec_every"], 0)
    dobs = mk.observed(p)
    dp, mis, gr, _ = run_gradient(F, batch, time, [v], np.concatenate([d.ravel() for d in dobs]),
                                  p["inv_sigma2"], [1.0])
    nt_rec = p["nt"] // p["rec_every"]
    gd = split_data(dp, batch, nt_rec)
    for s in range(len(sims)):
        assert abs(mis[s] / ref["misfit"][s] - 1) < TOL
        assert abs(np.linalg.norm(gd[s]) / ref["d_pred_norm"][s] - 1) < TOL
        pts = ref["d_pred_samples"][s]
        assert rel(np.array([gd[s][t, r] for t, r, _ in pts]), np.array([x for _, _, x in pts])) < TOL
    e = rel(gr, np.array(ref["gradient"]))
    say("  gradient rel %.2e" % e)
    assert e < TOL


# ------------------------------------------------------- encode, Langevin

def test_encode_matches_oracle(F):
    say("case encode")
    r = np.random.default_rng(3)
    d = f32(r.standard_normal((12, 37, 19)))
    gs, gw, kap = F.fwi_draw_encoding(9, 1, 0, 12, 4, 5)
    ptr = np.arange(0, 21, 4, dtype=np.int32)
    out = torch.zeros(5, 37, 19, device="cuda")
    F.fwi_encode(dev(d), dev(ptr, torch.int32), dev(gs, torch.int32), dev(gw), out)
    ref = oracle.encode(d, ptr, gs, gw)
    assert rel(out.cpu().numpy(), ref) < 1e-6
    # a malformed table poisons only its group
    bad = gs.copy()
    bad[5] = 12
    F.fwi_encode(dev(d), dev(ptr, torch.int32), dev(bad, torch.int32), dev(gw), out)
    o = out.cpu().numpy()
    assert np.isnan(o[1]).all() and np.isfinite(o[0]).all() and np.isfinite(o[2:]).all()


def test_langevin_matches_oracle(F):
    say("case langevin")
    off = np.array([0, 1001, 1001 + 4096, 1001 + 4096 + 7], dtype=np.int64)
    n = int(off[-1])
    r = np.random.default_rng(4)
    v0 = f32(r.uniform(1500, 4500, n))
    g = f32(r.standard_normal(n) * 50)
    xi = f32(r.standard_normal(n))
    eta, nu, lo, hi = 0.7, math.sqrt(1.4), 1600.0, 4400.0
    v = dev(v0)
    F.fwi_langevin(off, v, dev(g), dev(xi), 5, 3, eta, nu, lo, hi)
    ref = oracle.langevin(v0, g, xi, float(np.float32(eta)), float(np.float32(nu)), lo, hi)
    assert np.max(np.abs(v.cpu().numpy() - ref) / np.abs(ref)) < 1.2e-7
    # in-kernel Philox noise: with v = 0, eta = 0, nu = 1 and open bounds the update is xi
    v = torch.zeros(n, device="cuda")
    F.fwi_langevin(off, v, dev(g), None, 77, 12, 0.0, 1.0, -1e30, 1e30)
    got = v.cpu().numpy().astype(np.float64)
    for k in range(3):
        ref = oracle.normals(77, 12, k, off[k + 1] - off[k])
        assert np.max(np.abs(got[off[k]:off[k + 1]] - ref)) < 1e-6 * max(1.0, np.abs(ref).max())


def test_device_flags_model_above_vmax(F):
    say("case device flag")
    batch, time, models = edge_problem(F, 0, R=2, nt=20)
    models = [m.copy() for m in models]
    models[1][5] = 3400.0  # above v_max = 3300
    v = dev(np.concatenate([m.ravel() for m in models]))
    ws = F.alloc_workspace(batch, time)
    F.fwi_forward(batch, time, v, None, ws)
    with pytest.raises(F.FwiError) as e:
        F.fwi_poll_status(ws)
    assert e.value.status == F.FWI_E_NONFINITE
    F.fwi_poll_status(ws)  # cleared


# ------------------------------------------- per-sample imaging (2D adjoint)

def grouped_problem(F, counts, seed):
    """One sample per entry of counts (each on its own grid size), with that many
    supergathers of 1-3 random +-1 sources each; receivers every third column of row 1."""
    r = np.random.default_rng(seed)
    grids, models, sample_of, srcs, recs = [], [], [], [], []
    for k, G in enumerate(counts):
        nz, nx = 30 + 7 * k, 61 + 13 * k
        g = F.Grid(nz=nz, nx=nx, dz=10.0, dx=10.0, nb=6, v_ref=3000.0, v_max=3300.0)
        grids.append(g)
        models.append(f32(r.uniform(1800, 3200, g.nphys)))
        rec = (np.arange(0, nx, 3) + nx).astype(np.int32)
        for _ in range(G):
            n = int(r.integers(1, 4))
            srcs.append((r.integers(0, g.nphys, n).astype(np.int32), r.choice([-1.0, 1.0], n)))
            recs.append(rec)
            sample_of.append(k)
    return grids, models, sample_of, srcs, recs


@pytest.mark.parametrize("counts", [(1, 3, 7, 17), (32,)])
def test_per_sample_imaging_any_group_size(F, counts):
    # the 2D adjoint sums a sample's supergathers inside one workgroup; samples of 1, 3,
    # 7 and 17 supergathers share one launch (one wave count for all, idle waves in the
    # small samples), and 32 supergathers of one sample fill 16-wave workgroups.
    # Adjoint + imaging alone against a shared FP32 residual, kappa != 1.
    say("case per-sample imaging, supergathers per sample %s" % (counts,))
    grids, models, sample_of, srcs, recs = grouped_problem(F, counts, seed=sum(counts))
    nt, R = 120, 2
    batch = F.Batch(grids, sample_of, srcs, recs, W.ricker(15.0, 1e-3, nt))
    time = F.time_axis(1e-3, nt, R, 0)
    r = np.random.default_rng(7)
    rho = [f32(r.standard_normal((nt // R, batch.nrec[s])) * 1e-3) for s in range(batch.nsim)]
    kappa = [0.5 + k for k in range(len(counts))]
    v = dev(np.concatenate([m.ravel() for m in models]))
    ws = F.alloc_workspace(batch, time)
    F.fwi_forward(batch, time, v, None, ws)
    grad = torch.zeros(batch.model_size, device="cuda")
    F.fwi_adjoint(batch, time, v, dev(np.concatenate([x.ravel() for x in rho])), kappa, grad, None, ws)
    F.fwi_poll_status(ws)
    gg = split_model(grad.cpu().numpy().astype(np.float64), batch)
    for k in range(len(counts)):
        ref = np.zeros(grids[k].nphys)
        for s in range(batch.nsim):
            if sample_of[s] != k:
                continue
            a, b = batch.src_ptr[s], batch.src_ptr[s + 1]
            gs, _ = oracle.adjoint(ogrid(grids[k]), models[k], 1e-3, nt, R, batch.src_cell[a:b], f32(batch.src_w[a:b]),
                                   f32(batch.wavelet), batch.rec_cell[batch.rec_ptr[s]:batch.rec_ptr[s + 1]], rho[s],
                                   coef_fp32=True)
            ref += gs
        e = rel(gg[k], kappa[k] * ref)
        say("  sample %d (%d supergathers) gradient rel %.2e" % (k, counts[k], e))
        assert e < TOL
