"""GPU tests of the autograd form and of full-size sampled parity.

* autograd (torch.autograd.Function over fwi_forward / fwi_adjoint) on an uneven batch
  of three grid sizes with checkpoints every 10 steps: gradient vs the FP64 oracle and
  vs central differences of the loss;
* full-size sampled parity on the uneven 32-sample configuration (2000 steps, K = 10)
  and on the 400x150 / 160-simulation configuration the benchmark times, comparing the
  outputs of one sample (all of its simulations) with the oracle.
"""
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


def uneven_problem(F, sizes, nsample, nt, ckpt, h=10.0, nb=8, seed=0, s=2, smooth=3.0):
    """Salt models on grids of several sizes, samples round-robin over sizes, one
    supergather of s shots per sample (G = 1); starting models smoothed by `smooth` cells."""
    from paper_2512_12797_amd import problems
    cfg = W.C3
    grids = [F.Grid(nz=sizes[k % len(sizes)][0], nx=sizes[k % len(sizes)][1], dz=h, dx=h, nb=nb,
                    v_ref=cfg.vmax, v_max=cfg.vmax * 1.1) for k in range(nsample)]
    wav = W.ricker(cfg.freq, cfg.dt, nt)
    batch, groups = problems.encoded_batch(cfg, grids, wav, seed=seed, step=0, s=s, G=1,
                                           nshot_of=lambda g: max(s, g.nx // 16))
    models = [f32(W.salt_2d(g.nz, g.nx, seed=seed + k).ravel()) for k, g in enumerate(grids)]
    start = [f32(W.smooth(m.reshape(g.nz, g.nx), smooth).ravel()) for m, g in zip(models, grids)]
    time = F.time_axis(cfg.dt, nt, 1, ckpt)
    return batch, groups, time, models, start


def test_autograd_uneven_vs_oracle_and_fd(F):
    from paper_2512_12797_amd.autograd import FwiOperator
    sizes = [(24, 40), (30, 64), (30, 100)]
    batch, groups, time, truth, start = uneven_problem(F, sizes, 6, 300, 10)
    say("case autograd uneven 3 sizes, ckpt 10")
    dobs = [f32(d) for d in oracle_forward_sims(batch, time.dt, time.nt, 1, [m for m in truth], coef_fp32=False)]
    dobs_t = dev(np.concatenate([d.ravel() for d in dobs]))
    op = FwiOperator(batch, time)
    v = dev(np.concatenate(start)).requires_grad_(True)
    d = op(v)
    loss = 0.5 * ((d - dobs_t).double() ** 2).sum()
    loss.backward()
    g = v.grad.double().cpu().numpy()
    _, omis, ogr = oracle_batch_gradient(batch, time.dt, time.nt, 1, start, dobs, 1.0, [1.0] * batch.nsample)
    gg = split_model(g, batch)
    for k in range(batch.nsample):
        e = rel(gg[k], ogr[k])
        say("  sample %d (%dx%d) autograd gradient rel %.2e" % (k, batch.grids[k].nz, batch.grids[k].nx, e))
        assert e < TOL
    assert abs(loss.item() / omis.sum() - 1) < TOL
    # central differences of the FP32 loss along a smooth direction
    r = np.random.default_rng(3)
    dv = dev(np.concatenate([W.smooth(r.standard_normal((gr.nz, gr.nx)), 2.0).ravel() * 30.0
                             for gr in batch.grids]))
    eps = 0.5

    def L(x):
        with torch.no_grad():
            return float(0.5 * ((op(x) - dobs_t).double() ** 2).sum())

    fd = (L(v.detach() + eps * dv) - L(v.detach() - eps * dv)) / (2 * eps)
    an = float((v.grad.double() * dv.double()).sum())
    say("  FD %.6e  autograd %.6e  rel %.2e" % (fd, an, abs(fd - an) / abs(an)))
    assert abs(fd - an) <= 2e-3 * abs(an)


def test_autograd_two_forwards_before_backward(F):
    """A loss built from two forward calls of one operator (the second replaces the
    workspace state of the first): both gradients still match the oracle at their own
    models, and the earlier output's backward re-ran its forward once."""
    from paper_2512_12797_amd.autograd import FwiOperator
    sizes = [(24, 40), (30, 64)]
    batch, groups, time, truth, start = uneven_problem(F, sizes, 2, 200, 10)
    say("case autograd two forwards before backward")
    dobs = [f32(d) for d in oracle_forward_sims(batch, time.dt, time.nt, 1, [m for m in truth], coef_fp32=False)]
    dobs_t = dev(np.concatenate([d.ravel() for d in dobs]))
    op = FwiOperator(batch, time)
    m2 = [f32(1.04 * m) for m in start]
    v1 = dev(np.concatenate(start)).requires_grad_(True)
    v2 = dev(np.concatenate(m2)).requires_grad_(True)
    d1 = op(v1)
    d2 = op(v2)
    loss = 0.5 * ((d1 - dobs_t).double() ** 2).sum() + 0.25 * ((d2 - dobs_t).double() ** 2).sum()
    loss.backward()
    assert op.replays == 1
    for v, models, w in ((v1, start, 1.0), (v2, m2, 0.5)):
        _, _, ogr = oracle_batch_gradient(batch, time.dt, time.nt, 1, models, dobs, 1.0, [1.0] * batch.nsample)
        gg = split_model(v.grad.double().cpu().numpy(), batch)
        for k in range(batch.nsample):
            e = rel(gg[k], w * ogr[k])
            say("  weight %.2f sample %d gradient rel %.2e" % (w, k, e))
            assert e < TOL


def test_uneven_full_size_sampled(F):
    # the uneven configuration at full size: 32 samples on 256x128, 512x200, 800x200
    # (10 m, 20-cell sponge), 2000 steps, checkpoints every 10, one launch per step over
    # all 32 simulations; samples 0, 1 and 2 (one per grid size) are recomputed by the
    # oracle.  Starting models are smoothed by 10 cells so that every compared residual
    # ratio is above 0.3 (the gradient-parity condition).
    from paper_2512_12797_amd.autograd import FwiOperator
    sizes = list(W.C3_SIZES)
    batch, groups, time, truth, start = uneven_problem(F, sizes, 32, 2000, 10, nb=20, s=8, smooth=10.0)
    say("case uneven full size: %d sims, padded cells %d" % (batch.nsim, sum(
        (g.nz + 40) * (g.nx + 40) for g in batch.grids)))
    r = np.random.default_rng(9)
    nt_rec = time.nt
    cmp = [0, 1, 2]
    assert len({(batch.grids[k].nz, batch.grids[k].nx) for k in cmp}) == 3
    # observed data: the oracle for the compared samples' simulations, seeded noise elsewhere
    sb = _sub_batch(F, batch, cmp)
    dcmp = oracle_forward_sims(sb, time.dt, time.nt, 1, [truth[k] for k in cmp], coef_fp32=False)
    dobs = [f32(x) for x in dcmp] + [f32(1e-6 * r.standard_normal((nt_rec, batch.nrec[s])))
                                     for s in range(len(cmp), batch.nsim)]
    op = FwiOperator(batch, time)
    v = dev(np.concatenate(start)).requires_grad_(True)
    d = op(v)
    loss = 0.5 * ((d - dev(np.concatenate([x.ravel() for x in dobs]))).double() ** 2).sum()
    loss.backward()
    gs = split_model(v.grad.double().cpu().numpy(), batch)
    ds = split_data(d.detach().double().cpu().numpy(), batch, nt_rec)
    odp, _, ogr = oracle_batch_gradient(sb, time.dt, time.nt, 1, [start[k] for k in cmp], dobs[:len(cmp)], 1.0,
                                        [1.0] * len(cmp))
    for i, k in enumerate(cmp):
        e_d = rel(ds[k], odp[i])
        e_g = rel(gs[k], ogr[i])
        ratio = np.linalg.norm(odp[i] - dobs[i]) / np.linalg.norm(dobs[i])
        say("  sample %d (%dx%d): data rel %.2e, gradient rel %.2e, residual ratio %.2f" % (
            k, batch.grids[k].nz, batch.grids[k].nx, e_d, e_g, ratio))
        assert ratio >= 0.3
        assert e_d < TOL and e_g < TOL


def _sub_batch(F, batch, sims):
    """The simulations `sims` of a batch as their own batch (one sample each)."""
    sources, receivers, grids = [], [], []
    for s in sims:
        a, b = batch.src_ptr[s], batch.src_ptr[s + 1]
        sources.append((batch.src_cell[a:b], batch.src_w[a:b]))
        receivers.append(batch.rec_cell[batch.rec_ptr[s]:batch.rec_ptr[s + 1]])
        grids.append(batch.grids[batch.sample_of[s]])
    return F.Batch(grids, list(range(len(sims))), sources, receivers, batch.wavelet)


def test_bench_configuration_full_size_sampled(F):
    # the benchmark's configuration and launch shape: 400x150, 160 simulations (16
    # samples x 10 supergathers of 8), 4000 internal steps recorded every 2, keep-all
    # schedule; sample 0's 10 supergathers are recomputed by the oracle
    from paper_2512_12797_amd import problems
    cfg = W.C2
    grid = problems.grid_of(cfg)
    wav = W.ricker(cfg.freq, cfg.dt, cfg.nt)
    batch, groups = problems.encoded_batch(cfg, [grid] * cfg.nsample, wav, seed=1000, step=0)
    vtrue = f32(W.thrust_2d(cfg.nz, cfg.nx, seed=1000).ravel())
    vstart = f32(np.clip(W.smooth(vtrue.reshape(cfg.nz, cfg.nx), 16.0), cfg.vmin, cfg.vmax).ravel())
    time = F.time_axis(cfg.dt, cfg.nt, cfg.rec_every, 0)
    nt_rec = cfg.nt_rec
    s0 = [s for s in range(batch.nsim) if batch.sample_of[s] == 0]
    say("case bench configuration full size (oracle on %d simulations)" % len(s0))
    sb = _sub_batch(F, batch, s0)
    dobs0 = [f32(x) for x in oracle_forward_sims(sb, cfg.dt, cfg.nt, cfg.rec_every, [vtrue] * len(s0),
                                                 coef_fp32=False)]
    r = np.random.default_rng(1)
    dobs = dobs0 + [f32(1e-3 * r.standard_normal((nt_rec, batch.nrec[s]))) for s in range(len(s0), batch.nsim)]
    v = dev(np.tile(vstart, cfg.nsample))
    dpred = torch.zeros(batch.data_size(nt_rec), device="cuda")
    mis = torch.zeros(batch.nsim, dtype=torch.float64, device="cuda")
    grad = torch.zeros(batch.model_size, device="cuda")
    ws = F.alloc_workspace(batch, time)
    kappa = [g[2] for g in groups]
    F.fwi_gradient(batch, time, v, dev(np.concatenate([x.ravel() for x in dobs])), 1.0, kappa, dpred, mis, grad,
                   None, ws)
    F.fwi_poll_status(ws)
    del ws
    torch.cuda.empty_cache()
    odp, omis, ogr = oracle_batch_gradient(sb, cfg.dt, cfg.nt, cfg.rec_every, [vstart] * len(s0), dobs0, 1.0,
                                           [kappa[0]] * len(s0))
    gdp = split_data(dpred.double().cpu().numpy(), batch, nt_rec)
    gm = mis.cpu().numpy()
    for i, s in enumerate(s0):
        e = rel(gdp[s], odp[i])
        ratio = np.linalg.norm(odp[i] - dobs0[i]) / np.linalg.norm(dobs0[i])
        say("  sim %d data rel %.2e residual ratio %.2f misfit rel %.2e" % (s, e, ratio, abs(gm[s] / omis[i] - 1)))
        assert e < TOL and abs(gm[s] / omis[i] - 1) < TOL
        # gradient parity is claimed where the residual is not ill-conditioned (ratio >= 0.3)
        assert ratio >= 0.3
    g0 = grad.double().cpu().numpy()[:grid.nphys]
    ref = sum(ogr)  # each oracle "sample" here is one simulation, already scaled by kappa
    e = rel(g0, ref)
    say("  sample 0 gradient rel %.2e" % e)
    assert e < TOL


def test_3d_configuration_full_size_properties(F):
    """The 3D configuration at full size in the bench's launch shape: 200x200x100 physical
    (10-cell sponge), 32 simulations (8 samples x 4 supergathers of 16 +-1-encoded shots),
    1500 steps of 2 ms, every simulation in one launch per step.  A full-size 3D oracle
    gradient is out of reach (0.24 s per oracle step and simulation), so properties that
    hold at any size are checked instead:
    * linearity in the encoding: sample 0's first supergather's data equal the +-1-weighted
      sum of its 16 shots simulated one by one (rel L2 <= 1e-5);
    * the checkpoint schedule does not change the arithmetic: the gradients with
      checkpoints every 50 and every 30 steps, and with the bench's schedule (the kept
      tail and checkpoint interval fwi_schedule picks for the free memory), are identical
      bit for bit;
    * the gradient is finite and nonzero, and the per-sample norms match it."""
    from paper_2512_12797_amd import problems
    cfg = W.C5
    grid = problems.grid_of(cfg)
    wav = W.ricker(cfg.freq, cfg.dt, cfg.nt)
    vtrue = W.layered_salt_3d(cfg.nz, cfg.ny, cfg.nx, seed=0, vmin=cfg.vmin, vmax=cfg.vmax)
    vstart = f32(np.clip(W.smooth(vtrue, 8.0), cfg.vmin, cfg.vmax).ravel())
    batch, groups = problems.encoded_batch(cfg, [grid] * cfg.nsample, wav, seed=0, step=0)
    nt_rec = cfg.nt // cfg.rec_every
    say("case 3d full size: %d sims of %d padded cells, %d steps" % (batch.nsim, (grid.nz + 20) * (grid.ny + 20) *
                                                                    (grid.nx + 20), cfg.nt))
    torch.cuda.empty_cache()
    v = dev(np.tile(vstart, cfg.nsample))
    dobs = dev(1e-3 * np.random.default_rng(3).standard_normal(batch.data_size(nt_rec)))
    kappa = [g[2] for g in groups]
    outs = []
    for k in (50, 30, "schedule"):
        if k == "schedule":
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info()
            time = F.fwi_schedule(batch, F.time_axis(cfg.dt, cfg.nt, cfg.rec_every), free - (8 << 30))
            say("  schedule for %.1f GB: checkpoints every %d, last %d steps kept" % (
                (free - (8 << 30)) / 1e9, time.ckpt_every, time.keep_tail))
            assert time.ckpt_every >= 1 and time.keep_tail > 0
        else:
            time = F.time_axis(cfg.dt, cfg.nt, cfg.rec_every, k)
        ws = F.alloc_workspace(batch, time)
        dpred = torch.zeros(batch.data_size(nt_rec), device="cuda")
        mis = torch.zeros(batch.nsim, dtype=torch.float64, device="cuda")
        grad = torch.zeros(batch.model_size, device="cuda")
        gn = torch.zeros(batch.nsample, device="cuda")
        F.fwi_gradient(batch, time, v, dobs, 1.0, kappa, dpred, mis, grad, gn, ws)
        F.fwi_poll_status(ws)
        outs.append((dpred.cpu().numpy(), mis.cpu().numpy(), grad.cpu().numpy(), gn.cpu().numpy()))
        say("  checkpoints %s: |grad| %.3e" % (k, float(grad.double().norm())))
        del ws, dpred, mis, grad, gn
        torch.cuda.empty_cache()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    dpred, mis, grad, gn = outs[0]
    assert np.all(np.isfinite(grad)) and np.abs(grad).max() > 0
    per = split_model(grad.astype(np.float64), batch)
    assert np.allclose(gn, [np.linalg.norm(x) for x in per], rtol=1e-5)
    # linearity: supergather 0 of sample 0 against its 16 shots one by one
    gs, gw, _ = groups[0]
    s = cfg.shots_per_group
    shots = problems.shot_cells(cfg, grid)[gs[:s]]
    single = problems.single_shot_batch(cfg, grid, shots, wav)
    tf = F.time_axis(cfg.dt, cfg.nt, cfg.rec_every, -1)
    ws = F.alloc_workspace(single, tf)
    d1 = torch.zeros(single.data_size(nt_rec), device="cuda")
    F.fwi_forward(single, tf, dev(vstart), d1, ws)
    F.fwi_poll_status(ws)
    del ws
    d1 = split_data(d1.double().cpu().numpy(), single, nt_rec)
    ref = sum(float(w) * d for w, d in zip(gw[:s], d1))
    got = split_data(dpred.astype(np.float64), batch, nt_rec)[0]
    e = rel(got, ref)
    say("  encoded supergather vs sum of its 16 shots: rel %.2e" % e)
    assert np.abs(ref).max() > 0 and e < TOL


@pytest.mark.timeout(900)
def test_3d_full_grid_vs_oracle(F):
    """The 3D configuration's full grid (200x200x100 physical, 220x220x120 padded, 25 m)
    in the bench's launch shape: all 32 simulations (8 samples x 4 supergathers of 16
    shots) in one launch per time step, checkpoints every 10 steps.  The window is 100
    steps of 2 ms with an 8 Hz Ricker delayed by 0.08 s, so that the wavefield develops
    within what the oracle can keep (5.8 M cells x 8 B x 100 steps = 4.6 GB per
    simulation).  Sample 0's 4 supergathers are recomputed by the oracle: data per
    simulation, misfits and the sample's gradient within 1e-5.  The start is 0.85 x the
    true model (residual ratio about 0.43, above the 0.3 gradient-parity condition)."""
    from paper_2512_12797_amd import problems
    cfg = W.C5
    grid = problems.grid_of(cfg)
    nt = 100
    wav = W.ricker(8.0, cfg.dt, nt, t0=0.08)
    batch, groups = problems.encoded_batch(cfg, [grid] * cfg.nsample, wav, seed=0, step=0)
    vtrue = f32(W.layered_salt_3d(cfg.nz, cfg.ny, cfg.nx, seed=0, vmin=cfg.vmin, vmax=cfg.vmax).ravel())
    vstart = f32(0.85 * vtrue)
    s0 = [s for s in range(batch.nsim) if batch.sample_of[s] == 0]
    say("case 3d full grid vs oracle: %d sims of %d padded cells, %d steps; oracle on %d sims" % (
        batch.nsim, (grid.nz + 20) * (grid.ny + 20) * (grid.nx + 20), nt, len(s0)))
    sb = _sub_batch(F, batch, s0)
    dobs0 = [f32(x) for x in oracle_forward_sims(sb, cfg.dt, nt, 1, [vtrue] * len(s0), coef_fp32=False)]
    r = np.random.default_rng(4)
    dobs = dobs0 + [f32(1e-3 * r.standard_normal((nt, batch.nrec[s]))) for s in range(len(s0), batch.nsim)]
    torch.cuda.empty_cache()
    time = F.time_axis(cfg.dt, nt, 1, 10)
    ws = F.alloc_workspace(batch, time)
    v = dev(np.tile(vstart, cfg.nsample))
    dpred = torch.zeros(batch.data_size(nt), device="cuda")
    mis = torch.zeros(batch.nsim, dtype=torch.float64, device="cuda")
    grad = torch.zeros(batch.model_size, device="cuda")
    kappa = [g[2] for g in groups]
    F.fwi_gradient(batch, time, v, dev(np.concatenate([x.ravel() for x in dobs])), 1.0, kappa, dpred, mis, grad,
                   None, ws)
    F.fwi_poll_status(ws)
    del ws
    torch.cuda.empty_cache()
    gdp = split_data(dpred.double().cpu().numpy(), batch, nt)
    gm = mis.cpu().numpy()
    g0 = grad.double().cpu().numpy()[:grid.nphys]
    odp, omis, ogr = oracle_batch_gradient(sb, cfg.dt, nt, 1, [vstart] * len(s0), dobs0, 1.0, [kappa[0]] * len(s0))
    for i, s in enumerate(s0):
        e = rel(gdp[s], odp[i])
        ratio = np.linalg.norm(odp[i] - dobs0[i]) / np.linalg.norm(dobs0[i])
        say("  sim %d data rel %.2e residual ratio %.2f misfit rel %.2e" % (s, e, ratio, abs(gm[s] / omis[i] - 1)))
        assert ratio >= 0.3
        assert e < TOL and abs(gm[s] / omis[i] - 1) < TOL
    e = rel(g0, sum(ogr))
    say("  sample 0 gradient rel %.2e" % e)
    assert np.abs(g0).max() > 0 and e < TOL


# ------------------------------------------------ graphs, tile heights, tuner

def _edge_batch(F, seed, ckpt=0, nt=160, R=2):
    """Uneven 2-sample batch whose encodings are redrawn per `seed`."""
    from paper_2512_12797_amd import problems
    cfg = W.C3
    grids = [F.Grid(nz=37, nx=83, dz=10.0, dx=10.0, nb=7, v_ref=3500.0, v_max=3850.0),
             F.Grid(nz=50, nx=150, dz=10.0, dx=10.0, nb=6, v_ref=3500.0, v_max=3850.0)]
    wav = W.ricker(15.0, 1e-3, nt)
    batch, groups = problems.encoded_batch(cfg, grids, wav, seed=seed, step=seed, s=3, G=2,
                                           nshot_of=lambda g: 6)
    time = F.time_axis(1e-3, nt, R, ckpt)
    models = [f32(W.salt_2d(g.nz, g.nx, seed=k + 5, vtop=1500, vbot=2800, vsalt=3500).ravel())
              for k, g in enumerate(grids)]
    return batch, groups, time, models


def _run(F, batch, time, v, dobs, kappa, ws, stream=None):
    nd = batch.data_size(time.nt // time.rec_every)
    dpred = torch.zeros(nd, device="cuda")
    mis = torch.zeros(batch.nsim, dtype=torch.float64, device="cuda")
    grad = torch.zeros(batch.model_size, device="cuda")
    F.fwi_gradient(batch, time, v, dobs, 2.0, kappa, dpred, mis, grad, None, ws, stream=stream)
    torch.cuda.synchronize()
    return dpred.cpu().numpy(), mis.cpu().numpy(), grad.cpu().numpy()


def _overlap_problem(F, ndim):
    """97-step problems of the checkpoint-schedule tests (2D: uneven two-sample batch; 3D:
    one sample, three supergathers)."""
    if ndim == 2:
        batch, groups, _, models = _edge_batch(F, 3, 6, nt=97, R=1)
        dt = 1e-3
    else:
        g = F.Grid(nz=14, ny=11, nx=30, dz=20.0, dy=20.0, dx=20.0, nb=3, v_ref=3500.0, v_max=3850.0, ndim=3)
        r0 = np.random.default_rng(5)
        srcs = [(r0.integers(0, g.nphys, 2).astype(np.int32), [1.0, -1.0]) for _ in range(3)]
        rec = np.arange(0, g.nphys, 7, dtype=np.int32)
        batch = F.Batch([g], [0, 0, 0], srcs, [rec] * 3, W.ricker(9.0, 2e-3, 97))
        groups = [(None, None, 1.0)]
        models = [f32(r0.uniform(1800, 3400, g.nphys))]
        dt = 2e-3
    return batch, groups, models, dt


@pytest.mark.parametrize("ndim", [2, 3])
def test_overlapped_recomputation_is_bitwise_sequential(F, ndim):
    """Checkpointed schedules with the recomputation of segment s - 1 beside the adjoint of
    segment s (side stream, two imaging rings) give the sequential schedule's results bit
    for bit, directly and as a replayed graph, and match the oracle.  nt = 97 with
    checkpoints every 6 steps leaves a short last segment."""
    say("case overlapped recomputation %dD" % ndim)
    batch, groups, models, dt = _overlap_problem(F, ndim)
    time = F.time_axis(dt, 97, 1, 6)
    kappa = [gr[2] for gr in groups]
    r = np.random.default_rng(2)
    dobs_np = [f32(1e-3 * r.standard_normal((97, batch.nrec[s]))) for s in range(batch.nsim)]
    dobs = dev(np.concatenate([d.ravel() for d in dobs_np]))
    v = dev(np.concatenate(models))
    side = torch.cuda.Stream()
    outs = []
    try:
        for ov, graphs in ((False, False), (True, False), (True, True)):
            F.fwi_set_overlap(ov)
            F.fwi_graphs_enable(graphs)
            ws = F.alloc_workspace(batch, time)
            for _ in range(2 if graphs else 1):  # capture, then replay
                outs.append(_run(F, batch, time, v, dobs, kappa, ws, stream=side if graphs else None))
            del ws
    finally:
        F.fwi_set_overlap(False)
        F.fwi_graphs_enable(False)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    _, omis, ogr = oracle_batch_gradient(batch, dt, 97, 1, models, dobs_np, 2.0, kappa)
    gg = split_model(outs[0][2].astype(np.float64), batch)
    for k in range(batch.nsample):
        e = rel(gg[k], ogr[k])
        say("  sample %d gradient rel %.2e" % (k, e))
        assert e < TOL


# (ckpt_every, keep_tail, overlap): segments of 6 under a kept tail of 20 (77 = 12 x 6 + 5;
# the ring inside the tail's levels), a tail that leaves one checkpointed step, every step
# kept, an interval longer than the checkpointed part, a tail shorter than the ring (its own
# levels), and a kept tail beside the overlapped recomputation (two rings of their own)
TAIL_SCHEDULES = [(6, 0, False), (6, 20, False), (6, 96, False), (6, 97, False), (50, 60, False),
                  (10, 5, False), (4, 31, True)]


@pytest.mark.parametrize("ndim", [2, 3])
def test_kept_tail_schedules_are_bitwise_checkpointed(F, ndim):
    """A forward that also keeps the imaging operands of the last steps, so the adjoint
    recomputes only the checkpointed part, gives the keep-all schedule's results bit for
    bit (one adjoint step per launch, so every schedule adds the per-sample products in
    the same order), and the default two-step 2D adjoint matches the oracle."""
    say("case kept-tail schedules %dD" % ndim)
    batch, groups, models, dt = _overlap_problem(F, ndim)
    kappa = [gr[2] for gr in groups]
    r = np.random.default_rng(2)
    dobs_np = [f32(1e-3 * r.standard_normal((97, batch.nrec[s]))) for s in range(batch.nsim)]
    dobs = dev(np.concatenate([d.ravel() for d in dobs_np]))
    v = dev(np.concatenate(models))
    ref = None
    try:
        F.fwi_set_time_blocking(0, 1)
        for K, T, ov in [(0, 0, False)] + TAIL_SCHEDULES:
            F.fwi_set_overlap(ov)
            time = F.time_axis(dt, 97, 1, K, T)
            ws = F.alloc_workspace(batch, time)
            out = _run(F, batch, time, v, dobs, kappa, ws)
            F.fwi_poll_status(ws)
            del ws
            if ref is None:
                ref = out
                continue
            say("  K=%d T=%d overlap=%d: identical" % (K, T, ov))
            for a, b in zip(ref, out):
                assert np.array_equal(a, b), (K, T, ov)
    finally:
        F.fwi_set_overlap(False)
        F.fwi_set_time_blocking(0, 0)
    _, omis, ogr = oracle_batch_gradient(batch, dt, 97, 1, models, dobs_np, 2.0, kappa)
    for K, T, ov in TAIL_SCHEDULES[1:3]:  # default time blocking: two-step 2D adjoint launches
        time = F.time_axis(dt, 97, 1, K, T)
        ws = F.alloc_workspace(batch, time)
        _, mis, gr = _run(F, batch, time, v, dobs, kappa, ws)
        del ws
        gg = split_model(gr.astype(np.float64), batch)
        for k in range(batch.nsample):
            e = rel(gg[k], ogr[k])
            say("  K=%d T=%d sample %d gradient rel %.2e" % (K, T, k, e))
            assert e < TOL
        assert np.allclose(mis, omis, rtol=TOL, atol=0)


@pytest.mark.parametrize("ckpt", [0, 6])
def test_graph_replays_equal_eager(F, ckpt):
    say("case graph replays ckpt=%d" % ckpt)
    side = torch.cuda.Stream()
    batch, _, time, models = _edge_batch(F, 1, ckpt)
    nd = batch.data_size(time.nt // 2)
    r = np.random.default_rng(0)
    v = dev(np.concatenate(models))
    dobs = dev(1e-4 * r.standard_normal(nd))
    ws = F.alloc_workspace(batch, time)
    outs_eager = []
    for seed in (1, 2, 3):
        b, groups, _, _ = _edge_batch(F, seed, ckpt)
        outs_eager.append(_run(F, b, time, v, dobs, [g[2] for g in groups], ws))
    F.fwi_graphs_enable(True)
    try:
        c0, r0 = F.fwi_graphs_stats()
        for rep in range(2):
            for i, seed in enumerate((1, 2, 3)):
                b, groups, _, _ = _edge_batch(F, seed, ckpt)
                with torch.cuda.stream(side):
                    out = _run(F, b, time, v, dobs, [g[2] * (1.0 + 0.0 * rep) for g in groups], ws, stream=side)
                # unrelated eager work between replays
                junk = torch.randn(1 << 20, device="cuda").sum()
                torch.cuda.synchronize()
                for a, e in zip(out, outs_eager[i]):
                    assert np.array_equal(a, e), (rep, seed)
        c1, r1 = F.fwi_graphs_stats()
        say("  captures %d replays %d" % (c1 - c0, r1 - r0))
        assert c1 - c0 == 1 and r1 - r0 == 5
    finally:
        F.fwi_graphs_enable(False)


@pytest.mark.parametrize("ndim", [2, 3])
def test_results_identical_for_every_tile_height(F, ndim):
    say("case tile heights %dD" % ndim)
    if ndim == 2:
        # odd nt: with two time steps per launch the last forward and the first adjoint
        # step run alone, at the forced tile height
        batch, groups, time, models = _edge_batch(F, 4, 0, 123, R=3)
        cands = [8, 16, 32]
    else:
        g = F.Grid(nz=40, ny=13, nx=70, dz=20.0, dy=20.0, dx=20.0, nb=4, v_ref=3000.0, v_max=3300.0, ndim=3)
        rec = np.array([(1 * 13 + y) * 70 + x for y in range(0, 13, 3) for x in range(0, 70, 5)], dtype=np.int32)
        batch = F.Batch([g], [0, 0], [([(1 * 13 + 6) * 70 + 30], [1.0]), ([(20 * 13 + 2) * 70 + 3], [-1.0])],
                        [rec, rec], W.ricker(8.0, 2e-3, 80))
        time = F.time_axis(2e-3, 80, 1, 0)
        models = [f32(np.random.default_rng(1).uniform(1800, 3000, g.nphys))]
        groups = [(None, None, 1.0)]
        cands = [16, 24, 32, 40]
    nd = batch.data_size(time.nt // time.rec_every)
    v = dev(np.concatenate(models))
    dobs = dev(1e-4 * np.random.default_rng(2).standard_normal(nd))
    ws = F.alloc_workspace(batch, time)
    # 2D: with one time step per launch every step runs at the forced tile height; with
    # two the results must not depend on it either
    for blocking in (((1, 1), (2, 2)) if ndim == 2 else ((1, 1),)):
        outs = []
        try:
            F.fwi_set_time_blocking(*blocking)
            for bz in cands:
                F.fwi_set_tile(ndim, bz)
                outs.append(_run(F, batch, time, v, dobs, [g[2] for g in groups], ws))
        finally:
            F.fwi_set_tile(ndim, 0)
            F.fwi_set_time_blocking(0, 0)
        for o in outs[1:]:
            for a, b in zip(o, outs[0]):
                assert np.array_equal(a, b)


def test_tuner_and_cache(F, tmp_path):
    say("case tuner")
    batch, groups, time, models = _edge_batch(F, 7, 0, 120)
    v = dev(np.concatenate(models))
    ws = F.alloc_workspace(batch, time)
    path = str(tmp_path / "tune.json")
    bz, adj, ms = F.fwi_tune(batch, time, v, ws, path)
    say("  tuned bz %d, adjoint steps per launch %d, %.4f ms per gradient step" % (bz, adj, ms))
    assert bz in ((8, 16, 32) if batch.grids[0].ndim == 2 else (16, 32)) and ms > 0
    assert adj in (1, 2)  # 2D keep-all: both adjoints are candidates
    lines = open(path).read().strip().splitlines()
    assert len(lines) == 1 and '"bz": %d' % bz in lines[0] and '"adj_steps": %d' % adj in lines[0]
    bz2, adj2, ms2 = F.fwi_tune(batch, time, v, ws, path)  # read back, no new line
    assert bz2 == bz and adj2 == adj and abs(ms2 - ms) < 1e-5
    assert len(open(path).read().strip().splitlines()) == 1
    # the tuned choice is used and the result is still the oracle's
    nd = batch.data_size(time.nt // 2)
    dobs = f32(1e-4 * np.random.default_rng(3).standard_normal(nd))
    dp, mis, gr = _run(F, batch, time, v, dev(dobs), [g[2] for g in groups], ws)
    _, omis, ogr = oracle_batch_gradient(batch, time.dt, time.nt, 2, models,
                                         split_data(dobs, batch, time.nt // 2), 2.0, [g[2] for g in groups])
    for k, gk in enumerate(split_model(gr.astype(np.float64), batch)):
        assert rel(gk, ogr[k]) < TOL
