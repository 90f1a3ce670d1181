#!/usr/bin/env python3
"""Benchmark: encoded-shot FWI gradient + Langevin update on one MI355X.

Default workload (one "step" = one Langevin refinement of every posterior sample): 3D
200 x 200 x 100 grid at 25 m (220 x 220 x 120 with the 10-cell sponge), 64 surface shots
of a 4 Hz Ricker wavelet on an 8 x 8 lattice and 2500 receivers, 1500 steps of 2 ms; 8
posterior samples, each drawing 4 supergathers of 16 shots with +-1 polarity per step (32
simulations in one launch per time step), with the checkpoint interval and kept tail that
fwi_schedule picks for the free memory.  Per step: draw
encodings (host), encode observed data, forward + misfit + adjoint-state gradient,
Langevin update.  Inputs are seeded synthetic (dipping layers with a salt body, smoothed
start, 1 % Gaussian noise) and resident in HBM before the timed region.  The 2D encoded
workload (400 x 150, 16 samples x 10 supergathers) follows as an extra record.

Prints one JSON line.  Metric: physical cell-steps of the complete forward + adjoint
gradient per second (Gcell-steps/s).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

PEAK_HBM_GBS = 8000.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fwi_kernels.hip", "fwi_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2512_12797_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """Host core count and CPU model (for the CPU baseline's record)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": model}


def cpu_baseline(batch, grid, wav, nt_sample, R, vstart, cfg):
    """Time the oracle (as it stands) on one posterior sample's supergathers for nt_sample
    internal steps: a bounded sample of the workload, reported as a rate."""
    import oracle
    sims = [s for s in range(batch.nsim) if batch.sample_of[s] == 0]
    og = oracle.Grid(nz=grid.nz, nx=grid.nx, dz=grid.dz, dx=grid.dx, nb=grid.nb, v_ref=grid.v_ref, ny=grid.ny,
                     dy=grid.dy, ndim=grid.ndim)
    sp = np.zeros(len(sims) + 1, dtype=np.int32)
    rp = np.zeros(len(sims) + 1, dtype=np.int32)
    sc, sw, rc = [], [], []
    for i, s in enumerate(sims):
        a, b = batch.src_ptr[s], batch.src_ptr[s + 1]
        sc.extend(batch.src_cell[a:b]); sw.extend(batch.src_w[a:b])
        sp[i + 1] = sp[i] + (b - a)
        a, b = batch.rec_ptr[s], batch.rec_ptr[s + 1]
        rc.extend(batch.rec_cell[a:b])
        rp[i + 1] = rp[i] + (b - a)
    r = np.random.default_rng(99)
    dobs = [r.standard_normal((nt_sample // R, rp[i + 1] - rp[i])) for i in range(len(sims))]
    host = host_cpu()
    # the oracle runs its simulations in parallel (OpenMP, one thread per simulation)
    threads = min(len(sims), int(os.environ.get("OMP_NUM_THREADS", host["nproc"] or 1)), host["nproc"] or 1)
    t0 = time.perf_counter()
    oracle.gradient_batch([og] * len(sims), [vstart.ravel()] * len(sims), cfg.dt, nt_sample, R, sp,
                          np.array(sc, dtype=np.int32), np.array(sw, dtype=np.float64), wav[:nt_sample].astype(np.float64),
                          rp, np.array(rc, dtype=np.int32), dobs, 1.0)
    dt = time.perf_counter() - t0
    cells = len(sims) * grid.nphys * nt_sample
    return {"value": cells / dt / 1e9, "unit": "Gcell-steps/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle gradient (forward + misfit + adjoint + imaging) of one posterior sample's "
                      "%d supergathers over the first %d of the %d internal steps (physical cell-steps over wall "
                      "time, a bounded sample of the workload), one OpenMP thread per supergather; %.1f s wall"
                      % (len(sims), nt_sample, cfg.nt, dt),
            "host": host}


_COPY_GBS = []


def copy_probe(torch, fwi, dev):
    """Achievable streaming bandwidth on this GPU: the library's copy kernel over 1 GiB."""
    if _COPY_GBS:
        return _COPY_GBS[0]
    n4 = 1 << 28  # floats per buffer (1 GiB)
    a = torch.empty(n4, device=dev)
    b = torch.empty(n4, device=dev)
    fwi.fwi_copy_probe(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        fwi.fwi_copy_probe(a, b)
    e1.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * 4 * n4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    _COPY_GBS.append(gbs)
    return gbs


def gradient_bench(torch, fwi, problems, args, cfg, steps, warmup, with_cpu):
    """Encoded-shot gradient + Langevin update of every posterior sample of `cfg`, timed
    over `steps` refinement steps after `warmup`; returns the bench record."""
    dev = torch.device("cuda:0")
    nt = args.nt or cfg.nt
    R = cfg.rec_every
    nt_rec = nt // R
    grid = problems.grid_of(cfg)
    wav = W.ricker(cfg.freq, cfg.dt, nt)
    if cfg.ndim == 2:
        vtrue = W.thrust_2d(cfg.nz, cfg.nx, seed=args.seed)
        vstart = np.clip(W.smooth(vtrue, 16.0), cfg.vmin, cfg.vmax)
    else:
        vtrue = W.layered_salt_3d(cfg.nz, cfg.ny, cfg.nx, seed=args.seed, vmin=cfg.vmin, vmax=cfg.vmax)
        vstart = np.clip(W.smooth(vtrue, 8.0), cfg.vmin, cfg.vmax)
    shots = problems.shot_cells(cfg, grid)

    # ---- observed data: forward of the true model, one simulation per shot (setup)
    t_setup = time.perf_counter()
    obs_batch = problems.single_shot_batch(cfg, grid, shots, wav)
    tf = fwi.time_axis(cfg.dt, nt, R, -1)
    ws_obs = fwi.alloc_workspace(obs_batch, tf)
    d_shots = torch.empty(cfg.nshot, nt_rec, len(problems.receiver_cells(cfg, grid)), device=dev)
    fwi.fwi_forward(obs_batch, tf, torch.tensor(vtrue.ravel(), dtype=torch.float32, device=dev), d_shots, ws_obs)
    fwi.fwi_poll_status(ws_obs)
    del ws_obs
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    rms = float(d_shots.pow(2).mean().sqrt())
    sigma = 0.01 * rms
    d_shots += sigma * torch.randn(d_shots.shape, generator=gen, device=dev)
    inv_sigma2 = 1.0 / sigma ** 2

    # ---- the sampler state
    batch0, groups0 = problems.encoded_batch(cfg, [grid] * cfg.nsample, wav, args.seed, 0)
    v = torch.tensor(np.tile(vstart.ravel(), cfg.nsample), dtype=torch.float32, device=dev)
    nsim = batch0.nsim
    d_enc = torch.empty(nsim, nt_rec, d_shots.shape[2], device=dev)
    grad = torch.empty(batch0.model_size, device=dev)
    gnorm = torch.empty(cfg.nsample, device=dev)
    misfit = torch.empty(nsim, dtype=torch.float64, device=dev)

    fwi.fwi_set_overlap(bool(args.overlap))
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if args.ckpt == "auto":
        # the schedule with the fewest forward steps whose workspace fits: every imaging
        # operand kept, else checkpoints plus as long a kept tail as the memory holds
        time_ax = fwi.fwi_schedule(batch0, fwi.time_axis(cfg.dt, nt, R), free - (8 << 30))
    else:
        time_ax = fwi.time_axis(cfg.dt, nt, R, int(args.ckpt), int(args.keep_tail))
    ckpt, tail = time_ax.ckpt_every, time_ax.keep_tail
    ws = fwi.alloc_workspace(batch0, time_ax)
    log("[%s] setup %.1f s; workspace %.1f GB (ckpt_every=%d, keep_tail=%d); free %.1f of %.1f GB" % (
        cfg.name, time.perf_counter() - t_setup, ws.numel() / 1e9, ckpt, tail, free / 1e9, total / 1e9))

    fwi.fwi_set_tile_width(args.tile_width)
    tuned = None
    if args.tile:
        fwi.fwi_set_tile(cfg.ndim, args.tile)
        tuned = (args.tile, 0, float("nan"))
        log("tile height forced to %d" % args.tile)
    elif args.tune:
        cache = os.environ.get("FWI_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "fwi_tune_cache.json"))
        tuned = fwi.fwi_tune(batch0, time_ax, v, ws, cache)
        log("tuner: tile height %d, adjoint steps per launch %d, %.3f ms per gradient time step" % tuned)
    fwi.fwi_set_time_blocking(args.fwd_steps, args.adj_steps)
    stream = torch.cuda.Stream()  # graphs need a non-default stream
    prev_stream = torch.cuda.current_stream()
    torch.cuda.set_stream(stream)
    fwi.fwi_graphs_enable(bool(args.graphs))
    eta = [1e-3]
    v_lo, v_hi = cfg.vmin * 0.9, cfg.vmax * 1.1

    def step(t):
        batch, groups = problems.encoded_batch(cfg, [grid] * cfg.nsample, wav, args.seed, t)
        ptr, shot, w = problems.encode_tables(groups, cfg.shots_per_group)
        gp = torch.from_numpy(ptr).to(dev, non_blocking=True)
        gs = torch.from_numpy(shot).to(dev, non_blocking=True)
        gw = torch.from_numpy(w).to(dev, non_blocking=True)
        fwi.fwi_encode(d_shots, gp, gs, gw, d_enc)
        kappa = [g[2] for g in groups]
        fwi.fwi_gradient(batch, time_ax, v, d_enc, inv_sigma2, kappa, None, misfit, grad, gnorm, ws)
        fwi.fwi_langevin(batch.model_off, v, grad, None, args.seed, t, eta[0], math.sqrt(2 * eta[0]), v_lo, v_hi)

    for t in range(warmup):
        step(t)
        if t == 0:
            gmax = float(grad.abs().max())
            eta[0] = 10.0 / gmax if gmax > 0 else 1e-3  # ~10 m/s per refinement step
    fwi.fwi_poll_status(ws)
    torch.cuda.synchronize()

    # kernel durations: HIP events around every step launch of the timed region when the
    # launches are direct; graph replays cannot be timed per kernel, so with graphs the same
    # step is repeated once, untimed, with direct launches and events
    fwi.fwi_timing_read(0, True)
    fwi.fwi_timing_read(1, True)
    fwi.fwi_timing_enable(not args.graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup, warmup + steps):
        step(t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fwi.fwi_timing_enable(False)
    fwi.fwi_poll_status(ws)
    elapsed = t1 - t0
    gstats = fwi.fwi_graphs_stats()
    if args.graphs:
        fwi.fwi_graphs_enable(False)
        fwi.fwi_timing_enable(True)
        step(warmup + steps)
        torch.cuda.synchronize()
        fwi.fwi_timing_enable(False)
    fwd_ms, fwd_n = fwi.fwi_timing_read(0, True)
    adj_ms, adj_n = fwi.fwi_timing_read(1, True)
    torch.cuda.set_stream(prev_stream)

    ny_pad = cfg.ny + 2 * cfg.nb if cfg.ndim == 3 else 1
    phys_cells = nsim * cfg.nz * cfg.ny * cfg.nx
    pad_cells = nsim * (cfg.nz + 2 * cfg.nb) * ny_pad * (cfg.nx + 2 * cfg.nb)
    samp_cells = cfg.nsample * (cfg.nz + 2 * cfg.nb) * ny_pad * (cfg.nx + 2 * cfg.nb)
    cell_steps = phys_cells * nt * steps
    value = cell_steps / elapsed / 1e9
    log("[%s] step %.1f ms; %.1f Gcell-steps/s physical, %.1f padded; fwd kernel %.1f us x %d, adj kernel %.1f us "
        "x %d" % (cfg.name, 1e3 * elapsed / steps, value, pad_cells * nt * steps / elapsed / 1e9,
                  1e3 * fwd_ms / max(fwd_n, 1), fwd_n, 1e3 * adj_ms / max(adj_n, 1), adj_n))
    # two time steps per launch: the 2D keep-all schedule with an even step count (every
    # launch of the timed sweep is then a two-step launch)
    blk = cfg.ndim == 2 and ckpt == 0 and nt % 2 == 0
    adj_eff = args.adj_steps or (tuned[1] if tuned is not None and tuned[1] else 2)
    two_fwd = blk and args.fwd_steps == 2
    two_adj = blk and adj_eff == 2
    width = fwi.fwi_tile_shape(batch0, time_ax)[1] if cfg.ndim == 3 else None

    # ---- roofline of the dominant kernel (algorithmic bytes per launch / live duration)
    # forward step: u^n, u^{n-1} read and u^{n+1} written = 12 B per simulation cell, plus
    # c once per sample cell; W^n written where the imaging operand is kept or recomputed
    # (+4 B), the pair u^{n+1}, u^n where a checkpoint is taken (+8 B).  Launch counts per
    # gradient: keep-all: nt imaging launches; checkpoints every K over the first head =
    # nt - T steps with the last T kept: first pass head - (nseg - 1) plain, nseg - 1
    # checkpoint and T imaging launches, then head imaging launches (recomputation)
    if ckpt == 0:
        modes = {"plain": 0, "checkpoint": 0, "imaging": nt}
    else:
        head = nt - tail
        kk = min(ckpt, max(head, 1))
        nseg = (head + kk - 1) // kk
        nck = max(nseg - 1, 0)
        modes = {"plain": head - nck, "checkpoint": nck, "imaging": tail + head}
    n_fwd_launch = sum(modes.values())
    fwd_bytes = (pad_cells * (12 * n_fwd_launch + 8 * modes["checkpoint"] + 4 * modes["imaging"]) / n_fwd_launch
                 + samp_cells * 4)
    # adjoint + imaging: lt^{k+1}, lt^{k+2}, W^{k-1} read and lt^k written per simulation
    # cell; c read and the FP64 per-sample accumulator read + written per sample cell
    adj_bytes = pad_cells * 16 + samp_cells * 20
    if cfg.ndim == 2:
        adj_name = "adjoint+imaging step (k_adj2d<bzg>, per-sample imaging)"
        fwd_name = "forward step (k_fwd2d<bz>)"
        # per launch of two steps: u^{n-1}, u^n read, u^{n+1}, u^{n+2}, W^n, W^{n+1} written
        # (24 B per simulation cell), c read once; adjoint: lt^{k+2}, lt^{k+1}, W^{k-1},
        # W^{k-2} read, lt^k, lt^{k-1} written (24 B), c and the accumulator once (20 B)
        if two_fwd:
            fwd_bytes = pad_cells * 24 + samp_cells * 4
            fwd_name = "two-step forward (k_fwd2d2<16>)"
        if two_adj:
            adj_bytes = pad_cells * 24 + samp_cells * 20
            adj_name = "two-step adjoint+imaging (k_adj2d2<16>, per-sample imaging)"
    else:
        adj_name = "adjoint+imaging step (k_adj3d<%d,16>, per-sample imaging)" % width
        fwd_name = "forward step (k_fwd3d<%d,bz>)" % width
    if adj_ms >= fwd_ms:
        name, nbytes, ms, n = adj_name, adj_bytes, adj_ms, adj_n
    else:
        name, nbytes, ms, n = fwd_name, fwd_bytes, fwd_ms, fwd_n
    avg_s = ms / max(n, 1) / 1e3
    achieved = nbytes / avg_s / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_%s.json" % ("2d" if cfg.ndim == 2 else "3d"))
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            # counters are valid for the measured kernel sources, kernel and tile height only
            two = two_adj if name == adj_name else two_fwd
            rows = 16 if two else (tuned[0] if tuned is not None else None)
            # a record may hold counters for several tile heights (the tuner's pick varies)
            ent = tj.get("by_tile_rows", {}).get(str(rows), tj if tj.get("tile_rows") == rows else None)
            if (tj.get("kernel_source") == kernel_source_hash() and tj.get("kernel") == name
                    and rows is not None and ent is not None):
                traffic = ent.get("bytes_per_launch")
                pm = ent.get("per_mode")
                if pm and name == fwd_name:  # forward: weighted by this schedule's launches
                    traffic = int(round(1e6 * sum(modes[m] * (pm[m]["fetch_mb"] + pm[m]["write_mb"])
                                                  for m in modes) / n_fwd_launch))
        except (ValueError, OSError):
            traffic = None
    copy_gbs = copy_probe(torch, fwi, dev)

    if cfg.ndim == 3:
        wl = ("3d-200x200x100-salt-64shot-s16: 8 samples x 4 supergathers (+-1) of 16 shots, %d steps of 2 ms, "
              "gradient + Langevin" % nt)
    else:
        wl = ("2d-400x150-thrust-80shot-s8: 16 samples x 10 supergathers (+-1) of 8 shots, %d steps of 1 ms, "
              "gradient + Langevin" % nt)
    res = {
        "metric": "Gcell-steps/s fwd+adjoint FWI gradient",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(1e3 * elapsed / steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl,
                   "grid": [cfg.nz, cfg.ny, cfg.nx] if cfg.ndim == 3 else [cfg.nz, cfg.nx],
                   "padded": [cfg.nz + 2 * cfg.nb, ny_pad, cfg.nx + 2 * cfg.nb] if cfg.ndim == 3 else
                             [cfg.nz + 2 * cfg.nb, cfg.nx + 2 * cfg.nb],
                   "nsim": nsim, "nsample": cfg.nsample, "internal_steps": nt, "recorded": nt_rec,
                   "schedule": "all imaging operands kept" if ckpt == 0 else
                               "checkpoint every %d, last %d steps kept" % (ckpt, tail),
                   "forward_launches": modes,
                   "tile_rows": tuned[0] if tuned else None, "tile_width": width, "graphs": bool(args.graphs),
                   "time_steps_per_launch": {"forward": 2 if two_fwd else 1, "adjoint": 2 if two_adj else 1},
                   "graph_captures_replays": list(gstats),
                   "padded_gcell_steps_per_s": round(pad_cells * nt * steps / elapsed / 1e9, 3),
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(round(nbytes)), "avg_launch_us": round(avg_s * 1e6, 2), "launches": n,
                     "copy_probe_GBs": round(copy_gbs, 1)},
    }
    # all step kernels of one gradient together (forward and adjoint sweeps): their
    # algorithmic bytes over their summed live durations, and the share of the step's wall
    # time they take
    k_s = (fwd_ms + adj_ms) / 1e3
    if k_s > 0 and fwd_n and adj_n:
        all_gbs = (fwd_bytes * fwd_n + adj_bytes * adj_n) / k_s / 1e9
        res["roofline_step_kernels"] = {
            "bound": "hbm", "achieved": round(all_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(all_gbs / PEAK_HBM_GBS, 4), "of_copy_probe": round(all_gbs / copy_gbs, 3),
            "kernel_ms_per_gradient": round(1e3 * k_s, 2), "share_of_step": round(k_s / (elapsed / steps), 4),
            "forward_avg_us": round(1e3 * fwd_ms / max(fwd_n, 1), 2),
            "adjoint_avg_us": round(1e3 * adj_ms / max(adj_n, 1), 2)}
    del ws
    torch.cuda.empty_cache()
    if with_cpu:
        log("cpu baseline ...")
        # the oracle keeps every wavefield of a simulation in host memory: the 3D sample is a
        # short window of steps (5.8 M cells x 8 B per step and simulation)
        cpu_nt = args.cpu_steps or (nt if cfg.ndim == 2 else 60)
        res["cpu_baseline"] = cpu_baseline(batch0, grid, wav, min(cpu_nt, nt), R, vstart, cfg)
    return res


def uneven_bench(torch, fwi, problems, args):
    """The uneven batch in one launch per time step: 32 samples round-robin over 256x128,
    512x200 and 800x200 grids (10 m, 20-cell sponge), salt models, one supergather of 8
    shots per sample, 2000 steps of 1 ms, checkpoints every 10 steps; the encoded gradient
    of every sample timed over `steps` calls after `warmup`."""
    dev = torch.device("cuda:0")
    cfg = W.C3
    nt = args.nt or cfg.nt
    sizes = list(W.C3_SIZES)
    grids = [fwi.Grid(nz=sizes[k % 3][0], nx=sizes[k % 3][1], dz=cfg.h, dx=cfg.h, nb=cfg.nb, v_ref=cfg.vmax,
                      v_max=cfg.vmax * 1.1) for k in range(cfg.nsample)]
    wav = W.ricker(cfg.freq, cfg.dt, nt)
    nshot_of = lambda g: max(cfg.shots_per_group, g.nx // 16)  # noqa: E731
    truth = [W.salt_2d(g.nz, g.nx, seed=args.seed + k).ravel() for k, g in enumerate(grids)]
    start = [W.smooth(m.reshape(g.nz, g.nx), 10.0).ravel() for m, g in zip(truth, grids)]
    batch, groups = problems.encoded_batch(cfg, grids, wav, seed=args.seed, step=0, s=cfg.shots_per_group, G=1,
                                           nshot_of=nshot_of)
    ckpt = 10 if args.ckpt == "auto" else int(args.ckpt)
    time_ax = fwi.time_axis(cfg.dt, nt, 1, ckpt)
    # observed data: the library's forward of the true models (setup)
    tf = fwi.time_axis(cfg.dt, nt, 1, -1)
    ws = fwi.alloc_workspace(batch, tf)
    dobs = torch.empty(batch.data_size(nt), device=dev)
    fwi.fwi_forward(batch, tf, torch.tensor(np.concatenate(truth), dtype=torch.float32, device=dev), dobs, ws)
    fwi.fwi_poll_status(ws)
    del ws
    fwi.fwi_set_overlap(bool(args.overlap))
    ws = fwi.alloc_workspace(batch, time_ax)
    v = torch.tensor(np.concatenate(start), dtype=torch.float32, device=dev)
    grad = torch.empty(batch.model_size, device=dev)
    mis = torch.empty(batch.nsim, dtype=torch.float64, device=dev)
    kappa = [g[2] for g in groups]
    fwi.fwi_set_time_blocking(args.fwd_steps, args.adj_steps)
    # the library's default tile height unless --tile forces one (the tuner's timing of a
    # lone adjoint step mispredicts this checkpointed batch: it picks one step per adjoint
    # launch, 125 ms per gradient against 118 ms with two)
    if args.tile:
        fwi.fwi_set_tile(2, args.tile)
    bz, wx = fwi.fwi_tile_shape(batch, time_ax)
    stream = torch.cuda.Stream()
    prev_stream = torch.cuda.current_stream()
    torch.cuda.set_stream(stream)
    fwi.fwi_graphs_enable(bool(args.graphs))
    for _ in range(args.warmup):
        fwi.fwi_gradient(batch, time_ax, v, dobs, 1.0, kappa, None, mis, grad, None, ws)
    fwi.fwi_poll_status(ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwi.fwi_gradient(batch, time_ax, v, dobs, 1.0, kappa, None, mis, grad, None, ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fwi.fwi_graphs_enable(False)
    fwi.fwi_timing_read(0, True)
    fwi.fwi_timing_read(1, True)
    fwi.fwi_timing_enable(True)
    fwi.fwi_gradient(batch, time_ax, v, dobs, 1.0, kappa, None, mis, grad, None, ws)
    torch.cuda.synchronize()
    fwi.fwi_timing_enable(False)
    fwd_ms, fwd_n = fwi.fwi_timing_read(0, True)
    adj_ms, adj_n = fwi.fwi_timing_read(1, True)
    torch.cuda.set_stream(prev_stream)
    pad = sum((g.nz + 2 * g.nb) * (g.nx + 2 * g.nb) for g in grids)   # one simulation per sample
    phys = sum(g.nz * g.nx for g in grids)
    value = phys * nt * args.steps / elapsed / 1e9
    # bytes per launch as in the 2D and 3D lines: forward 14 + 4/K B per simulation cell
    # (first pass and recomputation averaged) + 4 B per sample cell; adjoint 16 + 20 B per
    # launch of one step, 24 + 20 B per launch of two (the timed gradient's launch count
    # tells which)
    fwd_bytes = pad * (14 + 4.0 / ckpt + 4)
    adj_two = adj_n > 0 and 2 * adj_n <= nt
    adj_bytes = pad * ((24 if adj_two else 16) + 20)
    adj_name = ("two-step adjoint+imaging (k_adj2d2<16>, per-sample imaging)" if adj_two else
                "adjoint+imaging step (k_adj2d<bzg>, per-sample imaging)")
    fwd_us, adj_us = 1e3 * fwd_ms / max(fwd_n, 1), 1e3 * adj_ms / max(adj_n, 1)
    if adj_ms >= fwd_ms:
        name, nbytes, us, n = adj_name, adj_bytes, adj_us, adj_n
    else:
        name, nbytes, us, n = "forward step (k_fwd2d<bz>)", fwd_bytes, fwd_us, fwd_n
    achieved = nbytes / (us / 1e6) / 1e9
    log("[uneven] %.1f ms per gradient; %.1f Gcell-steps/s physical; fwd %.1f us x %d, adj %.1f us x %d" % (
        1e3 * elapsed / args.steps, value, fwd_us, fwd_n, adj_us, adj_n))
    return {"metric": "Gcell-steps/s fwd+adjoint FWI gradient", "value": round(value, 3), "unit": "Gcell-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(1e3 * elapsed / args.steps, 2), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "2d-uneven-256x128/512x200/800x200-salt: 32 samples x 1 supergather of 8 shots, "
                                   "%d steps of 1 ms, gradient only, one launch per time step over all grids" % nt,
                       "nsim": batch.nsim, "schedule": "checkpoint every %d" % ckpt, "tile_rows": bz,
                       "graphs": bool(args.graphs), "padded_cells": pad, "parallelism": "1 GPU"},
            "roofline": {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                         "bytes_per_launch": int(round(nbytes)), "avg_launch_us": round(us, 2), "launches": n}}


PEAK_BF16_TFLOPS = 2500.0  # dense MFMA, BF16


def unet_bench(torch, args, b=8, n=256, chans=(32, 64, 128, 256)):
    """The preconditioner's 4-level U-Net on a batch of 256 x 256 inputs: inference (one HIP
    graph replay of the forward pass) and training-step time, and every convolution of the
    forward pass and weight gradient of the backward pass timed on its own against its
    roofline min(BF16 MFMA peak, arithmetic intensity x HBM peak).

    Per-kernel and training-step times are averages over back-to-back launches queued behind
    a GPU-side spin that outlasts the host's enqueueing, so that host launch overhead does
    not enter the device-side events."""
    from paper_2512_12797_amd import nn, precond
    from paper_2512_12797_amd.unet import UNet
    net = UNet(chans=chans, seed=0)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed)
    g = torch.randn(b, n, n, device="cuda", generator=gen)
    v = 1500.0 + 3000.0 * torch.rand(b, n, n, device="cuda", generator=gen)
    x16, res, scale = precond.prepare(g, v)
    tg = torch.randn(b, n, n, device="cuda", generator=gen)
    loss = torch.empty(1, device="cuda")
    work = torch.empty(2 * b * 256, device="cuda")
    rflat = res.reshape(-1)

    # spin length per millisecond (the spin counts the device clock)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.cuda._sleep(1 << 22)
    e1.record()
    torch.cuda.synchronize()
    assert e0.elapsed_time(e1) > 0.05, "the spin kernel did not spin"
    spin_per_ms = (1 << 22) / e0.elapsed_time(e1)

    def gpu_time(fn, reps):
        """Seconds per call of fn, device-side, over reps calls queued behind a spin."""
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        spin_ms = 2.0 * (time.perf_counter() - t0) * 1e3 + 1.0
        for _ in range(4):
            torch.cuda._sleep(int(spin_per_ms * spin_ms))
            e0.record()
            h0 = time.perf_counter()
            for _ in range(reps):
                fn()
            host_ms = (time.perf_counter() - h0) * 1e3
            e1.record()
            torch.cuda.synchronize()
            if host_ms < spin_ms:
                return e0.elapsed_time(e1) / 1e3 / reps
            spin_ms = 2.0 * host_ms + 1.0  # the host was slower than planned (e.g. under a profiler)
        raise RuntimeError("host enqueueing kept outlasting the spin")

    def train_step():
        out = net.forward(x16, rflat, b, n, n, keep=True)
        dp = torch.empty_like(out)
        dp16 = nn.bf16_empty(*out.shape)
        nn.rel_mse(out, 32, tg, b, n * n, loss, dp, dp16, work)
        net.backward(dp, dp16)
        net.adam_step(1e-4)

    # inference: the forward pass captured once as a HIP graph; every replay must reproduce
    # the eager result bit for bit
    ref = net.forward(x16, rflat, b, n, n).clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        net.forward(x16, rflat, b, n, n)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out_g = net.forward(x16, rflat, b, n, n)
    for _ in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_g, ref), "graph replay differs from the eager forward pass"
        net.forward(x16, rflat, b, n, n)
    reps = max(args.steps, 20)
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / 1e3 / reps
    t_inf_eager = gpu_time(lambda: net.forward(x16, rflat, b, n, n), 5)
    del graph

    # per-kernel: record the calls of one forward pass and one training step, then time each
    convs, wgrads = [], []
    orig = {k: getattr(nn, k) for k in ("conv3x3", "conv3x3_upcat", "wgrad", "wgrad_upcat")}

    def recorder(name, into):
        def rec(*a, **k):
            into.append((orig[name], a, k))
            orig[name](*a, **k)
        return rec

    # (call, shape, cout, keyword arguments) of every convolution and weight gradient
    for k in ("conv3x3", "conv3x3_upcat"):
        setattr(nn, k, recorder(k, convs))
    try:
        net.forward(x16, rflat, b, n, n)
    finally:
        for k in ("conv3x3", "conv3x3_upcat"):
            setattr(nn, k, orig[k])
    for k in ("wgrad", "wgrad_upcat"):
        setattr(nn, k, recorder(k, wgrads))
    try:
        train_step()
    finally:
        for k in ("wgrad", "wgrad_upcat"):
            setattr(nn, k, orig[k])
    torch.cuda.synchronize()
    t_train = gpu_time(train_step, max(args.steps, 5))

    def row(kind, h, w, cin, cout, fl, by, sec):
        ai = fl / by
        roof = min(PEAK_BF16_TFLOPS, ai * PEAK_HBM_GBS / 1e3)
        ach = fl / sec / 1e12
        return {"kernel": kind, "hw": [h, w], "cin": cin, "cout": cout, "us": round(sec * 1e6, 1),
                "tflops": round(ach, 1), "flop_per_byte": round(ai, 1),
                "bound": "mfma" if roof >= PEAK_BF16_TFLOPS else "hbm", "roof_tflops": round(roof, 1),
                "frac": round(ach / roof, 3)}

    rows, tot_fl, tot_s = [], 0.0, 0.0
    for fn, a, k in convs:
        shape, cout = (a[1], a[3]) if fn is orig["conv3x3"] else (a[3], a[5])
        nb_, h, w, cin = shape
        sec = gpu_time(lambda: fn(*a, **k), 10)
        fl = 2.0 * 9 * cin * cout * nb_ * h * w
        ca = 0 if fn is orig["conv3x3"] else a[1]  # channels read at half resolution
        by = nb_ * h * w * (2 * (cin - ca) + 2 * ca / 4.0
                            + cout * (4 * (k.get("out_f32") is not None) + 2 * (k.get("out_bf16") is not None)
                                      + 4 * (k.get("aux") is not None))
                            + 4 * (k.get("res") is not None)) + 2 * 9 * cin * cout
        rows.append(row("conv3x3 forward" + ("" if fn is orig["conv3x3"] else " [up2(a), b]"), h, w, cin, cout, fl,
                        by, sec))
        tot_fl += fl
        tot_s += sec
    wrows = []
    for fn, a, k in wgrads:
        shape, cout, db = (a[3], a[4], a[6]) if fn is orig["wgrad"] else (a[5], a[6], a[8])
        nb_, h, w, cin = shape
        sec = gpu_time(lambda: fn(*a), 10)
        fl = 2.0 * 9 * cin * cout * nb_ * h * w
        ca = 0 if fn is orig["wgrad"] else a[3]
        by = nb_ * h * w * (2 * (cin - ca) + 2 * ca / 4.0 + 2 * cout + 4 * cout * (db is not None)) + 4 * 9 * cin * cout
        wrows.append(row("weight gradient" + ("" if fn is orig["wgrad"] else " [up2(a), b]"), h, w, cin, cout, fl, by,
                         sec))
    # levels of net.layers(): encoder levels 0..L-1, decoder levels 0..L-2 (two convolutions
    # each), then the output convolution at level 0
    lv = [i for i in range(net.L) for _ in (0, 1)] + [i for i in range(net.L - 1) for _ in (0, 1)] + [0]
    real = sum(2.0 * 9 * (2 if l is net.enc[0][0] else l.cin) * l.cout_real * b * (n >> k) ** 2
               for k, l in zip(lv, net.layers()))
    return {"metric": "U-Net preconditioner inference throughput", "value": round(real / t_inf / 1e12, 2),
            "unit": "TFLOP/s", "n_gpus": 1, "higher_is_better": True, "dtype": "bf16 (fp32 accumulate)",
            "data": "synthetic", "config": {"workload": "unet-4level-32/64/128/256-256x256-batch%d" % b,
                                            "params": net.nparams(), "real_gflop_per_image": round(real / b / 1e9, 2)},
            "inference_ms": round(t_inf * 1e3, 3), "inference_eager_ms": round(t_inf_eager * 1e3, 3),
            "train_step_ms": round(t_train * 1e3, 3), "train_tflops": round(3.0 * real / t_train / 1e12, 2),
            "roofline": {"bound": "mixed", "achieved": round(tot_fl / tot_s / 1e12, 1),
                         "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tot_fl / tot_s / 1e12 / PEAK_BF16_TFLOPS, 4),
                         "note": "all forward convolutions, executed FLOPs / summed kernel time; per-layer bounds below"},
            "layers": rows, "weight_gradients": wrows}


def daps_bench(torch, args):
    """Diffusion-prior posterior sampling (the decoupled diffusion inference) against the
    prior-free encoded chains, on the 2D encoded workload: 16 samples from the smoothed
    start, the same number of encoded-gradient evaluations per sample for every sampler.
    Each sampler runs with the stochastic Langevin refinement and with the deterministic
    Adam guidance of the paper's experiments (the calibration ablation).  The predict-x0
    network is trained here on seeded procedural thrust models (not the test model's
    seed).  Reported per sampler: posterior-mean RMSE, mean sample RMSE, the mean
    posterior standard deviation and the share of cells whose error lies within two of
    them."""
    from paper_2512_12797_amd import chains, daps
    sv = chains.Survey(seed=args.seed, log=log)
    cfg = sv.cfg
    nsample = 16
    v0 = torch.tensor(np.tile(sv.vstart.ravel(), nsample), dtype=torch.float32, device=sv.dev).view(nsample, -1)
    eta = args.daps_max_update / float(sv.full_gradient(v0[:1], 1).abs().max())
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    t0 = time.perf_counter()
    models = daps.procedural_models(cfg, args.daps_models, seed0=20000)
    log("prior training set: %d models in %.1f s" % (args.daps_models, time.perf_counter() - t0))
    sched = daps.Schedule()
    den = daps.Denoiser(cfg.nz, cfg.nx, cfg.nz + chains.PAD_ROWS, lo, hi, seed=0)
    t1 = time.perf_counter()
    hist = den.train(models, sched, args.daps_tstart, steps=args.daps_train, log=log)
    t_train = time.perf_counter() - t1
    del models
    held = daps.procedural_models(cfg, 16, seed0=30000)
    ts = sorted({1, max(1, args.daps_tstart // 4), max(1, args.daps_tstart // 2), args.daps_tstart})
    ev = den.evaluate(held, sched, ts)
    for t, noise, err in ev:
        log("prior: level %d, noise %.1f m/s, clean-model estimate RMSE %.1f m/s" % (t, noise, err))
    vt = torch.tensor(sv.vtrue.ravel(), dtype=torch.float64, device=sv.dev)

    def stats(v, wall):
        return posterior_stats(v, vt, wall, nsample, cfg.nz)

    runs = {}
    ngrad = None
    for guide in ("langevin", "adam"):
        v, r_d, wall, ngrad = daps.sample(sv, den, sched, args.daps_tstart, args.daps_k, eta, args.seed, nsample,
                                          every=args.daps_every, renoise=args.daps_renoise, guide=guide,
                                          adam_lr=args.daps_lr, nu=None if guide == "langevin" else args.daps_adam_nu)
        runs["daps_" + guide] = dict(stats(v, wall), rmse_per_level_sampled=[
            [args.daps_tstart - i, round(r_d[i], 2)] for i in range(0, len(r_d), max(1, len(r_d) // 10))])
        log("daps, %s guidance: %s" % (guide, runs["daps_" + guide]))
    # the prior alone (no refinement): the spread the data have to narrow
    v, _, wall, _ = daps.sample(sv, den, sched, args.daps_tstart, 0, eta, args.seed, nsample,
                                every=args.daps_every, renoise=args.daps_renoise)
    runs["daps_prior_only"] = stats(v, wall)
    log("daps, prior only: %s" % runs["daps_prior_only"])
    for guide in ("langevin", "adam"):
        t2 = time.perf_counter()
        r_e, s_e, _, v = chains.run_chain(sv, "encoded", ngrad, eta, args.seed, nsample=nsample,
                                          nu=None if guide == "langevin" else args.daps_adam_nu,
                                          adam_lr=args.daps_lr if guide == "adam" else None, keep_samples=True)
        runs["encoded_" + guide] = dict(stats(v, time.perf_counter() - t2), s_per_step=round(s_e, 4))
        log("encoded chain, %s guidance: %s" % (guide, runs["encoded_" + guide]))
    start_rmse = float(np.sqrt(np.mean((sv.vstart - sv.vtrue) ** 2)))
    return {"metric": "posterior-mean RMSE after the same encoded-gradient evaluations", "unit": "m/s",
            "value": runs["daps_langevin"]["posterior_mean_rmse_mps"],
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "dtype": "f32 (network bf16)",
            "workload": "2d-400x150-thrust-80shot: 16 samples from a start smoothed by %g cells; encoded gradients "
                        "(10 supergathers of 8); Langevin eta=%.3e (largest first update %g m/s), nu=sqrt(2 eta); "
                        "Adam rate %g m/s, nu=%g" % (sv.start_sigma, eta, args.daps_max_update, args.daps_lr,
                                                      args.daps_adam_nu),
            "start_rmse_mps": round(start_rmse, 2), "gradient_evaluations_per_sample": ngrad,
            "daps": {"levels": args.daps_tstart, "steps_per_guided_level": args.daps_k, "guide_every": args.daps_every,
                     "renoise": args.daps_renoise, "T": sched.T,
                     "prior": {"models": args.daps_models, "train_steps": args.daps_train,
                               "train_s": round(t_train, 1), "loss_first_last": [hist[0][1], hist[-1][1]],
                               "heldout_level_noise_rmse_mps": [[t, round(n, 1), round(e, 1)] for t, n, e in ev]}},
            "runs": runs}


def posterior_stats(v, vt, wall, nsample, nz):
    """Posterior-mean and mean-sample RMSE, mean posterior standard deviation and the share
    of cells whose posterior-mean error is within two standard deviations (metrics of a
    batch of samples v, device [nsample, ncell], against the truth vt, f64), and the
    standard deviation and posterior-mean error by depth third (nz rows; the surface
    acquisition illuminates the shallow third best)."""
    vd = v.double()
    mean, std = vd.mean(0), vd.std(0)
    err = (mean - vt).abs()
    thirds = [(0, nz // 3), (nz // 3, 2 * nz // 3), (2 * nz // 3, nz)]
    sd2, er2 = std.view(nz, -1), err.view(nz, -1)
    return {"posterior_mean_rmse_mps": round(float((mean - vt).pow(2).mean().sqrt()), 2),
            "mean_sample_rmse_mps": round(float((vd - vt).pow(2).mean(1).sqrt().mean()), 2),
            "mean_posterior_std_mps": round(float(std.mean()), 2),
            "within_2std": round(float((err <= 2 * std).double().mean()), 3),
            "std_by_depth_third_mps": [round(float(sd2[a:b].mean()), 1) for a, b in thirds],
            "abs_error_by_depth_third_mps": [round(float(er2[a:b].mean()), 1) for a, b in thirds],
            "wall_s": round(wall, 2), "samples_per_hour": round(nsample / wall * 3600, 1)}


def svgd_bench(torch, args):
    """The SVGD baseline on the 2D encoded workload's survey: 16 particles from the
    smoothed start (each perturbed by 20 m/s of seeded white noise), RBF kernel with the
    median bandwidth, step set so that the largest first move is 300 m/s, or an Adam
    ascent along the Stein direction at --daps-lr m/s; with full-shot gradients (the
    paper's baseline) and with the encoded estimate."""
    from paper_2512_12797_amd import chains, svgd
    sv = chains.Survey(seed=args.seed, log=log)
    vt = torch.tensor(sv.vtrue.ravel(), dtype=torch.float64, device=sv.dev)
    runs = {}
    for kind, steps in (("full", args.svgd_full_steps), ("encoded", args.svgd_enc_steps)):
        for step_rule in ("", "_adam"):
            x, r, wall = svgd.run(sv, steps, 300.0, args.seed, gradient=kind,
                                  adam_lr=args.daps_lr if step_rule else None)
            name = "svgd_" + kind + step_rule
            runs[name] = dict(posterior_stats(x, vt, wall, 16, sv.cfg.nz), steps=steps,
                              s_per_step=round(wall / steps, 4),
                              rmse_sampled=[[i + 1, round(r[i], 2)] for i in range(0, len(r), max(1, len(r) // 10))])
            log("%s, %d steps: %s" % (name, steps, runs[name]))
    start_rmse = float(np.sqrt(np.mean((sv.vstart - sv.vtrue) ** 2)))
    return {"metric": "posterior-mean RMSE", "unit": "m/s", "value": runs["svgd_full"]["posterior_mean_rmse_mps"],
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "dtype": "f32",
            "workload": "2d-400x150-thrust-80shot: SVGD, 16 particles from a start smoothed by %g cells (+20 m/s "
                        "seeded white noise each), RBF kernel, median bandwidth, largest first move 300 m/s "
                        "(_adam runs: Adam ascent along the Stein direction at %g m/s)" % (sv.start_sigma, args.daps_lr),
            "start_rmse_mps": round(start_rmse, 2), "runs": runs}


def precond_bench(torch, args, nmodels=2500, enc_per_model=4, steps=20000, lr=1e-3, G=1):
    """The learned preconditioner at the pair configuration's full scale: about 10k pairs
    (2500 seeded thrust / salt models on 256 x 256 patches at 10 m, 32 surface shots of a
    10 Hz Ricker over 1500 steps, 4 encoded supergathers of 8 shots per model) generated by
    the library, split 90 / 10 by model, the network trained on the first part and scored
    on the held-out part: relative L2 error to the full-shot gradient of the plain encoded
    gradient, of the network's estimate and of the guarded result."""
    from paper_2512_12797_amd import precond
    from paper_2512_12797_amd.unet import UNet
    cfg = precond.PairConfig(G=G)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = precond.make_pairs(cfg, nmodels, enc_per_model, seed=args.seed, models_per_batch=6,
                               with_coverage=bool(args.pc_coverage),
                               log=lambda m: log(m) if ("%d models" % nmodels in m or m.count("00 models")) else None)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    npairs = int(pairs["scale"].shape[0])
    npad = cfg.n + 2 * cfg.nb
    cell_steps = float(pairs["solves"]) * npad * npad * cfg.nt
    mid = pairs["model_id"].numpy()
    held = mid >= int(round(0.9 * nmodels))
    val = ~held & (mid >= int(round(0.8 * nmodels)))   # fits the guard's blend weight
    train_idx = np.nonzero(~held & ~val)[0]
    val_idx = torch.from_numpy(np.nonzero(val)[0]).to("cuda")
    test_idx = torch.from_numpy(np.nonzero(held)[0]).to("cuda")
    net = UNet(seed=args.seed)
    t1 = time.perf_counter()
    hist = precond.train(net, pairs, train_idx, steps=steps, batch=8, lr=lr, lr_final=lr / 10, seed=args.seed,
                         log=lambda m: log(m) if m.startswith("validation") or (
                             m.startswith("train step") and int(m.split()[2]) % 2000 == 0) else None,
                         val_idx=val_idx, val_every=args.pc_val_every)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    x, res, tg = pairs["x16"][test_idx], pairs["res"][test_idx], pairs["target"][test_idx]
    plain = precond.rel_err(res, tg)
    out = precond.predict(net, x, res)
    netw = precond.rel_err(precond.channel0(out), tg)
    vres, vtg = pairs["res"][val_idx], pairs["target"][val_idx]
    alpha = precond.fit_blend(precond.channel0(precond.predict(net, pairs["x16"][val_idx], vres)), vres, vtg)
    guarded, keep = precond.guard(out, torch.ones(x.shape[0], device="cuda"), res, alpha=alpha)
    guard_err = precond.rel_err(guarded, tg)
    unblended, _ = precond.guard(out, torch.ones(x.shape[0], device="cuda"), res)
    unblended_err = precond.rel_err(unblended, tg)
    # the same scores on 1000 training pairs: under- or over-fitting
    tr = torch.from_numpy(np.random.default_rng(args.seed).choice(train_idx, size=min(1000, len(train_idx)),
                                                                  replace=False)).to("cuda")
    tr_plain = precond.rel_err(pairs["res"][tr], pairs["target"][tr])
    tr_net = precond.rel_err(precond.channel0(precond.predict(net, pairs["x16"][tr], pairs["res"][tr])),
                             pairs["target"][tr])
    return {"metric": "held-out relative L2 error to the full-shot gradient (plain encoded -> preconditioned)",
            "value": round(float(netw.mean()), 4), "unit": "relative L2", "higher_is_better": False, "n_gpus": 1,
            "dtype": "f32 solver, bf16 network (fp32 accumulate)", "data": "synthetic",
            "config": {"workload": "precond-256x256-10m-32shot-s8-1500steps", "models": nmodels,
                       "pairs": npairs, "train_pairs": int(len(train_idx)), "heldout_pairs": int(test_idx.numel()),
                       "supergathers": G, "shots_per_supergather": cfg.s, "kappa": cfg.kappa,
                       "train_steps": steps, "batch": 8, "lr": lr},
            "plain_encoded_error": round(float(plain.mean()), 4), "network_error": round(float(netw.mean()), 4),
            "guarded_error": round(float(guard_err.mean()), 4), "guard_kept": round(float(keep.float().mean()), 3),
            "guard_blend_alpha": round(alpha, 4), "guarded_error_alpha1": round(float(unblended_err.mean()), 4),
            "early_stop_step": net.val_best, "validation_error_by_step": [[s_, round(e_, 4)] for s_, e_ in net.val_hist],
            "heldout_guarded_worse_fraction": round(float(np.mean(guard_err > plain)), 3),
            "validation_pairs": int(val_idx.numel()),
            "median_plain_network_guarded": [round(float(np.median(x)), 4) for x in (plain, netw, guard_err)],
            "heldout_improved_fraction": round(float(np.mean(netw < plain)), 3),
            "train_subset_plain_network": [round(float(tr_plain.mean()), 4), round(float(tr_net.mean()), 4)],
            "shot_coverage_channel": bool(args.pc_coverage),
            "final_train_loss": round(hist[-1][1], 5),
            "pair_generation_s": round(t_pairs, 1), "pairs_per_s": round(npairs / t_pairs, 1),
            "pair_generation_padded_gcell_steps_per_s": round(cell_steps / t_pairs / 1e9, 1),
            "training_s": round(t_train, 1), "training_samples_per_s": round(steps * 8 / t_train, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nt", type=int, default=0, help="override internal steps (profiling runs only)")
    ap.add_argument("--ckpt", default="auto", help="auto | 0 (keep all imaging operands) | K (checkpoint)")
    ap.add_argument("--keep-tail", type=int, default=0, help="with --ckpt K: imaging operands of the last steps kept")
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graphs", type=int, default=1, help="replay each gradient as a captured HIP graph")
    ap.add_argument("--tune", type=int, default=1, help="pick the tile height with the library's tuner")
    ap.add_argument("--tile", type=int, default=0, help="force this tile height (rows per tile); 0: tuner or heuristic")
    ap.add_argument("--overlap", type=int, default=0, help="checkpoints: recompute beside the adjoint (0/1)")
    ap.add_argument("--tile-width", type=int, default=0, choices=[0, 32, 64],
                    help="3D tile width in cells (0: the library's choice by idle lanes)")
    ap.add_argument("--fwd-steps", type=int, default=0, choices=[0, 1, 2],
                    help="2D keep-all schedule: time steps per forward launch (0: automatic, 1)")
    ap.add_argument("--adj-steps", type=int, default=0, choices=[0, 1, 2],
                    help="2D keep-all schedule: time steps per adjoint launch (0: the tuner's choice, else 2)")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle steps for the CPU baseline (0: all)")
    ap.add_argument("--no-extra", action="store_true", help="3d: skip the 2D workload's extra record")
    ap.add_argument("--workload", default="3d",
                    choices=["2d", "3d", "uneven", "equal-error", "unet", "precond", "daps", "svgd"],
                    help="3d: 200x200x100, 32 simulations (the reported line; the 2D workload follows as an extra "
                         "record); 2d: 400x150, 160 simulations; uneven: 32 samples on 256x128 / 512x200 / 800x200 "
                         "grids in one launch per step (checkpoints every 10); "
                         "equal-error: posterior samples/hour of plain, encoded and preconditioned chains at equal "
                         "posterior-mean RMSE (several minutes); unet: the gradient preconditioner's network "
                         "(inference, training step, per-layer convolution rooflines); precond: ~10k solver-made "
                         "training pairs at 256^2, training, held-out error against the plain encoded gradient "
                         "(about 10 minutes)")
    ap.add_argument("--ee-forms", default="plain,encoded,preconditioned",
                    help="equal-error: chains to run (comma-separated; the target depends on the start only)")
    ap.add_argument("--ee-max-update", type=float, default=100.0,
                    help="equal-error: the largest first plain update (m/s), which sets eta for every form")
    ap.add_argument("--plain-steps", type=int, default=300,
                    help="equal-error: most plain-chain steps (the chain stops at the target: 0.9 x the start RMSE)")
    ap.add_argument("--max-steps", type=int, default=300, help="equal-error: most steps of the encoded chains")
    ap.add_argument("--net-seeds", type=int, default=3, help="equal-error: networks trained (seeds 0..n-1)")
    ap.add_argument("--chain-log", default=None, help="equal-error: directory for each chain's per-step JSONL log")
    ap.add_argument("--pc-models", type=int, default=2500, help="precond: seeded models (4 pairs each)")
    ap.add_argument("--pc-steps", type=int, default=1500,
                    help="precond: training steps (batch 8; the best validation point is kept)")
    ap.add_argument("--pc-lr", type=float, default=3e-4, help="precond: initial Adam learning rate (cosine to 1/10)")
    ap.add_argument("--pc-G", type=int, default=1, help="precond: supergathers of 8 shots summed per encoded gradient")
    ap.add_argument("--pc-coverage", type=int, default=1, help="precond: shot-coverage input channel (0/1)")
    ap.add_argument("--pc-val-every", type=int, default=100,
                    help="precond: training steps between validation scores (early stopping)")
    ap.add_argument("--daps-tstart", type=int, default=20, help="daps: first diffusion level (of T = 1000)")
    ap.add_argument("--daps-k", type=int, default=5, help="daps: Langevin steps per guided level")
    ap.add_argument("--daps-every", type=int, default=1, help="daps: guidance at every this many levels")
    ap.add_argument("--daps-renoise", default="marginal", choices=["posterior", "marginal", "mean"])
    ap.add_argument("--daps-max-update", type=float, default=300.0,
                    help="daps: eta is set so that the largest first update is this many m/s")
    ap.add_argument("--daps-lr", type=float, default=50.0, help="daps: Adam guidance rate, m/s")
    ap.add_argument("--svgd-full-steps", type=int, default=12, help="svgd: steps with full-shot gradients")
    ap.add_argument("--svgd-enc-steps", type=int, default=100, help="svgd: steps with encoded gradients")
    ap.add_argument("--daps-adam-nu", type=float, default=0.0, help="daps: noise weight after an Adam step")
    ap.add_argument("--daps-models", type=int, default=1024, help="daps: procedural models the prior is trained on")
    ap.add_argument("--daps-train", type=int, default=8000, help="daps: denoiser training steps (batch 8)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the workload shards by posterior sample with no exchange "
              "between GPUs, so one GPU's share is the whole measurement; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_12797_amd import fwi, problems

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.workload == "unet":
        print(json.dumps(unet_bench(torch, args)), flush=True)
        return
    if args.workload == "precond":
        print(json.dumps(precond_bench(torch, args, nmodels=args.pc_models, steps=args.pc_steps, lr=args.pc_lr,
                                       G=args.pc_G)), flush=True)
        return
    if args.workload == "daps":
        print(json.dumps(daps_bench(torch, args)), flush=True)
        return
    if args.workload == "svgd":
        print(json.dumps(svgd_bench(torch, args)), flush=True)
        return
    if args.workload == "equal-error":
        from paper_2512_12797_amd import chains
        res = chains.equal_error(seed=args.seed, plain_steps=args.plain_steps, max_steps=args.max_steps,
                                 log_dir=args.chain_log, max_update=args.ee_max_update,
                                 forms=tuple(args.ee_forms.split(",")),
                                 net_seeds=tuple(range(args.net_seeds)), log=log)
        res.update({"n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32"})
        print(json.dumps(res), flush=True)
        return
    if args.workload == "uneven":
        print(json.dumps(uneven_bench(torch, fwi, problems, args)), flush=True)
        return
    cfg = W.C2 if args.workload == "2d" else W.C5
    res = gradient_bench(torch, fwi, problems, args, cfg, args.steps, args.warmup, not args.no_cpu_baseline)
    if args.workload == "3d" and not args.no_extra and not args.nt:
        # the 2D encoded workload as a second record (its own measurement, not the value)
        r2 = gradient_bench(torch, fwi, problems, args, W.C2, min(args.steps, 10), min(args.warmup, 3), False)
        res["extra_workloads"] = {
            r2["config"]["workload"]: {k: r2[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup")} |
            {"roofline": r2["roofline"], "roofline_step_kernels": r2.get("roofline_step_kernels"),
             "config": r2["config"]}}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
