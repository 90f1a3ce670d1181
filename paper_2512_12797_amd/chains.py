"""Posterior samples per hour at equal posterior-model error.

Three gradient estimators drive the same clean-space Langevin refinement (Eqs. 8-9) of
16 posterior samples on the 2D encoded workload (400 x 150 at 20 m, 80 shots):

* plain: the full-shot gradient of Eq. 1 (every shot its own simulation);
* encoded: the Eq. 6 estimate from G = 10 supergathers of s = 8 +-1-encoded shots,
  redrawn every step (what the benchmark times);
* preconditioned: the encoded estimate mapped by the learned U-Net towards the
  full-shot gradient, with the plain-gradient guard.

The target posterior-mean RMSE (m/s against the true model, physical grid) is a fixed
fraction of the starting RMSE (0.9: a 10 % reduction); the plain chain runs until it
reaches it, which sets its step count.  Each form's wall time to the target is its number
of steps times its measured time per step, and samples per hour follow.  The plain form
is timed two ways: as a naive solver (one simulation per launch, samples one after the
other; one sample's full step of 80 single-shot gradient calls timed, times 16 samples)
and batched like the encoded form.
Each chain's trajectory is computed with the batched library (the estimator, not the
launch pattern, decides the trajectory).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

import workloads as W

from . import fwi, nn, precond, problems
from .unet import UNet


class Survey:
    """The 2D encoded workload: grid, acquisition, true and starting models, noisy data."""

    def __init__(self, seed=1000, start_sigma=6.0, device="cuda", log=print):
        self.cfg = cfg = W.C2
        self.dev = device
        self.log = log
        self.grid = problems.grid_of(cfg)
        self.wav = W.ricker(cfg.freq, cfg.dt, cfg.nt)
        self.shots = problems.shot_cells(cfg, self.grid)
        self.rec = problems.receiver_cells(cfg, self.grid)
        self.nrec = len(self.rec)
        self.nt_rec = cfg.nt_rec
        self.vtrue = W.thrust_2d(cfg.nz, cfg.nx, seed=seed)
        # starting model: the truth Gaussian-smoothed by start_sigma cells (120 m by default:
        # from the 320 m smoothing of the throughput benchmark the 6 Hz descent is
        # cycle-skipped and lowers the misfit while moving away from the truth)
        self.start_sigma = start_sigma
        self.vstart = np.clip(W.smooth(self.vtrue, start_sigma), cfg.vmin, cfg.vmax)
        self.t_fwd = fwi.time_axis(cfg.dt, cfg.nt, cfg.rec_every, -1)
        self.t_grad = fwi.time_axis(cfg.dt, cfg.nt, cfg.rec_every, 0)
        self.ws = None
        self.d_shots, self.sigma = self.observed(self.vtrue, seed)

    def workspace(self, batch, t):
        n = fwi.fwi_workspace_size(batch, t)
        if self.ws is None or self.ws.numel() < n:
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = torch.empty(n, dtype=torch.uint8, device=self.dev)
        return self.ws

    def observed(self, vtrue, seed, noise=0.01):
        """Single-shot data of a true model with Gaussian noise at `noise` x clean RMS."""
        b = problems.single_shot_batch(self.cfg, self.grid, self.shots, self.wav)
        d = torch.empty(len(self.shots), self.nt_rec, self.nrec, device=self.dev)
        fwi.fwi_forward(b, self.t_fwd, torch.tensor(vtrue.ravel(), dtype=torch.float32, device=self.dev), d,
                        self.workspace(b, self.t_fwd))
        g = torch.Generator(device=self.dev)
        g.manual_seed(seed)
        sigma = noise * float(d.pow(2).mean().sqrt())
        d += sigma * torch.randn(d.shape, generator=g, device=self.dev)
        return d, sigma

    # ---------------------------------------------------------------- gradients
    def full_gradient(self, v, nsample, d_shots=None, per_launch=2):
        """Full-shot gradient of each sample (device [nsample, nphys]); `per_launch`
        samples (x 80 single-shot simulations) per batched launch sequence."""
        d_shots = self.d_shots if d_shots is None else d_shots
        nphys = self.grid.nphys
        out = torch.empty(nsample, nphys, device=self.dev)
        for k0 in range(0, nsample, per_launch):
            m = min(per_launch, nsample - k0)
            b = problems.single_shot_batch(self.cfg, self.grid, self.shots, self.wav, nsample=m)
            dobs = d_shots.reshape(1, -1).expand(m, -1).reshape(-1).contiguous()
            fwi.fwi_gradient(b, self.t_grad, v[k0:k0 + m].reshape(-1).contiguous(), dobs, 1.0 / self.sigma ** 2,
                             None, None, None, out[k0:k0 + m].reshape(-1), None, self.workspace(b, self.t_grad))
        return out

    def encoded_gradient(self, v, nsample, seed, step, d_shots=None):
        """Eq. 6 estimate from G = 10 supergathers of 8 encoded shots per sample."""
        d_shots = self.d_shots if d_shots is None else d_shots
        cfg = self.cfg
        b, groups = problems.encoded_batch(cfg, [self.grid] * nsample, self.wav, seed, step)
        ptr, shot, w = problems.encode_tables(groups, cfg.shots_per_group)
        d_enc = torch.empty(b.nsim, self.nt_rec, self.nrec, device=self.dev)
        fwi.fwi_encode(d_shots, torch.from_numpy(ptr).to(self.dev), torch.from_numpy(shot).to(self.dev),
                       torch.from_numpy(w).to(self.dev), d_enc)
        out = torch.empty(nsample, self.grid.nphys, device=self.dev)
        fwi.fwi_gradient(b, self.t_grad, v.reshape(-1).contiguous(), d_enc, 1.0 / self.sigma ** 2,
                         [g[2] for g in groups], None, None, out.reshape(-1), None, self.workspace(b, self.t_grad))
        return out


# ------------------------------------------------------------------ network

PAD_ROWS = 2  # 150 rows -> 152, divisible by 2^3 for a 4-level U-Net


def make_pairs(sv: Survey, ntruth=32, fractions=(0.0, 0.35, 0.7), nenc=2, seed0=50000):
    """Training pairs at the workload's geometry: for seeded thrust models (not the test
    model), models between a smoothed start and the truth, their encoded gradients
    (input) and full-shot gradients (target), both scaled by the encoded gradient's RMS."""
    cfg = sv.cfg
    nf, hp = len(fractions), cfg.nz + PAD_ROWS
    xs, rs, tgs = [], [], []
    t0 = time.perf_counter()
    for i in range(ntruth):
        truth = W.thrust_2d(cfg.nz, cfg.nx, seed=seed0 + i)
        start = np.clip(W.smooth(truth, sv.start_sigma), cfg.vmin, cfg.vmax)
        d_i, _ = sv.observed(truth, seed0 + i)
        ms = np.stack([start + f * (truth - start) for f in fractions])
        v = torch.tensor(ms.reshape(nf, -1), dtype=torch.float32, device=sv.dev)
        gfull = sv.full_gradient(v, nf, d_shots=d_i).view(nf, cfg.nz, cfg.nx)
        for e in range(nenc):
            genc = sv.encoded_gradient(v, nf, seed0 + i, 1000 + e, d_shots=d_i).view(nf, cfg.nz, cfg.nx)
            x16, res, scale = precond.prepare(genc, v.view(nf, cfg.nz, cfg.nx), hp)
            xs.append(x16)
            rs.append(res)
            tgs.append(precond.scaled(gfull, scale, hp))
        sv.log("pairs: %d/%d truths, %.1f s" % (i + 1, ntruth, time.perf_counter() - t0))
    return {"x16": torch.cat(xs), "res": torch.cat(rs), "target": torch.cat(tgs)}


def precondition(net, g_enc, v, alpha=1.0):
    """Network estimate of the full-shot gradient, guarded by the plain encoded one and
    blended with it by alpha (fitted on validation pairs)."""
    S, nz, nx = g_enc.shape
    x16, res, scale = precond.prepare(g_enc, v, nz + PAD_ROWS)
    return precond.guard(precond.predict(net, x16, res), scale, g_enc, alpha=alpha)


# -------------------------------------------------------------------- chains

def run_chain(sv: Survey, form, steps, eta, seed, net=None, nsample=16, nu=None, adam_lr=None, keep_samples=False,
              v0=None, step0=0, log_jsonl=None, stop_below=None, elapsed0=0.0, alpha=1.0):
    """Langevin refinement of `nsample` samples from the smoothed start; returns the
    posterior-mean RMSE after each step, the mean wall time per step (direct launches,
    steps after the first: the first carries one-time host costs) and, for the
    preconditioned form, how many samples kept the network's gradient at each step (and
    the samples themselves with keep_samples).  Noise weight nu (default sqrt(2 eta)).
    With adam_lr the encoded gradient drives an Adam step of that rate (m/s) instead of
    -eta g, its moments kept over the chain, followed by the nu-weighted noise and the
    clamp (the guidance of the paper's experiments; nu = 0 makes it deterministic).
    Resume: v0 (device f32 [nsample, nphys]) and step0 continue a chain saved after step0
    steps; the encodings and the noise are counter-based (seed, step, sample), so the
    continuation equals the uninterrupted chain bit for bit (not for the Adam form, whose
    moments are not part of the saved state).  log_jsonl: a file that receives one JSON
    line per step (step, posterior-mean RMSE, mean posterior standard deviation, PDE solves
    per sample so far, seconds since the chain's start: elapsed0, the time a resumed chain
    had already run, plus this call's wall time).  stop_below: end the chain after the first
    step whose posterior-mean RMSE is at or below it."""
    nu = math.sqrt(2 * eta) if nu is None else nu
    if step0 and adam_lr is not None:
        raise ValueError("the Adam form cannot resume: its moments are not saved")
    cfg = sv.cfg
    nz, nx = cfg.nz, cfg.nx
    if v0 is None:
        v = torch.tensor(np.tile(sv.vstart.ravel(), nsample), dtype=torch.float32, device=sv.dev).view(nsample, -1)
    else:
        v = v0.reshape(nsample, -1).clone()
    off = np.arange(nsample + 1, dtype=np.int64) * sv.grid.nphys
    vt = torch.tensor(sv.vtrue.ravel(), dtype=torch.float64, device=sv.dev)
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    rmse, kept = [], []
    if adam_lr is not None:
        m1, m2 = torch.zeros_like(v).reshape(-1), torch.zeros_like(v).reshape(-1)
    torch.cuda.synchronize()
    t0 = t_log = time.perf_counter()  # t0 restarts after the first step (timing), t_log never
    for t in range(steps):
        if t == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        if form == "plain":
            g = sv.full_gradient(v, nsample)
        else:
            g = sv.encoded_gradient(v, nsample, seed, step0 + t)
            if form == "preconditioned":
                g, keep = precondition(net, g.view(nsample, nz, nx), v.view(nsample, nz, nx), alpha)
                g = g.reshape(nsample, -1).contiguous()
                kept.append(int(keep.sum()))
        g = g.reshape(-1).contiguous()
        if adam_lr is not None:
            nn.adam(v.reshape(-1), g, m1, m2, adam_lr, 0.9, 0.999, 1e-8, t + 1)
            fwi.fwi_langevin(off, v.reshape(-1), g, None, seed, t, 0.0, nu, lo, hi)
        else:
            fwi.fwi_langevin(off, v.reshape(-1), g, None, seed, step0 + t, eta, nu, lo, hi)
        rmse.append(float((v.double().mean(0) - vt).pow(2).mean().sqrt()))
        done = stop_below is not None and rmse[-1] <= stop_below
        if log_jsonl:
            # one forward and one adjoint solve per shot (plain) or per supergather (encoded)
            per_step = 2 * len(sv.shots) // (1 if form == "plain" else sv.cfg.shots_per_group)
            with open(log_jsonl, "a") as f:
                f.write(json.dumps({"step": step0 + t, "posterior_mean_rmse_mps": rmse[-1],
                                    "mean_posterior_std_mps": float(v.double().std(0).mean()) if nsample > 1 else 0.0,
                                    "pde_solves_per_sample": (step0 + t + 1) * per_step,
                                    "elapsed_s": elapsed0 + time.perf_counter() - t_log}) + "\n")
        if done:
            break
    torch.cuda.synchronize()
    out = (rmse, (time.perf_counter() - t0) / max(1, len(rmse) - 1), kept)
    return out + (v,) if keep_samples else out


def save_state(path, v, step, seed):
    """Chain state after `step` steps: the samples (device or host f32 [nsample, nphys]),
    the step count and the seed, as an .npz of plain arrays (no pickled objects)."""
    np.savez(path, v=np.ascontiguousarray(v.detach().cpu().numpy() if torch.is_tensor(v) else v, dtype=np.float32),
             step=np.int64(step), seed=np.int64(seed))


def load_state(path, device="cuda"):
    """(samples as device f32 [nsample, nphys], step, seed) saved by save_state."""
    with np.load(path, allow_pickle=False) as z:
        return torch.tensor(z["v"], device=device), int(z["step"]), int(z["seed"])


def time_naive_plain(sv: Survey, v, ncall=None):
    """Seconds per Langevin step of a naive plain solver: every shot of every sample its
    own gradient call (one simulation per launch), one after the other.  Times `ncall`
    calls (default: every shot, one sample's whole step) and scales to all shots of the
    16 samples."""
    ncall = ncall or len(sv.shots)
    cfg = sv.cfg
    calls = []
    for s in range(ncall):
        b = fwi.Batch([sv.grid], [0], [([int(sv.shots[s])], [1.0])], [sv.rec], sv.wav)
        calls.append((b, sv.d_shots[s].reshape(-1).contiguous()))
    ws = torch.empty(fwi.fwi_workspace_size(calls[0][0], sv.t_grad), dtype=torch.uint8, device=sv.dev)
    grad = torch.empty(sv.grid.nphys, device=sv.dev)
    vv = v[0].contiguous()
    fwi.fwi_gradient(calls[0][0], sv.t_grad, vv, calls[0][1], 1.0, None, None, None, grad, None, ws)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, d in calls:
        fwi.fwi_gradient(b, sv.t_grad, vv, d, 1.0, None, None, None, grad, None, ws)
    torch.cuda.synchronize()
    per_call = (time.perf_counter() - t0) / ncall
    return per_call * len(sv.shots) * 16


def first_reaching(rmse, target):
    for i, r in enumerate(rmse):
        if r <= target:
            return i + 1
    return None


def equal_error(seed=1000, plain_steps=300, max_steps=300, ntruth=32, train_steps=1500, max_update=100.0,
                start_sigma=6.0, net_seeds=(0,), target_frac=0.9, log=print, log_dir=None,
                forms=("plain", "encoded", "preconditioned")):
    """The whole comparison; returns a dict (one JSON object).  log_dir: a directory that
    receives each chain's per-step JSONL log (run_chain's log_jsonl).  forms: the chains to
    run (the target depends only on the start, so the forms can also run in separate
    calls and their records be put side by side)."""
    def jl(name):
        return None if log_dir is None else os.path.join(log_dir, "chain_%s.jsonl" % name)

    sv = Survey(seed=seed, start_sigma=start_sigma, log=log)
    nsample = 16
    v0 = torch.tensor(np.tile(sv.vstart.ravel(), nsample), dtype=torch.float32, device=sv.dev).view(nsample, -1)
    g0 = sv.full_gradient(v0[:1], 1)
    eta = max_update / float(g0.abs().max())  # the largest first update, m/s; all forms alike
    log("eta %.3e" % eta)

    start_rmse = float(np.sqrt(np.mean((sv.vstart - sv.vtrue) ** 2)))
    target = target_frac * start_rmse
    out_forms = {}
    if "plain" in forms:
        naive_s = time_naive_plain(sv, v0)
        log("plain, naive solver: %.1f s per step (one sample's 80 calls timed)" % naive_s)
        r_plain, s_plain, _ = run_chain(sv, "plain", plain_steps, eta, seed, stop_below=target, log_jsonl=jl("plain"))
        log("plain: %d steps, %.2f s per step, RMSE %.1f -> %.1f m/s (target %.1f)" % (
            len(r_plain), s_plain, start_rmse, r_plain[-1], target))
    if "encoded" in forms:
        r_enc, s_enc, _ = run_chain(sv, "encoded", max_steps, eta, seed, stop_below=target, log_jsonl=jl("encoded"))
        log("encoded: %.3f s per step, %d steps, RMSE %.1f" % (s_enc, len(r_enc), r_enc[-1]))
    runs = []
    if "preconditioned" not in forms:
        net_seeds = ()

    pairs = make_pairs(sv, ntruth=ntruth) if net_seeds else None
    P = pairs["x16"].shape[0] if net_seeds else 0
    if net_seeds:
        log("pairs: %d in %.1f s" % (P, time.perf_counter() - t0))
    # pairs come truth by truth (P / ntruth each): the last 4 truths validate (early
    # stopping and the guard's blend weight)
    per_truth = P // ntruth
    val_idx = torch.arange((ntruth - 4) * per_truth, P, device=sv.dev)
    train_idx = np.arange((ntruth - 4) * per_truth)
    for ns in net_seeds:
        t1 = time.perf_counter()
        net = UNet(chans=(32, 64, 128, 256), seed=ns)
        hist = precond.train(net, pairs, train_idx, steps=train_steps, batch=8, lr=1e-3, lr_final=1e-4,
                             seed=ns, log=log, val_idx=val_idx, val_every=100)
        vres = pairs["res"][val_idx]
        alpha = precond.fit_blend(precond.channel0(precond.predict(net, pairs["x16"][val_idx], vres)), vres,
                                  pairs["target"][val_idx])
        t_train = time.perf_counter() - t1
        log("network seed %d: validation best after %s steps, blend weight %.3f" % (ns, net.val_best, alpha))
        r_pre, s_pre, kept = run_chain(sv, "preconditioned", max_steps, eta, seed, net=net, stop_below=target,
                                       log_jsonl=jl("preconditioned_%d" % ns), alpha=alpha)
        log("preconditioned (network seed %d): %.3f s per step, reaches the target after %s steps" %
            (ns, s_pre, first_reaching(r_pre, target)))
        runs.append((ns, r_pre, s_pre, kept, t_train, hist, alpha, net.val_best, net.val_hist))
    del pairs

    def entry(rmse, s_step, label):
        n = first_reaching(rmse, target)
        wall = None if n is None else n * s_step
        return {"steps_to_target": n, "s_per_step": round(s_step, 4), "wall_s": None if wall is None else round(wall, 2),
                "samples_per_hour": None if wall is None else round(nsample / wall * 3600, 1), "timing": label,
                "rmse": [round(r, 2) for r in rmse]}

    if "plain" in forms:
        out_forms["plain_naive"] = {**entry(r_plain, naive_s, "one simulation per launch, samples in turn; one "
                                                              "sample's 80 single-shot gradient calls timed, x 16 "
                                                              "samples"), "rmse": None}
        out_forms["plain_batched"] = entry(r_plain, s_plain, "measured: 2 samples x 80 single-shot simulations per "
                                                             "launch")
    if "encoded" in forms:
        out_forms["encoded"] = entry(r_enc, s_enc, "measured: 16 samples x 10 supergathers of 8 in one launch per step")
    if runs:
        out_forms["preconditioned"] = [
            {**entry(r_pre, s_pre, "measured: encoded + U-Net inference + guard"), "network_seed": ns,
             "network_kept_fraction": round(float(np.mean(kept)) / nsample, 3) if kept else None,
             "training_s": round(t_train, 1), "train_loss_first_last": [hist[0][1], hist[-1][1]],
             "blend_alpha": round(alpha, 4), "early_stop_step": vbest,
             "validation_error_by_step": [[s_, round(e_, 4)] for s_, e_ in vhist]}
            for ns, r_pre, s_pre, kept, t_train, hist, alpha, vbest, vhist in runs]
    return {
        "metric": "posterior samples/hour at equal posterior-mean RMSE", "unit": "samples/hour",
        "workload": "2d-400x150-thrust-80shot: 16 samples from a start smoothed by %g cells, Langevin eta=%.3e "
                    "(largest first update %g m/s), nu=sqrt(2 eta)" % (start_sigma, eta, max_update),
        "target_rmse_mps": round(target, 2), "start_rmse_mps": round(start_rmse, 2), "target_fraction": target_frac,
        "plain_steps": len(r_plain) if "plain" in forms else None,
        "forms": out_forms,
    }
