"""Diffusion-prior posterior sampling around the encoded-gradient Langevin refinement
(Sec. 2, "Diffusion prior and reverse parameterization" and "Decoupled diffusion inference
with encoded shots data"; the proposed-framework table).

For a batch of posterior samples at diffusion level t, from t_start down to 1:
  (i)   predict the clean model x0^ = g(x_t, t) (Eq. 7) with the U-Net, in the
        normalised space (input: x_t and its noise level sqrt(1 - alpha_t); the network's
        output is added to x_t), and map it to m/s (fwi_daps_prep, fwi_daps_model);
  (ii)  take K Langevin steps from it with the encoded-shot gradient (Eq. 6 estimate,
        fwi_gradient + fwi_langevin);
  (iii) re-noise: x_{t-1} ~ N(mu~_t(x_t, z), beta~_t) in the normalised space (Eq. 10,
        fwi_daps_mix); at t = 1 the refined model is the sample.
The chain starts from the last levels: x_{t_start} is the forward diffusion of the
starting model (a warm start instead of pure noise).  Guidance may be injected every few
levels only (the synthetic experiments of Sec. 3 take 5 steps every 5 levels); a level
without it re-noises the network's estimate.  The modified sampler of the proposed-framework
table draws the Langevin noise with its own weight nu (sqrt(2 eta) by default) and makes
the re-noise optional: `renoise` picks the posterior draw (the equation), the draw from
q(x_{t-1} | z) (the table's line), or the posterior mean without noise.  The predict-x0
network is trained here, on the GPU network kernels, on seeded procedural models.  Python
only arranges tensors and scalars and calls the library.
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np
import torch

import workloads as W

from . import fwi, nn
from .unet import IN_CH, UNet

_bound = False


def _lib():
    global _bound
    L = fwi.lib()
    if not _bound:
        for name in ("fwi_daps_mix", "fwi_daps_prep", "fwi_daps_model"):
            getattr(L, name).restype = C.c_int32
        L.fwi_daps_last_error.restype = C.c_char_p
        L.fwi_daps_mix.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_float, C.c_float, C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p]
        L.fwi_daps_prep.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
        L.fwi_daps_model.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_float,
                                     C.c_float, C.c_void_p, C.c_void_p]
        _bound = True
    return L


def _ok(status):
    if status != fwi.FWI_OK:
        raise fwi.FwiError(status, _lib().fwi_daps_last_error().decode())


def fwi_daps_mix(nimg, n, z, x, c0, c1, sig, v_lo, v_hi, seed, step, out, stream=None):
    _ok(_lib().fwi_daps_mix(nimg, n, fwi._ptr(z), fwi._ptr(x), fwi._ptr(c0), fwi._ptr(c1), fwi._ptr(sig), v_lo, v_hi,
                            seed, step, fwi._ptr(out), fwi._stream(stream)))


def fwi_daps_prep(nimg, h, w, hp, x, level, x16, res, stream=None):
    _ok(_lib().fwi_daps_prep(nimg, h, w, hp, fwi._ptr(x), fwi._ptr(level), fwi._ptr(x16), fwi._ptr(res),
                             fwi._stream(stream)))


def fwi_daps_model(nimg, h, w, hp, c, pred, v_lo, v_hi, v, stream=None):
    _ok(_lib().fwi_daps_model(nimg, h, w, hp, c, fwi._ptr(pred), v_lo, v_hi, fwi._ptr(v), fwi._stream(stream)))


# ------------------------------------------------------------------ schedule

class Schedule:
    """Linear variance schedule beta_1 .. beta_T; alpha_t = prod_{s<=t} (1 - beta_s), alpha_0 = 1
    (host scalars: the per-level coefficients of the kernels)."""

    def __init__(self, T=1000, beta_1=1e-4, beta_T=0.02):
        self.T = T
        self.beta = [0.0] + [beta_1 + (beta_T - beta_1) * (t - 1) / (T - 1) for t in range(1, T + 1)]
        self.alpha = [1.0]
        for t in range(1, T + 1):
            self.alpha.append(self.alpha[-1] * (1.0 - self.beta[t]))

    def level(self, t):
        """Noise standard deviation of q(x_t | x_0): sqrt(1 - alpha_t)."""
        return math.sqrt(1.0 - self.alpha[t])

    def forward(self, t):
        """(c0, c1, sig) of the forward diffusion x_t = sqrt(alpha_t) x_0 + sqrt(1 - alpha_t) xi."""
        return math.sqrt(self.alpha[t]), 0.0, self.level(t)

    def posterior(self, t):
        """(c0, c1, sig) of the re-noise draw from q(x_{t-1} | x_t, x_0)."""
        bt, at, atm1 = self.beta[t], self.alpha[t], self.alpha[t - 1]
        c0 = math.sqrt(atm1) * bt / (1.0 - at)
        c1 = math.sqrt(1.0 - bt) * (1.0 - atm1) / (1.0 - at)
        return c0, c1, math.sqrt((1.0 - atm1) / (1.0 - at) * bt)


def _coefs(vals, n, device):
    """Per-image coefficient arrays (device f32 [n] x 3) from one (c0, c1, sig) or a list."""
    if isinstance(vals, tuple):
        vals = [vals] * n
    a = torch.tensor(vals, dtype=torch.float32).t().contiguous().to(device)
    return a[0].contiguous(), a[1].contiguous(), a[2].contiguous()


# -------------------------------------------------------------------- network

class Denoiser:
    """The predict-x0 network on models of h x w cells (rows padded to hp for the U-Net)."""

    def __init__(self, h, w, hp, v_lo, v_hi, seed=0, device="cuda"):
        self.h, self.w, self.hp = h, w, hp
        self.v_lo, self.v_hi = v_lo, v_hi
        self.dev = device
        self.net = UNet(chans=(32, 64, 128, 256), seed=seed, device=device, in_used=2)  # model, noise level

    def inputs(self, x, level):
        """x: normalised models (device f32 [S, h, w]); level: device f32 [S]."""
        S = x.shape[0]
        x16 = nn.bf16_empty(S, self.hp, self.w, IN_CH, device=self.dev)
        res = torch.empty(S, self.hp, self.w, device=self.dev)
        fwi_daps_prep(S, self.h, self.w, self.hp, x.contiguous(), level.contiguous(), x16, res)
        return x16, res

    def predict(self, x, level, batch=8):
        """Clean-model estimates in m/s (device f32 [S, h, w]) of normalised noisy models x."""
        S = x.shape[0]
        v = torch.empty(S, self.h, self.w, device=self.dev)
        for i in range(0, S, batch):
            b = min(batch, S - i)
            x16, res = self.inputs(x[i:i + b], level[i:i + b])
            out = self.net.forward(x16, res.reshape(-1).contiguous(), b, self.hp, self.w)
            fwi_daps_model(b, self.h, self.w, self.hp, out.shape[-1], out, self.v_lo, self.v_hi, v[i:i + b])
        return v

    def train(self, models, sched, t_max, steps=3000, batch=8, lr=5e-4, lr_final=5e-5, seed=0, log=None):
        """Adam on the relative squared error of the clean-model estimate: for a random batch
        of models (device f32 [N, h, w], m/s) and random levels t in 1..t_max, x_t is their
        forward diffusion and the target their normalised clean version.  Returns losses."""
        r = np.random.default_rng(seed)
        N = models.shape[0]
        hw = self.h * self.w
        loss = torch.empty(1, device=self.dev)
        work = torch.empty(2 * batch * 256, device=self.dev)
        ones, zeros = _coefs((1.0, 0.0, 0.0), batch, self.dev)[0], torch.zeros(batch, device=self.dev)
        xt = torch.empty(batch, self.h, self.w, device=self.dev)
        x0 = torch.empty(batch, self.h, self.w, device=self.dev)
        hist = []
        t0 = time.perf_counter()
        for it in range(steps):
            idx = torch.from_numpy(r.choice(N, size=batch, replace=False)).to(self.dev)
            zb = models[idx].reshape(batch, hw).contiguous()
            ts = r.integers(1, t_max + 1, size=batch)
            c0, c1, sig = _coefs([sched.forward(int(t)) for t in ts], batch, self.dev)
            fwi_daps_mix(batch, hw, zb, None, c0, c1, sig, self.v_lo, self.v_hi, seed, it, xt)
            fwi_daps_mix(batch, hw, zb, None, ones, zeros, zeros, self.v_lo, self.v_hi, seed, it, x0)
            x16, res = self.inputs(xt, sig)
            _, target = self.inputs(x0, zeros)
            out = self.net.forward(x16, res.reshape(-1).contiguous(), batch, self.hp, self.w, keep=True)
            dp = torch.empty_like(out)
            dp16 = nn.bf16_empty(*out.shape, device=self.dev)
            nn.rel_mse(out, out.shape[-1], target, batch, self.hp * self.w, loss, dp, dp16, work)
            self.net.backward(dp, dp16)
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * it / max(1, steps - 1)))
            self.net.adam_step(cur)
            if it % 100 == 0 or it == steps - 1:
                hist.append((it, float(loss.item())))
                if log and (it % 1000 == 0 or it == steps - 1):
                    log("denoiser step %d loss %.4f (%.1f s)" % (it, hist[-1][1], time.perf_counter() - t0))
        return hist

    def evaluate(self, models, sched, ts, seed=1):
        """RMSE (m/s) of the clean-model estimate from the forward diffusion of `models`
        (device f32 [N, h, w], m/s) at each level in ts, with the noise level itself."""
        N = models.shape[0]
        hw = self.h * self.w
        z = models.reshape(N, hw).contiguous()
        xt = torch.empty(N, hw, device=self.dev)
        out = []
        for t in ts:
            c0, c1, sig = _coefs(sched.forward(int(t)), N, self.dev)
            fwi_daps_mix(N, hw, z, None, c0, c1, sig, self.v_lo, self.v_hi, seed, int(t), xt)
            v = self.predict(xt.view(N, self.h, self.w), sig)
            err = float((v.double().reshape(N, hw) - z.double()).pow(2).mean().sqrt())
            out.append((int(t), sched.level(int(t)) * 0.5 * (self.v_hi - self.v_lo), err))
        return out


def procedural_models(cfg, n, seed0, device="cuda"):
    """n seeded thrust models at the workload's grid (device f32 [n, nz, nx], m/s)."""
    return torch.tensor(np.stack([W.thrust_2d(cfg.nz, cfg.nx, seed=seed0 + i) for i in range(n)]),
                        dtype=torch.float32, device=device)


# -------------------------------------------------------------------- sampler

RENOISE = ("posterior", "marginal", "mean")


GUIDE = ("langevin", "adam")


def sample(sv, den: Denoiser, sched: Schedule, t_start, K, eta, seed, nsample=16, every=1, nu=None,
           renoise="posterior", guide="langevin", adam_lr=50.0, langevin_bounds=None):
    """Decoupled diffusion inference of `nsample` posterior samples on the Survey `sv`
    (chains.Survey: geometry, observed data, starting model): K refinement steps at levels
    t_start, t_start - every, ...; re-noise mode one of RENOISE.  guide "langevin":
    z <- clamp(z - eta g + nu xi), nu default sqrt(2 eta); guide "adam": an Adam step of
    rate adam_lr (m/s) on the encoded gradient, moments restarted at each guided level,
    then z <- clamp(z + nu xi), nu default 0 (the deterministic guidance of the paper's
    experiments).  Returns (samples, device f32 [nsample, nphys]; posterior-mean RMSE
    after each level; wall seconds; gradient evaluations per sample)."""
    if renoise not in RENOISE or guide not in GUIDE or every < 1 or K < 0:
        raise ValueError("renoise must be one of %s, guide one of %s, every >= 1, K >= 0" % (RENOISE, GUIDE))
    if nu is None:
        nu = math.sqrt(2 * eta) if guide == "langevin" else 0.0
    cfg = sv.cfg
    nz, nx = cfg.nz, cfg.nx
    nphys = sv.grid.nphys
    dev = sv.dev
    lo, hi = langevin_bounds or (cfg.vmin * 0.9, cfg.vmax * 1.1)
    off = np.arange(nsample + 1, dtype=np.int64) * nphys
    vt = torch.tensor(sv.vtrue.ravel(), dtype=torch.float64, device=dev)
    v0 = torch.tensor(np.tile(sv.vstart.ravel(), nsample), dtype=torch.float32, device=dev).view(nsample, nphys)
    x = torch.empty(nsample, nphys, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # warm start: the starting model diffused to level t_start
    c0, c1, sig = _coefs(sched.forward(t_start), nsample, dev)
    fwi_daps_mix(nsample, nphys, v0, None, c0, c1, sig, den.v_lo, den.v_hi, seed, sched.T + 1, x)
    rmse, step = [], 0
    v = None
    for t in range(t_start, 0, -1):
        level = torch.full((nsample,), sched.level(t), device=dev)
        v = den.predict(x.view(nsample, nz, nx), level).reshape(nsample, nphys).contiguous()   # (i)
        if guide == "adam":
            m1, m2 = torch.zeros(nsample * nphys, device=dev), torch.zeros(nsample * nphys, device=dev)
        for k in range(K if (t_start - t) % every == 0 else 0):                                 # (ii)
            g = sv.encoded_gradient(v, nsample, seed, step).reshape(-1).contiguous()
            if guide == "adam":
                nn.adam(v.reshape(-1), g, m1, m2, adam_lr, 0.9, 0.999, 1e-8, k + 1)
                fwi.fwi_langevin(off, v.reshape(-1), g, None, seed, step, 0.0, nu, lo, hi)
            else:
                fwi.fwi_langevin(off, v.reshape(-1), g, None, seed, step, eta, nu, lo, hi)
            step += 1
        if t > 1:                                                                                 # (iii)
            if renoise == "marginal":
                c0, c1, sig = _coefs(sched.forward(t - 1), nsample, dev)
            else:
                c0, c1, sig = sched.posterior(t)
                c0, c1, sig = _coefs((c0, c1, sig if renoise == "posterior" else 0.0), nsample, dev)
            fwi_daps_mix(nsample, nphys, v, x if renoise != "marginal" else None, c0, c1, sig, den.v_lo, den.v_hi,
                         seed, t, x)
        rmse.append(float((v.double().mean(0) - vt).pow(2).mean().sqrt()))
    torch.cuda.synchronize()
    return v, rmse, time.perf_counter() - t0, step
