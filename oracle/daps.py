"""FP64 oracle of the diffusion outer loop around the Langevin refinement -- TEST
INFRASTRUCTURE (the import rule of this package applies).

Sec. 2, "Diffusion prior and reverse parameterization" and "Decoupled diffusion inference
with encoded shots data":
  * a variance schedule beta_t (t = 1..T) with alpha_t = prod_{s<=t} (1 - beta_s) and
    alpha_0 = 1; the forward diffusion q(x_t | x_0) = N(sqrt(alpha_t) x_0, (1 - alpha_t) I);
  * the re-noise step (Eq. 10): x_{t-1} ~ N(mu~_t(x_t, x_0), beta~_t I), with the DDPM
    posterior variance (Eq. 11) and mean (Eq. 12);
  * models normalised to [-1, 1] for the network; physical units for the likelihood.
The noise of a draw is the counter-based stream of ``normals_key`` with tag DAPS_TAG
(counter words a = step, b = image).
"""
from __future__ import annotations

import numpy as np

from . import normals_key

DAPS_TAG = 0x44415053


def linear_schedule(T, beta_1, beta_T):
    """(beta, alpha), arrays of length T + 1: beta_t linear from beta_1 to beta_T (beta_0 =
    0 unused), alpha_t = prod_{s<=t} (1 - beta_s), alpha_0 = 1."""
    beta = np.zeros(T + 1)
    beta[1:] = np.linspace(beta_1, beta_T, T)
    alpha = np.cumprod(1.0 - beta)
    return beta, alpha


def posterior(beta, alpha, t):
    """(c_x0, c_xt, beta_tilde) of q(x_{t-1} | x_t, x_0) at level t >= 1:
    mu~ = c_x0 x_0 + c_xt x_t (Eq. 12), beta~ (Eq. 11)."""
    bt, at, atm1 = beta[t], alpha[t], alpha[t - 1]
    c_x0 = np.sqrt(atm1) * bt / (1.0 - at)
    c_xt = np.sqrt(1.0 - bt) * (1.0 - atm1) / (1.0 - at)
    beta_tilde = (1.0 - atm1) / (1.0 - at) * bt
    return c_x0, c_xt, beta_tilde


def normalise(v, lo, hi):
    """Physical model -> the network's space: 2 (v - lo) / (hi - lo) - 1."""
    return 2.0 * (np.asarray(v, dtype=np.float64) - lo) / (hi - lo) - 1.0


def to_model(p, lo, hi):
    """The network's clean-model estimate -> physical units, clamped to [lo, hi]."""
    return np.clip(lo + (np.asarray(p, dtype=np.float64) + 1.0) / 2.0 * (hi - lo), lo, hi)


def mix(z, x, c0, c1, sig, lo, hi, seed, step):
    """Per image i (rows of the [nimg, n] arrays): c0[i] normalise(z_i) + c1[i] x_i +
    sig[i] xi_i, xi_i the stream (seed, DAPS_TAG, step, i).  z or x may be None."""
    ref = z if z is not None else x
    nimg, n = np.asarray(ref).shape
    out = np.zeros((nimg, n))
    for i in range(nimg):
        y = sig[i] * normals_key(seed, DAPS_TAG, step, i, n) if sig[i] != 0 else np.zeros(n)
        if z is not None:
            y = y + c0[i] * normalise(z[i], lo, hi)
        if x is not None:
            y = y + c1[i] * np.asarray(x[i], dtype=np.float64)
        out[i] = y
    return out


def prep(x, level, hp):
    """Network input channels for normalised models x [nimg, h, w]: (channel 0, channel 1,
    residual), each [nimg, hp, w]; channel 0 = residual = x and channel 1 = level[i] on the
    first h rows, zero below (the GPU stores the two channels in BF16)."""
    x = np.asarray(x, dtype=np.float64)
    nimg, h, w = x.shape
    ch0 = np.zeros((nimg, hp, w))
    ch1 = np.zeros((nimg, hp, w))
    ch0[:, :h] = x
    ch1[:, :h] = np.asarray(level, dtype=np.float64)[:, None, None]
    return ch0, ch1, ch0.copy()
