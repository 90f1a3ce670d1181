"""FP64 NumPy oracle of the U-Net gradient preconditioner -- TEST INFRASTRUCTURE.

Same architecture as the library's network (encoder levels of two 3x3 conv + SiLU
layers with 2x2 average pooling between them, decoder levels of nearest 2x upsampling,
channel concatenation with the encoder output of that level and two 3x3 conv + SiLU
layers, a 3x3 output conv to one channel plus the input gradient as a residual), with the
loss L = mean_i |pred_i - t_i|^2 / |t_i|^2.

With ``rounding=True`` the values the GPU rounds to BF16 are rounded here too: weights,
activations after SiLU, pooled activations, and the output-side gradients dL/dz used as
matrix operands in the weight and data gradients.  Everything else is FP64.  With
``rounding=False`` the network is plain FP64 (for finite-difference pins).

Weights are given as arrays [cout][9][cin] (tap = 3 ky + kx for offsets ky-1, kx-1) with
the real channel counts (no padding).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest BF16 (ties to even) through FP32; returns FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def conv3x3(x, w, b=None):
    """x [N, H, W, Ci], w [Co, 9, Ci]: zero-padded 3x3 correlation."""
    n, h, wd, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((n, h, wd, w.shape[0]))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        out += xp[:, ky:ky + h, kx:kx + wd, :] @ w[:, tap, :].T
    return out + (0.0 if b is None else b)


def conv3x3_wgrad(dz, x):
    """dW[co, tap, ci] = sum_p dz[p, co] x[p + offset(tap), ci]."""
    n, h, wd, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dzf = dz.reshape(-1, dz.shape[-1])
    dw = np.zeros((dz.shape[-1], 9, ci))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        dw[:, tap, :] = dzf.T @ xp[:, ky:ky + h, kx:kx + wd, :].reshape(-1, ci)
    return dw


def conv3x3_dgrad(dz, w):
    """dx[p, ci] = sum_{tap, co} w[co, tap, ci] dz[p - offset(tap), co]."""
    n, h, wd, co = dz.shape
    dzp = np.pad(dz, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros((n, h, wd, w.shape[2]))
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        dx += dzp[:, 2 - ky:2 - ky + h, 2 - kx:2 - kx + wd, :] @ w[:, tap, :]
    return dx


def pool2(a):
    n, h, w, c = a.shape
    return a.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def up2(a):
    return a.repeat(2, axis=1).repeat(2, axis=2)


class UNetOracle:
    """weights: list of (w [cout][9][cin], b [cout]) in the order encoder level 0 (a, b),
    ..., encoder level L-1 (a, b), decoder level L-2 (a, b), ..., decoder level 0 (a, b),
    output."""

    def __init__(self, chans, weights, rounding=True):
        self.chans, self.L, self.r = tuple(chans), len(chans), rounding
        R = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
        self.R = R
        self.W = [(R(w), np.asarray(b, dtype=np.float64)) for w, b in weights]

    def _idx(self):
        L = self.L
        enc = [(2 * i, 2 * i + 1) for i in range(L)]
        dec = {}
        k = 2 * L
        for i in range(L - 2, -1, -1):
            dec[i] = (k, k + 1)
            k += 2
        return enc, dec, k

    def forward(self, x, res):
        """x [N, H, W, 2] (input channels), res [N, H, W]: prediction [N, H, W]."""
        R = self.R
        enc, dec, ko = self._idx()
        c = {"x": R(x)}
        cur = c["x"]
        for i in range(self.L):
            if i > 0:
                cur = R(pool2(cur))
                c["pool%d" % i] = cur
            wa, ba = self.W[enc[i][0]]
            za = conv3x3(cur, wa, ba)
            aa = R(silu(za))
            wb, bb = self.W[enc[i][1]]
            zb = conv3x3(aa, wb, bb)
            ab = R(silu(zb))
            c["enc%d" % i] = (cur, za, aa, zb, ab)
            cur = ab
        for i in range(self.L - 2, -1, -1):
            cat = np.concatenate([up2(cur), c["enc%d" % i][4]], axis=-1)
            wa, ba = self.W[dec[i][0]]
            za = conv3x3(cat, wa, ba)
            aa = R(silu(za))
            wb, bb = self.W[dec[i][1]]
            zb = conv3x3(aa, wb, bb)
            ab = R(silu(zb))
            c["dec%d" % i] = (cat, za, aa, zb, ab)
            cur = ab
        wo, bo = self.W[ko]
        out = conv3x3(cur, wo, bo)[..., 0] + res
        c["top"] = cur
        self.cache = c
        return out

    @staticmethod
    def loss(pred, target):
        """Relative squared error averaged over images, and dL/dpred."""
        n = pred.shape[0]
        num = ((pred - target) ** 2).reshape(n, -1).sum(1)
        den = (target ** 2).reshape(n, -1).sum(1)
        L = float(np.mean(num / den))
        d = 2.0 * (pred - target) / (n * den[:, None, None])
        return L, d

    def backward(self, dpred):
        """Gradients [(dW, db)] in the constructor's order."""
        R = self.R
        enc, dec, ko = self._idx()
        c = self.cache
        grads = [None] * len(self.W)

        def layer_bwd(k, x, dz):
            dzr = R(dz)
            grads[k] = (conv3x3_wgrad(dzr, x), dz.reshape(-1, dz.shape[-1]).sum(0))
            return conv3x3_dgrad(dzr, self.W[k][0])

        dzo = dpred[..., None]
        dtop = layer_bwd(ko, c["top"], dzo)
        top = c["dec0"] if self.L > 1 else c["enc0"]
        dz = dtop * dsilu(top[3])
        d_skip = [None] * self.L
        for i in range(self.L - 1):
            cat, za, aa, zb, ab = c["dec%d" % i]
            da = layer_bwd(dec[i][1], aa, dz)
            dz = da * dsilu(za)
            dcat = layer_bwd(dec[i][0], cat, dz)
            cd = cat.shape[-1] - self.chans[i]
            dup, d_skip[i] = dcat[..., :cd], dcat[..., cd:]
            n, h, w, _ = dup.shape
            ddeep = dup.reshape(n, h // 2, 2, w // 2, 2, cd).sum(axis=(2, 4))
            zdeep = c["dec%d" % (i + 1)][3] if i + 1 < self.L - 1 else c["enc%d" % (self.L - 1)][3]
            dz = ddeep * dsilu(zdeep)
        for i in range(self.L - 1, -1, -1):
            xin, za, aa, zb, ab = c["enc%d" % i]
            if i < self.L - 1:
                dz = d_skip[i] * dsilu(zb)
            da = layer_bwd(enc[i][1], aa, dz)
            dz = da * dsilu(za)
            dx = layer_bwd(enc[i][0], xin, dz)
            if i > 0:
                d_skip[i - 1] = d_skip[i - 1] + 0.25 * up2(dx)
        return grads


def prep_input(g, v, hp, v_shift, v_scale, scale=None):
    """Network input of the gradient preconditioner, FP64: per image scale = RMS of g (1 for
    an all-zero image) unless given; channel 0 = g/scale, channel 1 = (v - v_shift)/v_scale
    (both rounded to BF16 as network inputs), rows padded with zeros to hp.  Returns
    (x [N, hp, W, 2] BF16-rounded, res [N, hp, W] = g/scale unrounded, scale [N])."""
    g = np.asarray(g, dtype=np.float64)
    n, h, w = g.shape
    if scale is None:
        rms = np.sqrt((g.reshape(n, -1) ** 2).mean(1))
        scale = np.where(rms > 0, rms, 1.0)
    scale = np.asarray(scale, dtype=np.float64)
    res = np.zeros((n, hp, w))
    res[:, :h] = g / scale[:, None, None]
    x = np.zeros((n, hp, w, 2))
    x[:, :h, :, 0] = res[:, :h]
    if v is not None:
        x[:, :h, :, 1] = (np.asarray(v, dtype=np.float64) - v_shift) / v_scale
    return bf16(x), res, scale


def guard(pred0, scale, g, cos_min, ratio_lo, ratio_hi, alpha=1.0):
    """Guarded gradient: p = scale * pred0 (first h rows of [N, hp, W]) is kept when
    cos(p, g) >= cos_min and |p|/|g| is in [ratio_lo, ratio_hi], else g is used.  A kept
    image is blended with the plain one, g + alpha (p - g) (alpha = 1: p itself)."""
    g = np.asarray(g, dtype=np.float64)
    n, h, w = g.shape
    p = np.asarray(pred0, dtype=np.float64)[:, :h] * np.asarray(scale, dtype=np.float64)[:, None, None]
    pf, gf = p.reshape(n, -1), g.reshape(n, -1)
    pn, gn = np.linalg.norm(pf, axis=1), np.linalg.norm(gf, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        cos = (pf * gf).sum(1) / (pn * gn)
        ratio = pn / gn
    keep = (pn > 0) & (gn > 0) & (cos >= cos_min) & (ratio >= ratio_lo) & (ratio <= ratio_hi)
    kept = p if alpha == 1.0 else g + alpha * (p - g)
    return np.where(keep[:, None, None], kept, g), keep
