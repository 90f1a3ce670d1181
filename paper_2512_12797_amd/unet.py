"""U-Net gradient preconditioner on the library's BF16-MFMA kernels (include/fwi_nn.h).

Architecture (levels L = len(chans)): encoder level i = two 3x3 conv + SiLU layers
(in -> c_i -> c_i), 2x2 average pooling between levels; decoder level i = nearest 2x
upsampling of the level below, channel concatenation with the encoder's level-i output,
two 3x3 conv + SiLU layers ((c_{i+1} + c_i) -> c_i -> c_i); output = 3x3 conv c_0 -> 1
(padded to 32 channels) without activation, plus a residual: channel 0 of the network
input (the encoded gradient) is added to the prediction, so an untrained network returns
the plain encoded gradient.

Activations are NHWC; convolution inputs are BF16 (matrix-core operands), pre-activations
FP32.  Parameters are FP32 masters updated by Adam and packed to BF16 (forward layout and
flipped/transposed data-gradient layout) after every step.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import nn

IN_CH = 16  # network input channels (padded)
IN_USED = 3  # channels in use: normalised gradient, normalised model, shot coverage


def _pad(c, m):
    return (c + m - 1) // m * m


class Conv:
    def __init__(self, cin, cout, cin_real, cout_real, rng, device, scale=1.0):
        self.cin, self.cout = cin, cout
        w = np.zeros((cout, 9, cin), dtype=np.float32)
        std = scale * math.sqrt(2.0 / (9 * cin_real))
        w[:cout_real, :, :cin_real] = rng.standard_normal((cout_real, 9, cin_real)) * std
        self.wf = torch.tensor(w, device=device)
        self.b = torch.zeros(cout, device=device)
        self.dw = torch.zeros_like(self.wf)
        self.db = torch.zeros_like(self.b)
        self.m = [torch.zeros_like(self.wf), torch.zeros_like(self.b)]
        self.v = [torch.zeros_like(self.wf), torch.zeros_like(self.b)]
        self.w16 = nn.bf16_empty(cout, 9, cin, device=device)
        self.wt16 = nn.bf16_empty(cin, 9, cout, device=device)
        self.cout_real = cout_real
        self.pack()

    def pack(self):
        nn.pack_weights(self.wf, self.cout, self.cin, self.w16, self.wt16)


class UNet:
    def __init__(self, chans=(32, 64, 128, 256), seed=0, device="cuda", in_used=IN_USED):
        """in_used: input channels that carry data (the first layer's initial weights on
        the others are zero)."""
        assert all(c % 32 == 0 for c in chans) and 1 <= in_used <= IN_CH
        self.chans = tuple(chans)
        self.in_used = in_used
        self.L = len(chans)
        self.device = device
        rng = np.random.default_rng(seed)
        self.enc = []
        for i, c in enumerate(chans):
            cin = IN_CH if i == 0 else chans[i - 1]
            cin_real = in_used if i == 0 else chans[i - 1]
            self.enc.append((Conv(cin, c, cin_real, c, rng, device), Conv(c, c, c, c, rng, device)))
        self.dec = [None] * (self.L - 1)
        for i in range(self.L - 2, -1, -1):
            cin = chans[i + 1] + chans[i]
            self.dec[i] = (Conv(cin, chans[i], cin, chans[i], rng, device),
                           Conv(chans[i], chans[i], chans[i], chans[i], rng, device))
        # zero output layer: the untrained network returns the residual (plain gradient)
        self.out = Conv(chans[0], 32, chans[0], 1, rng, device, scale=0.0)
        self.t = 0

    def layers(self):
        ls = []
        for a, b in self.enc:
            ls += [a, b]
        for d in self.dec:
            ls += list(d)
        ls.append(self.out)
        return ls

    def nparams(self):
        return sum(l.cout_real * 9 * (l.cin if l is not self.enc[0][0] else self.in_used) + l.cout_real
                   for l in self.layers())

    # ------------------------------------------------------------ forward
    def forward(self, x16, res, n, h, w, keep=False):
        """x16: bf16 [n, h, w, 16]; res: f32 [n*h*w] added to output channel 0.
        Returns f32 [n, h, w, 32] (channel 0 = prediction).  keep: store what the backward
        pass needs, including the FP32 pre-activations (inference writes only the BF16
        activations)."""
        assert h % (1 << (self.L - 1)) == 0 and w % (1 << (self.L - 1)) == 0
        dev = self.device
        st = {"x": x16, "n": n, "h": h, "w": w, "res": res}
        cur, cur_c = x16, IN_CH
        for i, (ca, cb) in enumerate(self.enc):
            hi, wi = h >> i, w >> i
            if i > 0:
                pooled = nn.bf16_empty(n, hi, wi, cur_c, device=dev)
                nn.pool2(cur, (n, 2 * hi, 2 * wi, cur_c), pooled)
                cur = pooled
                st["pool%d" % i] = pooled
            za = torch.empty(n, hi, wi, ca.cout, device=dev) if keep else None
            aa = nn.bf16_empty(n, hi, wi, ca.cout, device=dev)
            nn.conv3x3(cur, (n, hi, wi, cur_c), ca.w16, ca.cout, ca.b, act=True, out_f32=za, out_bf16=aa)
            zb = torch.empty(n, hi, wi, cb.cout, device=dev) if keep else None
            ab = nn.bf16_empty(n, hi, wi, cb.cout, device=dev)
            nn.conv3x3(aa, (n, hi, wi, ca.cout), cb.w16, cb.cout, cb.b, act=True, out_f32=zb, out_bf16=ab)
            st["enc%d" % i] = (cur, za, aa, zb, ab)
            cur, cur_c = ab, cb.cout
        for i in range(self.L - 2, -1, -1):
            hi, wi = h >> i, w >> i
            da, db = self.dec[i]
            # first convolution over [up2(cur), skip], read in place by the kernel
            skip = st["enc%d" % i][4]
            za = torch.empty(n, hi, wi, da.cout, device=dev) if keep else None
            aa = nn.bf16_empty(n, hi, wi, da.cout, device=dev)
            nn.conv3x3_upcat(cur, cur_c, skip, (n, hi, wi, cur_c + self.chans[i]), da.w16, da.cout, da.b, act=True,
                             out_f32=za, out_bf16=aa)
            zb = torch.empty(n, hi, wi, db.cout, device=dev) if keep else None
            ab = nn.bf16_empty(n, hi, wi, db.cout, device=dev)
            nn.conv3x3(aa, (n, hi, wi, da.cout), db.w16, db.cout, db.b, act=True, out_f32=zb, out_bf16=ab)
            st["dec%d" % i] = ((cur, skip), za, aa, zb, ab, cur_c)
            cur, cur_c = ab, db.cout
        out = torch.empty(n, h, w, 32, device=dev)
        nn.conv3x3(cur, (n, h, w, cur_c), self.out.w16, 32, self.out.b, res=res, out_f32=out)
        st["top"] = cur
        if keep:
            self.state = st
        return out

    # ----------------------------------------------------------- backward
    def _conv_bwd(self, conv, x16, shape_in, dz32, dz16, aux=None, want_dx=True):
        """Weight/bias gradients of `conv` and the gradient w.r.t. its input: with aux
        (the input's pre-activation) the result is dL/dz of the previous layer (f32, bf16);
        without, dL/dx in f32.  x16 is the input, or (a, b) for the concatenation
        [up2(a), b] of a decoder's first convolution."""
        n, h, w, cin = shape_in
        work = torch.empty(nn.wgrad_work(shape_in, conv.cout), device=self.device)
        if isinstance(x16, tuple):
            a, b = x16
            nn.wgrad_upcat(dz16, dz32, a, cin - b.shape[-1], b, shape_in, conv.cout, conv.dw, conv.db, work)
        else:
            nn.wgrad(dz16, dz32, x16, shape_in, conv.cout, conv.dw, conv.db, work)
        if not want_dx:
            return None
        o32 = torch.empty(n, h, w, cin, device=self.device)
        o16 = nn.bf16_empty(n, h, w, cin, device=self.device) if aux is not None else None
        nn.conv3x3(dz16, (n, h, w, conv.cout), conv.wt16, cin, aux=aux, out_f32=o32, out_bf16=o16)
        return (o32, o16) if aux is not None else o32

    def backward(self, dout32, dout16):
        st = self.state
        n, h, w = st["n"], st["h"], st["w"]
        dev = self.device
        top_c = self.chans[0]
        # output layer: input = decoder level 0 output (or encoder 0 when L == 1)
        top_src = st["dec0"] if self.L > 1 else st["enc0"]
        dz, dz16 = self._conv_bwd(self.out, st["top"], (n, h, w, top_c), dout32, dout16, aux=top_src[3])
        d_skip = [None] * self.L  # dL/d(encoder level i output activation), f32
        for i in range(self.L - 1):
            hi, wi = h >> i, w >> i
            da_conv, db_conv = self.dec[i]
            cat_src, za, aa, zb, ab, cdeep = st["dec%d" % i]
            # second conv of the level: input aa (pre-activation za)
            dz, dz16 = self._conv_bwd(db_conv, aa, (n, hi, wi, da_conv.cout), dz, dz16, aux=za)
            # first conv: input = concat(up(deeper), skip)
            dcat = self._conv_bwd(da_conv, cat_src, (n, hi, wi, cdeep + self.chans[i]), dz, dz16)
            dup = torch.empty(n, hi, wi, cdeep, device=dev)
            d_skip[i] = torch.empty(n, hi, wi, self.chans[i], device=dev)
            nn.split_bwd(dcat, cdeep, self.chans[i], n * hi * wi, dup, False, d_skip[i], False)
            ddeep = torch.empty(n, hi // 2, wi // 2, cdeep, device=dev)
            nn.up2_bwd(dup, (n, hi // 2, wi // 2, cdeep), ddeep)
            # the deeper tensor is decoder level i+1's output or the bottleneck's output
            zdeep = st["dec%d" % (i + 1)][3] if i + 1 < self.L - 1 else st["enc%d" % (self.L - 1)][3]
            dz = torch.empty_like(ddeep)
            dz16 = nn.bf16_empty(*ddeep.shape, device=dev)
            nn.silu_bwd(ddeep, zdeep, dz, dz16)
        # encoder, deepest first; dz currently belongs to the bottleneck's second conv
        for i in range(self.L - 1, -1, -1):
            hi, wi = h >> i, w >> i
            ca, cb = self.enc[i]
            xin, za, aa, zb, ab = st["enc%d" % i]
            if i < self.L - 1:
                # this level's output feeds the skip (d_skip) and the pooled input of level i+1
                dz = torch.empty_like(d_skip[i])
                dz16 = nn.bf16_empty(*d_skip[i].shape, device=dev)
                nn.silu_bwd(d_skip[i], zb, dz, dz16)
            dz, dz16 = self._conv_bwd(cb, aa, (n, hi, wi, ca.cout), dz, dz16, aux=za)
            cin = IN_CH if i == 0 else self.chans[i - 1]
            if i == 0:
                self._conv_bwd(ca, xin, (n, hi, wi, cin), dz, dz16, want_dx=False)
            else:
                dpool = self._conv_bwd(ca, xin, (n, hi, wi, cin), dz, dz16)
                # add the pooled path's gradient to level i-1's output gradient
                nn.pool2_bwd(dpool, (n, 2 * hi, 2 * wi, cin), d_skip[i - 1], True)
        self.state = None

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for l in self.layers():
            nn.adam(l.wf, l.dw, l.m[0], l.v[0], lr, b1, b2, eps, self.t)
            nn.adam(l.b, l.db, l.m[1], l.v[1], lr, b1, b2, eps, self.t)
            l.pack()

    # ---------------------------------------------------------- utilities
    def state_dict(self):
        return {"chans": self.chans, "t": self.t,
                "w": [l.wf.cpu().numpy() for l in self.layers()], "b": [l.b.cpu().numpy() for l in self.layers()]}

    def load_state_dict(self, sd):
        assert tuple(sd["chans"]) == self.chans
        for l, w, b in zip(self.layers(), sd["w"], sd["b"]):
            l.wf.copy_(torch.as_tensor(w))
            l.b.copy_(torch.as_tensor(b))
            l.pack()
        self.t = sd["t"]
