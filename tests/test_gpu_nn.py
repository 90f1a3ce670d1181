"""GPU parity of the preconditioner's network kernels and of the whole network against the
FP64 oracle evaluated on the same BF16-rounded operands.

Tolerances: single kernels with FP32 outputs 1e-5 relative L2 (FP32 accumulation order);
BF16 outputs within one BF16 ulp of the oracle's rounding of its FP64 value.  Whole
network: every BF16 rounding point of the forward and backward is reproduced by the
oracle; what remains are elements that land on the other side of a BF16 rounding boundary
because the GPU accumulated in FP32.  With K-term FP32 sums (K = 9 C <= 3456) the two
values differ by ~2^-24 sqrt(K) relative against a BF16 spacing of 2^-8, so ~1e-3 of the
rounded elements flip, each by 2^-8; these compound over the ~14 rounding stages of a
4-level forward + backward.  Bar: output and loss 2e-3, every parameter gradient 1e-2,
median over layers 3e-3 (relative L2).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet as U

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import nn
    nn.lib()
    return nn


def to_bf16_bits(a):
    """FP64 values that are exact BF16 -> int16 bit tensor on the GPU."""
    f = np.asarray(a, dtype=np.float32)
    bits = (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.tensor(bits, device="cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def f64(t, N=None):
    if t.dtype == torch.int16:
        from paper_2512_12797_amd import nn
        t = nn.as_float(t)
    return t.double().cpu().numpy()


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 9, 13, 16, 32), (1, 16, 16, 32, 64), (3, 8, 6, 96, 96),
                                         (1, 256, 256, 32, 64), (2, 181, 183, 16, 96), (1, 256, 257, 64, 32)])
def test_conv_fwd_dgrad_wgrad(N, n, h, w, ci, co):
    say("case conv %s" % ((n, h, w, ci, co),))
    r = np.random.default_rng(ci + co)
    x = U.bf16(r.standard_normal((n, h, w, ci)))
    wt = U.bf16(r.standard_normal((co, 9, ci)) / np.sqrt(9 * ci))
    b = r.standard_normal(co).astype(np.float32).astype(np.float64)
    aux = r.standard_normal((n, h, w, co)).astype(np.float32).astype(np.float64)
    res = r.standard_normal((n, h, w)).astype(np.float32).astype(np.float64)
    xg, wg = to_bf16_bits(x), to_bf16_bits(wt)
    bg = torch.tensor(b, dtype=torch.float32, device="cuda")
    out = torch.empty(n, h, w, co, device="cuda")
    o16 = N.bf16_empty(n, h, w, co)
    N.conv3x3(xg, (n, h, w, ci), wg, co, bias=bg, act=True, out_f32=out, out_bf16=o16)
    ref = U.conv3x3(x, wt, b)
    assert rel(f64(out), ref) < 1e-5
    got16 = f64(o16)
    ref16 = U.bf16(U.silu(ref))
    # one BF16 ulp of the result, plus the FP32 accumulation bound where a pre-activation
    # cancels to ~0: a K-term FP32 sum (K = 9 ci products, exact in FP32, and the bias) is
    # within K 2^-24 sum|x w| of the exact sum, and |SiLU'| <= 1.1 carries that through
    K = 9 * ci + 1
    acc = 1.1 * K * 2.0 ** -24 * U.conv3x3(np.abs(x), np.abs(wt), np.abs(b))
    assert np.all(np.abs(got16 - ref16) <= 2.0 ** -7 * np.abs(ref16) + acc)
    # aux (SiLU' of a pre-activation) and residual on channel 0
    auxg = torch.tensor(aux, dtype=torch.float32, device="cuda")
    resg = torch.tensor(res, dtype=torch.float32, device="cuda")
    N.conv3x3(xg, (n, h, w, ci), wg, co, aux=auxg, res=resg, out_f32=out)
    ref2 = U.conv3x3(x, wt) * U.dsilu(aux)
    ref2[..., 0] += res
    assert rel(f64(out), ref2) < 1e-5
    # data gradient through the packed flipped weights
    wf = torch.tensor(wt, dtype=torch.float32, device="cuda")
    w16 = N.bf16_empty(co, 9, ci)
    wt16 = N.bf16_empty(ci, 9, co)
    N.pack_weights(wf, co, ci, w16, wt16)
    assert torch.equal(w16, wg)
    dz = U.bf16(r.standard_normal((n, h, w, co)))
    dzg = to_bf16_bits(dz)
    if ci % 32 == 0:
        dx = torch.empty(n, h, w, ci, device="cuda")
        N.conv3x3(dzg, (n, h, w, co), wt16, ci, out_f32=dx)
        assert rel(f64(dx), U.conv3x3_dgrad(dz, wt)) < 1e-5
    # weight and bias gradients
    dz32 = torch.tensor(dz, dtype=torch.float32, device="cuda")
    dw = torch.empty(co, 9, ci, device="cuda")
    db = torch.empty(co, device="cuda")
    work = torch.empty(N.wgrad_work((n, h, w, ci), co), device="cuda")
    N.wgrad(dzg, dz32, xg, (n, h, w, ci), co, dw, db, work)
    assert rel(f64(dw), U.conv3x3_wgrad(dz, x)) < 1e-5
    assert rel(f64(db), dz.reshape(-1, co).sum(0)) < 1e-5


@pytest.mark.parametrize("n,h,w,ca,cb,co", [(2, 16, 20, 32, 16, 32), (1, 64, 66, 64, 32, 64), (3, 10, 8, 16, 48, 96)])
def test_upcat_conv_and_wgrad(N, n, h, w, ca, cb, co):
    """Convolution and weight gradient over [up2(a), b] read in place: against the oracle on
    the concatenated input, and bit for bit against the same kernels on the materialised
    concatenation (upsampling and concatenation only copy BF16 values)."""
    say("case upcat %s" % ((n, h, w, ca, cb, co),))
    r = np.random.default_rng(ca + 3 * cb + co)
    a = U.bf16(r.standard_normal((n, h // 2, w // 2, ca)))
    b = U.bf16(r.standard_normal((n, h, w, cb)))
    cat = np.concatenate([U.up2(a), b], axis=-1)
    ci = ca + cb
    wt = U.bf16(r.standard_normal((co, 9, ci)) / np.sqrt(9 * ci))
    bias = r.standard_normal(co).astype(np.float32).astype(np.float64)
    ag, bg, wg = to_bf16_bits(a), to_bf16_bits(b), to_bf16_bits(wt)
    biasg = torch.tensor(bias, dtype=torch.float32, device="cuda")
    out = torch.empty(n, h, w, co, device="cuda")
    o16 = N.bf16_empty(n, h, w, co)
    N.conv3x3_upcat(ag, ca, bg, (n, h, w, ci), wg, co, bias=biasg, act=True, out_f32=out, out_bf16=o16)
    assert rel(f64(out), U.conv3x3(cat, wt, bias)) < 1e-5
    catg = to_bf16_bits(cat)
    out2 = torch.empty_like(out)
    o216 = N.bf16_empty(n, h, w, co)
    N.conv3x3(catg, (n, h, w, ci), wg, co, bias=biasg, act=True, out_f32=out2, out_bf16=o216)
    assert torch.equal(out, out2) and torch.equal(o16, o216)
    dz = U.bf16(r.standard_normal((n, h, w, co)))
    dzg = to_bf16_bits(dz)
    dz32 = torch.tensor(dz, dtype=torch.float32, device="cuda")
    dw = torch.empty(co, 9, ci, device="cuda")
    db = torch.empty(co, device="cuda")
    work = torch.empty(N.wgrad_work((n, h, w, ci), co), device="cuda")
    N.wgrad_upcat(dzg, dz32, ag, ca, bg, (n, h, w, ci), co, dw, db, work)
    assert rel(f64(dw), U.conv3x3_wgrad(dz, cat)) < 1e-5
    assert rel(f64(db), dz.reshape(-1, co).sum(0)) < 1e-5
    dw2 = torch.empty_like(dw)
    N.wgrad(dzg, dz32, catg, (n, h, w, ci), co, dw2, None, work)
    assert torch.equal(dw, dw2)


def test_elementwise_kernels(N):
    say("case elementwise")
    r = np.random.default_rng(5)
    a = U.bf16(r.standard_normal((2, 8, 6, 32)))
    ag = to_bf16_bits(a)
    p = N.bf16_empty(2, 4, 3, 32)
    N.pool2(ag, (2, 8, 6, 32), p)
    assert np.array_equal(f64(p), U.bf16(U.pool2(a)))
    u = N.bf16_empty(2, 16, 12, 32)
    N.up2(ag, (2, 8, 6, 32), u)
    assert np.array_equal(f64(u), U.up2(a))
    d = r.standard_normal((2, 4, 3, 32)).astype(np.float32)
    dx = torch.ones(2, 8, 6, 32, device="cuda")
    N.pool2_bwd(torch.tensor(d, device="cuda"), (2, 8, 6, 32), dx, True)
    assert np.allclose(f64(dx), 1.0 + 0.25 * U.up2(d.astype(np.float64)), rtol=1e-7)
    dd = r.standard_normal((2, 16, 12, 32)).astype(np.float32)
    du = torch.empty(2, 8, 6, 32, device="cuda")
    N.up2_bwd(torch.tensor(dd, device="cuda"), (2, 8, 6, 32), du)
    assert rel(f64(du), dd.astype(np.float64).reshape(2, 8, 2, 6, 2, 32).sum(axis=(2, 4))) < 1e-6
    b = U.bf16(r.standard_normal((2, 8, 6, 64)))
    cat = N.bf16_empty(2, 8, 6, 96)
    N.concat(ag, 32, to_bf16_bits(b), 64, 96, cat)
    assert np.array_equal(f64(cat), np.concatenate([a, b], axis=-1))
    g = r.standard_normal((2, 8, 6, 96)).astype(np.float32)
    ga = torch.zeros(2, 8, 6, 32, device="cuda")
    gb = torch.ones(2, 8, 6, 64, device="cuda")
    N.split_bwd(torch.tensor(g, device="cuda"), 32, 64, 96, ga, False, gb, True)
    assert np.array_equal(f64(ga), g[..., :32].astype(np.float64))
    assert rel(f64(gb), 1.0 + g[..., 32:].astype(np.float64)) < 1e-6
    z = r.standard_normal(1000).astype(np.float32)
    da = r.standard_normal(1000).astype(np.float32)
    o = torch.empty(1000, device="cuda")
    o16 = N.bf16_empty(1000)
    N.silu_bwd(torch.tensor(da, device="cuda"), torch.tensor(z, device="cuda"), o, o16)
    ref = da.astype(np.float64) * U.dsilu(z.astype(np.float64))
    assert rel(f64(o), ref) < 1e-6
    # the scalar forms (channel counts and lengths that are not multiples of 4)
    a6 = U.bf16(r.standard_normal((1, 4, 6, 6)))
    p6 = N.bf16_empty(1, 2, 3, 6)
    N.pool2(to_bf16_bits(a6), (1, 4, 6, 6), p6)
    assert np.array_equal(f64(p6), U.bf16(U.pool2(a6)))
    d6 = r.standard_normal((1, 2, 3, 6)).astype(np.float32)
    dx6 = torch.zeros(1, 4, 6, 6, device="cuda")
    N.pool2_bwd(torch.tensor(d6, device="cuda"), (1, 4, 6, 6), dx6, False)
    assert np.allclose(f64(dx6), 0.25 * U.up2(d6.astype(np.float64)), rtol=1e-7)
    du6 = torch.empty(1, 2, 3, 6, device="cuda")
    N.up2_bwd(torch.tensor(np.repeat(np.repeat(d6, 2, 1), 2, 2).copy(), device="cuda"), (1, 2, 3, 6), du6)
    assert rel(f64(du6), 4.0 * d6.astype(np.float64)) < 1e-6
    g9 = r.standard_normal((5, 8)).astype(np.float32)
    ga3, gb5 = torch.empty(5, 3, device="cuda"), torch.empty(5, 5, device="cuda")
    N.split_bwd(torch.tensor(g9, device="cuda"), 3, 5, 5, ga3, False, gb5, False)
    assert np.array_equal(f64(ga3), g9[:, :3].astype(np.float64)) and np.array_equal(f64(gb5), g9[:, 3:])
    z7 = r.standard_normal(1001).astype(np.float32)
    da7 = r.standard_normal(1001).astype(np.float32)
    o7 = torch.empty(1001, device="cuda")
    N.silu_bwd(torch.tensor(da7, device="cuda"), torch.tensor(z7, device="cuda"), o7, None)
    assert rel(f64(o7), da7.astype(np.float64) * U.dsilu(z7.astype(np.float64))) < 1e-6
    # loss: relative squared error of channel 0
    pred = r.standard_normal((3, 40, 32)).astype(np.float32)
    tg = r.standard_normal((3, 40)).astype(np.float32)
    loss = torch.empty(1, device="cuda")
    dp = torch.empty(3, 40, 32, device="cuda")
    work = torch.empty(2 * 3 * 256, device="cuda")
    N.rel_mse(torch.tensor(pred, device="cuda"), 32, torch.tensor(tg, device="cuda"), 3, 40, loss, dp, None, work)
    Lr, dr = U.UNetOracle.loss(pred[..., 0].astype(np.float64).reshape(3, 40, 1),
                               tg.astype(np.float64).reshape(3, 40, 1))
    assert abs(float(loss.item()) / Lr - 1) < 1e-6
    assert rel(f64(dp)[..., 0], dr[..., 0]) < 1e-6 and np.all(f64(dp)[..., 1:] == 0)
    # Adam
    pp = r.standard_normal(777).astype(np.float32)
    gg = r.standard_normal(777).astype(np.float32)
    pt, m, v = torch.tensor(pp, device="cuda"), torch.zeros(777, device="cuda"), torch.zeros(777, device="cuda")
    N.adam(pt, torch.tensor(gg, device="cuda"), m, v, 1e-2, 0.9, 0.999, 1e-8, 1)
    mh = 0.1 * gg / (1 - 0.9)
    vh = 0.001 * gg.astype(np.float64) ** 2 / (1 - 0.999)
    assert np.allclose(f64(pt), pp - 1e-2 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-5, atol=1e-7)


def _oracle_weights(net):
    """The GPU network's parameters (real channels) in the oracle's order."""
    L = net.L
    out = []
    order = [l for pair in net.enc for l in pair] + [l for i in range(L - 2, -1, -1) for l in net.dec[i]] + [net.out]
    for k, l in enumerate(order):
        cin_real = net.in_used if l is net.enc[0][0] else l.cin
        w = l.wf.double().cpu().numpy()[:l.cout_real, :, :cin_real]
        b = l.b.double().cpu().numpy()[:l.cout_real]
        out.append((w, b))
    return order, out


@pytest.mark.parametrize("chans,hw", [((32, 64), 16), ((32, 64, 96, 128), 32)])
def test_network_forward_backward_vs_oracle(N, chans, hw):
    from paper_2512_12797_amd.unet import UNet
    say("case network %s %dx%d" % (chans, hw, hw))
    net = UNet(chans=chans, seed=1, in_used=2)  # two input channels carry data here
    # give the zero-initialised output layer weights so that every gradient is non-trivial
    r = np.random.default_rng(7)
    o = net.out
    w0 = np.zeros((o.cout, 9, o.cin), dtype=np.float32)
    w0[0] = r.standard_normal((9, o.cin)) * 0.05
    o.wf.copy_(torch.tensor(w0))
    o.pack()
    n = 2
    x = np.zeros((n, hw, hw, 16))
    x[..., :2] = r.standard_normal((n, hw, hw, 2))
    x = U.bf16(x)
    res = r.standard_normal((n, hw, hw)).astype(np.float32).astype(np.float64)
    tg = r.standard_normal((n, hw, hw)).astype(np.float32).astype(np.float64)
    out = net.forward(to_bf16_bits(x), torch.tensor(res.ravel(), dtype=torch.float32, device="cuda"), n, hw, hw,
                      keep=True)
    loss = torch.empty(1, device="cuda")
    dp = torch.empty_like(out)
    dp16 = N.bf16_empty(*out.shape)
    work = torch.empty(2 * n * 256, device="cuda")
    N.rel_mse(out, 32, torch.tensor(tg, dtype=torch.float32, device="cuda"), n, hw * hw, loss, dp, dp16, work)
    net.backward(dp, dp16)
    torch.cuda.synchronize()
    order, W = _oracle_weights(net)
    on = U.UNetOracle(chans, W, rounding=True)
    pred = on.forward(x[..., :2], res)
    Lr, d = on.loss(pred, tg)
    grads = on.backward(d)
    e_out = rel(f64(out)[..., 0], pred)
    say("  output rel %.2e, loss rel %.2e" % (e_out, abs(loss.item() / Lr - 1)))
    assert e_out < 2e-3 and abs(loss.item() / Lr - 1) < 2e-3
    errs = []
    for k, (l, (gw, gb)) in enumerate(zip(order, grads)):
        cin_real = net.in_used if l is net.enc[0][0] else l.cin
        ew = rel(f64(l.dw)[:l.cout_real, :, :cin_real], gw)
        eb = rel(f64(l.db)[:l.cout_real], gb)
        errs += [ew, eb]
        assert ew < 1e-2 and eb < 1e-2, (k, ew, eb)
    say("  parameter-gradient rel: median %.2e, worst %.2e over %d layers" % (np.median(errs), max(errs), len(order)))
    assert np.median(errs) < 3e-3


# ------------------------------------------------ preconditioner input and guard

def test_prep_matches_oracle():
    from paper_2512_12797_amd import nn
    r = np.random.default_rng(11)
    n, h, w, hp = 5, 37, 70, 40
    g = (r.standard_normal((n, h, w)) * 10.0 ** r.uniform(-6, 3, (n, 1, 1))).astype(np.float32)
    g[3] = 0.0  # an all-zero image keeps scale 1
    v = r.uniform(1500, 4500, (n, h, w)).astype(np.float32)
    tg, tv = torch.tensor(g, device="cuda"), torch.tensor(v, device="cuda")
    x16 = torch.empty(n, hp, w, 16, dtype=torch.int16, device="cuda")
    res = torch.empty(n, hp, w, device="cuda")
    scale = torch.empty(n, device="cuda")
    nn.prep(tg, tv, n, h, w, hp, 3000.0, 1500.0, None, scale, x16, res)
    ox, ores, oscale = U.prep_input(g, v, hp, 3000.0, 1500.0)
    assert rel(scale.cpu().numpy(), oscale) < 1e-6 and scale[3].item() == 1.0
    assert rel(res.cpu().numpy(), ores) < 1e-6
    xg = nn.as_float(x16).cpu().numpy().astype(np.float64)
    assert np.all(xg[..., 2:] == 0)
    # BF16 inputs: within one BF16 ulp of the oracle's rounding of its FP64 value
    for c in range(2):
        d = np.abs(xg[..., c] - ox[..., c])
        assert np.all(d <= 2.0 ** -7 * np.abs(ox[..., c]) + 1e-30)
    # targets scaled by given scales, v absent
    t2 = torch.empty(n, hp, w, device="cuda")
    nn.prep(tg, None, n, h, w, hp, 3000.0, 1500.0, scale, None, None, t2)
    assert torch.equal(t2, res)


def test_guard_matches_oracle():
    from paper_2512_12797_amd import nn
    r = np.random.default_rng(12)
    n, h, w, hp, C = 6, 30, 50, 32, 32
    g = r.standard_normal((n, h, w)).astype(np.float32)
    scale = r.uniform(0.5, 2.0, n).astype(np.float32)
    pred = np.zeros((n, hp, w, C), dtype=np.float32)
    base = g / scale[:, None, None]
    pred[0, :h, :, 0] = base[0] + 0.3 * r.standard_normal((h, w))   # agrees: kept
    pred[1, :h, :, 0] = -base[1]                                      # opposite: cosine < 0
    pred[2, :h, :, 0] = 10.0 * base[2]                                # too large: ratio > 5
    pred[3, :h, :, 0] = 0.1 * base[3]                                 # too small: ratio < 0.2
    pred[4] = 0.0                                                     # zero: rejected
    pred[5, :h, :, 0] = 2.0 * base[5] + r.standard_normal((h, w))     # kept
    pred[:, h:, :, 0] = 1e6                                           # padding rows are ignored
    out = torch.empty(n, h, w, device="cuda")
    keep = torch.empty(n, dtype=torch.int32, device="cuda")
    nn.guard(torch.tensor(pred, device="cuda"), C, torch.tensor(scale, device="cuda"), torch.tensor(g, device="cuda"),
             n, h, w, hp, 0.3, 0.2, 5.0, out, keep)
    oo, okeep = U.guard(pred[..., 0], scale, g, 0.3, 0.2, 5.0)
    assert list(keep.cpu().numpy().astype(bool)) == list(okeep) == [True, False, False, False, False, True]
    assert rel(out.cpu().numpy(), oo) < 1e-6


def test_guard_blend_matches_oracle():
    """Blend weights 0.25 and 0 on kept images (and none on rejected ones), against the
    oracle; a weight outside [0, 1] is refused."""
    from paper_2512_12797_amd import nn
    r = np.random.default_rng(13)
    n, h, w, hp, C = 3, 20, 40, 24, 32
    g = r.standard_normal((n, h, w)).astype(np.float32)
    scale = r.uniform(0.5, 2.0, n).astype(np.float32)
    pred = np.zeros((n, hp, w, C), dtype=np.float32)
    base = g / scale[:, None, None]
    pred[0, :h, :, 0] = base[0] + 0.3 * r.standard_normal((h, w))   # kept
    pred[1, :h, :, 0] = -base[1]                                      # rejected
    pred[2, :h, :, 0] = 1.5 * base[2] + 0.2 * r.standard_normal((h, w))  # kept
    args = (torch.tensor(pred, device="cuda"), C, torch.tensor(scale, device="cuda"), torch.tensor(g, device="cuda"),
            n, h, w, hp, 0.3, 0.2, 5.0)
    for alpha in (0.25, 0.0):
        out = torch.empty(n, h, w, device="cuda")
        keep = torch.empty(n, dtype=torch.int32, device="cuda")
        nn.guard(*args, out, keep, alpha=alpha)
        oo, okeep = U.guard(pred[..., 0], scale, g, 0.3, 0.2, 5.0, alpha=alpha)
        assert list(keep.cpu().numpy().astype(bool)) == list(okeep) == [True, False, True]
        if alpha == 0.0:
            assert np.array_equal(out.cpu().numpy(), g)
        else:
            assert rel(out.cpu().numpy(), oo) < 1e-6
    from paper_2512_12797_amd import fwi
    with pytest.raises(fwi.FwiError):
        nn.guard(*args, torch.empty(n, h, w, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"),
                 alpha=1.5)


def test_guard_exact_thresholds():
    """Cases that sit exactly on the guard's bounds (cosine 0.5, norm ratio 0.25 and 4, all
    exact in FP32 and FP64: p = (1, 1; 1, 1) with |p| = 2 against g = (8, 0; 0, 0) and
    (0.5, 0; 0, 0)) are kept, and one FP32 step past a bound falls back, as in the oracle."""
    from paper_2512_12797_amd import nn
    n, h, w, hp, C = 2, 2, 2, 4, 32
    g = np.array([[[8.0, 0.0], [0.0, 0.0]], [[0.5, 0.0], [0.0, 0.0]]], dtype=np.float32)
    scale = np.array([2.0, 2.0], dtype=np.float32)
    pred = np.zeros((n, hp, w, C), dtype=np.float32)
    pred[:, :h, :, 0] = 0.5                                          # p = scale * pred0 = 1
    pred[:, h:, :, 0] = -9.0                                         # padding rows are ignored
    up = lambda x: float(np.nextafter(np.float32(x), np.float32(np.inf)))
    down = lambda x: float(np.nextafter(np.float32(x), np.float32(-np.inf)))
    cases = [((0.5, 0.25, 4.0), [True, True]),
             ((up(0.5), 0.25, 4.0), [False, False]),
             ((0.5, up(0.25), 4.0), [False, True]),
             ((0.5, 0.25, down(4.0)), [True, False])]
    for (cmin, lo, hi), want in cases:
        out = torch.empty(n, h, w, device="cuda")
        keep = torch.empty(n, dtype=torch.int32, device="cuda")
        nn.guard(torch.tensor(pred, device="cuda"), C, torch.tensor(scale, device="cuda"),
                 torch.tensor(g, device="cuda"), n, h, w, hp, cmin, lo, hi, out, keep)
        oo, okeep = U.guard(pred[..., 0], scale, g, cmin, lo, hi)
        assert list(okeep) == want, (cmin, lo, hi)
        assert list(keep.cpu().numpy().astype(bool)) == want, (cmin, lo, hi)
        assert np.array_equal(out.cpu().numpy(), oo.astype(np.float32))
