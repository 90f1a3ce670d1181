"""GPU: the diffusion outer loop's kernels (include/fwi_daps.h) against the FP64 oracle
(oracle/daps.py), through the C ABI.

fwi_daps_mix evaluates in FP64 and rounds once: it matches the oracle to FP32 rounding
(the two normal streams share their construction; the device's log / cos / sin may differ
from the host's in the last FP64 bits).  fwi_daps_prep's BF16 channels equal the oracle's
values rounded to nearest even, bit for bit; fwi_daps_model matches exactly.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import daps as D
from oracle import unet as U

pytestmark = pytest.mark.gpu

LO, HI = 1350.0, 6600.0


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import daps
    return daps


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("terms,nimg,n", [("both", 3, 1001), ("z", 3, 1001), ("x", 3, 1001), ("inplace", 3, 1001),
                                          ("both", 16, 60000)])
def test_mix_matches_oracle(M, terms, nimg, n):
    # 1001 cells: a partial Philox block per image; 16 x 60000: the 2D workload's samples
    say("case daps mix, %s, %d x %d" % (terms, nimg, n))
    r = np.random.default_rng(3)
    z = f32(r.uniform(LO, HI, (nimg, n)))
    x = f32(r.uniform(-1.2, 1.2, (nimg, n)))
    c0 = f32(r.uniform(0.1, 1.0, nimg))
    c1 = f32(r.uniform(0.0, 1.0, nimg))
    sig = f32(([0.3, 0.0, 0.02] * nimg)[:nimg])
    seed, step = 77, 5
    zz = z if terms in ("both", "z", "inplace") else None
    xx = x if terms in ("both", "x", "inplace") else None
    ref = D.mix(zz, xx, c0, c1, sig, LO, HI, seed, step)
    zt = dev(z) if zz is not None else None
    xt = dev(x) if xx is not None else None
    out = xt if terms == "inplace" else torch.empty(nimg, n, device="cuda")
    M.fwi_daps_mix(nimg, n, zt, xt, dev(c0), dev(c1), dev(sig), LO, HI, seed, step, out)
    got = out.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("  max rel error %.2e" % err)
    assert err < 2e-7
    # the image with sig = 0 is deterministic
    assert np.array_equal(got[1], f32(ref[1]))


def test_forward_diffusion_statistics(M):
    # q(x_t | x_0) with the kernel's own draws: mean sqrt(alpha_t) x0, variance 1 - alpha_t
    sched = M.Schedule()
    t = 40
    n = 1 << 20
    z = torch.full((1, n), 4000.0, device="cuda")
    c0, c1, sig = (torch.tensor([v], dtype=torch.float32, device="cuda") for v in sched.forward(t))
    out = torch.empty(1, n, device="cuda")
    M.fwi_daps_mix(1, n, z, None, c0, c1, sig, LO, HI, 9, 0, out)
    x0 = D.normalise(4000.0, LO, HI)
    a = out.double()
    assert abs(float(a.mean()) - np.sqrt(sched.alpha[t]) * x0) < 5 * np.sqrt((1 - sched.alpha[t]) / n)
    assert abs(float(a.var()) / (1 - sched.alpha[t]) - 1) < 5 * np.sqrt(2.0 / n)


@pytest.mark.parametrize("nimg,w,hp", [(2, 40, 150), (2, 40, 152), (8, 400, 152)])
def test_prep_matches_oracle(M, nimg, w, hp):
    say("case daps prep, %d x 150 x %d -> %d rows" % (nimg, w, hp))
    r = np.random.default_rng(4)
    h = 150
    x = f32(r.uniform(-1, 1, (nimg, h, w)))
    level = f32(r.uniform(0.01, 0.5, nimg))
    x16 = torch.empty(nimg, hp, w, 16, dtype=torch.int16, device="cuda")
    res = torch.empty(nimg, hp, w, device="cuda")
    M.fwi_daps_prep(nimg, h, w, hp, dev(x), dev(level), x16, res)
    ch0, ch1, rref = D.prep(x, level, hp)
    got = (x16.to(torch.int32) << 16).view(torch.float32).cpu().numpy().astype(np.float64)
    assert np.array_equal(got[..., 0], U.bf16(ch0))
    assert np.array_equal(got[..., 1], U.bf16(ch1))
    assert np.all(got[..., 2:] == 0)
    assert np.array_equal(res.cpu().numpy().astype(np.float64), rref)


@pytest.mark.parametrize("nimg,w", [(2, 40), (8, 400)])
def test_model_matches_oracle(M, nimg, w):
    r = np.random.default_rng(5)
    h, hp, c = 150, 152, 32
    pred = f32(r.uniform(-1.3, 1.3, (nimg, hp, w, c)))
    v = torch.empty(nimg, h, w, device="cuda")
    M.fwi_daps_model(nimg, h, w, hp, c, dev(pred), LO, HI, v)
    ref = f32(D.to_model(pred[:, :h, :, 0], LO, HI))
    assert np.array_equal(v.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("renoise", ["posterior", "marginal", "mean"])
def test_sampler_plumbing_with_identity_network(M, renoise):
    # An untrained network returns its residual input (zero output layer), so with no
    # Langevin steps every level is: v = model(x_t); x_{t-1} = re-noise(v, x_t).  The oracle
    # replays that chain in FP64 with its own noise streams: this checks the warm start, the
    # coefficients of each mode and the counter words of every draw.
    from types import SimpleNamespace
    say("case daps sampler plumbing, %s" % renoise)
    nz, nx, ns, ts, seed = 14, 24, 3, 6, 21
    r = np.random.default_rng(6)
    vstart = 3000.0 + 1500.0 * r.random((nz, nx))
    cfg = SimpleNamespace(nz=nz, nx=nx, vmin=2000.0, vmax=6000.0)
    sv = SimpleNamespace(cfg=cfg, grid=SimpleNamespace(nphys=nz * nx), dev="cuda", vtrue=vstart + 50.0,
                         vstart=vstart)
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    den = M.Denoiser(nz, nx, 16, lo, hi, seed=0)
    sched = M.Schedule()
    v, rmse, _, ngrad = M.sample(sv, den, sched, ts, 0, 1e-5, seed, nsample=ns, renoise=renoise)
    beta, alpha = D.linear_schedule(1000, 1e-4, 0.02)
    z0 = np.tile(f32(vstart).ravel(), (ns, 1))
    x = D.mix(z0, None, [np.sqrt(alpha[ts])] * ns, [0.0] * ns, [np.sqrt(1 - alpha[ts])] * ns, lo, hi, seed, 1001)
    for t in range(ts, 0, -1):
        vo = D.to_model(x, lo, hi)
        if t > 1:
            if renoise == "marginal":
                c = (np.sqrt(alpha[t - 1]), 0.0, np.sqrt(1 - alpha[t - 1]))
            else:
                c0, c1, bt = D.posterior(beta, alpha, t)
                c = (c0, c1, np.sqrt(bt) if renoise == "posterior" else 0.0)
            x = D.mix(vo, x if renoise != "marginal" else None, *([ci] * ns for ci in c), lo, hi, seed, t)
    assert ngrad == 0 and len(rmse) == ts
    got = v.cpu().numpy().astype(np.float64)
    err = np.abs(got - vo).max()
    say("  max abs error %.3e m/s" % err)
    assert err < 5e-3


@pytest.mark.parametrize("guide,nu", [("langevin", 3.0), ("adam", 0.0), ("adam", 2.0)])
def test_sampler_guidance_steps(M, guide, nu):
    # The same identity-network chain with K = 2 refinement steps per level, the encoded
    # gradient replaced by that of (1/2)|v - v_ref|^2 (a stand-in whose value the oracle
    # can form): checks the Langevin and Adam guidance, the moment restart per level, the
    # noise counters and the clamp against an FP64 replay.
    import oracle
    from types import SimpleNamespace
    say("case daps sampler guidance, %s nu=%g" % (guide, nu))
    nz, nx, ns, ts, K, seed = 14, 24, 3, 4, 2, 23
    r = np.random.default_rng(8)
    vstart = 3000.0 + 1500.0 * r.random((nz, nx))
    vref = f32(vstart + r.normal(0.0, 80.0, (nz, nx)))
    vref_t = dev(vref.ravel())
    cfg = SimpleNamespace(nz=nz, nx=nx, vmin=2000.0, vmax=6000.0)
    sv = SimpleNamespace(cfg=cfg, grid=SimpleNamespace(nphys=nz * nx), dev="cuda", vtrue=vref, vstart=vstart,
                         encoded_gradient=lambda v, n, s, k: v.reshape(n, -1) - vref_t)
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    eta, lr = 0.1, 20.0
    den = M.Denoiser(nz, nx, 16, lo, hi, seed=0)
    v, _, _, ngrad = M.sample(sv, den, M.Schedule(), ts, K, eta, seed, nsample=ns, nu=nu, renoise="marginal",
                              guide=guide, adam_lr=lr)
    beta, alpha = D.linear_schedule(1000, 1e-4, 0.02)
    z0 = np.tile(f32(vstart).ravel(), (ns, 1))
    x = D.mix(z0, None, [np.sqrt(alpha[ts])] * ns, [0.0] * ns, [np.sqrt(1 - alpha[ts])] * ns, lo, hi, seed, 1001)
    step = 0
    for t in range(ts, 0, -1):
        vo = D.to_model(x, lo, hi)
        m1, m2 = np.zeros_like(vo), np.zeros_like(vo)
        for k in range(K):
            g = vo - vref.ravel()
            for i in range(ns):
                xi = oracle.normals(seed, step, i, vo.shape[1])
                if guide == "adam":
                    m1[i] = 0.9 * m1[i] + 0.1 * g[i]
                    m2[i] = 0.999 * m2[i] + 0.001 * g[i] ** 2
                    p = vo[i] - lr * (m1[i] / (1 - 0.9 ** (k + 1))) / (np.sqrt(m2[i] / (1 - 0.999 ** (k + 1))) + 1e-8)
                    vo[i] = oracle.langevin(p, np.zeros_like(p), xi, 0.0, nu, lo, hi)
                else:
                    vo[i] = oracle.langevin(vo[i], g[i], xi, eta, nu, lo, hi)
            step += 1
        if t > 1:
            x = D.mix(vo, None, [np.sqrt(alpha[t - 1])] * ns, [0.0] * ns, [np.sqrt(1 - alpha[t - 1])] * ns, lo, hi,
                      seed, t)
    assert ngrad == ts * K
    got = v.cpu().numpy().astype(np.float64)
    err = np.abs(got - vo).max()
    say("  max abs error %.3e m/s" % err)
    assert err < 2e-2


@pytest.mark.parametrize("nu", [0.0, 1.5])
def test_prior_free_adam_chain(M, nu):
    # chains.run_chain with Adam guidance: moments kept over the whole chain (bias
    # correction with the step count), then the noise and the clamp; the stand-in gradient
    # is that of (1/2)|v - v_ref|^2, replayed by the oracle in FP64
    import oracle
    from types import SimpleNamespace
    from paper_2512_12797_amd import chains
    say("case prior-free Adam chain, nu=%g" % nu)
    nz, nx, ns, steps, seed, lr = 6, 10, 2, 5, 31, 15.0
    r = np.random.default_rng(9)
    vstart = 3000.0 + 1000.0 * r.random((nz, nx))
    vref = f32(vstart + r.normal(0.0, 60.0, (nz, nx)))
    vref_t = dev(vref.ravel())
    cfg = SimpleNamespace(nz=nz, nx=nx, vmin=2000.0, vmax=6000.0)
    sv = SimpleNamespace(cfg=cfg, grid=SimpleNamespace(nphys=nz * nx), dev="cuda", vtrue=vref, vstart=vstart,
                         encoded_gradient=lambda v, n, s, k: v.reshape(n, -1) - vref_t)
    rmse, _, _, v = chains.run_chain(sv, "encoded", steps, 1e-3, seed, nsample=ns, nu=nu, adam_lr=lr,
                                     keep_samples=True)
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    vo = np.tile(f32(vstart).ravel(), (ns, 1))
    m1, m2 = np.zeros_like(vo), np.zeros_like(vo)
    for t in range(steps):
        g = vo - vref.ravel()
        m1 = 0.9 * m1 + 0.1 * g
        m2 = 0.999 * m2 + 0.001 * g ** 2
        p = vo - lr * (m1 / (1 - 0.9 ** (t + 1))) / (np.sqrt(m2 / (1 - 0.999 ** (t + 1))) + 1e-8)
        for i in range(ns):
            vo[i] = oracle.langevin(p[i], np.zeros_like(p[i]), oracle.normals(seed, t, i, p.shape[1]), 0.0, nu, lo,
                                    hi)
    err = np.abs(v.cpu().numpy().astype(np.float64) - vo).max()
    say("  max abs error %.3e m/s" % err)
    assert len(rmse) == steps and err < 1e-2


@pytest.mark.parametrize("adam_lr", [None, 12.0])
def test_svgd_loop_against_oracle_steps(adam_lr):
    # svgd.run's particle loop (start perturbation, step size from the first direction,
    # buffer swap; or the Adam ascent along the Stein direction) with the full-shot
    # gradient replaced by that of (1/2)|v - v_ref|^2
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from types import SimpleNamespace
    from oracle import svgd as S
    from paper_2512_12797_amd import svgd
    say("case svgd loop, adam %s" % adam_lr)
    nz, nx, n, steps, seed = 8, 12, 5, 4, 17
    r = np.random.default_rng(10)
    vstart = 3000.0 + 1000.0 * r.random((nz, nx))
    vref = f32(vstart + r.normal(0.0, 60.0, (nz, nx)))
    vref_t = dev(vref.ravel())
    cfg = SimpleNamespace(nz=nz, nx=nx, vmin=2000.0, vmax=6000.0)
    sv = SimpleNamespace(cfg=cfg, grid=SimpleNamespace(nphys=nz * nx), dev="cuda", vtrue=vref, vstart=vstart,
                         full_gradient=lambda v, k: v.reshape(k, -1) - vref_t)
    x, rmse, _ = svgd.run(sv, steps, 40.0, seed, n=n, gradient="full", adam_lr=adam_lr)
    lo, hi = cfg.vmin * 0.9, cfg.vmax * 1.1
    xo = f32(np.clip(vstart.ravel()[None, :] + np.random.default_rng(seed).normal(0.0, 20.0, (n, nz * nx)), lo, hi))
    eps = None
    m1, m2 = np.zeros_like(xo), np.zeros_like(xo)
    for k in range(steps):
        g = xo - vref.ravel()
        if adam_lr is not None:
            phi = S.direction(xo, g)[0]
            m1 = 0.9 * m1 + 0.1 * phi
            m2 = 0.999 * m2 + 0.001 * phi ** 2
            xo = np.clip(xo + adam_lr * (m1 / (1 - 0.9 ** (k + 1))) / (np.sqrt(m2 / (1 - 0.999 ** (k + 1))) + 1e-8),
                         lo, hi)
            continue
        if eps is None:
            eps = 40.0 / np.abs(S.direction(xo, g)[0]).max()
        xo, _, _ = S.step(xo, g, eps, lo, hi)
    err = np.abs(x.cpu().numpy().astype(np.float64) - xo).max()
    say("  max abs error %.3e m/s" % err)
    assert len(rmse) == steps and err < 1e-2
