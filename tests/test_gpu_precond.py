"""Learned preconditioner end to end on the GPU: training pairs from the solver, training
on the library's BF16-MFMA kernels, the guard's blend weight fitted on validation pairs,
and the gain over the plain encoded gradient on held-out pairs, on a small patch where
every shot illuminates most of it and at the 256 x 256 pair configuration."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_trained_network_beats_plain_encoded_gradient():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import precond
    from paper_2512_12797_amd.unet import UNet
    cfg = precond.PairConfig(n=64, nb=16, nt=700, freq=12.0, nshot=16, s=4)
    say("case precond pairs")
    pairs = precond.make_pairs(cfg, nmodels=64, enc_per_model=4, seed=3, models_per_batch=16, log=say)
    P = pairs["x16"].shape[0]
    test_models = set(range(56, 64))
    val_models = set(range(48, 56))
    mid = pairs["model_id"].numpy()
    train_idx = np.array([i for i in range(P) if mid[i] not in test_models | val_models])
    val_idx = torch.tensor([i for i in range(P) if mid[i] in val_models], device="cuda")
    test_idx = torch.tensor([i for i in range(P) if mid[i] in test_models], device="cuda")
    net = UNet(chans=(32, 64, 128), seed=0)
    # untrained network = plain gradient (zero output layer + residual)
    x, res, tg = pairs["x16"][test_idx], pairs["res"][test_idx], pairs["target"][test_idx]
    plain = precond.rel_err(res, tg)
    p0 = precond.rel_err(precond.channel0(precond.predict(net, x, res)), tg)
    assert np.allclose(p0, plain, rtol=1e-2)
    say("case precond training")
    hist = precond.train(net, pairs, train_idx, steps=400, batch=8, lr=2e-3, lr_final=2e-4, log=say)
    assert hist[-1][1] < hist[0][1]
    out = precond.predict(net, x, res)
    trained = precond.rel_err(precond.channel0(out), tg)
    say("held-out relative error vs full-shot gradient: plain %.3f -> network %.3f" % (plain.mean(), trained.mean()))
    assert trained.mean() < 0.9 * plain.mean()
    ones = torch.ones(x.shape[0], device="cuda")
    guarded, keep = precond.guard(out, ones, res)
    g_err = precond.rel_err(guarded, tg)
    assert np.all(g_err <= np.maximum(trained, plain) + 1e-6)
    # the blend weight fitted on validation pairs keeps most of a network that helps
    vres = pairs["res"][val_idx]
    alpha = precond.fit_blend(precond.channel0(precond.predict(net, pairs["x16"][val_idx], vres)), vres,
                              pairs["target"][val_idx])
    blended, _ = precond.guard(out, ones, res, alpha=alpha)
    b_err = precond.rel_err(blended, tg)
    say("blend weight %.3f: held-out error %.3f" % (alpha, b_err.mean()))
    assert alpha > 0.5 and b_err.mean() < 0.9 * plain.mean()
    # a prediction unrelated to the plain gradient falls back to it
    bad = torch.zeros_like(out)
    bad[..., 0] = -res
    fallback, keep_bad = precond.guard(bad, ones, res)
    assert not keep_bad.any() and torch.equal(fallback, res)


def test_network_gains_at_256():
    """The 256 x 256 pair configuration (32 shots, one supergather of 8, 1500 steps) with 64
    models: 48 to train on, 8 for validation (early stopping and the guard's blend weight),
    8 held out.  The network, given the drawn shots' coverage, cuts the held-out error of
    the plain encoded gradient by more than 10 %, and the blended guard keeps that gain."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12797_amd import precond
    from paper_2512_12797_amd.unet import UNet
    cfg = precond.PairConfig()
    say("case precond 256x256 pairs")
    pairs = precond.make_pairs(cfg, nmodels=64, enc_per_model=4, seed=5, models_per_batch=8, log=say)
    P = pairs["x16"].shape[0]
    mid = pairs["model_id"].numpy()
    train_idx = np.nonzero(mid < 48)[0]
    val_idx = torch.from_numpy(np.nonzero((mid >= 48) & (mid < 56))[0]).to("cuda")
    test_idx = torch.from_numpy(np.nonzero(mid >= 56)[0]).to("cuda")
    assert len(train_idx) + val_idx.numel() + test_idx.numel() == P
    net = UNet(seed=0)
    precond.train(net, pairs, train_idx, steps=600, batch=8, lr=1e-3, lr_final=1e-4, val_idx=val_idx, val_every=100)
    assert net.val_best is not None and net.val_hist[0][0] == 0
    vres = pairs["res"][val_idx]
    alpha = precond.fit_blend(precond.channel0(precond.predict(net, pairs["x16"][val_idx], vres)), vres,
                              pairs["target"][val_idx])
    x, res, tg = pairs["x16"][test_idx], pairs["res"][test_idx], pairs["target"][test_idx]
    out = precond.predict(net, x, res)
    ones = torch.ones(x.shape[0], device="cuda")
    blended, _ = precond.guard(out, ones, res, alpha=alpha)
    plain = precond.rel_err(res, tg)
    netw = precond.rel_err(precond.channel0(out), tg)
    b_err = precond.rel_err(blended, tg)
    say("256x256: plain %.4f, network %.4f (validation best after %d steps), blend weight %.3f -> %.4f" % (
        plain.mean(), netw.mean(), net.val_best, alpha, b_err.mean()))
    assert 0.0 <= alpha <= 1.0
    assert netw.mean() < 0.9 * plain.mean()
    assert b_err.mean() < 0.9 * plain.mean()
