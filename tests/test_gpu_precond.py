"""Learned preconditioner end to end on the GPU (small configuration): training pairs
from the solver, training on the library's BF16-MFMA kernels, and the gain over the plain
encoded gradient on held-out pairs (what the method gains from the network)."""
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
    mid = pairs["model_id"].numpy()
    train_idx = np.array([i for i in range(P) if mid[i] not in test_models])
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
    # a prediction unrelated to the plain gradient falls back to it
    bad = torch.zeros_like(out)
    bad[..., 0] = -res
    fallback, keep_bad = precond.guard(bad, ones, res)
    assert not keep_bad.any() and torch.equal(fallback, res)
