"""Pins of the FP64 network oracle (CPU): convolution against SciPy, adjoint identities of
its data and weight gradients, and central differences of the loss through the network."""
import numpy as np
from scipy.signal import correlate2d

from oracle import unet as U


def test_conv_matches_scipy_correlate():
    r = np.random.default_rng(0)
    x = r.standard_normal((2, 7, 9, 3))
    w = r.standard_normal((4, 9, 3))
    out = U.conv3x3(x, w)
    for n in range(2):
        for co in range(4):
            ref = sum(correlate2d(x[n, :, :, ci], w[co, :, ci].reshape(3, 3), mode="same") for ci in range(3))
            assert np.allclose(out[n, :, :, co], ref, atol=1e-12)


def test_gradients_are_adjoints_of_the_convolution():
    r = np.random.default_rng(1)
    x = r.standard_normal((2, 6, 5, 3))
    w = r.standard_normal((4, 9, 3))
    y = r.standard_normal((2, 6, 5, 4))
    lhs = np.sum(U.conv3x3(x, w) * y)
    assert abs(lhs - np.sum(x * U.conv3x3_dgrad(y, w))) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(w * U.conv3x3_wgrad(y, x))) < 1e-10 * abs(lhs)


def test_pool_up_adjoint():
    r = np.random.default_rng(2)
    a = r.standard_normal((1, 4, 6, 2))
    b = r.standard_normal((1, 2, 3, 2))
    assert abs(np.sum(U.pool2(a) * b) - np.sum(a * 0.25 * U.up2(b))) < 1e-12


def _weights(chans, r, scale=0.3):
    L = len(chans)
    shapes = []
    for i, c in enumerate(chans):
        shapes += [(c, 2 if i == 0 else chans[i - 1]), (c, c)]
    for i in range(L - 2, -1, -1):
        shapes += [(chans[i], chans[i + 1] + chans[i]), (chans[i], chans[i])]
    shapes.append((1, chans[0]))
    return [(r.standard_normal((co, 9, ci)) * scale / np.sqrt(9 * ci), r.standard_normal(co) * 0.1)
            for co, ci in shapes]


def test_network_gradient_central_differences():
    r = np.random.default_rng(3)
    chans = (4, 6, 8)
    W = _weights(chans, r)
    x = r.standard_normal((2, 8, 8, 2))
    res = r.standard_normal((2, 8, 8))
    t = r.standard_normal((2, 8, 8))
    net = U.UNetOracle(chans, W, rounding=False)
    pred = net.forward(x, res)
    L0, d = net.loss(pred, t)
    g = net.backward(d)
    dirs = [(r.standard_normal(w.shape), r.standard_normal(b.shape)) for w, b in W]
    an = sum(np.sum(gw * dw) + np.sum(gb * db) for (gw, gb), (dw, db) in zip(g, dirs))
    eps = 1e-5

    def Lof(s):
        Ws = [(w + s * dw, b + s * db) for (w, b), (dw, db) in zip(W, dirs)]
        n2 = U.UNetOracle(chans, Ws, rounding=False)
        return n2.loss(n2.forward(x, res), t)[0]

    fd = (Lof(eps) - Lof(-eps)) / (2 * eps)
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 0.0, 1e-30])
    r = U.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0  # tie to even
    assert r[2] == 1.0 + 2 ** -7  # round up
    assert abs(r[3] + 3.140625) < 1e-12
    assert r[4] == 0.0
