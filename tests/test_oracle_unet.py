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


# ---------------------------------------------------- input preparation and the guard

def test_prep_input_hand_computed_scale_and_padding():
    """RMS scale over the image's own h x w cells (padded rows never count), BF16 inputs,
    zero rows below h, and scale 1 for an all-zero image."""
    g = np.array([[[3.0, 4.0], [0.0, 0.0]],        # RMS sqrt(25 / 4) = 2.5 over the 2 x 2 image
                  [[0.0, 0.0], [0.0, 0.0]]])       # all zero: scale 1
    v = np.array([[[3000.0, 2500.0], [3500.0, 2000.0]]] * 2)
    x, res, scale = U.prep_input(g, v, 4, 2500.0, 1000.0)
    assert x.shape == (2, 4, 2, 2) and res.shape == (2, 4, 2)
    assert scale[0] == 2.5 and scale[1] == 1.0      # an RMS over the 4 padded rows would be 1.768
    assert np.array_equal(res[0, :2], [[1.2, 1.6], [0.0, 0.0]])
    # 1.2 and 1.6 rounded to BF16 (8 significant bits): 154/128 and 205/128
    assert np.array_equal(x[0, :2, :, 0], [[154 / 128, 205 / 128], [0.0, 0.0]])
    assert np.array_equal(x[0, :2, :, 1], [[0.5, 0.0], [1.0, -0.5]])
    assert not x[:, 2:].any() and not res[:, 2:].any()
    assert not x[1, :, :, 0].any()
    # no model: channel 1 stays zero
    x2, _, _ = U.prep_input(g, None, 2, 0.0, 1.0)
    assert not x2[..., 1].any()


def test_prep_input_scale_equivariance_and_given_scale():
    r = np.random.default_rng(5)
    g = r.standard_normal((3, 5, 7))
    x, res, scale = U.prep_input(g, None, 8, 0.0, 1.0)
    xs, ress, scales = U.prep_input(4.0 * g, None, 8, 0.0, 1.0)
    assert np.allclose(scales, 4.0 * scale, rtol=1e-15)
    assert np.allclose(ress, res, rtol=1e-14, atol=0) and np.array_equal(xs, x)
    # a given scale replaces the RMS
    _, res2, scale2 = U.prep_input(g, None, 5, 0.0, 1.0, scale=np.array([2.0, 4.0, 0.5]))
    assert np.array_equal(scale2, [2.0, 4.0, 0.5])
    assert np.array_equal(res2[1], g[1] / 4.0)


def _guard_case(p, g, hp=3, scale=2.0, junk=7.0):
    """pred0 rows of a padded height hp (rows past h hold junk the guard must ignore)."""
    g = np.asarray(g, dtype=np.float64)[None]
    pred0 = np.full((1, hp, g.shape[2]), junk)
    pred0[0, :g.shape[1]] = np.asarray(p, dtype=np.float64) / scale
    return pred0, np.array([scale]), g


def test_guard_thresholds_are_inclusive():
    """p = (3, 9; 3, 1) has |p| = 10.  Against g = (2, 0; 0, 0): cos = 0.3, |p|/|g| = 5;
    against g = (50, 0; 0, 0): cos = 0.3, |p|/|g| = 0.2.  All exact in FP64, so the
    bounds cos >= 0.3 and 0.2 <= ratio <= 5 are hit exactly: kept; one ulp past: fallback."""
    p = [[3.0, 9.0], [3.0, 1.0]]
    for gv, lo, hi in (([[2.0, 0.0], [0.0, 0.0]], 0.2, 5.0), ([[50.0, 0.0], [0.0, 0.0]], 0.2, 5.0)):
        pred0, sc, g = _guard_case(p, gv)
        out, keep = U.guard(pred0, sc, g, 0.3, lo, hi)
        assert keep[0] and np.array_equal(out[0], p)
        # one ulp stricter in each threshold that is active: the plain gradient comes back
        ratio = 10.0 / np.abs(g).max()
        strict = [(np.nextafter(0.3, 1.0), lo, hi)]
        if ratio == hi:
            strict.append((0.3, lo, np.nextafter(hi, 0.0)))
        else:
            strict.append((0.3, np.nextafter(lo, 1.0), hi))
        for c, l, h in strict:
            out, keep = U.guard(pred0, sc, g, c, l, h)
            assert not keep[0] and np.array_equal(out[0], g[0])


def test_guard_zero_norms_fall_back():
    p = [[3.0, 9.0], [3.0, 1.0]]
    # zero plain gradient: the network output is never kept (the ratio is undefined)
    pred0, sc, g = _guard_case(p, [[0.0, 0.0], [0.0, 0.0]])
    out, keep = U.guard(pred0, sc, g, -1.0, 0.0, np.inf)
    assert not keep[0] and not out.any()
    # zero network output: fall back to g even with the loosest thresholds
    pred0, sc, g = _guard_case([[0.0, 0.0], [0.0, 0.0]], [[1.0, 2.0], [3.0, 4.0]])
    out, keep = U.guard(pred0, sc, g, -1.0, 0.0, np.inf)
    assert not keep[0] and np.array_equal(out[0], g[0])


def test_guard_blend_weight():
    """A kept image with blend weight alpha is g + alpha (p - g): p = (3, 9; 3, 1), g =
    (2, 0; 0, 0) (cos 0.3, ratio 5: kept) gives (2.25, 2.25; 0.75, 0.25) at alpha = 1/4,
    g itself at alpha = 0 and p at alpha = 1; a rejected image stays g at any alpha."""
    p = [[3.0, 9.0], [3.0, 1.0]]
    pred0, sc, g = _guard_case(p, [[2.0, 0.0], [0.0, 0.0]])
    out, keep = U.guard(pred0, sc, g, 0.3, 0.2, 5.0, alpha=0.25)
    assert keep[0] and np.array_equal(out[0], [[2.25, 2.25], [0.75, 0.25]])
    out, _ = U.guard(pred0, sc, g, 0.3, 0.2, 5.0, alpha=0.0)
    assert np.array_equal(out[0], g[0])
    out, _ = U.guard(pred0, sc, g, 0.3, 0.2, 5.0, alpha=1.0)
    assert np.array_equal(out[0], p)
    out, keep = U.guard(pred0, sc, g, np.nextafter(0.3, 1.0), 0.2, 5.0, alpha=0.25)
    assert not keep[0] and np.array_equal(out[0], g[0])


def test_guard_per_image_decision_and_scale():
    """Two images in one call, one kept and one rejected (cosine -0.3 < 0), each decided on
    its own; the kept output is scale * pred0."""
    p0 = np.array([[3.0, 9.0], [3.0, 1.0]])
    g = np.array([[[2.0, 0.0], [0.0, 0.0]], [[-2.0, 0.0], [0.0, 0.0]]])
    pred0 = np.full((2, 4, 2), -3.0)
    pred0[:, :2] = p0 / 8.0
    out, keep = U.guard(pred0, np.array([8.0, 8.0]), g, 0.0, 0.2, 5.0)
    assert list(keep) == [True, False]
    assert np.array_equal(out[0], p0) and np.array_equal(out[1], g[1])
