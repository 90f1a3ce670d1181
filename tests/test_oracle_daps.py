"""CPU pins of the diffusion outer-loop oracle (oracle/daps.py) against what the
mathematics fixes: the DDPM posterior derived independently by Gaussian conditioning, the
marginal it must reproduce, its t = 1 limit, and the noise stream's construction."""
import numpy as np
import pytest

import oracle
from oracle import daps as D

T, B1, BT = 1000, 1e-4, 0.02


def test_schedule():
    beta, alpha = D.linear_schedule(T, B1, BT)
    assert alpha[0] == 1.0 and beta[1] == B1 and abs(beta[T] - BT) < 1e-18
    assert np.all(np.diff(alpha) < 0) and np.all(alpha > 0)
    # alpha_t / alpha_{t-1} = 1 - beta_t
    assert np.allclose(alpha[1:] / alpha[:-1], 1.0 - beta[1:], rtol=1e-14, atol=0)


def test_posterior_equals_gaussian_conditioning():
    # Bayes' rule on q(x_t | x_{t-1}) = N(sqrt(1 - beta_t) x_{t-1}, beta_t) and
    # q(x_{t-1} | x_0) = N(sqrt(alpha_{t-1}) x_0, 1 - alpha_{t-1}): the posterior precision is
    # the sum of the two precisions (the first seen as a function of x_{t-1}), the mean the
    # precision-weighted combination -- a different route from the closed form
    beta, alpha = D.linear_schedule(T, B1, BT)
    for t in range(2, T + 1):
        bt, atm1 = beta[t], alpha[t - 1]
        prec = 1.0 / (1.0 - atm1) + (1.0 - bt) / bt
        var = 1.0 / prec
        ref = (np.sqrt(atm1) / (1.0 - atm1) * var, np.sqrt(1.0 - bt) / bt * var, var)
        got = D.posterior(beta, alpha, t)
        for g, r in zip(got, ref):
            assert abs(g - r) <= 1e-12 * abs(r), (t, got, ref)


def test_renoise_preserves_the_forward_marginal():
    # x_t ~ q(x_t | x_0) followed by the re-noise draw with the true x_0 must give
    # x_{t-1} ~ q(x_{t-1} | x_0) = N(sqrt(alpha_{t-1}) x_0, 1 - alpha_{t-1}): exactly in the
    # coefficients, and in the sample moments of draws from the counter-based stream
    beta, alpha = D.linear_schedule(T, B1, BT)
    for t in (2, 10, 100, 500, T):
        c0, c1, bt = D.posterior(beta, alpha, t)
        # (FP64 rounding grows as eps / (1 - alpha_t): 1 - alpha_2 is 3e-4)
        assert abs(c0 + c1 * np.sqrt(alpha[t]) - np.sqrt(alpha[t - 1])) < 1e-11
        assert abs(c1 ** 2 * (1.0 - alpha[t]) + bt - (1.0 - alpha[t - 1])) < 1e-11
    t = 50
    c0, c1, bt = D.posterior(beta, alpha, t)
    n = 400_000
    x0 = np.full((1, n), 0.37)
    lo, hi = 1500.0, 5500.0
    z = D.to_model(x0, lo, hi)  # physical model whose normalised value is x0
    xt = D.mix(z, None, [np.sqrt(alpha[t])], [0.0], [np.sqrt(1 - alpha[t])], lo, hi, seed=3, step=0)
    xtm1 = D.mix(z, xt, [c0], [c1], [np.sqrt(bt)], lo, hi, seed=3, step=1)[0]
    mean, var = xtm1.mean(), xtm1.var()
    se = np.sqrt((1 - alpha[t - 1]) / n)
    assert abs(mean - np.sqrt(alpha[t - 1]) * 0.37) < 5 * se
    assert abs(var / (1 - alpha[t - 1]) - 1) < 5 * np.sqrt(2.0 / n)


def test_first_level_returns_the_clean_model():
    # alpha_0 = 1: the last re-noise (t = 1) is deterministic and lands on x_0
    beta, alpha = D.linear_schedule(T, B1, BT)
    c0, c1, bt = D.posterior(beta, alpha, 1)
    assert abs(c0 - 1.0) < 1e-12 and c1 == 0.0 and bt == 0.0


def test_noise_stream_construction():
    # the same Philox / Box-Muller construction as the Langevin noise, with its own key
    assert np.array_equal(oracle.normals_key(11, 0x4C414E47, 4, 2, 37), oracle.normals(11, 4, 2, 37))
    a = oracle.normals_key(11, D.DAPS_TAG, 4, 2, 200_001)
    assert abs(a.mean()) < 0.01 and abs(a.var() - 1) < 0.01
    assert not np.array_equal(a[:37], oracle.normals(11, 4, 2, 37))


def test_normalisation():
    lo, hi = 1500.0, 5500.0
    v = np.linspace(lo, hi, 101)
    x = D.normalise(v, lo, hi)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.allclose(D.to_model(x, lo, hi), v, rtol=0, atol=1e-9)
    assert D.to_model(np.array([-1.5, 1.5]), lo, hi).tolist() == [lo, hi]


@pytest.mark.parametrize("hp", [7, 9])
def test_prep_layout(hp):
    x = np.arange(2 * 7 * 3, dtype=np.float64).reshape(2, 7, 3)
    ch0, ch1, res = D.prep(x, [0.5, 0.25], hp)
    assert ch0.shape == (2, hp, 3) and np.array_equal(ch0[:, :7], x) and np.all(ch0[:, 7:] == 0)
    assert np.all(ch1[0, :7] == 0.5) and np.all(ch1[1, :7] == 0.25) and np.all(ch1[:, 7:] == 0)
    assert np.array_equal(res, ch0)
