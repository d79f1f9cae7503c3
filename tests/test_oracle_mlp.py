"""Pins of the oracle MLP: backward against central finite differences of the
loss, softmax-CE closed forms, Adam's first step."""
import numpy as np

from oracle import mlp as OM


def _data(rng, N=37):
    X = rng.standard_normal((N, OM.NIN)) * 3 + 1
    y = rng.integers(0, OM.NOUT, size=N)
    mu = X.mean(axis=0)
    sigma = X.std(axis=0) + 0.5
    return X, y, mu, sigma


def test_param_count():
    assert OM.NPARAM == 5443


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    X, y, mu, sigma = _data(rng)
    th = OM.init_params(rng)
    th[OM.NPARAM - 3:] = rng.standard_normal(3) * 0.1
    g = OM.backward(th, X, y, mu, sigma)
    h = 1e-6
    idx = rng.choice(OM.NPARAM, size=300, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (OM.loss(th + e, X, y, mu, sigma) - OM.loss(th - e, X, y, mu, sigma)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_uniform_logits_loss_is_log3():
    rng = np.random.default_rng(1)
    X, y, mu, sigma = _data(rng)
    th = np.zeros(OM.NPARAM)
    assert abs(OM.loss(th, X, y, mu, sigma) - np.log(3)) < 1e-15
    g = OM.backward(th, X, y, mu, sigma)
    # only b3 has a gradient: mean(softmax - onehot) = 1/3 - class frequency
    gb3 = g[-3:]
    freq = np.bincount(y, minlength=3) / len(y)
    np.testing.assert_allclose(gb3, 1 / 3 - freq, atol=1e-15)
    assert np.all(g[:-3] == 0)


def test_adam_first_step_is_sign_times_lr():
    rng = np.random.default_rng(2)
    th = rng.standard_normal(OM.NPARAM)
    g = rng.standard_normal(OM.NPARAM)
    th1, m, v = OM.adam_step(th, g, np.zeros_like(th), np.zeros_like(th), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(th1, th - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
