"""Pins of the FP64 learned-stage oracle (CPU only): closed forms of the
activation, finite-difference gradients, the first Adam step, and planted
mistakes in the backward pass."""
import math

import numpy as np
import pytest

import oracle.fcc_oracle as O
import oracle.mlp_oracle as N


def test_gelu_closed_forms():
    assert N.gelu(0.0) == 0.0
    assert abs(N.gelu_grad(0.0) - 0.5) < 1e-15
    assert abs(N.gelu(10.0) - 10.0) < 1e-12 and abs(N.gelu(-10.0)) < 1e-12
    # the tanh form stays within 1e-3 of x Phi(x), the exact definition
    for x in np.linspace(-6, 6, 61):
        exact = 0.5 * x * (1.0 + math.erf(x / math.sqrt(2.0)))
        assert abs(N.gelu(x) - exact) < 1e-3


def test_gelu_grad_finite_difference():
    x = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (N.gelu(x + h) - N.gelu(x - h)) / (2 * h)
    assert np.abs(fd - N.gelu_grad(x)).max() < 1e-8


def _fd_check(loss_grad, theta, coef, delta, hidden, idx, h=1e-6):
    _, g = loss_grad(theta, coef, delta, hidden)
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (N.loss_and_grad(tp, coef, delta, hidden)[0] - N.loss_and_grad(tm, coef, delta, hidden)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def _case(seed=0, in_dim=10, hidden=16, R=40):
    rng = np.random.default_rng(seed)
    theta = N.init_params(in_dim, hidden, seed) + 0.01 * rng.standard_normal(N.num_params(in_dim, hidden))
    coef = rng.standard_normal((R, in_dim)) * rng.uniform(0.1, 50.0, size=(R, 1))
    delta = rng.uniform(-4, 4, R)
    return theta, coef, delta


def test_loss_grad_finite_difference():
    theta, coef, delta, hidden = *_case(), 16
    idx = np.random.default_rng(1).choice(theta.size, 60, replace=False)
    idx = np.concatenate([idx, [theta.size - 1, theta.size - 2, 0, 10 * 16]])
    _fd_check(N.loss_and_grad, theta, coef, delta, hidden, idx)


def test_loss_closed_form_and_clip():
    # with every weight zero, mu = b3[0] and s = b3[1] for every row
    in_dim, hidden = 4, 8
    theta = np.zeros(N.num_params(in_dim, hidden))
    theta[-2], theta[-1] = 0.5, 1.0
    coef = np.ones((3, in_dim))
    delta = np.array([0.0, 1.0, -1.0])
    L, g = N.loss_and_grad(theta, coef, delta, hidden)
    e = 0.5 - delta
    assert abs(L - np.mean(0.5 * (np.exp(-1.0) * e * e + 1.0))) < 1e-15
    assert abs(g[-2] - np.mean(np.exp(-1.0) * e)) < 1e-15
    # clipped log-variance passes no gradient
    theta[-1] = 20.0
    _, g = N.loss_and_grad(theta, coef, delta, hidden)
    assert g[-1] == 0.0


def test_features_scale_free():
    rng = np.random.default_rng(3)
    c = rng.standard_normal((5, 6))
    u = N.features(c)
    assert np.allclose((u * u).sum(1), 1.0)
    assert np.allclose(N.features(7.5 * c), u)
    assert np.all(N.features(np.zeros((2, 6))) == 0)


def test_adam_first_step():
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    t1, m, v = N.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.1, eps=1e-12)
    # bias-corrected moments equal g and g^2, so each step is lr * sign(g)
    assert np.allclose(t1, theta - 0.1 * np.sign(g), atol=1e-9)


def test_parabolic_lag_from_corr():
    tau = np.arange(-4, 5)
    for vertex in (-2.3, 0.0, 0.4, 3.2):
        y = 10.0 - (tau - vertex) ** 2
        assert abs(O.tdoa_parabolic_from_corr(y[None], 4)[0] - vertex) < 1e-12
    y = -np.abs(tau - 4.0)          # peak at the window edge: no refinement
    assert O.tdoa_parabolic_from_corr(y[None], 4)[0] == 4.0


# --------------------------------------------------------- planted mistakes --

def _bad_no_gelu_grad(theta, coef, delta, hidden):
    orig = N.gelu_grad
    try:
        N.gelu_grad = lambda x: np.ones_like(np.asarray(x, dtype=np.float64))
        return N.loss_and_grad(theta, coef, delta, hidden)
    finally:
        N.gelu_grad = orig


def _bad_transposed_w2(theta, coef, delta, hidden):
    L, g = N.loss_and_grad(theta, coef, delta, hidden)
    in_dim = coef.shape[1]
    o = in_dim * hidden + hidden
    gw2 = g[o:o + hidden * hidden].reshape(hidden, hidden).T.copy()
    g = g.copy()
    g[o:o + hidden * hidden] = gw2.ravel()
    return L, g


@pytest.mark.parametrize("bad", [_bad_no_gelu_grad, _bad_transposed_w2])
def test_planted_backward_mistake_is_caught(bad):
    theta, coef, delta = _case(5)
    idx = np.arange(theta.size)
    with pytest.raises(AssertionError):
        _fd_check(bad, theta, coef, delta, 16, idx)
