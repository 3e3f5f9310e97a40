"""Pins for the oracle's per-particle MLP likelihood and gradient (CPU only)."""
import math

import numpy as np
import pytest

from oracle import mlp
import smc_inputs


def _brute_loglik(theta_j, X, y, widths, act, likelihood="categorical", noise_std=1.0):
    """Per-sample log-likelihood by explicit Python loops and math.fsum (independent of numpy)."""
    shapes = mlp.layer_shapes(widths)
    total = []
    for i in range(X.shape[0]):
        a = [float(v) for v in X[i]]
        off = 0
        for l, (o, n_in) in enumerate(shapes):
            z = []
            for r in range(o):
                row = theta_j[off + r * (n_in + 1): off + (r + 1) * (n_in + 1)]
                z.append(math.fsum([float(row[c]) * a[c] for c in range(n_in)] + [float(row[n_in])]))
            off += o * (n_in + 1)
            if l + 1 < len(shapes):
                a = [math.tanh(v) if act == "tanh" else max(v, 0.0) for v in z]
            else:
                a = z
        if likelihood == "categorical":
            mx = max(a)
            lse = mx + math.log(math.fsum(math.exp(v - mx) for v in a))
            total.append(a[int(y[i])] - lse)
        else:
            r = float(y[i]) - a[0]
            total.append(-0.5 * math.log(2 * math.pi * noise_std ** 2) - r * r / (2 * noise_std ** 2))
    return math.fsum(total)


def _fd_grad(f, theta, idx, eps=1e-6):
    out = []
    for k in idx:
        tp = theta.copy(); tp[k] += eps
        tm = theta.copy(); tm[k] -= eps
        out.append((f(tp) - f(tm)) / (2 * eps))
    return np.array(out)


def test_layout_sizes():
    assert mlp.n_params([2, 16, 2]) == 82
    assert mlp.n_params([784, 100, 10]) == 79510
    assert mlp.n_params([784, 256, 256, 10]) == 269322


def test_zero_weights_closed_form():
    # all-zero weights: every class has probability 1/C, LL = -M log C
    X, y = smc_inputs.templates28(37, seed=3)
    theta = np.zeros((3, mlp.n_params([784, 8, 10])))
    ll = mlp.loglik(theta, X, y, [784, 8, 10], "relu")
    np.testing.assert_allclose(ll, -37 * math.log(10), rtol=1e-14)


@pytest.mark.parametrize("widths,act", [([2, 16, 2], "tanh"), ([5, 4, 3, 4], "relu"), ([3, 6, 5, 3], "tanh")])
def test_forward_matches_brute_force(widths, act):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((9, widths[0]))
    y = rng.integers(0, widths[-1], 9)
    theta = rng.standard_normal((3, mlp.n_params(widths)))
    ll = mlp.loglik(theta, X, y, widths, act)
    for j in range(3):
        assert abs(ll[j] - _brute_loglik(theta[j], X, y, widths, act)) < 1e-11 * max(1.0, abs(ll[j]))


def test_gaussian_linear_matches_brute_force():
    X, y, _ = smc_inputs.linreg(11, 3, seed=2)
    theta = np.random.default_rng(0).standard_normal((2, 4))
    ll = mlp.loglik(theta, X, y, [3, 1], "relu", "gaussian", noise_std=0.7)
    for j in range(2):
        assert abs(ll[j] - _brute_loglik(theta[j], X, y, [3, 1], "relu", "gaussian", 0.7)) < 1e-11 * abs(ll[j])


@pytest.mark.parametrize("widths,act,lik", [
    ([2, 16, 2], "tanh", "categorical"),
    ([6, 5, 4, 3], "relu", "categorical"),
    ([3, 1], "relu", "gaussian"),
    ([4, 7, 1], "tanh", "gaussian"),
])
def test_gradient_matches_finite_differences(widths, act, lik):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((13, widths[0]))
    y = rng.integers(0, widths[-1], 13) if lik == "categorical" else rng.standard_normal(13)
    theta = 0.7 * rng.standard_normal((2, mlp.n_params(widths)))
    scale = np.array([1.0, 2.5])
    ll, g = mlp.loglik_grad(theta, X, y, widths, act, lik, 0.8, scale=scale)
    np.testing.assert_allclose(ll, mlp.loglik(theta, X, y, widths, act, lik, 0.8), rtol=1e-13)
    for j in range(2):
        f = lambda t: mlp.loglik(t[None, :], X, y, widths, act, lik, 0.8)[0]
        idx = np.arange(theta.shape[1])
        fd = _fd_grad(f, theta[j].copy(), idx) * scale[j]
        np.testing.assert_allclose(g[j], fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(fd)))


def test_gradient_fd_mnist_shaped():
    X, y = smc_inputs.templates28(20, seed=5)
    widths = [784, 8, 10]
    theta = 0.1 * np.random.default_rng(3).standard_normal((1, mlp.n_params(widths)))
    ll, g = mlp.loglik_grad(theta, X, y, widths, "relu")
    idx = np.random.default_rng(4).choice(theta.shape[1], 40, replace=False)
    f = lambda t: mlp.loglik(t[None, :], X, y, widths, "relu")[0]
    fd = _fd_grad(f, theta[0].copy(), idx)
    np.testing.assert_allclose(g[0, idx], fd, rtol=1e-5, atol=1e-6 * np.max(np.abs(fd)))


def test_relu_derivative_at_zero_is_zero():
    # ReLU'(0) := 0: a hidden unit with exactly zero pre-activation passes no gradient
    widths = [1, 1, 2]
    theta = np.array([[0.0, 0.0, 1.0, 0.0, -1.0, 0.0]])  # W1 = 0, b1 = 0 -> z1 = 0
    ll, g = mlp.loglik_grad(theta, np.array([[2.0]]), np.array([0]), widths, "relu")
    assert g[0, 0] == 0.0 and g[0, 1] == 0.0
