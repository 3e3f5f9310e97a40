"""Pins for the oracle's LeNet-5 network (the Table 1 study's MNIST model, Section 4): the
parameter count the paper gives, the convolutions against a library correlation, and the
log-likelihood and hand-written gradient against an independent PyTorch float64 network
with autograd (CPU only)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn
from scipy.signal import correlate2d

from oracle import lenet


def test_lenet5_has_the_papers_parameter_count():
    sh = lenet.LeNetShape(*lenet.LENET5_MNIST)
    assert sh.D == 61706
    assert sh.F == 400 and (sh.H2, sh.Hq) == (10, 5)


def test_shape_checks():
    with pytest.raises(ValueError):
        lenet.LeNetShape(28, 28, 1, 4, 6, 16, 120, 84, 10)   # even kernel
    assert lenet.LeNetShape(12, 12, 1, 5, 2, 3, 8, 8, 3).F == 3   # second convolution 2 x 2, pooled 1 x 1
    with pytest.raises(ValueError):
        lenet.LeNetShape(10, 10, 1, 5, 2, 3, 8, 8, 3)        # second convolution 1 x 1
    with pytest.raises(ValueError):
        lenet.LeNetShape(14, 14, 1, 5, 2, 3, 8, 8, 3)        # second convolution 3 x 3


def test_convolution_against_a_library_correlation():
    rng = np.random.default_rng(0)
    n, H, W, cin, cout, k = 2, 7, 6, 3, 4, 3
    a = rng.standard_normal((n, H + k - 1, W + k - 1, cin))
    w = rng.standard_normal((cout, k * k * cin))
    b = rng.standard_normal(cout)
    z = lenet._conv(a, w, b, k, H, W)
    wk = w.reshape(cout, k, k, cin)
    for i in range(n):
        for o in range(cout):
            ref = b[o] + sum(correlate2d(a[i, :, :, c], wk[o, :, :, c], mode="valid") for c in range(cin))
            np.testing.assert_allclose(z[i, :, :, o], ref, rtol=1e-12, atol=1e-12)


def _torch_net(theta_j, X, y, sh, act):
    """The same network written with torch's float64 CPU layers; returns (LL, grad) by autograd."""
    t = torch.tensor(theta_j, dtype=torch.float64, requires_grad=True)
    blocks, off = [], 0
    for o, i in sh.blocks:
        blk = t[off:off + o * (i + 1)].reshape(o, i + 1)
        blocks.append((blk[:, :i], blk[:, i]))
        off += o * (i + 1)
    f_act = torch.tanh if act == "tanh" else torch.relu
    k = sh.k
    x = torch.tensor(X, dtype=torch.float64).reshape(-1, sh.H, sh.W, sh.Cin).permute(0, 3, 1, 2)
    (w1, b1), (w2, b2), (w3, b3), (w4, b4), (w5, b5) = blocks
    # weight index (ky k + kx) cin + c  ->  torch's [out, cin, ky, kx]
    k1 = w1.reshape(sh.C1, k, k, sh.Cin).permute(0, 3, 1, 2)
    k2 = w2.reshape(sh.C2, k, k, sh.C1).permute(0, 3, 1, 2)
    a = Fn.avg_pool2d(f_act(Fn.conv2d(x, k1, b1, padding=sh.pad)), 2)
    a = Fn.avg_pool2d(f_act(Fn.conv2d(a, k2, b2)), 2)
    f = a.permute(0, 2, 3, 1).reshape(a.shape[0], -1)  # features in (py, px, c) order
    h = f_act(Fn.linear(f, w3, b3))
    h = f_act(Fn.linear(h, w4, b4))
    lp = Fn.log_softmax(Fn.linear(h, w5, b5), dim=1)
    ll = lp[torch.arange(len(y)), torch.tensor(y)].sum()
    ll.backward()
    return ll.item(), t.grad.numpy()


@pytest.mark.parametrize("shape,act", [
    ((12, 12, 1, 5, 3, 4, 8, 6, 3), "tanh"),
    ((8, 12, 2, 3, 4, 3, 5, 7, 4), "relu"),
    ((16, 12, 1, 5, 2, 3, 6, 5, 10), "tanh"),
])
def test_loglik_and_gradient_against_torch_autograd(shape, act):
    sh = lenet.LeNetShape(*shape)
    rng = np.random.default_rng(sum(shape))
    J, n = 3, 5
    theta = 0.4 * rng.standard_normal((J, sh.D))
    X = rng.uniform(0, 1, (n, sh.H * sh.W * sh.Cin))
    y = rng.integers(0, sh.n_cls, n)
    scale = np.array([1.0, 0.5, 2.0])
    ll, g = lenet.loglik_grad(theta, X, y, sh, act, scale)
    np.testing.assert_allclose(ll, lenet.loglik(theta, X, y, sh, act), rtol=1e-13)
    for j in range(J):
        ll_t, g_t = _torch_net(theta[j], X, y, sh, act)
        assert abs(ll[j] - ll_t) <= 1e-12 * abs(ll_t)
        np.testing.assert_allclose(g[j], scale[j] * g_t, rtol=1e-10, atol=1e-12)


def test_lenet5_gradient_against_central_differences():
    sh = lenet.LeNetShape(*lenet.LENET5_MNIST)
    rng = np.random.default_rng(5)
    theta = 0.1 * rng.standard_normal((2, sh.D))
    X = rng.uniform(0, 1, (3, 784))
    y = np.array([1, 7, 3])
    v = rng.standard_normal(theta.shape)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    _, g = lenet.loglik_grad(theta, X, y, sh)
    eps = 1e-5
    fd = (lenet.loglik(theta + eps * v, X, y, sh) - lenet.loglik(theta - eps * v, X, y, sh)) / (2 * eps)
    np.testing.assert_allclose(fd, np.sum(g * v, axis=1), rtol=1e-7, atol=1e-9)


def test_predictive_probabilities_normalise_and_zero_weights_are_uniform():
    sh = lenet.LeNetShape(12, 12, 1, 5, 3, 4, 8, 6, 3)
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, (4, 144))
    lp = lenet.predict_logprobs(0.5 * rng.standard_normal((2, sh.D)), X, sh)
    np.testing.assert_allclose(np.exp(lp).sum(axis=2), 1.0, rtol=1e-13)
    lp0 = lenet.predict_logprobs(np.zeros((1, sh.D)), X, sh)
    np.testing.assert_allclose(lp0, np.log(1 / 3), rtol=1e-14)
