"""FP64 per-particle MLP likelihood and gradient (test infrastructure).

The sampler targets a neural-network posterior built from the network's
likelihood p(y | theta) and a prior q0 (Section 2).  The likelihood and its
gradient are evaluated on the current annealed subset y_{1:M_k} and scaled by
N/M_k to estimate the full-batch quantities (Section 3, Eq. approx-grad).  This
module computes the *unscaled* subset sums

    LL(theta)      = sum_{i < M} log p(y_i | x_i, theta)
    grad LL(theta) = sum_{i < M} d/dtheta log p(y_i | x_i, theta)

for a population of J parameter vectors at once.  Scaling by lambda = N/M_k
and the prior term are applied by the caller (oracle.smc).

Parameter layout (one particle, D values):  for each layer l = 1..L with
n_in inputs and n_out outputs, the block [W_l | b_l] of shape
[n_out x (n_in + 1)] stored row-major, i.e. each output unit's n_in weights
followed by its bias.  D = sum_l n_out * (n_in + 1).

Networks:  a_0 = x;  z_l = W_l a_{l-1} + b_l;  a_l = phi(z_l) for l < L;
the output layer is linear.  phi is tanh or ReLU (ReLU'(0) := 0).
Likelihoods:  categorical (softmax over the output layer; the paper's image
classification) or Gaussian N(y; z_L, sigma^2) with one output (used for the
closed-form Bayesian linear-regression check).
"""
from __future__ import annotations

import numpy as np

TANH = "tanh"
RELU = "relu"
CATEGORICAL = "categorical"
GAUSSIAN = "gaussian"


def layer_shapes(widths):
    """[(n_out, n_in), ...] for widths = [n_0, n_1, ..., n_L]."""
    return [(widths[i + 1], widths[i]) for i in range(len(widths) - 1)]


def n_params(widths) -> int:
    return sum(o * (i + 1) for (o, i) in layer_shapes(widths))


def unpack(theta: np.ndarray, widths):
    """Split theta [J x D] into per-layer (W [J x out x in], b [J x out]) views."""
    theta = np.asarray(theta, dtype=np.float64)
    out = []
    off = 0
    J = theta.shape[0]
    for (o, i) in layer_shapes(widths):
        blk = theta[:, off:off + o * (i + 1)].reshape(J, o, i + 1)
        out.append((blk[:, :, :i], blk[:, :, i]))
        off += o * (i + 1)
    assert off == theta.shape[1], "theta has the wrong length for these widths"
    return out


def _act(z, act):
    if act == TANH:
        return np.tanh(z)
    if act == RELU:
        return np.maximum(z, 0.0)
    raise ValueError(act)


def _act_grad(z, act):
    if act == TANH:
        t = np.tanh(z)
        return 1.0 - t * t
    if act == RELU:
        return (z > 0.0).astype(np.float64)
    raise ValueError(act)


def forward(theta, X, widths, act):
    """Pre-activations z_1..z_L, each [J x M x n_l], in FP64."""
    X = np.asarray(X, dtype=np.float64)
    params = unpack(theta, widths)
    a = X[None, :, :]  # shared input for every particle
    zs = []
    for l, (W, b) in enumerate(params):
        z = np.matmul(a, np.transpose(W, (0, 2, 1))) + b[:, None, :]
        zs.append(z)
        if l + 1 < len(params):
            a = _act(z, act)
    return zs


def log_softmax(z):
    m = np.max(z, axis=-1, keepdims=True)
    return z - (m + np.log(np.sum(np.exp(z - m), axis=-1, keepdims=True)))


def per_sample_loglik(theta, X, y, widths, act, likelihood=CATEGORICAL, noise_std=1.0):
    """log p(y_i | x_i, theta_j) as [J x M]."""
    zL = forward(theta, X, widths, act)[-1]
    if likelihood == CATEGORICAL:
        lp = log_softmax(zL)
        idx = np.asarray(y, dtype=np.int64)
        return np.take_along_axis(lp, idx[None, :, None].repeat(lp.shape[0], 0), axis=2)[:, :, 0]
    if likelihood == GAUSSIAN:
        r = np.asarray(y, dtype=np.float64)[None, :] - zL[:, :, 0]
        return -0.5 * np.log(2.0 * np.pi * noise_std ** 2) - r * r / (2.0 * noise_std ** 2)
    raise ValueError(likelihood)


def loglik(theta, X, y, widths, act, likelihood=CATEGORICAL, noise_std=1.0):
    """LL_j = sum_i log p(y_i | x_i, theta_j) over the given samples, [J]."""
    return per_sample_loglik(theta, X, y, widths, act, likelihood, noise_std).sum(axis=1)


def loglik_grad(theta, X, y, widths, act, likelihood=CATEGORICAL, noise_std=1.0, scale=None):
    """(LL [J], scale_j * grad LL_j [J x D]) by hand-written backpropagation.

    ``scale`` (per particle, default 1) multiplies the gradient only; the
    sampler passes lambda_k = N / M_k here (Section 3, Eq. approx-grad).
    """
    X = np.asarray(X, dtype=np.float64)
    params = unpack(theta, widths)
    J = theta.shape[0]
    L = len(params)
    # forward, keeping pre-activations and activations
    acts = [np.broadcast_to(X[None, :, :], (J,) + X.shape)]
    zs = []
    for l, (W, b) in enumerate(params):
        z = np.matmul(acts[-1], np.transpose(W, (0, 2, 1))) + b[:, None, :]
        zs.append(z)
        if l + 1 < L:
            acts.append(_act(z, act))
    zL = zs[-1]
    # output-layer error delta_L = d log p / d z_L
    if likelihood == CATEGORICAL:
        lp = log_softmax(zL)
        idx = np.asarray(y, dtype=np.int64)
        onehot = np.zeros_like(zL)
        onehot[:, np.arange(len(idx)), idx] = 1.0
        ll = np.sum(lp * onehot, axis=(1, 2))
        delta = onehot - np.exp(lp)
    elif likelihood == GAUSSIAN:
        r = np.asarray(y, dtype=np.float64)[None, :] - zL[:, :, 0]
        ll = np.sum(-0.5 * np.log(2.0 * np.pi * noise_std ** 2) - r * r / (2.0 * noise_std ** 2), axis=1)
        delta = (r / noise_std ** 2)[:, :, None]
    else:
        raise ValueError(likelihood)
    s = np.ones(J) if scale is None else np.asarray(scale, dtype=np.float64).reshape(J)
    delta = delta * s[:, None, None]
    grads = []
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        a_prev = acts[l]
        dW = np.matmul(np.transpose(delta, (0, 2, 1)), a_prev)  # [J x out x in]
        db = delta.sum(axis=1)                                  # [J x out]
        grads.append(np.concatenate([dW, db[:, :, None]], axis=2).reshape(J, -1))
        if l > 0:
            delta = np.matmul(delta, W) * _act_grad(zs[l - 1], act)
    grads.reverse()
    return ll, np.concatenate(grads, axis=1)


def predict_logprobs(theta, X, widths, act):
    """Per-particle class log-probabilities log softmax(f_theta(x)), [J x M x C]."""
    return log_softmax(forward(theta, X, widths, act)[-1])
