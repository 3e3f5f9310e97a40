"""FP64 per-particle convolutional network likelihood and gradient (test infrastructure).

The paper's image classifiers are convolutional networks whose weights are the
SMC particles (Section 4); the sampler needs, per particle, the log-likelihood
of the current annealed subset and its gradient (Section 3, Eq. approx-grad).
This module computes the unscaled subset sums for the network

    conv3x3(C1) -> ReLU -> conv3x3(C2) -> ReLU -> 2x2 average pool -> linear (n_cls)

on images of H x W pixels with Cin channels, stored channel-last (NHWC, one
sample per row of H*W*Cin values).  Convolutions use "same" zero padding and
stride 1; H and W are even.

Parameter layout (one particle), three blocks [W | b] as for the dense
networks, each output unit's weights followed by its bias:
  conv1  [C1 x (9 Cin + 1)]      weight index (ky * 3 + kx) * Cin + c
  conv2  [C2 x (9 C1 + 1)]       weight index (ky * 3 + kx) * C1 + c
  linear [n_cls x (Hp Wp C2 + 1)] input index (py * Wp + px) * C2 + c,  Hp = H/2, Wp = W/2
Output pixel (y, x) of a convolution reads input pixel (y + ky - 1, x + kx - 1).
The likelihood is categorical (softmax over the linear layer's outputs).
"""
from __future__ import annotations

import numpy as np


class CNNShape:
    def __init__(self, H, W, Cin, C1, C2, n_cls):
        if H % 2 or W % 2:
            raise ValueError("H and W must be even")
        self.H, self.W, self.Cin, self.C1, self.C2, self.n_cls = H, W, Cin, C1, C2, n_cls
        self.Hp, self.Wp = H // 2, W // 2
        self.F3 = self.Hp * self.Wp * C2
        self.blocks = [(C1, 9 * Cin), (C2, 9 * C1), (n_cls, self.F3)]
        self.D = sum(o * (i + 1) for o, i in self.blocks)


def unpack(theta, sh: CNNShape):
    """[(W [J x out x in], b [J x out])] for conv1, conv2, linear."""
    theta = np.asarray(theta, dtype=np.float64)
    J = theta.shape[0]
    out, off = [], 0
    for o, i in sh.blocks:
        blk = theta[:, off:off + o * (i + 1)].reshape(J, o, i + 1)
        out.append((blk[:, :, :i], blk[:, :, i]))
        off += o * (i + 1)
    assert off == theta.shape[1], "theta has the wrong length for this network"
    return out


def _pad(a):
    return np.pad(a, ((0, 0), (1, 1), (1, 1), (0, 0)))


def _conv(a, w, b, cin):
    """'same' 3x3 convolution of a [n x H x W x cin] with w [out x 9 cin] (tap-major), bias b [out]."""
    n, H, W, _ = a.shape
    p = _pad(a)
    z = np.broadcast_to(b, (n, H, W, b.shape[0])).copy()
    for ky in range(3):
        for kx in range(3):
            t = ky * 3 + kx
            z += p[:, ky:ky + H, kx:kx + W, :] @ w[:, t * cin:(t + 1) * cin].T
    return z


def _pool(a):
    n, H, W, c = a.shape
    return a.reshape(n, H // 2, 2, W // 2, 2, c).mean(axis=(2, 4))


def _forward_one(Wb, X, sh):
    (w1, b1), (w2, b2), (w3, b3) = Wb
    x = np.asarray(X, dtype=np.float64).reshape(-1, sh.H, sh.W, sh.Cin)
    z1 = _conv(x, w1, b1, sh.Cin)
    a1 = np.maximum(z1, 0.0)
    z2 = _conv(a1, w2, b2, sh.C1)
    a2 = np.maximum(z2, 0.0)
    pooled = _pool(a2).reshape(x.shape[0], -1)
    logits = pooled @ w3.T + b3
    return x, z1, a1, z2, pooled, logits


def _log_softmax(z):
    m = np.max(z, axis=1, keepdims=True)
    return z - m - np.log(np.sum(np.exp(z - m), axis=1, keepdims=True))


def predict_logprobs(theta, X, sh: CNNShape):
    """log softmax of every particle's outputs, [J x n x n_cls]."""
    params = unpack(theta, sh)
    J = params[0][0].shape[0]
    return np.stack([_log_softmax(_forward_one([(w[j], b[j]) for w, b in params], X, sh)[-1])
                     for j in range(J)])


def loglik(theta, X, y, sh: CNNShape):
    y = np.asarray(y, dtype=np.int64)
    lp = predict_logprobs(theta, X, sh)
    return lp[:, np.arange(len(y)), y].sum(axis=1)


def loglik_grad(theta, X, y, sh: CNNShape, scale=None):
    """(LL [J], scale_j * grad LL [J x D]) on the samples (X, y), by hand-written backpropagation."""
    y = np.asarray(y, dtype=np.int64)
    params = unpack(theta, sh)
    J = params[0][0].shape[0]
    scale = np.ones(J) if scale is None else np.asarray(scale, dtype=np.float64)
    lls, grads = [], []
    for j in range(J):
        (w1, b1), (w2, b2), (w3, b3) = [(w[j], b[j]) for w, b in params]
        x, z1, a1, z2, pooled, logits = _forward_one([(w1, b1), (w2, b2), (w3, b3)], X, sh)
        n = x.shape[0]
        lp = _log_softmax(logits)
        lls.append(lp[np.arange(n), y].sum())
        d3 = -np.exp(lp)
        d3[np.arange(n), y] += 1.0                                  # d LL / d logits
        gW3, gb3 = d3.T @ pooled, d3.sum(axis=0)
        dpool = (d3 @ w3).reshape(n, sh.Hp, sh.Wp, sh.C2)
        da2 = np.repeat(np.repeat(dpool, 2, axis=1), 2, axis=2) / 4.0
        dz2 = da2 * (z2 > 0.0)
        p1 = _pad(a1)
        gW2 = np.zeros_like(w2)
        dp1 = np.zeros_like(p1)
        for ky in range(3):
            for kx in range(3):
                t = ky * 3 + kx
                sl = (slice(None), slice(ky, ky + sh.H), slice(kx, kx + sh.W), slice(None))
                gW2[:, t * sh.C1:(t + 1) * sh.C1] = np.einsum("nyxo,nyxc->oc", dz2, p1[sl])
                dp1[sl] += dz2 @ w2[:, t * sh.C1:(t + 1) * sh.C1]
        gb2 = dz2.sum(axis=(0, 1, 2))
        dz1 = dp1[:, 1:sh.H + 1, 1:sh.W + 1, :] * (z1 > 0.0)
        p0 = _pad(x)
        gW1 = np.zeros_like(w1)
        for ky in range(3):
            for kx in range(3):
                t = ky * 3 + kx
                gW1[:, t * sh.Cin:(t + 1) * sh.Cin] = np.einsum(
                    "nyxo,nyxc->oc", dz1, p0[:, ky:ky + sh.H, kx:kx + sh.W, :])
        gb1 = dz1.sum(axis=(0, 1, 2))
        g = np.concatenate([np.concatenate([gW1, gb1[:, None]], 1).ravel(),
                            np.concatenate([gW2, gb2[:, None]], 1).ravel(),
                            np.concatenate([gW3, gb3[:, None]], 1).ravel()])
        grads.append(scale[j] * g)
    return np.asarray(lls), np.stack(grads)


class Model:
    """Adapter with the interface the oracle sampler uses for its network."""

    def __init__(self, sh: CNNShape):
        self.sh = sh
        self.D = sh.D

    def loglik_grad(self, theta, X, y, scale):
        return loglik_grad(theta, X, y, self.sh, scale)

    def predict_logprobs(self, theta, X):
        return predict_logprobs(theta, X, self.sh)
