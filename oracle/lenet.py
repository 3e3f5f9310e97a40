"""FP64 per-particle LeNet-5 likelihood and gradient (test infrastructure).

The paper's MNIST study trains a LeNet-5 network (Section 4, the Table 1 study: tanh
activations, D = 61,706 parameters) whose weights are the SMC particles; the sampler
needs, per particle, the log-likelihood of the current subset and its gradient
(Section 3, Eq. approx-grad).  This module computes the unscaled subset sums for

    conv kxk "same" (C1) -> act -> 2x2 average pool -> conv kxk "valid" (C2) -> act
    -> 2x2 average pool -> dense (F1) -> act -> dense (F2) -> act -> dense (n_cls)

on images of H x W pixels with Cin channels stored channel-last (NHWC, one sample per
row of H*W*Cin values), stride 1, zero padding (k - 1) / 2 on the first convolution and
none on the second.  With (H, W, Cin, k, C1, C2, F1, F2, n_cls) = (28, 28, 1, 5, 6, 16,
120, 84, 10) this is LeNet-5 with D = 61,706 (the count the paper gives; parameter-free
average pooling and the padded first convolution are what reproduce it).

Parameter layout (one particle), five blocks [W | b], each output unit's weights followed
by its bias:
  conv1  [C1 x (k k Cin + 1)]   weight index (ky * k + kx) * Cin + c
  conv2  [C2 x (k k C1 + 1)]    weight index (ky * k + kx) * C1 + c
  dense1 [F1 x (F + 1)]         input index (py * Wq + px) * C2 + c, F = Hq Wq C2
  dense2 [F2 x (F1 + 1)]
  output [n_cls x (F2 + 1)]
Output pixel (y, x) of the first convolution reads input pixel (y + ky - p, x + kx - p),
p = (k - 1) / 2; of the second, pooled pixel (y + ky, x + kx).  The likelihood is
categorical (softmax over the output layer).
"""
from __future__ import annotations

import numpy as np


class LeNetShape:
    def __init__(self, H, W, Cin, k, C1, C2, F1, F2, n_cls):
        if k < 1 or k % 2 == 0:
            raise ValueError("k must be odd")
        if H % 2 or W % 2:
            raise ValueError("H and W must be even")
        self.H, self.W, self.Cin, self.k = H, W, Cin, k
        self.C1, self.C2, self.F1, self.F2, self.n_cls = C1, C2, F1, F2, n_cls
        self.pad = (k - 1) // 2
        self.Hp, self.Wp = H // 2, W // 2                    # after the first pooling
        self.H2, self.W2 = self.Hp - k + 1, self.Wp - k + 1  # second convolution
        if self.H2 < 2 or self.W2 < 2 or self.H2 % 2 or self.W2 % 2:
            raise ValueError("the second convolution's output must be even and at least 2 x 2")
        self.Hq, self.Wq = self.H2 // 2, self.W2 // 2
        self.F = self.Hq * self.Wq * C2
        self.blocks = [(C1, k * k * Cin), (C2, k * k * C1), (F1, self.F), (F2, F1), (n_cls, F2)]
        self.D = sum(o * (i + 1) for o, i in self.blocks)


LENET5_MNIST = (28, 28, 1, 5, 6, 16, 120, 84, 10)


def unpack(theta, sh: LeNetShape):
    """[(W [J x out x in], b [J x out])] for the five layers."""
    theta = np.asarray(theta, dtype=np.float64)
    J = theta.shape[0]
    out, off = [], 0
    for o, i in sh.blocks:
        blk = theta[:, off:off + o * (i + 1)].reshape(J, o, i + 1)
        out.append((blk[:, :, :i], blk[:, :, i]))
        off += o * (i + 1)
    assert off == theta.shape[1], "theta has the wrong length for this network"
    return out


def _act(z, act):
    return np.tanh(z) if act == "tanh" else np.maximum(z, 0.0)


def _act_grad(a, act):
    """derivative of the activation, from its output"""
    return 1.0 - a * a if act == "tanh" else (a > 0.0).astype(np.float64)


def _conv(a, w, b, k, Ho, Wo):
    """correlation of a [n x Hi x Wi x cin] (already padded) with w [out x k k cin], output
    [n x Ho x Wo x out]: z[y, x] = b + sum_taps a[y + ky, x + kx] . w[tap]"""
    cin = a.shape[3]
    z = np.broadcast_to(b, (a.shape[0], Ho, Wo, b.shape[0])).copy()
    for ky in range(k):
        for kx in range(k):
            t = ky * k + kx
            z += a[:, ky:ky + Ho, kx:kx + Wo, :] @ w[:, t * cin:(t + 1) * cin].T
    return z


def _pool(a):
    n, H, W, c = a.shape
    return a.reshape(n, H // 2, 2, W // 2, 2, c).mean(axis=(2, 4))


def _unpool(d):
    """adjoint of the 2x2 average pool"""
    return np.repeat(np.repeat(d, 2, axis=1), 2, axis=2) / 4.0


def _forward_one(Wb, X, sh, act):
    (w1, b1), (w2, b2), (w3, b3), (w4, b4), (w5, b5) = Wb
    p = sh.pad
    x = np.asarray(X, dtype=np.float64).reshape(-1, sh.H, sh.W, sh.Cin)
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    a1 = _act(_conv(xp, w1, b1, sh.k, sh.H, sh.W), act)
    p1 = _pool(a1)
    a2 = _act(_conv(p1, w2, b2, sh.k, sh.H2, sh.W2), act)
    f = _pool(a2).reshape(x.shape[0], -1)
    h1 = _act(f @ w3.T + b3, act)
    h2 = _act(h1 @ w4.T + b4, act)
    logits = h2 @ w5.T + b5
    return xp, a1, p1, a2, f, h1, h2, logits


def _log_softmax(z):
    m = np.max(z, axis=1, keepdims=True)
    return z - m - np.log(np.sum(np.exp(z - m), axis=1, keepdims=True))


def predict_logprobs(theta, X, sh: LeNetShape, act="tanh"):
    """log softmax of every particle's outputs, [J x n x n_cls]."""
    params = unpack(theta, sh)
    J = params[0][0].shape[0]
    return np.stack([_log_softmax(_forward_one([(w[j], b[j]) for w, b in params], X, sh, act)[-1])
                     for j in range(J)])


def loglik(theta, X, y, sh: LeNetShape, act="tanh"):
    y = np.asarray(y, dtype=np.int64)
    lp = predict_logprobs(theta, X, sh, act)
    return lp[:, np.arange(len(y)), y].sum(axis=1)


def _block(gw, gb):
    return np.concatenate([gw, gb[:, None]], 1).ravel()


def loglik_grad(theta, X, y, sh: LeNetShape, act="tanh", scale=None):
    """(LL [J], scale_j * grad LL [J x D]) on the samples (X, y), by hand-written backpropagation."""
    y = np.asarray(y, dtype=np.int64)
    params = unpack(theta, sh)
    J = params[0][0].shape[0]
    scale = np.ones(J) if scale is None else np.asarray(scale, dtype=np.float64)
    k = sh.k
    lls, grads = [], []
    for j in range(J):
        Wb = [(w[j], b[j]) for w, b in params]
        (w1, _), (w2, _), (w3, _), (w4, _), (w5, _) = Wb
        xp, a1, p1, a2, f, h1, h2, logits = _forward_one(Wb, X, sh, act)
        n = xp.shape[0]
        lp = _log_softmax(logits)
        lls.append(lp[np.arange(n), y].sum())
        d5 = -np.exp(lp)
        d5[np.arange(n), y] += 1.0                                  # d LL / d logits
        d4 = (d5 @ w5) * _act_grad(h2, act)
        d3 = (d4 @ w4) * _act_grad(h1, act)
        df = (d3 @ w3).reshape(n, sh.Hq, sh.Wq, sh.C2)
        dz2 = _unpool(df) * _act_grad(a2, act)
        gW2 = np.zeros_like(w2)
        dp1 = np.zeros_like(p1)
        for ky in range(k):
            for kx in range(k):
                t = ky * k + kx
                sl = (slice(None), slice(ky, ky + sh.H2), slice(kx, kx + sh.W2), slice(None))
                gW2[:, t * sh.C1:(t + 1) * sh.C1] = np.einsum("nyxo,nyxc->oc", dz2, p1[sl])
                dp1[sl] += dz2 @ w2[:, t * sh.C1:(t + 1) * sh.C1]
        dz1 = _unpool(dp1) * _act_grad(a1, act)
        gW1 = np.zeros_like(w1)
        for ky in range(k):
            for kx in range(k):
                t = ky * k + kx
                gW1[:, t * sh.Cin:(t + 1) * sh.Cin] = np.einsum(
                    "nyxo,nyxc->oc", dz1, xp[:, ky:ky + sh.H, kx:kx + sh.W, :])
        g = np.concatenate([_block(gW1, dz1.sum(axis=(0, 1, 2))),
                            _block(gW2, dz2.sum(axis=(0, 1, 2))),
                            _block(d3.T @ f, d3.sum(axis=0)),
                            _block(d4.T @ h1, d4.sum(axis=0)),
                            _block(d5.T @ h2, d5.sum(axis=0))])
        grads.append(scale[j] * g)
    return np.asarray(lls), np.stack(grads)


class Model:
    """Adapter with the interface the oracle sampler uses for its network."""

    def __init__(self, sh: LeNetShape, act="tanh"):
        self.sh = sh
        self.act = act
        self.D = sh.D

    def loglik_grad(self, theta, X, y, scale):
        return loglik_grad(theta, X, y, self.sh, self.act, scale)

    def predict_logprobs(self, theta, X):
        return predict_logprobs(theta, X, self.sh, self.act)
