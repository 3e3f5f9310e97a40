"""Pins for the oracle's convolutional network: brute-force loops, finite differences, closed forms."""
import math

import numpy as np

from oracle import cnn, smc
import smc_inputs


def _brute_logits(theta_j, x, sh):
    """The network written out with scalar loops (tiny shapes only)."""
    (w1, b1), (w2, b2), (w3, b3) = [(w[0], b[0]) for w, b in cnn.unpack(theta_j[None], sh)]
    img = x.reshape(sh.H, sh.W, sh.Cin)

    def conv(a, w, b, cin, cout):
        out = np.zeros((sh.H, sh.W, cout))
        for y in range(sh.H):
            for xx in range(sh.W):
                for o in range(cout):
                    acc = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            yy, xs = y + ky - 1, xx + kx - 1
                            if 0 <= yy < sh.H and 0 <= xs < sh.W:
                                for c in range(cin):
                                    acc += a[yy, xs, c] * w[o, (ky * 3 + kx) * cin + c]
                    out[y, xx, o] = max(acc, 0.0)
        return out

    a1 = conv(img, w1, b1, sh.Cin, sh.C1)
    a2 = conv(a1, w2, b2, sh.C1, sh.C2)
    pooled = []
    for py in range(sh.Hp):
        for px in range(sh.Wp):
            for c in range(sh.C2):
                pooled.append((a2[2 * py, 2 * px, c] + a2[2 * py + 1, 2 * px, c] + a2[2 * py, 2 * px + 1, c]
                               + a2[2 * py + 1, 2 * px + 1, c]) / 4.0)
    pooled = np.asarray(pooled)
    return np.array([b3[k] + sum(w3[k, f] * pooled[f] for f in range(sh.F3)) for k in range(sh.n_cls)])


SMALL = cnn.CNNShape(4, 6, 2, 3, 2, 3)


def _case(seed, n=5, scale=0.5):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal((2, SMALL.D)) * scale
    X = rng.uniform(0, 1, (n, SMALL.H * SMALL.W * SMALL.Cin))
    y = rng.integers(0, SMALL.n_cls, n)
    return theta, X, y


def test_shape_and_parameter_count():
    sh = cnn.CNNShape(32, 32, 3, 16, 32, 10)
    assert sh.D == 16 * 28 + 32 * 145 + 10 * (16 * 16 * 32 + 1) == 87018


def test_forward_matches_scalar_loops():
    theta, X, y = _case(0)
    lp = cnn.predict_logprobs(theta, X, SMALL)
    for j in range(2):
        for i in range(X.shape[0]):
            z = _brute_logits(theta[j], X[i], SMALL)
            ref = z - max(z) - math.log(sum(math.exp(v - max(z)) for v in z))
            np.testing.assert_allclose(lp[j, i], ref, rtol=1e-12, atol=1e-12)


def test_zero_weights_give_uniform_likelihood():
    _, X, y = _case(1)
    ll = cnn.loglik(np.zeros((1, SMALL.D)), X, y, SMALL)
    assert abs(ll[0] + X.shape[0] * math.log(SMALL.n_cls)) < 1e-12


def test_gradient_matches_finite_differences():
    theta, X, y = _case(2)
    ll, g = cnn.loglik_grad(theta, X, y, SMALL, scale=[1.0, 2.5])
    np.testing.assert_allclose(ll, cnn.loglik(theta, X, y, SMALL), rtol=1e-13)
    rng = np.random.default_rng(3)
    for j, s in ((0, 1.0), (1, 2.5)):
        # every block: conv1, conv2, linear (weights and biases)
        idx = np.concatenate([rng.choice(SMALL.D, 40, replace=False), [27 - 1, 3 * 19 + 18, SMALL.D - 1]])
        for e in idx:
            tp = theta[j:j + 1].copy(); tp[0, e] += 1e-6
            tm = theta[j:j + 1].copy(); tm[0, e] -= 1e-6
            fd = (cnn.loglik(tp, X, y, SMALL)[0] - cnn.loglik(tm, X, y, SMALL)[0]) / 2e-6
            assert abs(s * fd - g[j, e]) < 1e-6 * (1.0 + abs(s * fd)), (j, e, fd, g[j, e])


def test_oracle_sampler_runs_the_cnn():
    sh = cnn.CNNShape(8, 8, 3, 4, 4, 3)
    X, y = smc_inputs.textures32(64, seed=0, size=8, n_cls=3)
    X = X.reshape(64, -1)
    o = smc.Sampler(X, y, None, "relu", step_size=1e-3, model=cnn.Model(sh))
    o.init(smc_inputs.prior_draw(1, 6, sh.D, 0.1), 32, 2.0)
    o.step(48, 64 / 48, smc_inputs.momenta(2, (6, sh.D)))
    assert np.all(np.isfinite(o.logw)) and abs(np.exp(o.logw).sum() - 1.0) < 1e-12
    probs, acc, _ = o.predictive(X[:10], y[:10])
    np.testing.assert_allclose(probs.sum(axis=1), 1.0, rtol=1e-12)
