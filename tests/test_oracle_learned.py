"""Pins for the oracle's learned proposal density, network gradient and Adam (CPU only)."""
import math

import numpy as np

from oracle import learned, mlp, smc
import smc_inputs


def _sampler(h=0.01):
    X, y = smc_inputs.blobs(128, seed=0)
    return smc.Sampler(X, y, [2, 16, 2], "tanh", step_size=h, leapfrog_steps=1), X, y


def test_group_index():
    gid = learned.group_index([2, 3, 2])
    # layer 1: 3 rows of [w w b]; layer 2: 2 rows of [w w w b]
    assert gid.tolist() == [0, 0, 1] * 3 + [2, 2, 2, 3] * 2
    assert learned.blob_size(4) == 8 + 256 + 64 + 4096 + 64 + 5 * 64 + 5


def test_constant_outputs_reduce_to_fixed_step_langevin():
    # zero output layer -> o = 0 -> h = h0, m = 1: the learned move and its Gaussian
    # forward/reverse densities must reproduce the fixed-step S = 1 update exactly
    h0 = 0.02
    G = learned.n_groups([2, 16, 2])
    blob = learned.init_blob(G, seed=0)
    p = learned.unpack_blob(blob, G)
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    th0 = smc_inputs.prior_draw(1, 16, 82, 1.0)
    xi = smc_inputs.momenta(2, (16, 82))
    a, _, _ = _sampler(h0)
    b, _, _ = _sampler(h0)
    a.init(th0, 64, 2.0)
    b.init(th0, 64, 2.0)
    a.step(96, 128 / 96, xi)
    learned.learned_step(b, 96, 128 / 96, xi, blob, h0, k=1, K=10, N=128)
    np.testing.assert_allclose(b.theta, a.theta, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(b.last_increment, a.last_increment, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(b.logw, a.logw, atol=1e-9)


def _log_ratio(s, theta, theta1, blob, h0, m, lam, G, gid):
    """log L(theta | theta1) - log q(theta1 | theta) with the learned scales."""
    ll0, g0 = s.loglik_grad(theta, m, lam)
    ll1, g1 = s.loglik_grad(theta1, m, lam)
    h, mg = learned.scales(learned.net_forward(blob, learned.features(ll0, g0, m, 1, 10, 128), G)[0], h0)
    h1, mg1 = learned.scales(learned.net_forward(blob, learned.features(ll1, g1, m, 1, 10, 128), G)[0], h0)
    me, me1 = mg[:, gid], mg1[:, gid]
    mf = theta + 0.5 * (h * h)[:, None] * g0 / me
    mr = theta1 + 0.5 * (h1 * h1)[:, None] * g1 / me1
    lq = np.sum(-0.5 * math.log(2 * math.pi) - np.log(h[:, None] / np.sqrt(me))
                - 0.5 * ((theta1 - mf) * np.sqrt(me) / h[:, None]) ** 2, axis=1)
    ll = np.sum(-0.5 * math.log(2 * math.pi) - np.log(h1[:, None] / np.sqrt(me1))
                - 0.5 * ((theta - mr) * np.sqrt(me1) / h1[:, None]) ** 2, axis=1)
    return ll - lq


def test_density_ratio_is_antisymmetric():
    G = learned.n_groups([2, 16, 2])
    gid = learned.group_index([2, 16, 2])
    blob = learned.init_blob(G, seed=3)
    s, _, _ = _sampler()
    th = smc_inputs.prior_draw(4, 5, 82, 1.0).astype(np.float64)
    th1 = th + 0.01 * smc_inputs.momenta(5, th.shape)
    r01 = _log_ratio(s, th, th1, blob, 0.01, 64, 2.0, G, gid)
    r10 = _log_ratio(s, th1, th, blob, 0.01, 64, 2.0, G, gid)
    np.testing.assert_allclose(r01, -r10, rtol=1e-10, atol=1e-10)


def test_learned_step_uses_general_weight_form():
    # the learned step's increment equals log pi_k(theta') - lp + log L - log q with
    # densities evaluated independently here
    G = learned.n_groups([2, 16, 2])
    gid = learned.group_index([2, 16, 2])
    blob = learned.init_blob(G, seed=8)
    s, _, _ = _sampler()
    th0 = smc_inputs.prior_draw(6, 6, 82, 1.0)
    s.init(th0, 64, 2.0)
    theta, lp = s.theta.copy(), s.lp.copy()
    learned.learned_step(s, 64, 2.0, smc_inputs.momenta(9, (6, 82)), blob, 0.01, k=1, K=10, N=128)
    r = _log_ratio(s, theta, s.theta, blob, 0.01, 64, 2.0, G, gid)
    np.testing.assert_allclose(s.last_increment, s.lp - lp + r, rtol=1e-9, atol=1e-9)


def test_mse_gradient_matches_finite_differences():
    G = 4
    blob = learned.init_blob(G, seed=1, mu=[0.1, -0.2, 0.5, 0.3], sd=[1.5, 0.7, 0.3, 0.4])
    rng = np.random.default_rng(2)
    f = rng.standard_normal((11, 4))
    t = rng.standard_normal((11, 5))
    _, g = learned.mse_loss_grad(blob, f, t, G)
    idx = rng.choice(np.arange(8, blob.shape[0]), 60, replace=False)
    for k in idx:
        bp = blob.copy(); bp[k] += 1e-6
        bm = blob.copy(); bm[k] -= 1e-6
        fd = (learned.mse_loss_grad(bp, f, t, G)[0] - learned.mse_loss_grad(bm, f, t, G)[0]) / 2e-6
        assert abs(fd - g[k]) < 1e-7 + 1e-6 * abs(fd)
    assert np.all(g[:8] == 0.0)


def test_adam_first_step_is_signed_learning_rate():
    # after one step the bias-corrected moments are g and g^2: the update is lr * g / (|g| + eps)
    blob = np.array([1.0, -2.0, 3.0])
    grad = np.array([0.5, -4.0, 1e-3])
    new, _ = learned.adam_update(blob, grad, (np.zeros(3), np.zeros(3), 0), lr=0.1)
    np.testing.assert_allclose(new, blob - 0.1 * grad / (np.abs(grad) + 1e-8), rtol=1e-12)


def test_scales_fallback_and_bounds():
    o = np.array([[0.0, 0.0], [50.0, -50.0], [np.nan, 1.0]])
    h, mg = learned.scales(o, 0.01)
    np.testing.assert_allclose(h, [0.01, 0.08, 0.01], rtol=1e-12)
    np.testing.assert_allclose(mg[:, 0], [1.0, 0.1, 1.0], rtol=1e-12)


def test_step_size_targets_prefer_stable_steps():
    # on a sharply curved target, very large steps are rejected by the Metropolis factor
    s, _, _ = _sampler(0.01)
    s.init(smc_inputs.prior_draw(3, 12, 82, 1.0), 128, 1.0)
    logh, logm = learned.step_size_targets(s, 128, 1.0, smc_inputs.momenta(4, (12, 82)), 0.01)
    assert np.all(logh >= math.log(0.01 / 8) - 1e-12) and np.all(logh <= math.log(0.08) + 1e-12)
    np.testing.assert_allclose(logm.mean(axis=1), 0.0, atol=1e-12)


def test_step_size_targets_without_acceptance_pick_the_longest_jump():
    # accept_power = 0 scores a step by its squared jump alone; for a Langevin move from
    # gradient g with noise xi that jump is |h^2/2 g + h xi|^2, computed here directly
    s, _, _ = _sampler(0.01)
    s.init(smc_inputs.prior_draw(5, 10, 82, 1.0), 128, 1.0)
    xi = smc_inputs.momenta(6, (10, 82)).astype(np.float64)
    logh, _ = learned.step_size_targets(s, 128, 1.0, xi, 0.01, accept_power=0.0)
    _, g = s.loglik_grad(s.theta, 128, 1.0)  # gradient of log pi_k (likelihood and prior)
    hs = 0.01 * 2.0 ** np.arange(-3, 4)
    jumps = np.stack([np.sum((0.5 * h * h * g + h * xi) ** 2, axis=1) for h in hs], axis=1)
    np.testing.assert_allclose(logh, np.log(hs[np.argmax(jumps, axis=1)]), rtol=1e-12)
    # a larger exponent never prefers a step with a lower score at exponent 1 and a worse increment
    lh1, _ = learned.step_size_targets(s, 128, 1.0, xi, 0.01, accept_power=1.0)
    lh4, _ = learned.step_size_targets(s, 128, 1.0, xi, 0.01, accept_power=4.0)
    assert np.all(lh4 <= logh + 1e-12) and np.all(lh1 <= logh + 1e-12)


def _torch_net(blob, G):
    """The proposal network written independently with torch float64 library layers."""
    import torch
    import torch.nn.functional as F

    b = torch.tensor(blob, dtype=torch.float64)
    n_out = 1 + G
    sizes = [4, 4, 64 * 4, 64, 64 * 64, 64, n_out * 64, n_out]
    parts = list(torch.split(b, sizes))
    mu, sd = parts[0], parts[1]
    W1, b1 = parts[2].reshape(64, 4).clone().requires_grad_(), parts[3].clone().requires_grad_()
    W2, b2 = parts[4].reshape(64, 64).clone().requires_grad_(), parts[5].clone().requires_grad_()
    W3, b3 = parts[6].reshape(n_out, 64).clone().requires_grad_(), parts[7].clone().requires_grad_()

    def fwd(f):
        u = torch.clamp((torch.as_tensor(f, dtype=torch.float64) - mu) / sd, -3.0, 3.0)
        return F.linear(torch.tanh(F.linear(torch.tanh(F.linear(u, W1, b1)), W2, b2)), W3, b3)

    return fwd, (W1, b1, W2, b2, W3, b3)


def test_net_forward_matches_torch_float64_network_with_active_clip():
    # standardise, clip to +-3 sd, tanh, tanh, linear; some feature columns lie far outside
    # the training statistics so that the clip is active in both directions
    G = 4
    rng = np.random.default_rng(5)
    blob = learned.init_blob(G, seed=7, mu=[0.1, -0.2, 0.5, 0.3], sd=[1.5, 0.7, 0.3, 0.4])
    blob[8:] += 0.1 * rng.standard_normal(blob.shape[0] - 8)  # non-zero biases too
    f = rng.standard_normal((9, 4))
    f[0] = [100.0, -100.0, 0.5, 0.3]     # clipped at +3 and -3
    f[1] = [0.1 + 4.8, -0.2 - 2.0, 0.5 + 0.91, 0.3 - 1.19]  # clipped / inside / clipped / inside
    fwd, _ = _torch_net(blob, G)
    o, (u, _, _) = learned.net_forward(blob, f, G)
    np.testing.assert_allclose(o, fwd(f).detach().numpy(), rtol=1e-12, atol=1e-13)
    assert u[0].tolist() == [3.0, -3.0, 0.0, 0.0]
    np.testing.assert_allclose(u[1], [3.0, -2.0 / 0.7, 3.0, -1.19 / 0.4], rtol=1e-12)
    # without the clip the first row would differ
    p = learned.unpack_blob(blob, G)
    u_noclip = (f[0] - p["mu"]) / p["sd"]
    o_noclip = np.tanh(np.tanh(u_noclip @ p["W1"].T + p["b1"]) @ p["W2"].T + p["b2"]) @ p["W3"].T + p["b3"]
    assert np.max(np.abs(o_noclip - o[0])) > 1e-3


def test_mse_loss_gradient_matches_torch_autograd():
    import torch

    G = 6
    rng = np.random.default_rng(11)
    blob = learned.init_blob(G, seed=2, mu=[-0.3, 0.2, 0.1, 0.6], sd=[0.8, 1.1, 0.5, 0.25])
    blob[8:] += 0.05 * rng.standard_normal(blob.shape[0] - 8)
    f = rng.standard_normal((13, 4))
    f[3] = [50.0, 0.0, -50.0, 0.6]
    t = rng.standard_normal((13, 1 + G))
    loss, grad = learned.mse_loss_grad(blob, f, t, G)
    fwd, params = _torch_net(blob, G)
    o = fwd(f)
    tl = 0.5 * ((o - torch.tensor(t)) ** 2).sum() / f.shape[0]
    tl.backward()
    ref = np.concatenate([np.zeros(8)] + [p.grad.numpy().ravel() for p in params])
    np.testing.assert_allclose(loss, tl.item(), rtol=1e-13)
    np.testing.assert_allclose(grad, ref, rtol=1e-11, atol=1e-14)


def test_adam_matches_torch_optim_over_several_steps():
    # the bias corrections 1 - beta^t for t = 1..7 with gradients that change from step to step
    import torch

    rng = np.random.default_rng(3)
    x0 = rng.standard_normal(17)
    grads = [rng.standard_normal(17) * s for s in (1.0, 0.1, 3.0, 0.5, 2.0, 1e-3, 1.0)]
    p = torch.tensor(x0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.03, betas=(0.9, 0.999), eps=1e-8)
    blob = x0.copy()
    state = (np.zeros(17), np.zeros(17), 0)
    for g in grads:
        p.grad = torch.tensor(g)
        opt.step()
        blob, state = learned.adam_update(blob, g, state, lr=0.03)
        np.testing.assert_allclose(blob, p.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert state[2] == 7


def test_features_worked_by_hand():
    # (log |grad log pi|, LL / M_k, k / K, M_k / N): gradients (3, 4, 0) and (0, 0, 2) have
    # norms 5 and 2
    grad = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 2.0]])
    ll = np.array([-20.0, -5.0])
    f = learned.features(ll, grad, m=10, k=3, K=12, N=40)
    np.testing.assert_allclose(f, [[math.log(5.0), -2.0, 0.25, 0.25],
                                   [math.log(2.0), -0.5, 0.25, 0.25]], rtol=1e-15)
