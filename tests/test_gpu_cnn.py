"""GPU parity of the convolutional network's likelihood, gradient, predictive and sampler
trajectory against the oracle (CIFAR-shaped textures; conv3x3 -> conv3x3 -> avgpool -> linear)."""
import numpy as np
import pytest

from gpu_helpers import cuda, lib, print_case, rel_err, to_dev, torch
from oracle import cnn, smc
from oracle import schedules as osched
import smc_inputs

pytestmark = pytest.mark.gpu

CASES = [
    # (H, W, Cin, C1, C2, n_cls), J, M, precision, act_budget_bytes (small budgets force chunks)
    ((8, 8, 3, 8, 8, 3), 6, 20, "fp32", 0),
    ((8, 8, 3, 8, 8, 3), 6, 20, "fp32", 400_000),
    ((8, 6, 2, 16, 8, 4), 5, 9, "fp32", 0),
    ((32, 32, 3, 16, 32, 10), 4, 12, "fp32", 0),
    ((32, 32, 3, 16, 32, 10), 4, 12, "bf16", 0),
    ((32, 32, 3, 16, 32, 10), 3, 7, "bf16", 2_000_000),
]


def _data(dims, n, seed):
    H, W, Cin, C1, C2, ncls = dims
    assert H == W and Cin == 3
    X, y = smc_inputs.textures32(n, seed=seed, size=H, n_cls=ncls)
    return X.reshape(n, -1), y


def _data_any(dims, n, seed):
    H, W, Cin, C1, C2, ncls = dims
    if H == W and Cin == 3:
        return _data(dims, n, seed)
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (n, H * W * Cin)).astype(np.float32), rng.integers(0, ncls, n)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_cnn_loglik_and_gradient_vs_oracle(case):
    cuda()
    P = lib()
    dims, J, M, prec, budget = CASES[case]
    sh = cnn.CNNShape(*dims)
    print_case("cnn-net", dims=dims, J=J, M=M, prec=prec, budget=budget)
    X, y = _data_any(dims, M + 3, seed=case)
    theta = smc_inputs.prior_draw(case + 40, J, sh.D, 0.08)
    cfg = P.SMCConfig(widths=list(dims), n_particles=J, model="cnn", precision=prec, act_budget_bytes=budget)
    Xd, yd, td = to_dev(X), to_dev(y.astype(np.int32)), to_dev(theta)
    s = P.SMCSampler(cfg, Xd, yd, m0=M, lambda0=1.0, theta0=td)
    assert s.D == sh.D
    if budget:
        assert s.chunk_samples() < M
    scale = np.linspace(0.5, 2.0, J)
    sd = to_dev(scale)
    ll_g, g_g = s.nn_backward(td, M, sd)
    ll_f = s.nn_forward(td, M)
    torch.cuda.synchronize()
    ll_ref, g_ref = cnn.loglik_grad(theta, X[:M], y[:M], sh, scale=scale)
    ll_g, ll_f, g_g = ll_g.cpu().numpy(), ll_f.cpu().numpy(), g_g.cpu().numpy()
    tol_ll = 1e-5 if prec == "fp32" else 2e-2
    assert rel_err(ll_g, ll_ref) < tol_ll
    assert rel_err(ll_f, ll_ref) < tol_ll
    gs = np.max(np.abs(g_ref), axis=1, keepdims=True)
    err = np.max(np.abs(g_g - g_ref) / gs)
    print(f"ll rel err {rel_err(ll_g, ll_ref):.3g}, grad err {err:.3g}", flush=True)
    # BF16: the error is rounding the back-propagated errors at four stages (linear-layer output
    # error, pooled error, conv2 patch errors, conv1 output error) before the conv1 weight
    # gradient sums them over all pixels; an FP64 emulation of exactly these rounding points on
    # case 4 gives 6.9% of the largest gradient entry, the value the GPU reaches
    assert err < (2e-4 if prec == "fp32" else 1e-1), err
    s.close()


def test_cnn_predictive_vs_oracle():
    cuda()
    P = lib()
    dims = (32, 32, 3, 16, 32, 10)
    sh = cnn.CNNShape(*dims)
    J = 5
    X, y = _data(dims, 16, seed=3)
    Xt, yt = _data(dims, 40, seed=4)
    theta = smc_inputs.prior_draw(7, J, sh.D, 0.08)
    print_case("cnn-predictive", J=J, n_test=40)
    cfg = P.SMCConfig(widths=list(dims), n_particles=J, model="cnn")
    s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=16, lambda0=1.0, theta0=to_dev(theta))
    r = s.predict(to_dev(Xt), to_dev(yt.astype(np.int32)), probs=True)
    st = s.state()
    lw = st["logw"].cpu().numpy()
    probs, acc, mlpd = smc.predictive(theta.astype(np.float64), lw, Xt, yt, None, "relu", cnn.Model(sh))
    np.testing.assert_allclose(r["probs"].cpu().numpy(), probs, rtol=1e-4, atol=1e-6)
    assert abs(r["accuracy"] - acc) <= 0.005
    assert abs(r["mean_log_pred"] - mlpd) < 1e-4 * max(1.0, abs(mlpd))
    s.close()


def test_cnn_trajectory_and_adaptive_growth_vs_oracle():
    """Lockstep sampler run on the CIFAR-shaped network with injected momenta and offsets; the
    subset grows by the posterior-mean criterion, decided from the GPU's values and checked
    against the oracle's."""
    cuda()
    P = lib()
    dims = (32, 32, 3, 16, 32, 10)
    sh = cnn.CNNShape(*dims)
    J, N, kappa, tol, h = 8, 24, 8, 0.02, 2e-3
    X, y = _data(dims, N, seed=5)
    th0 = smc_inputs.prior_draw(9, J, sh.D, 0.08)
    print_case("cnn-trajectory", J=J, N=N, kappa=kappa)
    o = smc.Sampler(X, y, None, "relu", step_size=h, prior_std=1.0, model=cnn.Model(sh))
    o.init(th0, kappa, N / kappa)
    cfg = P.SMCConfig(widths=list(dims), n_particles=J, model="cnn", step_size=h, seed=2)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=kappa, lambda0=N / kappa, theta0=to_dev(th0))
    u = smc_inputs.uniforms(31, 8)
    assert o.resample(u[0]) == g.resample("if_needed", float(u[0]), want=True)[0]
    g.posterior_mean_change()
    st = g.state()
    prev = osched.posterior_mean(st["theta"].cpu().numpy(), st["logw"].cpu().numpy())
    m, sizes = kappa, []
    for k in range(1, 6):
        xi = smc_inputs.momenta(500 + k, (J, sh.D))
        g.set_noise(to_dev(xi))
        g.step(m, N / m)
        o.step(m, N / m, xi)
        sizes.append(m)
        res_g, anc_g = g.resample("if_needed", float(u[k]), want=True)
        res_o = o.resample(u[k])
        assert res_g == res_o, k
        if res_o:
            assert anc_g == o.ancestors.tolist(), k
        st = g.state()
        th = st["theta"].cpu().numpy()
        assert np.max(np.abs(th - o.theta)) < 1e-4 * np.max(np.abs(o.theta)), k
        lw = st["logw"].cpu().numpy()
        big = o.logw > np.log(1e-6)
        assert np.max(np.abs(lw[big] - o.logw[big])) < 2e-3, k
        # the criterion on the GPU's own population, and the growth rule applied to it
        change = g.posterior_mean_change()
        cur = osched.posterior_mean(th, lw)
        ref = osched.mean_change(prev, cur)
        assert abs(change - ref) <= 1e-9 * ref + 1e-15, (k, change, ref)
        m = osched.adaptive_next(m, change, tol, kappa, N)
        prev = cur
    print(f"subset sizes {sizes}", flush=True)
    g.close()
