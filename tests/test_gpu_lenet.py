"""GPU parity of the LeNet-5 network (the MNIST model of the paper's Table 1 study, Section 4):
likelihood, gradient, predictive and an HMC sampler trajectory against the oracle, on
MNIST-shaped images and on small shapes with odd channel counts and 3x3 kernels."""
import numpy as np
import pytest

from gpu_helpers import cuda, lib, print_case, rel_err, to_dev, torch
from oracle import lenet, smc
import smc_inputs

pytestmark = pytest.mark.gpu

LENET5 = lenet.LENET5_MNIST

CASES = [
    # (H, W, Cin, k, C1, C2, F1, F2, n_cls), act, J, M, act_budget_bytes (small budgets force chunks)
    (LENET5, "tanh", 4, 40, 0),
    (LENET5, "tanh", 3, 300, 1),       # two chunks of 256 and 44 images
    (LENET5, "relu", 3, 21, 0),
    ((12, 12, 1, 5, 3, 4, 8, 8, 3), "relu", 6, 37, 0),
    ((12, 12, 2, 3, 3, 5, 8, 4, 3), "tanh", 5, 20, 0),   # odd C1 and C2, k = 3, two input channels
    ((8, 12, 2, 3, 5, 6, 8, 4, 4), "tanh", 2, 9, 0),
    (LENET5, "tanh", 1, 1, 0),         # one particle, one image
    (LENET5, "relu", 2, 257, 1),       # chunks of 256 and 1 image
]


def _data(dims, n, seed):
    if tuple(dims) == LENET5:
        X, y = smc_inputs.templates28(n, seed=seed)
        return X, y.astype(np.int64)
    H, W, Cin = dims[:3]
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (n, H * W * Cin)).astype(np.float32), rng.integers(0, dims[-1], n)


def _sampler(P, dims, act, J, X, y, m0, theta, **kw):
    cfg = P.SMCConfig(widths=list(dims), n_particles=J, model="lenet", activation=act, **kw)
    return P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=m0, lambda0=1.0, theta0=to_dev(theta))


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lenet_loglik_and_gradient_vs_oracle(case):
    cuda()
    P = lib()
    dims, act, J, M, budget = CASES[case]
    sh = lenet.LeNetShape(*dims)
    print_case("lenet-net", dims=dims, act=act, J=J, M=M, budget=budget)
    X, y = _data(dims, M + 3, seed=case)
    theta = smc_inputs.prior_draw(case + 60, J, sh.D, 0.2)
    s = _sampler(P, dims, act, J, X, y, M, theta, act_budget_bytes=budget)
    assert s.D == sh.D
    if budget:
        assert s.chunk_samples() < M
    scale = np.linspace(0.5, 2.0, J)
    td = to_dev(theta)
    ll_g, g_g = s.nn_backward(td, M, to_dev(scale))
    ll_f = s.nn_forward(td, M)
    torch.cuda.synchronize()
    ll_ref, g_ref = lenet.loglik_grad(theta, X[:M], y[:M], sh, act, scale=scale)
    ll_g, ll_f, g_g = ll_g.cpu().numpy(), ll_f.cpu().numpy(), g_g.cpu().numpy()
    e_ll = max(rel_err(ll_g, ll_ref), rel_err(ll_f, ll_ref))
    gs = np.max(np.abs(g_ref), axis=1, keepdims=True)
    err = np.max(np.abs(g_g - g_ref) / gs)
    # the two convolution blocks on their own: they are summed over every pixel of every image
    Dc = sh.blocks[0][0] * (sh.blocks[0][1] + 1) + sh.blocks[1][0] * (sh.blocks[1][1] + 1)
    err_c = np.max(np.abs(g_g[:, :Dc] - g_ref[:, :Dc]) / np.max(np.abs(g_ref[:, :Dc]), axis=1, keepdims=True))
    print(f"ll rel err {e_ll:.3g}, grad err {err:.3g}, conv blocks {err_c:.3g}", flush=True)
    assert e_ll < 1e-5, e_ll
    assert err < 2e-4 and err_c < 2e-4, (err, err_c)
    s.close()


@pytest.mark.parametrize("n_test,budget", [(70, 0), (300, 1)])  # 300 test images in chunks of 256 and 44
def test_lenet_predictive_vs_oracle(n_test, budget):
    cuda()
    P = lib()
    sh = lenet.LeNetShape(*LENET5)
    J = 5
    X, y = _data(LENET5, 16, seed=3)
    Xt, yt = _data(LENET5, n_test, seed=4)
    theta = smc_inputs.prior_draw(7, J, sh.D, 0.2)
    print_case("lenet-predictive", J=J, n_test=n_test, budget=budget)
    s = _sampler(P, LENET5, "tanh", J, X, y, 16, theta, act_budget_bytes=budget)
    if budget:
        assert s.chunk_samples() < n_test
    r = s.predict(to_dev(Xt), to_dev(yt.astype(np.int32)), probs=True)
    lw = s.state()["logw"].cpu().numpy()
    probs, acc, mlpd = smc.predictive(theta.astype(np.float64), lw, Xt, yt, None, "tanh", lenet.Model(sh, "tanh"))
    np.testing.assert_allclose(r["probs"].cpu().numpy(), probs, rtol=1e-4, atol=1e-6)
    assert abs(r["accuracy"] - acc) <= 1 / n_test + 1e-12
    assert abs(r["mean_log_pred"] - mlpd) < 1e-4 * max(1.0, abs(mlpd))
    s.close()


def test_lenet_hmc_trajectory_vs_oracle():
    """Lockstep HMC (S = 3, h = 0.002, the study's move) on LeNet-5 with injected momenta and
    resampling offsets, the subset growing by a fixed step as in the naive schedules."""
    cuda()
    P = lib()
    sh = lenet.LeNetShape(*LENET5)
    J, N, kappa, h, S = 8, 30, 10, 2e-3, 3
    X, y = _data(LENET5, N, seed=5)
    th0 = smc_inputs.prior_draw(9, J, sh.D, 0.2)
    print_case("lenet-trajectory", J=J, N=N, kappa=kappa, S=S)
    o = smc.Sampler(X, y, None, "tanh", step_size=h, prior_std=1.0, leapfrog_steps=S, model=lenet.Model(sh, "tanh"))
    o.init(th0, kappa, N / kappa)
    cfg = P.SMCConfig(widths=list(LENET5), n_particles=J, model="lenet", activation="tanh", step_size=h,
                      leapfrog_steps=S, seed=2)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=kappa, lambda0=N / kappa, theta0=to_dev(th0))
    u = smc_inputs.uniforms(31, 8)
    assert o.resample(u[0]) == g.resample("if_needed", float(u[0]), want=True)[0]
    for k, m in enumerate([10, 10, 20, 20, 30], start=1):
        xi = smc_inputs.momenta(700 + k, (J, sh.D))
        g.set_noise(to_dev(xi))
        g.step(m, N / m)
        o.step(m, N / m, xi)
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
    g.close()


@pytest.mark.parametrize("bad", [
    dict(precision="bf16"),
    dict(proposal="learned"),
    dict(widths=[28, 28, 1, 4, 6, 16, 120, 84, 10]),    # even kernel
    dict(widths=[26, 26, 1, 5, 6, 16, 120, 84, 10]),    # second convolution 9 x 9
    dict(widths=[28, 28, 1, 5, 9, 16, 120, 84, 10]),    # C1 > 8
    dict(widths=[28, 28, 1, 5, 6, 16, 122, 84, 10]),    # F1 not a multiple of 4
    dict(likelihood="gaussian", noise_std=1.0),
])
def test_lenet_rejects_unsupported_configs(bad):
    cuda()
    P = lib()
    kw = dict(widths=list(LENET5), n_particles=2, model="lenet", activation="tanh")
    kw.update(bad)
    X, y = _data(LENET5, 8, seed=1)
    cfg = P.SMCConfig(**kw)
    with pytest.raises(Exception):
        yv = y.astype(np.float32) if kw.get("likelihood") == "gaussian" else y.astype(np.int32)
        P.SMCSampler(cfg, to_dev(X), to_dev(yv), m0=8, lambda0=1.0)
