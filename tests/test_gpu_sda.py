"""GPU parity of the two-segment tempered target of smooth data annealing (Section 3.1):
segment log-likelihoods, log-target and gradient through every likelihood kernel (FP32 output
layer, fused BF16 and split-BF16 kernels, the deep-network output layer, the convolutional
network), the weighted moments, and an SDA run in lockstep with the oracle."""
import numpy as np
import pytest

from gpu_helpers import bf16_round, cuda, lib, print_case, rel_err, to_dev, torch
from oracle import cnn, lenet, mlp, sda, smc
import smc_inputs

pytestmark = pytest.mark.gpu

CASES = [
    # widths, model, act, precision, J, n_data, m0, m, split, lam_a, lam_b, act_budget_bytes
    ([784, 100, 10], "mlp", "relu", "fp32", 8, 320, 130, 300, 130, 1.0, 0.3, 8 * 100 * 4 * 2 * 64),
    ([784, 100, 10], "mlp", "relu", "bf16", 8, 640, 260, 600, 260, 1.0, 0.45, 0),
    ([784, 100, 10], "mlp", "tanh", "bf16x3", 8, 640, 300, 520, 0, 1.0, 0.2, 0),
    ([784, 100, 10], "mlp", "relu", "bf16x3", 8, 640, 200, 600, 333, 1.0, 0.7, 8 * 100 * 2 * 3 * 128),
    ([784, 64, 32, 10], "mlp", "relu", "fp32", 6, 400, 200, 333, 200, 1.0, 0.6, 6 * 96 * 4 * 3 * 64),
    ([784, 64, 32, 10], "mlp", "tanh", "bf16", 6, 400, 200, 333, 200, 1.0, 0.6, 0),
    ([2, 16, 2], "mlp", "tanh", "fp32", 16, 200, 75, 150, 75, 2.0, 0.25, 0),
    ((8, 8, 3, 8, 8, 3), "cnn", "relu", "fp32", 4, 40, 17, 30, 17, 1.0, 0.5, 400_000),
    ((8, 8, 3, 8, 8, 3), "cnn", "relu", "bf16", 4, 40, 17, 30, 17, 1.0, 0.5, 0),
    ((28, 28, 1, 5, 6, 16, 120, 84, 10), "lenet", "tanh", "fp32", 4, 60, 20, 45, 20, 1.0, 0.4, 0),
    # chunks of 256 and 44 images, the second segment starting inside the second chunk
    ((28, 28, 1, 5, 6, 16, 120, 84, 10), "lenet", "tanh", "fp32", 3, 320, 100, 300, 280, 1.0, 0.4, 1),
]


def _data(widths, model, n, seed):
    if model == "cnn":
        H, W, Cin, _, _, ncls = widths
        rng = np.random.default_rng(seed)
        return rng.uniform(0, 1, (n, H * W * Cin)).astype(np.float32), rng.integers(0, ncls, n).astype(np.int32)
    if widths[0] == 784 or model == "lenet":
        X, y = smc_inputs.templates28(n, seed=seed)
    else:
        X, y = smc_inputs.blobs(n, seed=seed)
    return X, y.astype(np.int32)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_tempered_target_vs_oracle(case):
    """After one tempered step: the GPU's log-likelihood, cached log-target and gradient at its
    new particles against the oracle's FP64 two-segment target at the same particles, and the
    weighted segment moments under the GPU's weights."""
    cuda()
    P = lib()
    widths, model, act, prec, J, n, m0, m, split, la, lb, budget = CASES[case]
    print_case("sda-target", widths=widths, model=model, prec=prec, J=J, m=m, split=split, budget=budget)
    X, y = _data(widths, model, n, seed=case)
    if model == "cnn":
        sh = cnn.CNNShape(*widths)
        D, omodel = sh.D, cnn.Model(sh)
    elif model == "lenet":
        sh = lenet.LeNetShape(*widths)
        D, omodel = sh.D, lenet.Model(sh, act)
    else:
        D, omodel = mlp.n_params(widths), None
    prior = {"cnn": 0.08, "lenet": 0.2}.get(model, 0.3 if widths[0] == 784 else 1.0)
    th0 = smc_inputs.prior_draw(case + 70, J, D, prior)
    cfg = P.SMCConfig(widths=list(widths), n_particles=J, activation=act, precision=prec, model=model,
                      step_size=1e-3, prior_std=prior, act_budget_bytes=budget, seed=case)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y), m0=m0, lambda0=1.0, theta0=to_dev(th0))
    if budget:
        assert g.chunk_samples() < m
    g.set_noise(to_dev(smc_inputs.momenta(case + 80, (J, D))))
    info = g.step_tempered(m, split, la, lb)
    assert info["grad_evals"] == J * m * 2  # the new target's gradient, then one leapfrog step
    st = g.state()
    th = st["theta"].cpu().numpy().astype(np.float64)
    Xo = bf16_round(X) if prec == "bf16x3" else X
    o = smc.Sampler(Xo, y, None if omodel is not None else widths, act, prior_std=prior, model=omodel)
    ll, ll_b, grad = o.segment_loglik_grad(th, m, split, la, lb)
    lp = o.segment_log_target(ll, ll_b, th, la, lb)
    ll_g, lp_g, grad_g = st["loglik"].cpu().numpy(), st["logpi"].cpu().numpy(), st["grad"].cpu().numpy()
    tol_ll = {"fp32": 1e-5, "bf16": 2e-2, "bf16x3": 1e-4}[prec]
    tol_g = {"fp32": 2e-4, "bf16": 1e-1 if model == "cnn" else 3e-2, "bf16x3": 5e-3}[prec]
    e_ll, e_lp = rel_err(ll_g, ll), rel_err(lp_g, lp)
    e_g = np.max(np.abs(grad_g - grad) / np.max(np.abs(grad), axis=1, keepdims=True))
    # moments of Omega^ = -LL[split, m), Omega = -LL[0, split) under the GPU's weights
    w = np.exp(st["logw"].cpu().numpy())
    mo = g.segment_moments()
    var_o, cov_o = sda.weighted_moments(w, -(ll - ll_b), -ll_b)
    eb_o = np.sum(w * -ll_b)
    print(f"ll {e_ll:.3g} logpi {e_lp:.3g} grad {e_g:.3g}; var {mo['var_hat']:.6g} vs {var_o:.6g}, "
          f"cov {mo['cov']:.6g} vs {cov_o:.6g}", flush=True)
    assert e_ll < tol_ll and e_lp < tol_ll, (e_ll, e_lp)
    assert e_g < tol_g, e_g
    assert abs(mo["mean_hat"] - eb_o) <= tol_ll * max(1.0, abs(eb_o))
    if split == 0:
        assert mo["mean"] == 0.0 and mo["cov"] == 0.0
    # the variance is a difference of second moments: compare on the scale of E[Omega^2]
    m2 = np.sum(w * ll_b * ll_b)
    assert abs(mo["var_hat"] - var_o) <= 4 * tol_ll * m2, (mo["var_hat"], var_o)
    assert abs(mo["cov"] - cov_o) <= 4 * tol_ll * np.sqrt(m2 * np.sum(w * (ll - ll_b) ** 2)) + 1e-12
    g.close()


def test_one_segment_tempered_step_is_the_plain_step():
    """m_split >= m_k is the one-segment target: bitwise the same state as smc_step."""
    cuda()
    P = lib()
    widths, J, N = [784, 100, 10], 8, 512
    X, y = _data(widths, "mlp", N, seed=3)
    D = mlp.n_params(widths)
    th0 = smc_inputs.prior_draw(5, J, D, 0.3)
    xi = to_dev(smc_inputs.momenta(6, (J, D)))
    out = []
    for tempered in (False, True):
        cfg = P.SMCConfig(widths=widths, n_particles=J, precision="bf16x3", step_size=1e-3, prior_std=0.3)
        g = P.SMCSampler(cfg, to_dev(X), to_dev(y), m0=256, lambda0=2.0, theta0=to_dev(th0))
        g.set_noise(xi)
        if tempered:
            g.step_tempered(384, 384, N / 384, 0.77)
        else:
            g.step(384, N / 384)
        st = g.state()
        out.append((st["theta"].cpu().numpy(), st["logw"].cpu().numpy(), st["logpi"].cpu().numpy()))
        g.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_sda_run_matches_the_oracle():
    """The SDA schedule on the GPU (moments from the device) against the oracle's sampler and
    annealing rule, with the same momenta and resampling offsets; appends and beta values
    are decided by the GPU and checked against the oracle's."""
    cuda()
    P = lib()
    from paper_2601_21983_amd.schedules import SDASchedule
    widths, act, J, C, kappa, N, h, dS = [2, 16, 2], "tanh", 32, 64, 64, 256, 2e-3, 1.0
    X, y = smc_inputs.blobs(N, seed=21)
    D = mlp.n_params(widths)
    th0 = smc_inputs.prior_draw(22, J, D, 1.0)
    print_case("sda-run", J=J, C=C, kappa=kappa, N=N, dS=dS)
    o = smc.Sampler(X, y, widths, act, step_size=h, prior_std=1.0)
    o.init(th0, C, 0.1)
    cfg = P.SMCConfig(widths=widths, n_particles=J, activation=act, step_size=h, prior_std=1.0, seed=4)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=C, lambda0=0.1, theta0=to_dev(th0))
    sched = SDASchedule(C, kappa, N, beta0=0.1, dS=dS)
    u = smc_inputs.uniforms(23, 200)
    assert o.resample(u[0]) == g.resample("if_needed", float(u[0]), want=True)[0]
    appended, k = 0, 0
    while not sched.done() and k < 150:
        k += 1
        m, split, beta = sched.target
        xi = smc_inputs.momenta(300 + k, (J, D))
        g.set_noise(to_dev(xi))
        g.step_tempered(m, split, 1.0, beta)
        o.step_tempered(m, split, 1.0, beta, xi)
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
        prev = sched.target
        nxt = sched.next(g)
        ref = sda.next_target(prev, np.exp(o.logw), o.ll, o.ll_b, N, kappa, beta0=0.1, dS=dS)
        assert nxt[:2] == ref[:2], (k, nxt, ref)
        assert abs(nxt[2] - ref[2]) <= 1e-5 * ref[2], (k, nxt, ref)
        appended += nxt[0] > prev[0]
    print(f"{k} iterations, {appended} appends, targets {sched.history[-3:]}", flush=True)
    assert sched.done() and appended == (N - C) // kappa
    g.close()
