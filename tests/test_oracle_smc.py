"""Pins for the oracle's SMC sampler: weights, ESS, resampling, move, closed forms (CPU only)."""
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import blr, mlp, schedules, smc
from oracle.philox import philox4x32
import smc_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- normalisation and ESS
def test_log_sum_exp_against_decimal():
    getcontext().prec = 60
    rng = np.random.default_rng(0)
    for scale in [1.0, 50.0, 700.0]:
        v = scale * rng.standard_normal(17)
        exact = sum(Decimal(float(x)).exp() for x in v).ln()
        assert abs(smc.log_sum_exp(v) - float(exact)) <= 4e-16 * max(1.0, abs(float(exact)))


def test_normalised_weights_sum_to_one_and_ess_bounds():
    rng = np.random.default_rng(1)
    for J in [1, 2, 7, 256]:
        lw, _ = smc.normalise(30 * rng.standard_normal(J))
        assert abs(np.sum(np.exp(lw)) - 1.0) < 1e-14
        e = smc.ess(lw)
        assert 1.0 - 1e-12 <= e <= J + 1e-9


def test_ess_special_cases():
    lw, _ = smc.normalise(np.zeros(64))
    assert abs(smc.ess(lw) - 64.0) < 1e-10
    one_hot = np.full(64, -np.inf)
    one_hot[5] = 3.0
    lw, _ = smc.normalise(one_hot)
    assert smc.ess(lw) == 1.0


# ----------------------------------------------------------------- systematic resampling
def _golden_systematic():
    rows = []
    for line in open(os.path.join(GOLDEN, "systematic.txt")):
        if line.startswith("#") or not line.strip():
            continue
        u, w, a = [p.strip() for p in line.split(";")]
        rows.append((float(u), np.array([float(x) for x in w.split()]), [int(x) for x in a.split()]))
    return rows


@pytest.mark.parametrize("case", range(3))
def test_systematic_worked_examples(case):
    u, w, a = _golden_systematic()[case]
    assert list(smc.systematic_ancestors(w, u)) == a


def test_systematic_identity_for_equal_weights():
    rng = np.random.default_rng(2)
    for J in [1, 3, 64, 100, 1000]:
        for u in [0.0, rng.random(), 1.0 - 2 ** -53]:
            w = np.full(J, 1.0 / J)
            assert np.array_equal(smc.systematic_ancestors(w, u), np.arange(J))


def test_systematic_counts_and_order():
    rng = np.random.default_rng(3)
    for J in [5, 64, 300]:
        lw, _ = smc.normalise(3 * rng.standard_normal(J))
        w = np.exp(lw)
        a = smc.systematic_ancestors(w, rng.random())
        assert np.all(np.diff(a) >= 0)
        counts = np.bincount(a, minlength=J)
        assert counts.sum() == J
        lo = np.floor(J * w) - 1
        hi = np.ceil(J * w) + 1
        # up to the 2^-50 quantisation each count is floor or ceil of J w
        assert np.all(counts >= lo) and np.all(counts <= hi)
        assert np.all((counts == np.floor(J * w)) | (counts == np.ceil(J * w)) | (np.abs(J * w - np.round(J * w)) < 1e-9))


# ----------------------------------------------------------------- multinomial resampling
def _golden_multinomial():
    rows = []
    for line in open(os.path.join(GOLDEN, "multinomial.txt")):
        if line.startswith("#") or not line.strip():
            continue
        u, w, a = [p.strip() for p in line.split(";")]
        rows.append((np.array([float(x) for x in u.split()]), np.array([float(x) for x in w.split()]),
                     [int(x) for x in a.split()]))
    return rows


@pytest.mark.parametrize("case", range(3))
def test_multinomial_worked_examples(case):
    u, w, a = _golden_multinomial()[case]
    assert list(smc.multinomial_ancestors(w, u)) == a


def test_multinomial_agrees_with_the_float_inverse_cdf_and_ignores_uniform_order():
    rng = np.random.default_rng(14)
    J = 300
    for _ in range(10):
        lw, _ = smc.normalise(2 * rng.standard_normal(J))
        w = np.exp(lw)
        u = rng.random(J)
        a = smc.multinomial_ancestors(w, u)
        assert np.all(np.diff(a) >= 0)
        assert np.array_equal(a, smc.multinomial_ancestors(w, u[rng.permutation(J)]))
        cdf = np.cumsum(w)
        ref = np.sort(np.minimum(np.searchsorted(cdf, u, side="right"), J - 1))
        for k in np.nonzero(a != ref)[0]:
            # only a uniform within rounding distance of a boundary may land differently
            assert np.min(np.abs(cdf[:, None] - u[None, :])) < 1e-12


def test_multinomial_counts_follow_the_binomial_law():
    """Over 4000 draws with J = 8 the mean count of particle j is J w_j and its variance
    J w_j (1 - w_j); the sample means must lie within 5 standard errors."""
    rng = np.random.default_rng(15)
    w = np.array([0.02, 0.08, 0.1, 0.2, 0.25, 0.05, 0.3, 0.0])
    J, R = 8, 4000
    counts = np.zeros((R, J))
    for r in range(R):
        counts[r] = np.bincount(smc.multinomial_ancestors(w, rng.random(J)), minlength=J)
    mean = counts.mean(axis=0)
    se = np.sqrt(J * w * (1 - w) / R)
    assert np.all(np.abs(mean - J * w) <= 5 * se + 1e-12)
    assert np.all(counts[:, 7] == 0)
    var = counts.var(axis=0)
    assert np.all(np.abs(var - J * w * (1 - w)) <= 0.15 * J * w * (1 - w) + 1e-12)


def test_systematic_agrees_with_textbook_float_rule():
    rng = np.random.default_rng(4)
    J = 257
    for _ in range(20):
        lw, _ = smc.normalise(2 * rng.standard_normal(J))
        w = np.exp(lw)
        u = rng.random()
        a = smc.systematic_ancestors(w, u)
        cdf = np.cumsum(w)
        pts = (np.arange(J) + u) / J
        ref = np.minimum(np.searchsorted(cdf, pts, side="right"), J - 1)
        # disagreements may only occur when a point sits within rounding distance of a boundary
        for k in np.nonzero(a != ref)[0]:
            assert np.min(np.abs(cdf - pts[k])) < 1e-12


def test_placement_is_valid_in_place_arrangement():
    rng = np.random.default_rng(5)
    for J in [4, 50, 333]:
        lw, _ = smc.normalise(4 * rng.standard_normal(J))
        a = smc.systematic_ancestors(np.exp(lw), rng.random())
        p = smc.placement(a)
        assert sorted(p.tolist()) == sorted(a.tolist())
        counts = np.bincount(a, minlength=J)
        survivors = np.nonzero(counts > 0)[0]
        assert np.all(p[survivors] == survivors)
        # every source is a survivor, so copying slot p[k] -> k in any order is safe
        assert np.all(counts[p] > 0)


# ----------------------------------------------------------------- schedules
def test_schedule_golden_values():
    for line in open(os.path.join(GOLDEN, "schedules.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, K, N, C, kap, k, mk = line.split()
        f = schedules.SCHEDULES[name]
        assert f(int(k), int(K), int(N), int(C), int(kap)) == int(mk), line


def test_schedules_monotone_and_bounded():
    for name in schedules.SCHEDULES:
        s = schedules.sizes(name, 200, 60000, 500, 500)
        assert all(500 <= m <= 60000 for m in s)
        if name != "constant":
            assert all(b >= a for a, b in zip(s, s[1:]))
        assert s[0] == 500


# ----------------------------------------------------------------- Philox
def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        assert philox4x32(v[0:4], v[4:6]) == tuple(v[6:10])


# ----------------------------------------------------------------- move and weights
def _blr_sampler(n=40, d=2, h=0.02, S=1, seed=0, noise=0.5, prior=1.0):
    X, y, _ = smc_inputs.linreg(n, d, seed=seed, noise_std=noise)
    return smc.Sampler(X, y, [d, 1], "relu", "gaussian", noise_std=noise, prior_std=prior,
                       step_size=h, leapfrog_steps=S), X, y


def test_leapfrog_is_reversible():
    s, X, y = _blr_sampler(S=4, h=0.03)
    widths = [4, 6, 3]
    Xc = np.random.default_rng(0).standard_normal((30, 4))
    yc = np.random.default_rng(1).integers(0, 3, 30)
    for sampler in [s, smc.Sampler(Xc, yc, widths, "tanh", step_size=0.01, leapfrog_steps=3)]:
        D = sampler.D
        rng = np.random.default_rng(2)
        th = rng.standard_normal((3, D))
        P = rng.standard_normal((3, D))
        m = sampler.X.shape[0]
        _, g = sampler.loglik_grad(th, m, 1.7)
        th1, P1, _, g1 = sampler.leapfrog(th, P, g, m, 1.7)
        th2, P2, _, _ = sampler.leapfrog(th1, -P1, g1, m, 1.7)
        np.testing.assert_allclose(th2, th, atol=1e-11)
        np.testing.assert_allclose(-P2, P, atol=1e-11)


def test_weight_increment_is_minus_energy_error():
    # with a fixed target the L-kernel weight is exp(-(H(theta_k, P_k) - H(theta_{k-1}, P_{k-1})))
    # and the one-step energy error of leapfrog shrinks at least like h^2
    errs = []
    hs = [0.04, 0.02, 0.01, 0.005]
    for h in hs:
        s, X, y = _blr_sampler(h=h, S=1)
        th0 = smc_inputs.prior_draw(1, 16, 3, 1.0).astype(np.float64)
        s.init(th0, 40, 1.0)
        xi = smc_inputs.momenta(2, (16, 3))
        lp0 = s.lp.copy()
        H0 = -lp0 + 0.5 * np.sum(xi.astype(np.float64) ** 2, axis=1)
        s.step(40, 1.0, xi)
        inc = s.last_increment
        k0, k1 = s.kinetic
        H1 = -s.lp + k1
        np.testing.assert_allclose(inc, -(H1 - H0), rtol=1e-10, atol=1e-10)
        errs.append(np.max(np.abs(inc)))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert slope >= 2.0


def test_zero_step_telescopes_to_final_loglik():
    # h = 0 and no resampling: particles never move and
    # log w_K = lambda_K LL_K(theta_0) + const after normalisation
    X, y = smc_inputs.blobs(256, seed=0)
    widths = [2, 16, 2]
    s = smc.Sampler(X, y, widths, "tanh", step_size=0.0)
    th0 = smc_inputs.prior_draw(3, 32, mlp.n_params(widths), 1.0)
    sizes = schedules.sizes("linear", 5, 256, 32, 32)
    s.init(th0, sizes[0], 256 / sizes[0])
    for k in range(1, 6):
        s.step(sizes[k], 256 / sizes[k], smc_inputs.momenta(10 + k, th0.shape))
    lam = 256 / sizes[-1]
    expect, _ = smc.normalise(lam * mlp.loglik(th0, X[:sizes[-1]], y[:sizes[-1]], widths, "tanh"))
    np.testing.assert_allclose(s.logw, expect, atol=1e-9)


def test_nonfinite_particle_gets_zero_weight():
    X, y = smc_inputs.blobs(64, seed=0)
    s = smc.Sampler(X, y, [2, 16, 2], "tanh", step_size=1e-3)
    th0 = smc_inputs.prior_draw(3, 8, 82, 1.0).astype(np.float64)
    th0[3, 5] = np.nan
    s.init(th0, 64, 1.0)
    assert s.logw[3] == -np.inf and np.all(np.isfinite(np.delete(s.logw, 3)))
    th0[:, 0] = np.nan
    with pytest.raises(FloatingPointError):
        smc.Sampler(X, y, [2, 16, 2], "tanh").init(th0, 64, 1.0)


def test_blr_smc_matches_exact_posterior():
    # Data-annealed SMC with Langevin moves on Bayesian linear regression:
    # the weighted particle mean and covariance at the full data set (lambda = 1)
    # must match the closed-form Gaussian posterior.
    n, d, noise = 48, 2, 0.5
    X, y, _ = smc_inputs.linreg(n, d, seed=11, noise_std=noise)
    J = 4096
    s = smc.Sampler(X, y, [d, 1], "relu", "gaussian", noise_std=noise, prior_std=1.0,
                    step_size=0.03, leapfrog_steps=1)
    sizes = [8, 16, 24, 32, 40, 48] + [48] * 40
    s.init(smc_inputs.prior_draw(5, J, d + 1, 1.0), sizes[0], n / sizes[0])
    s.resample(smc_inputs.uniforms(6, 1)[0])
    for k in range(1, len(sizes)):
        s.step(sizes[k], n / sizes[k], smc_inputs.momenta(100 + k, (J, d + 1)))
        s.resample(smc_inputs.uniforms(200 + k, 1)[0])
    mu, cov = blr.posterior(X, y, noise, 1.0)
    w = np.exp(s.logw)
    mean = w @ s.theta
    sd = np.sqrt(np.diag(cov))
    # Across seeds this configuration's error has rms ~0.05 sd (resampling correlates
    # particles, so sd / sqrt(ESS) underestimates it); a dropped kinetic term in the
    # weight shrinks the spread to ~0.7 sd.
    assert np.all(np.abs(mean - mu) < 0.25 * sd)
    c = (s.theta - mean).T @ ((s.theta - mean) * w[:, None])
    np.testing.assert_allclose(np.sqrt(np.diag(c)), sd, rtol=0.08)


def test_blr_importance_sampling_only():
    # h = 0, no resampling: pure importance sampling from the prior to the lambda-scaled target
    n, d, noise = 6, 1, 1.0
    X, y, _ = smc_inputs.linreg(n, d, seed=12, noise_std=noise)
    J = 200000
    s = smc.Sampler(X, y, [d, 1], "relu", "gaussian", noise_std=noise, prior_std=1.0, step_size=0.0)
    s.init(smc_inputs.prior_draw(7, J, d + 1, 1.0), 3, 2.0)
    # the initial weights target the lambda-scaled 3-point posterior
    mu0, cov0 = blr.posterior(X[:3], y[:3], noise, 1.0, lam=2.0)
    w0 = np.exp(s.logw)
    assert np.all(np.abs(w0 @ s.theta - mu0) < 5 * np.sqrt(np.diag(cov0)) / math.sqrt(s.ess))
    s.step(6, 1.0, np.zeros((J, d + 1), np.float32))
    mu, cov = blr.posterior(X, y, noise, 1.0)
    w = np.exp(s.logw)
    mean = w @ s.theta
    assert np.all(np.abs(mean - mu) < 5 * np.sqrt(np.diag(cov)) / math.sqrt(s.ess))
    # evidence: the sum of log-normaliser increments estimates log p(y_{1:6}) when lambda_K = 1
    # (init uses lambda_0 = 2 on 3 points, then the 6-point target with lambda = 1)


def test_predictive_single_particle_is_softmax():
    X, y = smc_inputs.blobs(20, seed=1)
    widths = [2, 16, 2]
    th = smc_inputs.prior_draw(1, 1, 82, 1.0)
    probs, acc, mlpd = smc.predictive(th, np.zeros(1), X, y, widths, "tanh")
    ref = np.exp(mlp.predict_logprobs(th, X, widths, "tanh")[0])
    np.testing.assert_allclose(probs, ref, rtol=1e-14)
    assert acc == np.mean(np.argmax(ref, 1) == y)
    np.testing.assert_allclose(mlpd, np.mean(np.log(ref[np.arange(20), y])), rtol=1e-13)


def test_predictive_ties_take_lowest_class():
    theta = np.zeros((1, 82))
    X = np.zeros((3, 2))
    _, acc0, _ = smc.predictive(theta, np.zeros(1), X, np.zeros(3, int), [2, 16, 2], "tanh")
    _, acc1, _ = smc.predictive(theta, np.zeros(1), X, np.ones(3, int), [2, 16, 2], "tanh")
    assert acc0 == 1.0 and acc1 == 0.0


def test_predictive_mixture_of_three_particles_worked_by_hand():
    # Section 2 (posterior estimates): p(y | x) = sum_j w~_j p(y | x, theta_j) and the mean log
    # predictive is mean_i log sum_j w~_j p(y_i | x_i, theta_j).  A network without hidden
    # layer, widths [2, 2]: class 0 has weights and bias zero, class 1 weight (a_j, 0) and bias
    # c_j, so p_j(1 | x) = r / (1 + r) with r = exp(c_j + a_j x_1).  Particle j is chosen with
    # p_j(1 | x_1 = 0) = P0[j] and p_j(1 | x_1 = 1) = P1[j].
    P0 = np.array([0.5, 0.2, 0.9])
    P1 = np.array([0.25, 0.6, 0.1])
    w = np.array([0.2, 0.3, 0.5])
    c = np.log(P0 / (1 - P0))
    a = np.log(P1 / (1 - P1)) - c
    theta = np.zeros((3, 6))          # rows [w00 w01 b0 | w10 w11 b1]
    theta[:, 3] = a
    theta[:, 5] = c
    X = np.array([[0.0, 7.0], [1.0, -3.0], [0.0, 0.5]])   # x_2 has zero weight everywhere
    y = np.array([1, 0, 0])
    probs, acc, mlpd = smc.predictive(theta, np.log(w), X, y, [2, 2], "relu")
    # mixture probabilities of class 1, worked by hand: 0.2*0.5 + 0.3*0.2 + 0.5*0.9 = 0.61 and
    # 0.2*0.25 + 0.3*0.6 + 0.5*0.1 = 0.28
    np.testing.assert_allclose(probs[:, 1], [0.61, 0.28, 0.61], rtol=1e-13)
    np.testing.assert_allclose(probs.sum(1), 1.0, rtol=1e-14)
    # labels 1, 0, 0: the arg-max is 1, 0, 1, so two of three are right
    assert acc == 2.0 / 3.0
    ref = (math.log(0.61) + math.log(0.72) + math.log(0.39)) / 3.0
    np.testing.assert_allclose(mlpd, ref, rtol=1e-13)
    # the two plausible mistakes give other values: averaging log-probabilities over particles
    # and weighting log p linearly
    avg_log = np.mean([np.mean(np.log(p)) for p in ([0.5, 0.2, 0.9], [0.75, 0.4, 0.9], [0.5, 0.8, 0.1])])
    lin_log = np.mean([w @ np.log(p) for p in ([0.5, 0.2, 0.9], [0.75, 0.4, 0.9], [0.5, 0.8, 0.1])])
    assert abs(mlpd - avg_log) > 0.05 and abs(mlpd - lin_log) > 0.05


def test_predictive_weights_are_used_as_normalised_log_weights():
    # the same mixture with the weights supplied as log w~ of unequal particles in another
    # order: the estimate does not depend on the particles' order
    P0 = np.array([0.9, 0.5, 0.2])
    w = np.array([0.5, 0.2, 0.3])
    theta = np.zeros((3, 6))
    theta[:, 5] = np.log(P0 / (1 - P0))
    X = np.zeros((2, 2))
    probs, acc, mlpd = smc.predictive(theta, np.log(w), X, np.array([1, 1]), [2, 2], "tanh")
    np.testing.assert_allclose(probs[:, 1], 0.61, rtol=1e-13)
    assert acc == 1.0
    np.testing.assert_allclose(mlpd, math.log(0.61), rtol=1e-13)
