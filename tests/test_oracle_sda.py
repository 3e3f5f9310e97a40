"""Pins for the oracle's smooth data annealing (Section 3.1): weighted moments, the beta
updates, the mini-batch append rule and the two-segment tempered target (CPU only)."""
import numpy as np
import pytest

from oracle import mlp, sda, smc
import smc_inputs


# ----------------------------------------------------------------- weighted moments (Eq. E{XY})
def test_uniform_weights_give_the_population_moments():
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(37), 3.0 + 2.0 * rng.standard_normal(37)
    var_b, cov = sda.weighted_moments(np.full(37, 1 / 37), a, b)
    assert abs(var_b - np.var(b)) < 1e-12
    assert abs(cov - np.cov(a, b, bias=True)[0, 1]) < 1e-12


def test_moments_under_a_point_mass_vanish_and_are_shift_invariant():
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(8), rng.standard_normal(8)
    w = np.zeros(8)
    w[3] = 1.0
    assert sda.weighted_moments(w, a, b) == (0.0, 0.0)
    w = rng.uniform(size=8)
    w /= w.sum()
    v0, c0 = sda.weighted_moments(w, a, b)
    v1, c1 = sda.weighted_moments(w, a + 5.0, b - 7.0)
    assert abs(v0 - v1) < 1e-12 and abs(c0 - c1) < 1e-12


def test_zero_weight_particles_do_not_enter():
    w = np.array([0.5, 0.0, 0.5])
    a = np.array([1.0, np.inf, 3.0])
    b = np.array([2.0, -np.inf, 4.0])
    assert sda.weighted_moments(w, a, b) == sda.weighted_moments(np.array([0.5, 0.5]), a[[0, 2]], b[[0, 2]])
    assert sda.weighted_moments(w, a, b) == (1.0, 1.0)


# ----------------------------------------------------------------- beta updates
W4 = np.full(4, 0.25)
OH = np.array([1.0, 2.0, 3.0, 4.0])  # E = 2.5, Var = 1.25


def test_beta_update_without_new_data_flips_the_sign():
    # beta - dS / Var = 0.1 - 0.8 would decrease beta, so the step is +0.8
    assert abs(sda.next_beta(0.1, W4, np.zeros(4), OH, annealed=False) - 0.9) < 1e-15
    # the covariance term is ignored before any mini-batch was appended
    assert abs(sda.next_beta(0.1, W4, -OH, OH, annealed=False) - 0.9) < 1e-15


def test_beta_update_after_an_append_uses_var_plus_cov():
    # Omega = Omega^: Var + Cov = 2.5, step 0.4 after the sign flip
    assert abs(sda.next_beta(0.1, W4, OH, OH, annealed=True) - 0.5) < 1e-15
    # Omega = -2 Omega^: Var + Cov = -1.25, so beta - dS / (Var + Cov) = beta + 0.8 already increases
    assert abs(sda.next_beta(0.1, W4, -2.0 * OH, OH, annealed=True) - 0.9) < 1e-15


def test_beta_is_clipped_to_one():
    assert sda.next_beta(0.7, W4, np.zeros(4), OH, annealed=False) == 1.0
    assert sda.next_beta(0.1, W4, np.zeros(4), 0.1 * OH, annealed=False) == 1.0


def test_next_target_appends_a_mini_batch_after_beta_reached_one():
    w, ll = W4, -OH
    assert sda.next_target((100, 0, 1.0), w, ll, ll, N=1000, kappa=100) == (200, 100, 0.1)
    assert sda.next_target((900, 800, 1.0), w, ll, ll, N=1000, kappa=300) == (1000, 900, 0.1)
    assert sda.next_target((1000, 900, 1.0), w, ll, ll, N=1000, kappa=100) == (1000, 900, 1.0)
    # otherwise beta moves and the subset stays
    m, split, beta = sda.next_target((100, 0, 0.1), w, ll, ll, N=1000, kappa=100)
    assert (m, split) == (100, 0) and abs(beta - 0.9) < 1e-15


def test_next_target_splits_the_log_likelihood_into_its_segments():
    # ll on [0, m) and ll_b on [split, m): Omega = -(ll - ll_b), Omega^ = -ll_b
    ll_b = -OH
    ll = ll_b + (-OH)  # Omega = Omega^: as in the Var + Cov pin above
    _, _, beta = sda.next_target((200, 100, 0.1), W4, ll, ll_b, N=1000, kappa=100)
    assert abs(beta - 0.5) < 1e-15


# ----------------------------------------------------------------- two-segment tempered target
WIDTHS = [2, 5, 2]


def _sampler(n=40, act="tanh"):
    X, y = smc_inputs.blobs(n, seed=3)
    return smc.Sampler(X, y, WIDTHS, act, prior_std=1.3), X, y


def _theta(J, seed=4):
    return smc_inputs.prior_draw(seed, J, mlp.n_params(WIDTHS), 0.8).astype(np.float64)


def test_segment_target_reduces_to_the_one_segment_target():
    s, _, _ = _sampler()
    th = _theta(5)
    ll, g = s.loglik_grad(th, 30, 1.7)
    ll2, llb, g2 = s.segment_loglik_grad(th, 30, 30, 1.7, 0.3)
    assert np.array_equal(ll, ll2) and np.array_equal(g, g2) and np.all(llb == 0.0)
    ll3, llb3, g3 = s.segment_loglik_grad(th, 30, 12, 1.7, 1.7)
    np.testing.assert_allclose(ll3, ll, rtol=1e-13)
    np.testing.assert_allclose(g3, g, rtol=1e-11, atol=1e-12)


def test_segment_target_against_per_sample_sums():
    """Brute force: log pi = 0.6 sum_{i<12} log p_i + 0.25 sum_{12<=i<30} log p_i + log q0."""
    s, X, y = _sampler()
    th = _theta(4)
    Xs = s.X
    per = mlp.per_sample_loglik(th, Xs[:30], s.y[:30], WIDTHS, "tanh")  # [J x n]
    ll, llb, _ = s.segment_loglik_grad(th, 30, 12, 0.6, 0.25)
    np.testing.assert_allclose(ll, per.sum(axis=1), rtol=1e-13)
    np.testing.assert_allclose(llb, per[:, 12:].sum(axis=1), rtol=1e-13)
    lp = s.segment_log_target(ll, llb, th, 0.6, 0.25)
    ref = 0.6 * per[:, :12].sum(axis=1) + 0.25 * per[:, 12:].sum(axis=1) - np.sum(th * th, axis=1) / (2 * 1.3 ** 2)
    np.testing.assert_allclose(lp, ref, rtol=1e-13)


def test_segment_gradient_against_central_differences():
    s, _, _ = _sampler()
    th = _theta(3)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(th.shape)
    v /= np.linalg.norm(v, axis=1, keepdims=True)

    def lp(t):
        ll, llb, _ = s.segment_loglik_grad(t, 30, 12, 0.6, 0.25)
        return s.segment_log_target(ll, llb, t, 0.6, 0.25)

    _, _, g = s.segment_loglik_grad(th, 30, 12, 0.6, 0.25)
    eps = 1e-5
    fd = (lp(th + eps * v) - lp(th - eps * v)) / (2 * eps)
    np.testing.assert_allclose(fd, np.sum(g * v, axis=1), rtol=1e-7, atol=1e-9)


def test_tempered_step_with_the_split_at_m_is_the_plain_step():
    th0 = _theta(6, seed=7)
    xi = smc_inputs.momenta(8, th0.shape).astype(np.float64)
    a, _, _ = _sampler()
    b, _, _ = _sampler()
    a.init(th0, 20, 2.0)
    b.init(th0, 20, 2.0)
    a.step(30, 40 / 30, xi)
    b.step_tempered(30, 30, 40 / 30, 0.5, xi)
    assert np.array_equal(a.theta, b.theta) and np.array_equal(a.logw, b.logw)


def test_sda_run_anneals_every_sample_in():
    """A small SDA run with the oracle: beta rises within each phase, a mini-batch is appended
    after each iteration at beta = 1, and the run ends on the full posterior."""
    s, _, _ = _sampler(n=40)
    J, C, kappa, N = 16, 10, 10, 40
    s.init(_theta(J, seed=11), C, 0.1)
    state = (C, 0, 0.1)
    seen = [state]
    for k in range(200):
        xi = smc_inputs.momenta(100 + k, (J, s.D)).astype(np.float64)
        s.step_tempered(state[0], state[1], 1.0, state[2], xi)
        s.resample(smc_inputs.uniforms(200 + k, 1)[0])
        nxt = sda.next_target(state, np.exp(s.logw), s.ll, s.ll_b, N, kappa)
        if nxt[0] == state[0]:
            assert nxt[2] > state[2] or nxt[2] == 1.0
        else:
            assert state[2] == 1.0 and nxt == (state[0] + kappa, state[0], 0.1)
        state = nxt
        seen.append(state)
        if state == (N, N - kappa, 1.0) and seen[-2] == state:
            break
    assert state[0] == N and state[2] == 1.0
    assert len({m for m, _, _ in seen}) == (N - C) // kappa + 1
