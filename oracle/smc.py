"""FP64 SMC sampler with gradient-based moves and data annealing (test infrastructure).

Follows Section 2 (SMC samplers), Section 2.1 (Markov and L-kernels) and
Section 3 (batch inference and data annealing) step by step:

* initialisation: theta_0 ~ q0, w_0 = pi_0(theta_0) / q0(theta_0)      (Eq. init_weight)
* move: S leapfrog steps (Eqs. mom_first, pos_update, mom_second);
        Langevin dynamics is S = 1
* reweighting with the reversed-momentum L-kernel, whose Jacobians cancel
  (Eqs. q_prop, l=q_deriv, weight_update_fp):
        w_k = w_{k-1} * pi_k(theta_k) / pi_{k-1}(theta_{k-1})
                      * N(-P_k; 0, M) / N(P_{k-1}; 0, M)
* normalisation (Eq. normalise), effective sample size (Eq. jeff), resampling
  when the ESS falls below J/2, weights reset to 1/J
* posterior estimates E[f] ~ sum_j w~_j f(theta_j)

Readings taken where the paper is silent:
* target: log pi_k(theta) = lambda_k * LL_k(theta) - |theta|^2 / (2 sigma_p^2),
  lambda_k = N / M_k scales both the log-likelihood and its gradient
  (Section 3: stochastic estimates of log-likelihoods and gradients);
* the weight's denominator is the previous target at the previous state,
  cached from the previous iteration;
* the gradient at theta_{k-1} is recomputed on the new subset when the subset
  (and so lambda) changed, otherwise the final gradient of the previous move is
  reused;
* mass matrix M = I;
* resampling is systematic (the paper uses multinomial, also provided) with
  the exact integer rule of ``systematic_ancestors``; the ESS test is strict (< J/2) and
  is applied after every reweighting, including the initial one;
* a particle whose log-likelihood is not finite gets log-weight -inf.

All arithmetic is float64.  The random numbers the method consumes (momenta,
the resampling offset u) are passed in by the caller.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp

FIX_BITS = 50  # weight quantisation for the exact systematic-resampling rule


# --------------------------------------------------------------------------- weights
def log_sum_exp(v):
    """log sum_j exp(v_j), shifted by the maximum; -inf if every entry is -inf."""
    v = np.asarray(v, dtype=np.float64)
    m = np.max(v)
    if not np.isfinite(m):
        return m
    return m + math.log(np.sum(np.exp(v - m)))


def normalise(logw):
    """Normalised log-weights log w~ and the normaliser log sum_j w_j (Eq. normalise)."""
    lz = log_sum_exp(logw)
    return np.asarray(logw, dtype=np.float64) - lz, lz


def ess(logw_normalised):
    """J_eff = 1 / sum_j w~_j^2 (Eq. jeff), from normalised log-weights."""
    w = np.exp(np.asarray(logw_normalised, dtype=np.float64))
    return 1.0 / np.sum(w * w)


# --------------------------------------------------------------------------- resampling
def systematic_ancestors(w, u):
    """Systematic resampling with exact integer arithmetic.

    One offset u in [0, 1) places the J points (k + u) / J, k = 0..J-1, on the
    cumulative distribution of the normalised weights w.  To make the result
    independent of summation order, the weights are quantised first:

        Q_j = floor(w_j * 2^50)          (exact: power-of-two scale, then floor)
        S_j = Q_0 + ... + Q_j            (exact integer prefix sums), T = S_{J-1}
        R   = min(floor(u * T), T - 1)   (one correctly rounded FP64 product)
        t_k = floor((k * T + R) / J)     (exact integer division)
        a_k = #{ j : S_j <= t_k }        (the first j whose S_j exceeds t_k)

    The ancestors are non-decreasing and each particle is chosen
    floor(J w_j) or ceil(J w_j) times, up to the quantisation.
    """
    w = np.asarray(w, dtype=np.float64)
    J = w.shape[0]
    Q = [int(math.floor(float(x) * float(2 ** FIX_BITS))) for x in w]
    S = []
    acc = 0
    for q in Q:
        acc += q
        S.append(acc)
    T = S[-1]
    if T <= 0:
        raise ValueError("all weights quantise to zero")
    R = min(int(math.floor(float(u) * float(T))), T - 1)
    anc = np.empty(J, dtype=np.int64)
    for k in range(J):
        t = (k * T + R) // J
        # first index whose inclusive prefix sum exceeds t
        lo, hi = 0, J - 1
        while lo < hi:
            mid = (lo + hi) // 2
            if S[mid] > t:
                hi = mid
            else:
                lo = mid + 1
        anc[k] = lo
    return anc


def multinomial_ancestors(w, uniforms):
    """Multinomial resampling (the paper's scheme, Section 2) with the same exact integer rule.

    J independent uniforms U_k in [0, 1) are placed on the quantised cumulative
    distribution of ``systematic_ancestors``:

        t_k = min(floor(U_k * T), T - 1)   (one correctly rounded FP64 product each)
        a_k = #{ j : S_j <= t_k }

    and the ancestors are returned in non-decreasing order (the order of the
    uniforms does not matter).  Particle j is chosen Binomial(J, Q_j / T) times.
    """
    w = np.asarray(w, dtype=np.float64)
    u = np.asarray(uniforms, dtype=np.float64)
    J = w.shape[0]
    if u.shape != (J,):
        raise ValueError("one uniform per particle")
    Q = [int(math.floor(float(x) * float(2 ** FIX_BITS))) for x in w]
    S = []
    acc = 0
    for q in Q:
        acc += q
        S.append(acc)
    T = S[-1]
    if T <= 0:
        raise ValueError("all weights quantise to zero")
    anc = []
    for k in range(J):
        t = min(int(math.floor(float(u[k]) * float(T))), T - 1)
        lo, hi = 0, J - 1
        while lo < hi:
            mid = (lo + hi) // 2
            if S[mid] > t:
                hi = mid
            else:
                lo = mid + 1
        anc.append(lo)
    return np.array(sorted(anc), dtype=np.int64)


def placement(ancestors):
    """In-place arrangement of the resampled population.

    Every particle that survives keeps its own slot; the slots of particles
    that die receive the surplus copies, dead slots in increasing order paired
    with surplus copies in increasing source order.  The multiset of sources
    equals the ancestor vector.
    """
    anc = np.asarray(ancestors, dtype=np.int64)
    J = anc.shape[0]
    counts = np.bincount(anc, minlength=J)
    extra = []
    for j in range(J):
        extra.extend([j] * max(int(counts[j]) - 1, 0))
    p = np.arange(J, dtype=np.int64)
    r = 0
    for k in range(J):
        if counts[k] == 0:
            p[k] = extra[r]
            r += 1
    assert r == len(extra)
    return p


# --------------------------------------------------------------------------- sampler
class Sampler:
    """Data-annealed SMC sampler over an MLP posterior, FP64.

    X, y hold the data already in annealing order: the subset at iteration k
    is the first M_k rows (mini-batches drawn without replacement and appended
    cumulatively, Section 3).
    """

    def __init__(self, X, y, widths, act, likelihood=mlp.CATEGORICAL, noise_std=1.0,
                 prior_std=1.0, step_size=1e-3, leapfrog_steps=1, ess_frac=0.5, model=None):
        self.X = np.asarray(X, dtype=np.float64)
        self.y = np.asarray(y)
        self.widths = list(widths) if widths is not None else None
        self.act = act
        self.likelihood = likelihood
        self.noise_std = float(noise_std)
        self.prior_std = float(prior_std)
        self.h = float(step_size)
        self.S = int(leapfrog_steps)
        self.ess_frac = float(ess_frac)
        # another network (e.g. oracle.cnn.Model) replaces the dense one when given
        self.model = model
        self.D = model.D if model is not None else mlp.n_params(self.widths)

    # ---- target (reading: lambda scales LL and gradient; Gaussian prior)
    def loglik_grad(self, theta, m, lam):
        """(LL_m(theta) [J], grad log pi(theta) [J x D]) on the first m samples."""
        if self.model is not None:
            ll, g = self.model.loglik_grad(theta, self.X[:m], self.y[:m], np.full(theta.shape[0], lam))
        else:
            ll, g = mlp.loglik_grad(theta, self.X[:m], self.y[:m], self.widths, self.act,
                                    self.likelihood, self.noise_std,
                                    scale=np.full(theta.shape[0], lam))
        return ll, g - theta / self.prior_std ** 2

    def log_target(self, ll, theta, lam):
        return lam * ll - np.sum(theta * theta, axis=1) / (2.0 * self.prior_std ** 2)

    # ---- two-segment target (smooth data annealing, Section 3.1):
    #      log pi(theta) = lam_a LL[0, split) + lam_b LL[split, m) + log q0(theta)
    def _segment(self, theta, lo, hi, lam):
        """(LL on samples [lo, hi) [J], lam * its gradient [J x D]); zeros when the range is empty."""
        J = theta.shape[0]
        if hi <= lo:
            return np.zeros(J), np.zeros_like(theta)
        sc = np.full(J, lam)
        if self.model is not None:
            return self.model.loglik_grad(theta, self.X[lo:hi], self.y[lo:hi], sc)
        return mlp.loglik_grad(theta, self.X[lo:hi], self.y[lo:hi], self.widths, self.act,
                               self.likelihood, self.noise_std, scale=sc)

    def segment_loglik_grad(self, theta, m, split, lam_a, lam_b):
        """(LL on the first m samples [J], LL on samples [split, m) [J], grad log pi(theta) [J x D])."""
        split = min(int(split), int(m))
        ll_a, g_a = self._segment(theta, 0, split, lam_a)
        ll_b, g_b = self._segment(theta, split, int(m), lam_b)
        return ll_a + ll_b, ll_b, g_a + g_b - theta / self.prior_std ** 2

    def segment_log_target(self, ll, ll_b, theta, lam_a, lam_b):
        return lam_a * (ll - ll_b) + lam_b * ll_b - np.sum(theta * theta, axis=1) / (2.0 * self.prior_std ** 2)

    # ---- Eq. init_weight
    def init(self, theta0, m0, lam0):
        self.theta = np.asarray(theta0, dtype=np.float64).copy()
        self.m, self.lam = int(m0), float(lam0)
        self.tgt = None
        ll, g = self.loglik_grad(self.theta, self.m, self.lam)
        self.ll, self.g = ll, g
        self.lp = self.log_target(ll, self.theta, self.lam)
        # pi_0 / q0 with q0 the prior: the prior factors cancel
        logw = self.lam * ll
        logw = np.where(np.isfinite(logw), logw, -np.inf)
        self._finish_reweight(logw, np.zeros_like(logw))
        return self

    def _finish_reweight(self, logw_unnormalised, prev_logw):
        if not np.any(np.isfinite(logw_unnormalised)):
            raise FloatingPointError("every particle has a non-finite log-weight")
        self.logw, lz = normalise(logw_unnormalised)
        self.log_z_increment = lz - log_sum_exp(prev_logw)
        self.ess = ess(self.logw)

    # ---- S leapfrog steps with M = I (Eqs. mom_first, pos_update, mom_second)
    def leapfrog(self, theta, P, g, m, lam):
        """(theta_S, P_S, LL(theta_S), grad log pi(theta_S)) from (theta, P) with g at theta."""
        ll = None
        for _ in range(self.S):
            P = P + 0.5 * self.h * g
            theta = theta + self.h * P
            ll, g = self.loglik_grad(theta, m, lam)
            P = P + 0.5 * self.h * g
        return theta, P, ll, g

    # ---- one move + reweight (Eqs. mom_first .. weight_update_fp)
    def step(self, m, lam, xi):
        """Move every particle with S leapfrog steps from momentum xi, then reweight."""
        m, lam = int(m), float(lam)
        if m < self.m:
            raise ValueError("the annealed subset only grows")
        if (m, lam) != (self.m, self.lam) or self.tgt is not None:
            self.m, self.lam, self.tgt = m, lam, None
            _, self.g = self.loglik_grad(self.theta, m, lam)
        P = np.asarray(xi, dtype=np.float64).copy()
        kinetic0 = 0.5 * np.sum(P * P, axis=1)
        theta, P, ll, g = self.leapfrog(self.theta, P, self.g, m, lam)
        kinetic1 = 0.5 * np.sum(P * P, axis=1)
        lp_new = self.log_target(ll, theta, lam)
        incr = lp_new - self.lp - kinetic1 + kinetic0
        self.last_increment = incr
        logw = self.logw + incr
        logw = np.where(np.isfinite(incr) & np.isfinite(ll), logw, -np.inf)
        self.theta, self.g, self.ll, self.lp = theta, g, ll, lp_new
        self.kinetic = (kinetic0, kinetic1)
        self._finish_reweight(logw, self.logw)
        return self

    def step_tempered(self, m, split, lam_a, lam_b, xi):
        """step() for the two-segment target: samples [0, split) weigh lam_a, samples
        [split, m) weigh lam_b (a split at or beyond m is the one-segment target with lam_a).
        Keeps the second segment's log-likelihood at the new state in ll_b."""
        m = int(m)
        split = min(int(split), m)
        lam_a = float(lam_a)
        lam_b = float(lam_b) if split < m else lam_a
        if m < self.m:
            raise ValueError("the annealed subset only grows")
        tgt = (m, split, lam_a, lam_b)
        if tgt != self.tgt:
            self.m, self.lam, self.tgt = m, None, tgt
            _, _, self.g = self.segment_loglik_grad(self.theta, *tgt)
        P = np.asarray(xi, dtype=np.float64).copy()
        kinetic0 = 0.5 * np.sum(P * P, axis=1)
        theta, g = self.theta, self.g
        for _ in range(self.S):
            P = P + 0.5 * self.h * g
            theta = theta + self.h * P
            ll, ll_b, g = self.segment_loglik_grad(theta, *tgt)
            P = P + 0.5 * self.h * g
        kinetic1 = 0.5 * np.sum(P * P, axis=1)
        lp_new = self.segment_log_target(ll, ll_b, theta, lam_a, lam_b)
        incr = lp_new - self.lp - kinetic1 + kinetic0
        self.last_increment = incr
        logw = self.logw + incr
        logw = np.where(np.isfinite(incr) & np.isfinite(ll), logw, -np.inf)
        self.theta, self.g, self.ll, self.ll_b, self.lp = theta, g, ll, ll_b, lp_new
        self.kinetic = (kinetic0, kinetic1)
        self._finish_reweight(logw, self.logw)
        return self

    # ---- resampling when the ESS drops below ess_frac * J
    def resample(self, u, mode="if_needed", scheme="systematic"):
        """u: the systematic offset, or for scheme="multinomial" the J uniforms."""
        J = self.theta.shape[0]
        if mode == "never" or (mode == "if_needed" and not (self.ess < self.ess_frac * J)):
            self.ancestors = None
            return False
        w = np.exp(self.logw)
        if scheme == "multinomial":
            self.ancestors = multinomial_ancestors(w, u)
        else:
            self.ancestors = systematic_ancestors(w, u)
        p = placement(self.ancestors)
        self.placement = p
        self.theta = self.theta[p]
        self.g = self.g[p]
        self.ll = self.ll[p]
        if getattr(self, "ll_b", None) is not None:
            self.ll_b = self.ll_b[p]
        self.lp = self.lp[p]
        self.logw = np.full(J, -math.log(J))
        self.ess = float(J)
        return True

    # ---- posterior predictive (Section 2, posterior estimates)
    def predictive(self, Xt, yt=None):
        """Weighted mixture of per-particle softmax probabilities.

        Returns (probs [n x C], accuracy or None, mean log predictive or None).
        Accuracy uses the arg-max with the lowest class index on ties.
        """
        return predictive(self.theta, self.logw, Xt, yt, self.widths, self.act, self.model)

    def posterior_mean(self):
        return np.exp(self.logw) @ self.theta


def predictive(theta, logw, Xt, yt, widths, act, model=None):
    if model is not None:
        lp = model.predict_logprobs(theta, Xt)                 # [J x n x C]
    else:
        lp = mlp.predict_logprobs(theta, Xt, widths, act)      # [J x n x C]
    lw = np.asarray(logw, dtype=np.float64)
    probs = np.einsum("j,jnc->nc", np.exp(lw), np.exp(lp))
    if yt is None:
        return probs, None, None
    yt = np.asarray(yt, dtype=np.int64)
    pred = np.argmax(probs, axis=1)  # numpy returns the first maximum
    acc = float(np.mean(pred == yt))
    lpy = lp[:, np.arange(len(yt)), yt] + lw[:, None]            # [J x n]
    mlpd = float(np.mean([log_sum_exp(lpy[:, i]) for i in range(lpy.shape[1])]))
    return probs, acc, mlpd
