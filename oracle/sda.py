"""Smooth data annealing (SDA) moments and tempering updates (test infrastructure).

Section 3.1: with Omega_k = -log p(y_{1:M_{k-1}} | theta) on the data already
annealed in and Omega^_k = -log p(y_{M_{k-1}+1:M_k} | theta) on the newest
mini-batch, the tempering exponent beta is moved so that the entropy changes
at a constant rate dS.  Weighted moments use the normalised weights (Eq. E{XY}
and the lines before it).

Readings: the update without new data is Eq. beta_initial_data_k and the
update after a mini-batch was appended is Eq. beta_annealed_k; if an update
would not increase beta the sign of dS is flipped (equivalently the magnitude
of the step is used); beta is clipped to 1, and after an iteration whose
target had beta = 1 a new mini-batch is appended and beta restarts at 0.1.
The initial phase tempers the first C samples (Eq. sda_initial_target): it is
the two-segment target with nothing fully annealed in (Omega = 0).  Once every
sample is annealed in and beta = 1 the target stays the full posterior.
"""
from __future__ import annotations

import numpy as np


def weighted_moments(w, omega, omega_hat):
    """(Var(Omega^), Cov(Omega, Omega^)) under normalised weights w.  A particle of zero
    weight does not enter the sums (its log-likelihood may be infinite)."""
    w = np.asarray(w, dtype=np.float64)
    keep = w > 0.0
    w = w[keep]
    a = np.asarray(omega, dtype=np.float64)[keep]
    b = np.asarray(omega_hat, dtype=np.float64)[keep]
    e_b = np.sum(w * b)
    var_b = np.sum(w * b * b) - e_b * e_b
    e_a = np.sum(w * a)
    cov = np.sum(w * a * b) - e_a * e_b
    return var_b, cov


def next_beta(beta, w, omega, omega_hat, annealed: bool, dS: float = 1.0):
    """beta_{k+1} from beta_k (Eqs. beta_initial_data_k, beta_annealed_k)."""
    var_b, cov = weighted_moments(w, omega, omega_hat)
    denom = var_b + cov if annealed else var_b
    step = -dS / denom
    if not np.isfinite(step) or step <= 0.0:
        step = abs(dS / denom) if np.isfinite(denom) and denom != 0.0 else 1.0
    return min(1.0, beta + step)


def next_target(state, w, ll, ll_b, N, kappa, beta0=0.1, dS=1.0):
    """The SDA target after the iteration run at state = (m, split, beta).

    The target is p(y[0:split] | theta) p(y[split:m] | theta)^beta q0(theta); ll and
    ll_b are the particles' log-likelihoods on [0, m) and [split, m) at the current
    state and w their normalised weights.  Returns the next (m, split, beta).
    """
    m, split, beta = int(state[0]), int(state[1]), float(state[2])
    if beta >= 1.0:
        if m >= N:
            return m, split, 1.0
        return min(m + int(kappa), int(N)), m, float(beta0)
    ll = np.asarray(ll, dtype=np.float64)
    ll_b = np.asarray(ll_b, dtype=np.float64)
    omega_hat = -ll_b
    omega = -(ll - ll_b)
    return m, split, next_beta(beta, w, omega, omega_hat, annealed=split > 0, dS=dS)
