"""Exact posterior of Bayesian linear regression (test infrastructure, closed-form pin).

With a Gaussian likelihood N(y_i; x_i^T w + b, sigma^2), a N(0, sigma_p^2 I)
prior on theta = (w, b) and the subset likelihood raised to lambda = N / M
(the scaled target of Section 3), the target is Gaussian with

    Sigma = (I / sigma_p^2 + lambda * Xa^T Xa / sigma^2)^{-1}
    mu    = Sigma * lambda * Xa^T y / sigma^2

where Xa = [X | 1] appends the bias input.  SMC weighted means and covariances
must converge to (mu, Sigma).
"""
from __future__ import annotations

import numpy as np


def posterior(X, y, noise_std, prior_std, lam=1.0):
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Xa = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    prec = np.eye(Xa.shape[1]) / prior_std ** 2 + lam * Xa.T @ Xa / noise_std ** 2
    cov = np.linalg.inv(prec)
    mean = cov @ (lam * Xa.T @ y / noise_std ** 2)
    return mean, cov


def log_evidence(X, y, noise_std, prior_std):
    """log p(y_{1:M}) for lambda = 1 (marginal likelihood of the linear model)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Xa = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    cov_y = prior_std ** 2 * Xa @ Xa.T + noise_std ** 2 * np.eye(X.shape[0])
    sign, logdet = np.linalg.slogdet(cov_y)
    return -0.5 * (y @ np.linalg.solve(cov_y, y) + logdet + X.shape[0] * np.log(2 * np.pi))
