"""The five naive data-annealing schedules of Section 3.1 (test infrastructure).

C is the initial batch size, kappa the mini-batch increment, K the number of
iterations and N the dataset size; M_k is the subset size at iteration k.
Iteration 0 is the initial weighting with M_0 = C; moves run for k = 1..K.
The test k < 0.9 K compares real numbers.

Readings where the paper is silent or its formula can leave [C, N]:
* Linear is clamped to N (kappa k + C can exceed N before 0.9 K);
* Automated rounds C + floor((N - C) / (0.9 K)) k to the nearest multiple of
  kappa, halves rounding up, and clamps to [C, N].
"""
from __future__ import annotations

from fractions import Fraction


def _before_refine(k: int, K: int) -> bool:
    return Fraction(k) < Fraction(9, 10) * K


def constant(k, K, N, C, kappa):
    return C


def full_batch(k, K, N, C, kappa):
    return N


def constant_to_refine(k, K, N, C, kappa):
    return C if _before_refine(k, K) else N


def linear(k, K, N, C, kappa):
    if _before_refine(k, K):
        return min(kappa * k + C, N)
    return N


def automated(k, K, N, C, kappa):
    if not _before_refine(k, K):
        return N
    slope = (Fraction(N - C) / (Fraction(9, 10) * K)).__floor__()
    raw = C + slope * k
    mult = (2 * raw + kappa) // (2 * kappa)  # nearest multiple, halves up
    return max(C, min(N, mult * kappa))


SCHEDULES = {
    "constant": constant,
    "fb": full_batch,
    "ctr": constant_to_refine,
    "linear": linear,
    "automated": automated,
}


def sizes(name, K, N, C, kappa):
    """[M_0, M_1, ..., M_K] for the named schedule (M_0 = C)."""
    f = SCHEDULES[name]
    return [C] + [f(k, K, N, C, kappa) for k in range(1, K + 1)]


# ---------------------------------------------------------------------------
# Adaptive growth by the posterior-mean criterion.  The paper motivates growing
# the subset only once the sampler has settled on the current one; here the
# settling test is the relative change of the weighted posterior mean
# theta_bar_k = sum_j w~_j theta_j (the Section 2 estimator with f = identity):
# a mini-batch of kappa points is appended when
#     |theta_bar_k - theta_bar_{k-1}| / |theta_bar_{k-1}| < tol.

def posterior_mean(theta, logw):
    """sum_j w~_j theta_j with w~ the normalised weights of the log-weights."""
    import numpy as np
    lw = np.asarray(logw, dtype=np.float64)
    m = np.max(lw)
    w = np.exp(lw - m)
    w = w / np.sum(w)
    return w @ np.asarray(theta, dtype=np.float64)


def mean_change(prev, cur):
    """|cur - prev| / |prev| (Euclidean norms); +inf when prev is zero and cur is not."""
    import numpy as np
    num = float(np.sqrt(np.sum((np.asarray(cur, np.float64) - np.asarray(prev, np.float64)) ** 2)))
    den = float(np.sqrt(np.sum(np.asarray(prev, np.float64) ** 2)))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def adaptive_next(m, change, tol, kappa, N):
    """Subset size of the next iteration: grow by kappa (clamped to N) once the change is below tol."""
    return min(N, m + kappa) if change < tol else m
