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
