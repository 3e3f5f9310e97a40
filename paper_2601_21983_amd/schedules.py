"""Data-annealing schedules: the subset size M_k per iteration (Section 3.1).

Host-side control logic of the sampler (the device kernels only see m_k and
lambda_k = N / M_k).  C is the initial batch size, kappa the mini-batch
increment, K the number of iterations and N the data-set size.  Iteration 0 is
the initial weighting with M_0 = C; moves run for k = 1..K; "k < 0.9 K" compares
real numbers (10 k < 9 K in integers).  Linear is clamped to N; Automated is
rounded to the nearest multiple of kappa (halves up) and clamped to [C, N].
"""
from __future__ import annotations


def _before_refine(k: int, K: int) -> bool:
    return 10 * k < 9 * K


def subset_size(name: str, k: int, K: int, N: int, C: int, kappa: int) -> int:
    if name == "constant":
        return C
    if name == "fb":
        return N
    if name == "ctr":
        return C if _before_refine(k, K) else N
    if name == "linear":
        return min(kappa * k + C, N) if _before_refine(k, K) else N
    if name == "automated":
        if not _before_refine(k, K):
            return N
        slope = (10 * (N - C)) // (9 * K)  # floor((N - C) / (0.9 K))
        raw = C + slope * k
        mult = (2 * raw + kappa) // (2 * kappa)
        return max(C, min(N, mult * kappa))
    raise ValueError(f"unknown schedule {name!r}")


def sizes(name: str, K: int, N: int, C: int, kappa: int) -> list[int]:
    """[M_0, ..., M_K]."""
    return [C] + [subset_size(name, k, K, N, C, kappa) for k in range(1, K + 1)]


NAMES = ("constant", "fb", "ctr", "linear", "automated")


class PosteriorMeanSchedule:
    """Adaptive subset growth: append kappa points (up to N) once the relative change of the
    weighted posterior mean between consecutive iterations falls below tol.

    Call ``start(sampler)`` after initialisation, then ``next(sampler)`` after every
    iteration for the next subset size.  The change is computed on the device
    (smc_posterior_mean_change)."""

    def __init__(self, m0: int, kappa: int, tol: float, N: int):
        if not (0 < m0 <= N) or kappa < 1 or not tol > 0:
            raise ValueError("need 0 < m0 <= N, kappa >= 1 and tol > 0")
        self.m, self.kappa, self.tol, self.N = int(m0), int(kappa), float(tol), int(N)
        self.changes = []

    def start(self, sampler) -> None:
        sampler.posterior_mean_change()

    def next(self, sampler) -> int:
        c = sampler.posterior_mean_change()
        self.changes.append(c)
        if c < self.tol:
            self.m = min(self.N, self.m + self.kappa)
        return self.m
