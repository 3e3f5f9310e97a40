"""Data-annealing schedules: the subset size M_k per iteration (Section 3.1).

Host-side control logic of the sampler (the device kernels only see m_k and
lambda_k = N / M_k, or for smooth data annealing the two-segment target
(m_k, split, 1, beta) and the weighted moments the device computes).  C is the initial batch size, kappa the mini-batch
increment, K the number of iterations and N the data-set size.  Iteration 0 is
the initial weighting with M_0 = C; moves run for k = 1..K; "k < 0.9 K" compares
real numbers (10 k < 9 K in integers).  Linear is clamped to N; Automated is
rounded to the nearest multiple of kappa (halves up) and clamped to [C, N].
"""
from __future__ import annotations

import math


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


class SDASchedule:
    """Smooth data annealing (Section 3.1): the subset grows one mini-batch of kappa points at a
    time, and the newest batch enters the target tempered by beta,

        pi(theta) ~ p(y[0:split] | theta) p(y[split:m] | theta)^beta q0(theta),

    with beta moved after every iteration so that the entropy changes by dS:
    beta <- beta - dS / Var(Omega^) before the first append (Eq. beta_initial_data_k; the
    initial phase tempers the first C points, split = 0) and beta <- beta - dS / (Var(Omega^) +
    Cov(Omega, Omega^)) after it (Eq. beta_annealed_k), the sign of dS flipped when the update
    would not increase beta and beta clipped to 1.  After an iteration whose target had
    beta = 1 the next batch is appended and beta restarts at beta0.  The moments come from the
    device (smc_segment_moments).

    Use: ``m, split, beta = sched.target`` for ``sampler.step_tempered(m, split, 1.0, beta)``,
    then ``sched.next(sampler)`` after every iteration.  Initialise the sampler with
    m0 = C and lambda0 = beta0 (the initial target is p(y[0:C])^beta0 q0)."""

    def __init__(self, C: int, kappa: int, N: int, beta0: float = 0.1, dS: float = 1.0):
        if not (0 < C <= N) or kappa < 1 or not (0.0 < beta0 <= 1.0) or not dS > 0:
            raise ValueError("need 0 < C <= N, kappa >= 1, 0 < beta0 <= 1 and dS > 0")
        self.kappa, self.N, self.beta0, self.dS = int(kappa), int(N), float(beta0), float(dS)
        self.target = (int(C), 0, float(beta0))
        self.history = [self.target]

    def done(self) -> bool:
        return self.target[0] >= self.N and self.target[2] >= 1.0

    def _beta_update(self, beta: float, denom: float) -> float:
        step = -self.dS / denom if denom != 0.0 else math.nan
        if not math.isfinite(step) or step <= 0.0:
            step = abs(self.dS / denom) if math.isfinite(denom) and denom != 0.0 else 1.0
        return min(1.0, beta + step)

    def next(self, sampler):
        """The target of the next iteration, from the iteration just run."""
        m, split, beta = self.target
        if beta >= 1.0:
            if m < self.N:
                self.target = (min(m + self.kappa, self.N), m, self.beta0)
        else:
            mo = sampler.segment_moments()
            denom = mo["var_hat"] + (mo["cov"] if split > 0 else 0.0)
            self.target = (m, split, self._beta_update(beta, denom))
        self.history.append(self.target)
        return self.target
