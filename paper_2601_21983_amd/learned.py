"""Learned proposal-scale network: trace collection, initialisation and GPU training.

An extension of the method (the paper's moves use a fixed step size): a
4 -> 64 -> 64 -> (1+G) MLP maps per-particle features (log |grad log pi|,
LL / M_k, k / K, M_k / N) to a step size and per-group masses of a
preconditioned Langevin move whose Gaussian forward/reverse densities enter the
importance weight.  Targets come from replaying states of the plain fixed-step
sampler: the best step of a grid by squared jump times the Metropolis factor,
and the centred log RMS gradient of each parameter group.  Training runs on the
GPU through the library's forward/backward/Adam kernels.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib as L

N_FEAT = 4
HIDDEN = 64


def n_params(n_groups: int) -> int:
    return L.smc_mlp_n_params(n_groups)


def init_params(n_groups: int, mu, sd, seed: int = 0) -> torch.Tensor:
    """Glorot-uniform weights, zero biases, and the input statistics (mu, sd)."""
    rng = np.random.default_rng(seed)
    n_out = 1 + n_groups
    parts = [np.asarray(mu, np.float64).reshape(N_FEAT), np.asarray(sd, np.float64).reshape(N_FEAT)]
    for (o, i) in [(HIDDEN, N_FEAT), (HIDDEN, HIDDEN), (n_out, HIDDEN)]:
        lim = math.sqrt(6.0 / (o + i))
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    blob = np.concatenate(parts).astype(np.float32)
    assert blob.shape[0] == n_params(n_groups)
    return torch.from_numpy(blob).cuda()


def collect_traces(sampler, sizes, N: int, h_grid, every: int = 1, resample: str = "if_needed",
                   accept_power: float = 1.0, reference: "JudgeReference | None" = None):
    """Run the plain sampler over the schedule `sizes` ([M_0, ..., M_K]) and, every `every`
    iterations, record (features, targets) of its population before the move.  With
    `reference`, also record the run's post-move ESS and held-out log predictive for the
    run-level judge of the learned move.

    Returns (feat [R x 4], tgt [R x (1+G)]) float32 GPU tensors.
    """
    K = len(sizes) - 1
    feats, tgts = [], []
    for k in range(1, K + 1):
        lam = N / sizes[k]
        if (k - 1) % every == 0:
            # the move of iteration k sees the feature k / K
            f, t = sampler.proposal_targets(sizes[k], lam, h_grid, k / K, accept_power)
            feats.append(f)
            tgts.append(t)
        info = sampler.step(sizes[k], lam, info=reference is not None)
        if reference is not None:
            reference.record(sampler, k, info["ess"])
        sampler.resample(resample)
    return torch.cat(feats), torch.cat(tgts)


def traces_from_runs(make_sampler, seeds, sizes, N: int, h_grid, every: int = 1, accept_power: float = 1.0,
                     reference: "JudgeReference | None" = None):
    """Traces of several plain-sampler runs (one per seed) concatenated.

    make_sampler(seed) must return a fresh plain (fixed-step) SMCSampler at M_0 =
    sizes[0]; several runs cover more of the state space the learned sampler visits.
    With `reference`, every run also adds to the judge's reference (averaged over the runs).
    """
    fs, ts = [], []
    for sd in seeds:
        s = make_sampler(sd)
        s.resample()
        if reference is not None:
            reference.start_run()
        f, t = collect_traces(s, sizes, N, h_grid, every, accept_power=accept_power, reference=reference)
        s.close()
        fs.append(f)
        ts.append(t)
    return torch.cat(fs), torch.cat(ts)


def judge_checkpoints(K: int):
    """Iterations at which the run-level judge compares a learned run with the fixed-step
    reference: 1, 2, 4, 8, ... and K.  A losing learned move is caught after its first
    iteration, before it can spoil the population; later checks cover ever longer stretches."""
    ks, k = {int(K)}, 1
    while k <= K:
        ks.add(k)
        k *= 2
    return sorted(ks)


class JudgeReference:
    """What the fixed-step plain sampler achieves over one schedule: its post-move ESS / J at
    every iteration and its held-out mean log predictive at the judge's checkpoints, averaged
    over the recorded runs."""

    def __init__(self, X_val: torch.Tensor, y_val: torch.Tensor, checkpoints):
        self.X_val, self.y_val = X_val, y_val
        self.checkpoints = sorted(set(int(k) for k in checkpoints))
        if not self.checkpoints or self.checkpoints[0] < 1:
            raise ValueError("checkpoints must be iterations >= 1")
        self._cp = set(self.checkpoints)
        self._ess: dict = {}
        self._heldout: dict = {}
        self.runs = 0

    def start_run(self) -> None:
        self.runs += 1

    def record(self, sampler, k: int, ess: float) -> None:
        self._ess.setdefault(k, []).append(ess / sampler.J)
        if k in self._cp:
            r = sampler.predict(self.X_val, self.y_val)
            self._heldout.setdefault(k, []).append(r["mean_log_pred"])

    def is_checkpoint(self, k: int) -> bool:
        return k in self._cp

    def ess_frac(self, k: int) -> float:
        return float(np.mean(self._ess[k]))

    def heldout(self, k: int) -> float:
        return float(np.mean(self._heldout[k]))

    def covers(self, k: int) -> bool:
        return k in self._ess and (k not in self._cp or k in self._heldout)


class ProposalJudge:
    """Run-level fallback of the learned proposal to the fixed-step move.

    The fixed-step plain sampler is the judge (its figures come from a JudgeReference over the
    same schedule).  At each checkpoint k of the reference the judge compares, over the
    iterations since the previous checkpoint,
      * the mean post-move ESS / J with `ratio` times the reference's mean over the same
        iterations, and
      * the held-out mean log predictive at k with the reference's at k.
    The learned move loses if either comparison fails; the sampler then runs the fixed-step
    move (switched through smc_set_proposal) for the rest of the run.  Both moves reweight
    with the L-kernel of their own step, so the population stays properly weighted across the
    switch.  Non-finite network outputs already fall back to the fixed step per particle
    inside the move kernel; this is the run-level rule on top of it.
    """

    def __init__(self, reference: JudgeReference, ratio: float = 0.9):
        self.ref = reference
        self.ratio = float(ratio)
        self._ess = []
        self._last_cp = 0
        self.fired_at = None
        self.reason = None
        self.checks = []
        self.learned_iterations = 0

    def after_step(self, sampler, k: int, ess: float) -> None:
        """Call once per iteration k (1-based) with the step's post-move ESS, before resampling."""
        if sampler.proposal != "learned":
            return
        self.learned_iterations += 1
        self._ess.append((k, ess / sampler.J))
        if not self.ref.is_checkpoint(k) or not self.ref.covers(k):
            return
        win = [(i, e) for i, e in self._ess if i > self._last_cp]
        self._last_cp = k
        got = float(np.mean([e for _, e in win]))
        want = self.ratio * float(np.mean([self.ref.ess_frac(i) for i, _ in win]))
        held = sampler.predict(self.ref.X_val, self.ref.y_val)["mean_log_pred"]
        held_ref = self.ref.heldout(k)
        check = {"iteration": k, "ess_frac": round(got, 4), "ess_frac_needed": round(want, 4),
                 "heldout": round(held, 6), "heldout_reference": round(held_ref, 6)}
        self.checks.append(check)
        reasons = []
        if not got >= want:
            reasons.append("ess")
        if not held >= held_ref:
            reasons.append("heldout")
        if reasons:
            self.fired_at = k
            self.reason = "+".join(reasons)
            sampler.set_proposal("fixed")

    def report(self) -> dict:
        return {"fired": self.fired_at is not None, "iteration": self.fired_at, "reason": self.reason,
                "learned_iterations": self.learned_iterations, "checkpoints": self.ref.checkpoints,
                "ess_ratio": self.ratio, "checks": self.checks}


def train(feat: torch.Tensor, tgt: torch.Tensor, n_groups: int, steps: int = 600, lr: float = 3e-3,
          seed: int = 0, chunk: int = 200):
    """Full-batch Adam on the GPU.  Returns (params, losses): the loss at the first step, then at the
    last step of every chunk (each loss is evaluated before that step's update)."""
    feat = feat.contiguous()
    tgt = tgt.contiguous()
    f = feat.double()
    mu = f.mean(0).cpu().numpy()
    sd = f.std(0).clamp_min(1e-3).cpu().numpy()
    params = init_params(n_groups, mu, sd, seed)
    adam = torch.zeros(2 * params.numel(), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    losses = []
    done = 0
    while done < steps:
        n = 1 if done == 0 else min(chunk, steps - done)  # the first entry is the initial loss
        losses.append(L.smc_mlp_train(params.data_ptr(), adam.data_ptr(), feat.data_ptr(), tgt.data_ptr(),
                                      feat.shape[0], n_groups, done + 1, n, lr, stream))
        done += n
    return params, losses


def default_grid(h0: float):
    """h0 * 2^e for e = -3..3."""
    return [h0 * 2.0 ** e for e in range(-3, 4)]
