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
                   accept_power: float = 1.0):
    """Run the plain sampler over the schedule `sizes` ([M_0, ..., M_K]) and, every `every`
    iterations, record (features, targets) of its population before the move.

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
        sampler.step(sizes[k], lam, info=False)
        sampler.resample(resample)
    return torch.cat(feats), torch.cat(tgts)


def traces_from_runs(make_sampler, seeds, sizes, N: int, h_grid, every: int = 1, accept_power: float = 1.0):
    """Traces of several plain-sampler runs (one per seed) concatenated.

    make_sampler(seed) must return a fresh plain (fixed-step) SMCSampler at M_0 =
    sizes[0]; several runs cover more of the state space the learned sampler visits.
    """
    fs, ts = [], []
    for sd in seeds:
        s = make_sampler(sd)
        s.resample()
        f, t = collect_traces(s, sizes, N, h_grid, every, accept_power=accept_power)
        s.close()
        fs.append(f)
        ts.append(t)
    return torch.cat(fs), torch.cat(ts)


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
