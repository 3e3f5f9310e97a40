"""Torch-facing wrapper of the C ABI: an SMC sampler handle and an autograd Function.

PyTorch supplies device memory and the stream; every step of the method runs in
libsmc's HIP kernels.  Tensors passed in must be contiguous CUDA (HIP) tensors of
the stated dtype; the wrapper only checks and marshals them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

from . import _lib as L

_ACT = {"tanh": L.SMC_ACT_TANH, "relu": L.SMC_ACT_RELU}
_LIK = {"categorical": L.SMC_LIK_CATEGORICAL, "gaussian": L.SMC_LIK_GAUSSIAN}
_PREC = {"fp32": L.SMC_PREC_FP32, "bf16": L.SMC_PREC_BF16, "bf16x3": L.SMC_PREC_BF16X3}
_PROP = {"fixed": L.SMC_PROPOSAL_FIXED, "learned": L.SMC_PROPOSAL_LEARNED}
_RES = {"if_needed": L.SMC_RESAMPLE_IF_NEEDED, "always": L.SMC_RESAMPLE_ALWAYS, "never": L.SMC_RESAMPLE_NEVER}


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def n_params(widths: Sequence[int], model: str = "mlp") -> int:
    """Parameters per particle: dense layers [n_0, ..., n_L], or for the convolutional network
    widths = [H, W, Cin, C1, C2, n_cls] (blocks [C1 x (9 Cin + 1)], [C2 x (9 C1 + 1)],
    [n_cls x ((H/2)(W/2) C2 + 1)]), or for LeNet widths = [H, W, Cin, k, C1, C2, F1, F2, n_cls]
    (conv blocks [C1 x (k^2 Cin + 1)], [C2 x (k^2 C1 + 1)], then dense F -> F1 -> F2 -> n_cls
    with F = ((H/2 - k + 1)/2) ((W/2 - k + 1)/2) C2)."""
    if model == "cnn":
        H, W, Cin, C1, C2, n = widths
        return C1 * (9 * Cin + 1) + C2 * (9 * C1 + 1) + n * ((H // 2) * (W // 2) * C2 + 1)
    if model == "lenet":
        H, W, Cin, k, C1, C2, F1, F2, n = widths
        F = (H // 2 - k + 1) // 2 * ((W // 2 - k + 1) // 2) * C2
        return C1 * (k * k * Cin + 1) + C2 * (k * k * C1 + 1) + F1 * (F + 1) + F2 * (F1 + 1) + n * (F2 + 1)
    return sum(widths[i + 1] * (widths[i] + 1) for i in range(len(widths) - 1))


@dataclass
class SMCConfig:
    widths: Sequence[int]
    n_particles: int
    activation: str = "relu"
    likelihood: str = "categorical"
    precision: str = "fp32"
    proposal: str = "fixed"
    leapfrog_steps: int = 1
    step_size: float = 1e-3
    prior_std: float = 1.0
    noise_std: float = 1.0
    ess_frac: float = 0.5
    seed: int = 0
    act_budget_bytes: int = 0
    n_iterations: int = 0
    model: str = "mlp"  # "mlp", "cnn" (widths = [H, W, Cin, C1, C2, n_cls]) or "lenet"
    #                     (widths = [H, W, Cin, k, C1, C2, F1, F2, n_cls])

    def to_c(self) -> L.smc_config:
        c = L.smc_config()
        c.n_particles = self.n_particles
        if self.model == "cnn":
            if len(self.widths) != 6:
                raise ValueError("the convolutional network takes widths [H, W, Cin, C1, C2, n_cls]")
            c.n_layers = 3
        elif self.model == "lenet":
            if len(self.widths) != 9:
                raise ValueError("LeNet takes widths [H, W, Cin, k, C1, C2, F1, F2, n_cls]")
            c.n_layers = 5
        elif self.model == "mlp":
            c.n_layers = len(self.widths) - 1
        else:
            raise ValueError(f"unknown model {self.model!r}")
        for i, w in enumerate(self.widths):
            c.widths[i] = int(w)
        c.activation = _ACT[self.activation]
        c.model_kind = {"mlp": L.SMC_MODEL_MLP, "cnn": L.SMC_MODEL_CNN, "lenet": L.SMC_MODEL_LENET}[self.model]
        c.likelihood = _LIK[self.likelihood]
        c.precision = _PREC[self.precision]
        c.proposal = _PROP[self.proposal]
        c.leapfrog_steps = self.leapfrog_steps
        c.step_size = self.step_size
        c.prior_std = self.prior_std
        c.noise_std = self.noise_std
        c.ess_frac = self.ess_frac
        c.seed = self.seed
        c.act_budget_bytes = self.act_budget_bytes
        c.n_iterations = self.n_iterations
        return c


class SMCSampler:
    """One data-annealed SMC sampler on the current GPU (see include/smc.h)."""

    def __init__(self, cfg: SMCConfig, X: torch.Tensor, y: torch.Tensor, m0: int, lambda0: float,
                 theta0: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
        self.cfg = cfg
        self.J = cfg.n_particles
        self.D = n_params(cfg.widths, cfg.model)
        self.C = cfg.widths[-1]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        xp = _dev(X, torch.float32, "X")
        yp = _dev(y, torch.float32 if cfg.likelihood == "gaussian" else torch.int32, "y")
        tp = None
        if theta0 is not None:
            tp = _dev(theta0, torch.float32, "theta0")
            if tuple(theta0.shape) != (self.J, self.D):
                raise ValueError("theta0 must be [J x D]")
        F = cfg.widths[0] * cfg.widths[1] * cfg.widths[2] if cfg.model in ("cnn", "lenet") else cfg.widths[0]
        if X.dim() != 2 or X.shape[1] != F:
            raise ValueError("X has the wrong number of features")
        self.N = X.shape[0]
        self._h = None
        self._h = L.smc_init(cfg.to_c(), xp, yp, self.N, tp, int(m0), float(lambda0), self.stream.cuda_stream)
        self.m = int(m0)
        self.proposal = cfg.proposal

    # ---------------------------------------------------------------- lifecycle
    def close(self) -> None:
        if self._h is not None:
            L.smc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("sampler is closed")
        return self._h

    # ---------------------------------------------------------------- method
    def step(self, m: int, lam: float, info: bool = True) -> Optional[dict]:
        r = L.smc_step(self.handle, int(m), float(lam), want_info=info)
        self.m = int(m)
        if r is None:
            return None
        return {"ess": r.ess, "log_z_increment": r.log_z_increment, "mean_loglik": r.mean_loglik,
                "max_loglik": r.max_loglik, "n_nonfinite": r.n_nonfinite,
                "resample_recommended": bool(r.resample_recommended), "grad_evals": r.grad_evals}

    def step_tempered(self, m: int, m_split: int, lam_a: float, lam_b: float, info: bool = True) -> Optional[dict]:
        """One iteration targeting lam_a LL[0, m_split) + lam_b LL[m_split, m) + log q0 (smooth data
        annealing: lam_a = 1, lam_b = beta)."""
        r = L.smc_step_tempered(self.handle, int(m), int(m_split), float(lam_a), float(lam_b), want_info=info)
        self.m = int(m)
        if r is None:
            return None
        return {"ess": r.ess, "log_z_increment": r.log_z_increment, "mean_loglik": r.mean_loglik,
                "max_loglik": r.max_loglik, "n_nonfinite": r.n_nonfinite,
                "resample_recommended": bool(r.resample_recommended), "grad_evals": r.grad_evals}

    def segment_moments(self) -> dict:
        """Weighted moments of Omega^ = -LL[m_split, m) and Omega = -LL[0, m_split) at the current particles."""
        e_b, var_b, e_a, cov = L.smc_segment_moments(self.handle)
        return {"mean_hat": e_b, "var_hat": var_b, "mean": e_a, "cov": cov}

    def resample(self, mode: str = "if_needed", u: Optional[float] = None, want: bool = False,
                 scheme: str = "systematic", uniforms: Optional[torch.Tensor] = None):
        """Systematic (offset u, host float, or None: drawn on the device) or multinomial
        (uniforms: float64 GPU tensor [J], or None: drawn on the device) resampling."""
        if scheme == "multinomial":
            if u is not None:
                raise ValueError("multinomial resampling takes `uniforms`, not `u`")
            up = None
            if uniforms is not None:
                up = _dev(uniforms, torch.float64, "uniforms")
                if tuple(uniforms.shape) != (self.J,):
                    raise ValueError("uniforms must be [J]")
            res, anc = L.smc_resample_multinomial(self.handle, _RES[mode], up, want_result=want,
                                                  want_ancestors=want, J=self.J)
        elif scheme == "systematic":
            if uniforms is not None:
                raise ValueError("systematic resampling takes one offset `u`")
            res, anc = L.smc_resample(self.handle, _RES[mode], u, want_result=want, want_ancestors=want, J=self.J)
        else:
            raise ValueError("scheme must be 'systematic' or 'multinomial'")
        return (res, anc) if want else None

    def predict(self, Xt: torch.Tensor, yt: Optional[torch.Tensor] = None, probs: bool = False):
        xp = _dev(Xt, torch.float32, "Xt")
        yp = _dev(yt, torch.int32, "yt") if yt is not None else None
        n = Xt.shape[0]
        out = torch.empty((n, self.C), dtype=torch.float32, device=Xt.device) if probs else None
        acc, mlp = L.smc_posterior_predict(self.handle, xp, yp, n, out.data_ptr() if out is not None else None,
                                           want_metrics=yt is not None)
        return {"accuracy": acc, "mean_log_pred": mlp, "probs": out}

    def posterior_mean(self) -> torch.Tensor:
        out = torch.empty(self.D, dtype=torch.float64, device="cuda")
        L.smc_posterior_mean(self.handle, out.data_ptr())
        return out

    def posterior_mean_change(self) -> float:
        """|theta_bar - theta_bar_prev| / |theta_bar_prev| against the previous call (+inf on the first)."""
        return L.smc_posterior_mean_change(self.handle)

    def state(self) -> dict:
        dev = torch.device("cuda")
        th = torch.empty((self.J, self.D), dtype=torch.float32, device=dev)
        g = torch.empty_like(th)
        lw = torch.empty(self.J, dtype=torch.float64, device=dev)
        ll = torch.empty_like(lw)
        lp = torch.empty_like(lw)
        L.smc_get_state(self.handle, th.data_ptr(), lw.data_ptr(), ll.data_ptr(), lp.data_ptr(), g.data_ptr())
        return {"theta": th, "logw": lw, "loglik": ll, "logpi": lp, "grad": g,
                "rng_counter": L.smc_get_rng_counter(self.handle), "m": self.m}

    def set_state(self, theta: torch.Tensor, logw: Optional[torch.Tensor] = None,
                  logpi: Optional[torch.Tensor] = None, rng_counter: int = 0) -> None:
        L.smc_set_state(self.handle, _dev(theta, torch.float32, "theta"),
                        _dev(logw, torch.float64, "logw") if logw is not None else None,
                        _dev(logpi, torch.float64, "logpi") if logpi is not None else None, rng_counter)

    def set_noise(self, momenta: torch.Tensor) -> None:
        if tuple(momenta.shape) != (self.J, self.D):
            raise ValueError("momenta must be [J x D]")
        L.smc_set_noise(self.handle, _dev(momenta, torch.float32, "momenta"))

    def chunk_samples(self) -> int:
        return L.smc_chunk_samples(self.handle)

    def profile(self, enable: bool = True) -> None:
        """Bracket every kernel launch with HIP events on the sampler's stream."""
        L.smc_profile(self.handle, enable)

    def profile_read(self) -> dict:
        """{kernel class: (total_ms, launches, algorithmic flops, algorithmic bytes)}; clears the records."""
        return L.smc_profile_read(self.handle)

    # ---------------------------------------------------------------- learned proposal
    @property
    def n_groups(self) -> int:
        """Parameter groups of the learned proposal: the weights and the biases of every layer
        (LeNet's five layers count, although LeNet runs with the fixed proposal)."""
        layers = {"cnn": 3, "lenet": 5}.get(self.cfg.model, len(self.cfg.widths) - 1)
        return 2 * layers

    def set_proposal_net(self, params: torch.Tensor, h0: float) -> None:
        L.smc_set_proposal_net(self.handle, _dev(params, torch.float32, "params"), params.numel(), float(h0))

    def set_proposal(self, proposal: str) -> None:
        """Switch the move of the following iterations: "fixed" or "learned"."""
        L.smc_set_proposal(self.handle, _PROP[proposal])
        self.proposal = proposal

    def proposal_features(self, k_over_K: float, m_over_N: float) -> torch.Tensor:
        out = torch.empty((self.J, 4), dtype=torch.float64, device="cuda")
        L.smc_proposal_features(self.handle, float(k_over_K), float(m_over_N), out.data_ptr())
        return out

    def proposal_targets(self, m: int, lam: float, h_grid, k_over_K: float, accept_power: float = 1.0):
        """(features [J x 4], raw-output targets [J x (1+G)]) at the current population."""
        feat = torch.empty((self.J, 4), dtype=torch.float32, device="cuda")
        tgt = torch.empty((self.J, 1 + self.n_groups), dtype=torch.float32, device="cuda")
        L.smc_proposal_targets(self.handle, int(m), float(lam), list(h_grid), float(k_over_K), float(accept_power),
                               feat.data_ptr(), tgt.data_ptr())
        self.m = int(m)
        return feat, tgt

    # ---------------------------------------------------------------- network passes
    def nn_forward(self, theta: torch.Tensor, m: int) -> torch.Tensor:
        ll = torch.empty(self.J, dtype=torch.float64, device=theta.device)
        L.smc_nn_forward(self.handle, _dev(theta, torch.float32, "theta"), int(m), ll.data_ptr())
        return ll

    def nn_backward(self, theta: torch.Tensor, m: int, scale: Optional[torch.Tensor] = None):
        ll = torch.empty(self.J, dtype=torch.float64, device=theta.device)
        g = torch.empty_like(theta)
        sp = _dev(scale, torch.float64, "scale") if scale is not None else None
        L.smc_nn_backward(self.handle, _dev(theta, torch.float32, "theta"), int(m), sp, ll.data_ptr(), g.data_ptr())
        return ll, g


class ParticleMLPFn(torch.autograd.Function):
    """LL_j(theta_j) = sum_{i<m} log p(y_i | x_i, theta_j) with the hand-written backward.

    forward saves only theta; backward recomputes the forward activations chunk by
    chunk inside the library (activation recomputation) and returns
    grad_output_j * d LL_j / d theta_j.
    """

    @staticmethod
    def forward(ctx, theta: torch.Tensor, sampler: SMCSampler, m: int):
        ctx.sampler = sampler
        ctx.m = m
        ctx.save_for_backward(theta)
        return sampler.nn_forward(theta.contiguous(), m)

    @staticmethod
    def backward(ctx, grad_ll):
        (theta,) = ctx.saved_tensors
        _, g = ctx.sampler.nn_backward(theta.contiguous(), ctx.m, grad_ll.to(torch.float64).contiguous())
        return g, None, None
