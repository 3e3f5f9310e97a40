"""Learned proposal-scale network and its Langevin move density (test infrastructure).

An extension beyond the paper, whose moves use one fixed step size h and an
identity mass matrix (Section 2.1).  Here a small MLP maps four per-particle
features to a per-particle step size h_j and a per-parameter-group diagonal
mass m_{j,g}; the move is the S = 1 (Langevin) leapfrog in preconditioned
form,

    theta' = theta + (h^2 / 2) m^{-1} * grad log pi(theta) + h m^{-1/2} * xi,

and because (h, m) depend on the state the Jacobian cancellation of Eqs.
q_prop / l=q_deriv no longer applies.  The weight therefore uses the Gaussian
forward density q and a Gaussian reverse L-kernel whose parameters are
recomputed at theta' (the general form of Eq. weight_update):

    log w += log pi_k(theta') - log pi_{k-1}(theta) + log L(theta | theta') - log q(theta' | theta)

With constant network outputs (h, m = 1) this reduces exactly to the fixed-step
S = 1 update.

Network:  u = clip((f - mu) / sd, -3, 3);  a1 = tanh(W1 u + b1);
a2 = tanh(W2 a1 + b2);  o = W3 a2 + b3, with 4 inputs, two hidden layers of 64
and 1 + G outputs.  The standardised inputs are clipped to three training
standard deviations so that states outside the training traces do not
extrapolate the network.
Outputs map to bounded scales:  log h = log h0 + ln(8) tanh(o_0) (the range
of the step-size grid the targets come from), log m_g = ln(10) tanh(o_g).  Features: f = (log |grad log pi|, LL / M_k,
k / K, M_k / N).  Groups: the weight matrix and the bias vector of each layer
(G = 2 L).

Parameter blob (flat): mu[4], sd[4], W1[64x4], b1[64], W2[64x64], b2[64],
W3[(1+G)x64], b3[1+G], matrices row-major [out x in].
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp
from .smc import Sampler, normalise, log_sum_exp, ess

N_FEAT = 4
HIDDEN = 64
U_CLIP = 3.0
LN10 = math.log(10.0)
LN_H = math.log(8.0)   # bound of log(h / h0)


def n_groups(widths):
    return 2 * (len(widths) - 1)


def group_index(widths):
    """Group id of every parameter: 2 l for W_l entries, 2 l + 1 for b_l entries."""
    gid = []
    for l, (o, i) in enumerate(mlp.layer_shapes(widths)):
        row = [2 * l] * i + [2 * l + 1]
        gid.extend(row * o)
    return np.asarray(gid, dtype=np.int64)


def blob_size(G):
    n_out = 1 + G
    return 2 * N_FEAT + HIDDEN * N_FEAT + HIDDEN + HIDDEN * HIDDEN + HIDDEN + n_out * HIDDEN + n_out


def unpack_blob(blob, G):
    blob = np.asarray(blob, dtype=np.float64)
    n_out = 1 + G
    sizes = [("mu", (N_FEAT,)), ("sd", (N_FEAT,)), ("W1", (HIDDEN, N_FEAT)), ("b1", (HIDDEN,)),
             ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)), ("W3", (n_out, HIDDEN)), ("b3", (n_out,))]
    out, off = {}, 0
    for name, shp in sizes:
        n = int(np.prod(shp))
        out[name] = blob[off:off + n].reshape(shp)
        off += n
    assert off == blob.shape[0], "blob size does not match the group count"
    return out


def init_blob(G, seed, mu=None, sd=None):
    """Random initial network (Glorot-uniform weights, zero biases)."""
    rng = np.random.default_rng(seed)
    n_out = 1 + G
    parts = [np.zeros(N_FEAT) if mu is None else np.asarray(mu, np.float64),
             np.ones(N_FEAT) if sd is None else np.asarray(sd, np.float64)]
    for (o, i) in [(HIDDEN, N_FEAT), (HIDDEN, HIDDEN), (n_out, HIDDEN)]:
        lim = math.sqrt(6.0 / (o + i))
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def net_forward(blob, f, G):
    """Network outputs o [R x (1+G)] and the activations for backpropagation."""
    p = unpack_blob(blob, G)
    u = np.clip((np.asarray(f, dtype=np.float64) - p["mu"]) / p["sd"], -U_CLIP, U_CLIP)
    a1 = np.tanh(u @ p["W1"].T + p["b1"])
    a2 = np.tanh(a1 @ p["W2"].T + p["b2"])
    o = a2 @ p["W3"].T + p["b3"]
    return o, (u, a1, a2)


def mse_loss_grad(blob, f, t, G):
    """Loss (1/R) sum_r 1/2 |o_r - t_r|^2 and its gradient w.r.t. the blob.

    mu and sd are fixed input statistics and get zero gradient.
    """
    p = unpack_blob(blob, G)
    o, (u, a1, a2) = net_forward(blob, f, G)
    R = o.shape[0]
    d3 = (o - t) / R
    loss = 0.5 * np.sum((o - t) ** 2) / R
    gW3 = d3.T @ a2
    gb3 = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (1.0 - a2 * a2)
    gW2 = d2.T @ a1
    gb2 = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - a1 * a1)
    gW1 = d1.T @ u
    gb1 = d1.sum(0)
    grad = np.concatenate([np.zeros(2 * N_FEAT), gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grad


def adam_update(blob, grad, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015); state = (m, v, t) is updated in place."""
    m, v, t = state
    t += 1
    m[:] = beta1 * m + (1.0 - beta1) * grad
    v[:] = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    new = blob - lr * mhat / (np.sqrt(vhat) + eps)
    return new, (m, v, t)


def features(ll, grad, m, k, K, N):
    """Per-particle features (log |grad log pi|, LL / M_k, k / K, M_k / N), [J x 4]."""
    gn = np.sqrt(np.sum(np.asarray(grad, dtype=np.float64) ** 2, axis=1))
    J = gn.shape[0]
    return np.stack([np.log(gn), np.asarray(ll, np.float64) / m,
                     np.full(J, k / K), np.full(J, m / N)], axis=1)


def scales(o, h0):
    """Bounded step sizes h [J] and group masses mg [J x G] from raw outputs.

    A particle whose outputs are not finite falls back to the fixed step
    (h = h0, m = 1).
    """
    o = np.asarray(o, dtype=np.float64)
    ok = np.all(np.isfinite(o), axis=1)
    o = np.where(ok[:, None], o, 0.0)
    h = h0 * np.exp(LN_H * np.tanh(o[:, 0]))
    mg = np.exp(LN10 * np.tanh(o[:, 1:]))
    return h, mg


def _normal_logpdf(x, mean, sd):
    z = (x - mean) / sd
    return -0.5 * math.log(2.0 * math.pi) - np.log(sd) - 0.5 * z * z


def learned_step(s: Sampler, m, lam, xi, blob, h0, k, K, N):
    """One learned-scale Langevin move and reweight of the oracle sampler ``s``."""
    m, lam = int(m), float(lam)
    if m < s.m:
        raise ValueError("the annealed subset only grows")
    if (m, lam) != (s.m, s.lam):
        s.m, s.lam = m, lam
        s.ll, s.g = s.loglik_grad(s.theta, m, lam)
    G = n_groups(s.widths)
    gid = group_index(s.widths)
    xi = np.asarray(xi, dtype=np.float64)
    theta, g = s.theta, s.g
    h, mg = scales(net_forward(blob, features(s.ll, g, m, k, K, N), G)[0], h0)
    me = mg[:, gid]
    mean_f = theta + 0.5 * (h * h)[:, None] * g / me
    sd_f = h[:, None] / np.sqrt(me)
    theta1 = mean_f + sd_f * xi
    ll1, g1 = s.loglik_grad(theta1, m, lam)
    h1, mg1 = scales(net_forward(blob, features(ll1, g1, m, k, K, N), G)[0], h0)
    me1 = mg1[:, gid]
    mean_r = theta1 + 0.5 * (h1 * h1)[:, None] * g1 / me1
    sd_r = h1[:, None] / np.sqrt(me1)
    log_q = np.sum(_normal_logpdf(theta1, mean_f, sd_f), axis=1)
    log_l = np.sum(_normal_logpdf(theta, mean_r, sd_r), axis=1)
    lp1 = s.log_target(ll1, theta1, lam)
    incr = lp1 - s.lp + log_l - log_q
    s.last_increment = incr
    s.last_scales = (h, mg, h1, mg1)
    logw = s.logw + incr
    logw = np.where(np.isfinite(incr) & np.isfinite(ll1), logw, -np.inf)
    s.theta, s.g, s.ll, s.lp = theta1, g1, ll1, lp1
    s._finish_reweight(logw, s.logw)
    return s


def step_size_targets(s: Sampler, m, lam, xi, h0, grid=tuple(range(-3, 4)), accept_power=1.0, return_scores=False):
    """Per-particle training targets from one replayed sampler state.

    For every step h = h0 2^e on the grid, one preconditioning-free Langevin
    move from the current state with the shared noise xi is scored by
    |theta' - theta|^2 min(1, exp(D))^p, where D is the Metropolis log-ratio of
    that move under the fixed target pi_k (also the move's log-weight
    increment) and p = accept_power (p = 1: the expected-squared-jump proxy;
    larger p prefers steps whose increments stay near zero).  The
    target for log h is the best grid value.  The mass targets are the log
    RMS gradient per parameter group, centred over the groups.
    Returns (log h* [J], log m* [J x G]), and with return_scores also the score of
    every grid step [J x len(grid)].
    """
    m, lam = int(m), float(lam)
    if (m, lam) != (s.m, s.lam):
        ll, g = s.loglik_grad(s.theta, m, lam)
    else:
        ll, g = s.ll, s.g
    theta = s.theta
    lp0 = s.log_target(ll, theta, lam)
    xi = np.asarray(xi, dtype=np.float64)
    best = np.full(theta.shape[0], -np.inf)
    best_h = np.full(theta.shape[0], math.log(h0))
    all_scores = []
    for e in grid:
        h = h0 * 2.0 ** e
        theta1 = theta + 0.5 * h * h * g + h * xi
        ll1, g1 = s.loglik_grad(theta1, m, lam)
        lp1 = s.log_target(ll1, theta1, lam)
        log_q = np.sum(_normal_logpdf(theta1, theta + 0.5 * h * h * g, h), axis=1)
        log_l = np.sum(_normal_logpdf(theta, theta1 + 0.5 * h * h * g1, h), axis=1)
        d = lp1 - lp0 + log_l - log_q
        score = np.sum((theta1 - theta) ** 2, axis=1) * np.exp(accept_power * np.minimum(d, 0.0))
        score = np.where(np.isfinite(score), score, -np.inf)
        all_scores.append(score)
        better = score > best
        best = np.where(better, score, best)
        best_h = np.where(better, math.log(h), best_h)
    G = n_groups(s.widths)
    gid = group_index(s.widths)
    rms = np.stack([np.sqrt(np.mean(g[:, gid == q] ** 2, axis=1)) for q in range(G)], axis=1)
    logm = np.log(rms)
    logm = logm - logm.mean(axis=1, keepdims=True)
    if return_scores:
        return best_h, logm, np.stack(all_scores, axis=1)
    return best_h, logm


def output_targets(log_h, log_m, h0, clip=0.95):
    """Raw-output regression targets: the inverse of ``scales`` on clipped values."""
    t0 = np.arctanh(np.clip((np.asarray(log_h) - math.log(h0)) / LN_H, -clip, clip))
    tg = np.arctanh(np.clip(np.asarray(log_m) / LN10, -clip, clip))
    return np.concatenate([t0[:, None], tg], axis=1)


__all__ = ["n_groups", "group_index", "blob_size", "unpack_blob", "init_blob", "net_forward",
           "mse_loss_grad", "adam_update", "features", "scales", "learned_step",
           "step_size_targets", "output_targets", "normalise", "log_sum_exp", "ess"]
