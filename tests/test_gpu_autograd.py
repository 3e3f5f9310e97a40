"""The hand-written backward behind torch.autograd (ParticleMLPFn) at the scale of the
784-256-256-10 network: directional finite differences, the oracle's gradient on sampled
particles, and activation recomputation over several chunks."""
import numpy as np
import pytest

from gpu_helpers import cuda, lib, print_case, rel_err, to_dev, torch
from oracle import mlp
import smc_inputs

pytestmark = pytest.mark.gpu

WIDTHS = [784, 256, 256, 10]


def _sampler(P, J, M, budget, seed=0, act="relu"):
    X, y = smc_inputs.templates28(M, seed=seed)
    D = mlp.n_params(WIDTHS)
    theta = smc_inputs.prior_draw(seed + 1, J, D, 0.05)
    cfg = P.SMCConfig(widths=WIDTHS, n_particles=J, activation=act, precision="fp32", act_budget_bytes=budget)
    s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=M, lambda0=1.0, theta0=to_dev(theta))
    return s, X, y, theta


@pytest.mark.parametrize("act", ["tanh", "relu"])
def test_autograd_function_matches_finite_differences(act):
    """tanh: central differences along the gradient direction and along gradient + random
    directions (unit length), where the derivative is large against the FP32 rounding of the
    log-likelihood (~0.1 absolute at |LL| ~ 7e3); in FP64 the step 1e-2 has a truncation error of
    1.4e-5 relative on these directions.  ReLU: its kinks make differences unreliable (1.9% at
    step 1e-2 in FP64 along random directions), so only the oracle's exact gradient is compared."""
    cuda()
    P = lib()
    J, M = 16, 3000
    budget = 16 * (256 + 256) * 4 * 4 * 256  # a few hundred samples per chunk: several recomputed chunks
    print_case("autograd-fd", J=J, M=M, budget=budget, act=act)
    s, X, y, theta = _sampler(P, J, M, budget, act=act)
    assert s.chunk_samples() < M // 4
    th = to_dev(theta).requires_grad_(True)
    ll = P.ParticleMLPFn.apply(th, s, M)
    w = torch.linspace(0.5, 1.5, J, dtype=torch.float64, device="cuda")
    (ll * w).sum().backward()
    g = th.grad.detach().double()
    # directional derivatives along random unit directions, central differences in FP32 passes
    rng = np.random.default_rng(5)
    eps = 1e-2
    gu = (g / g.norm(dim=1, keepdim=True)).cpu().numpy()
    for q in range(3 if act == "tanh" else 0):
        v = gu.copy()
        if q > 0:
            r = rng.standard_normal(theta.shape)
            v = v + r / np.linalg.norm(r, axis=1, keepdims=True)
        v = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
        vd = to_dev(v)
        lp = s.nn_forward((th.detach() + eps * vd).contiguous(), M)
        lm = s.nn_forward((th.detach() - eps * vd).contiguous(), M)
        fd = ((lp - lm) / (2 * eps)).cpu().numpy()
        an = ((g * vd.double()).sum(dim=1) / w).cpu().numpy()
        err = np.max(np.abs(fd - an) / np.abs(an))
        print(f"direction {q}: max relative error {err:.2e}", flush=True)
        assert err < 1e-3, err
    # against the FP64 oracle on three particles
    idx = [0, 7, 15]
    _, gref = mlp.loglik_grad(theta[idx], X, y, WIDTHS, act)
    gg = (g / w[:, None]).cpu().numpy()[idx]
    assert np.max(np.abs(gg - gref) / np.max(np.abs(gref), axis=1, keepdims=True)) < 2e-4
    s.close()


def test_config3_scale_sampled_parity():
    """J = 1024 particles of the 784-256-256-10 network over 4000 samples (several recomputed
    chunks under the default 8 GiB budget at this J), checked on sampled particles."""
    cuda()
    P = lib()
    J, M = 1024, 4000
    print_case("config3-scale", J=J, M=M)
    s, X, y, theta = _sampler(P, J, M, 0, seed=3)
    assert s.chunk_samples() < M
    td = to_dev(theta)
    ll, g = s.nn_backward(td, M)
    torch.cuda.synchronize()
    idx = [0, 511, 1023]
    llref, gref = mlp.loglik_grad(theta[idx], X, y, WIDTHS, "relu")
    assert rel_err(ll.cpu().numpy()[idx], llref) < 1e-5
    gg = g.cpu().numpy()[idx]
    assert np.max(np.abs(gg - gref) / np.max(np.abs(gref), axis=1, keepdims=True)) < 2e-4
    s.close()
