"""The learned-scale Langevin move at the benchmark's network size (784-100-10 ReLU,
D = 79,510): every particle's move runs over 78 workgroups whose partial sums feed the
proposal densities, the features reduce over all D parameters, and the four parameter
groups (W1, b1, W2, b2) carry their own masses.  Three lockstep steps with injected noise
against the oracle's learned step (Section 2.1 move with state-dependent step and mass,
general L-kernel weight of Eq. weight_update), in FP32 and in split BF16 (against the
oracle on BF16-rounded inputs, the quantity that mode approximates)."""
import numpy as np
import pytest

from gpu_helpers import bf16_round, cuda, lib, print_case, to_dev
from oracle import learned as olearned
from oracle import smc
import smc_inputs

pytestmark = pytest.mark.gpu

WIDTHS = [784, 100, 10]
G = 4
J = 12
PRIOR = 0.05
H0 = 0.002
K = 10
EPS_SCALE = 1e-2  # bound on the relative change of the learned step sizes and masses from BF16 features


def _blob():
    # input statistics near the features this workload produces (log |grad| ~ 6-8,
    # LL / M ~ -2.3), moderate outputs so that steps and masses vary over the particles
    b = olearned.init_blob(G, 21, mu=[7.0, -2.3, 0.2, 0.05], sd=[1.0, 0.2, 0.1, 0.02])
    p = olearned.unpack_blob(b, G)
    p["W3"][:] *= 1.5
    p["b3"][:] = [0.3, -0.4, 0.2, 0.5, -0.3]
    return b.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_learned_step_at_benchmark_size(precision):
    cuda()
    P = lib()
    N = 3000
    X, y = smc_inputs.templates28(N, seed=7)
    y = y.astype(np.int32)
    D = 79510
    th0 = smc_inputs.prior_draw(8, J, D, PRIOR)
    blob = _blob()
    cfg = P.SMCConfig(widths=WIDTHS, n_particles=J, activation="relu", precision=precision, step_size=H0,
                      prior_std=PRIOR, proposal="learned", n_iterations=K, seed=4)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y), m0=1000, lambda0=1.0, theta0=to_dev(th0))
    g.set_proposal_net(to_dev(blob.astype(np.float32)), H0)
    Xo = bf16_round(X) if precision == "bf16x3" else X
    o = smc.Sampler(Xo, y, WIDTHS, "relu", prior_std=PRIOR, step_size=H0)
    o.init(th0, 1000, 1.0)
    # split BF16 approximates the rounded-input oracle to ~1e-5 of |LL| (products carry ~16 bits)
    ll_rel = 1e-5 if precision == "fp32" else 1e-4
    for k, m in [(1, 1000), (2, 2000), (3, 2000)]:
        xi = smc_inputs.momenta(60 + k, (J, D))
        print_case("learned-step-784-100-10", precision=precision, k=k, m=m, J=J)
        g.set_noise(to_dev(xi))
        g.step(m, 1.0)
        g_start = o.g if m == o.m else o.loglik_grad(o.theta, m, 1.0)[1]  # the move's starting gradient
        olearned.learned_step(o, m, 1.0, xi, blob, H0, k=k, K=K, N=N)
        st = g.state()
        th = st["theta"].cpu().numpy()
        assert np.all(np.isfinite(th))
        # the step sizes and masses differ over the particles (the per-particle scales are exercised)
        h, mg, h1, mg1 = o.last_scales
        if k == 1:
            assert np.ptp(np.log(h)) > 0.05 and np.ptp(np.log(mg)) > 0.05
        ll = st["loglik"].cpu().numpy()
        lw = st["logw"].cpu().numpy()
        fin = np.isfinite(o.logw)
        assert np.array_equal(fin, np.isfinite(lw))
        e_th = np.max(np.abs(th - o.theta))
        e_lw = np.max(np.abs(lw[fin] - o.logw[fin]))
        # log-likelihood and the features kernel's reduction over all D parameters, both on the GPU's
        # own particles (in split BF16 the trajectories part: see the theta bound below)
        feat = g.proposal_features(k / K, m / N).cpu().numpy()
        ll_g, gr_g = o.loglik_grad(th.astype(np.float64), m, 1.0)
        e_ll = np.max(np.abs(ll - ll_g) / np.abs(ll_g))
        f_ref = olearned.features(ll_g, gr_g, m, k, K, N)
        e_f0 = np.max(np.abs(feat[:, 0] - f_ref[:, 0]))
        e_f1 = np.max(np.abs(feat[:, 1] - f_ref[:, 1]) / np.abs(f_ref[:, 1]))
        assert np.array_equal(feat[:, 2:], f_ref[:, 2:])
        # theta: FP32 rounding; in split BF16 also (i) the drift term (h^2 / 2m) g with the single-BF16
        # backward's gradient error (up to 3% of the largest entry) and (ii) the noise term h / sqrt(m) xi
        # with the step sizes and masses computed from that gradient's features (relative change eps)
        gid = olearned.group_index(WIDTHS)
        drift = 0.5 * (h * h)[:, None] / mg[:, gid] * np.abs(g_start)
        noise = (h[:, None] / np.sqrt(mg[:, gid])) * np.abs(xi)
        tol_th = 1e-4 * np.max(np.abs(o.theta))
        if precision != "fp32":
            tol_th += 3e-2 * np.max(drift) + EPS_SCALE * np.max(noise)
        print(f"[measured] {precision} k={k} theta {e_th:.2e} (tol {tol_th:.2e}) ll {e_ll:.2e} (tol {ll_rel:.0e}) "
              f"logw {e_lw:.2e} features log|g| {e_f0:.2e} LL/M {e_f1:.2e}", flush=True)
        assert e_th < tol_th, (k, e_th, tol_th)
        assert e_ll < ll_rel, (k, e_ll)
        if precision == "fp32":
            assert e_f0 < 1e-5 and e_f1 < 1e-5, (e_f0, e_f1)
            # log w: the GPU's step sizes and masses are FP32 values (about four roundings from the
            # network output, 4 ulps = 2.4e-7 relative) and the proposal densities carry -D log(h'/h):
            # D = 79,510 multiplies that rounding to ~0.02 nats per step, and the steps add up.  Each
            # side's weight is exact for its own step sizes, so this is a parity bound, not a bias.
            tol_lw = 2e-3 + k * D * 2.4e-7
            assert e_lw < tol_lw, (k, e_lw, tol_lw)
        else:
            # the feature log|g| comes from the single-BF16 backward (its norm error averages over D)
            assert e_f0 < 2e-3 and e_f1 < ll_rel, (e_f0, e_f1)
            # no lockstep bound on log w: the single-BF16 gradient moves theta' through the drift term
            # by (h^2 / 2m) dg per coordinate, and log pi(theta') answers with ~ sum_i g_i dtheta_i, of
            # order D (tens of nats here).  Each side's weight is exact for its own move (the reverse
            # kernel uses the same gradient), so this is trajectory divergence, not a bias; the FP32
            # case checks the weight arithmetic in lockstep
            assert np.all(np.isfinite(lw[fin]))
    g.close()
