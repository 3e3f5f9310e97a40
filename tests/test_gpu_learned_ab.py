"""What the trained proposal-scale network gains over the fixed-step method.

MNIST-shaped workload (784-100-10 ReLU, N = 6000, J = 64, Linear 500 -> 6000 over
K = 12 iterations, base step h0 = 0.002).  The network is trained on traces of three
plain runs; then plain and learned samplers run from the same seeds and are compared
on held-out accuracy and mean log predictive.  Measured on MI355X: the learned
sampler reaches 99.2-99.6 % accuracy (mean log predictive -0.01 .. -0.09) where the
plain one reaches 74-85 % (-2.5 .. -5.7), with a higher mean ESS."""
import numpy as np
import pytest

from gpu_helpers import cuda, lib, print_case, to_dev, torch
import smc_inputs

pytestmark = pytest.mark.gpu


def test_learned_proposal_beats_fixed_step():
    cuda()
    P = lib()
    from paper_2601_21983_amd import learned as PL, schedules
    N, NT, J, K, h0 = 6000, 1000, 64, 12, 0.002
    X, y = smc_inputs.templates28(N, seed=0)
    Xt, yt = smc_inputs.templates28(NT, seed=1)
    perm = smc_inputs.annealing_permutation(N, seed=2)
    X, y = X[perm], y[perm]
    Xd, yd, Xtd, ytd = to_dev(X), to_dev(y.astype(np.int32)), to_dev(Xt), to_dev(yt.astype(np.int32))
    sizes = schedules.sizes("linear", K, N, 500, 500)

    def make(proposal, seed):
        cfg = P.SMCConfig(widths=[784, 100, 10], n_particles=J, step_size=h0, proposal=proposal, n_iterations=K,
                          seed=seed)
        return P.SMCSampler(cfg, Xd, yd, m0=sizes[0], lambda0=N / sizes[0])

    print_case("learned-ab", N=N, J=J, K=K, h0=h0)
    feat, tgt = PL.traces_from_runs(lambda sd: make("fixed", sd), [7, 8, 9], sizes, N, PL.default_grid(h0))
    assert feat.shape == (3 * K * J, 4) and torch.isfinite(tgt).all()
    params, losses = PL.train(feat, tgt, 4, steps=600)
    assert losses[-1] < 0.5 * losses[0]

    def run(s, params=None):
        if params is not None:
            s.set_proposal_net(params, h0)
        s.resample()
        ess = []
        for k in range(1, K + 1):
            ess.append(s.step(sizes[k], N / sizes[k])["ess"])
            s.resample()
        r = s.predict(Xtd, ytd)
        s.close()
        return np.mean(ess), r["accuracy"], r["mean_log_pred"]

    for seed in (1, 2):
        ep, ap, mp = run(make("fixed", seed))
        el, al, ml = run(make("learned", seed), params)
        print(f"seed {seed}: plain ess {ep:.2f} acc {ap:.4f} mlp {mp:.4f} | learned ess {el:.2f} acc {al:.4f} "
              f"mlp {ml:.4f}", flush=True)
        assert al >= ap + 0.05
        assert ml > mp
