"""GPU parity of multinomial resampling (the paper's scheme, Section 2) with the exact integer
rule: ancestors and in-place placement bit for bit against the oracle, inside the sampler with
host-given uniforms, and the device-drawn uniforms' reproducibility and binomial counts."""
import os

import numpy as np
import pytest

from gpu_helpers import cuda, lib, print_case, to_dev, torch
from oracle import mlp, smc
import smc_inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _multi_case(w, u):
    P = lib()
    J = len(w)
    anc = torch.empty(J, dtype=torch.int32, device="cuda")
    pl = torch.empty(J, dtype=torch.int32, device="cuda")
    d_w, d_u = to_dev(np.asarray(w, np.float64)), to_dev(np.asarray(u, np.float64))
    P._lib.smc_multinomial_resample(d_w.data_ptr(), J, d_u.data_ptr(), anc.data_ptr(), pl.data_ptr(), None)
    torch.cuda.synchronize()
    return anc.cpu().numpy(), pl.cpu().numpy()


def test_multinomial_worked_examples():
    cuda()
    for line in open(os.path.join(GOLDEN, "multinomial.txt")):
        if line.startswith("#") or not line.strip():
            continue
        u, w, a = [p.strip() for p in line.split(";")]
        u = [float(x) for x in u.split()]
        w = [float(x) for x in w.split()]
        print_case("multinomial-worked", J=len(w))
        got, _ = _multi_case(w, u)
        assert got.tolist() == [int(x) for x in a.split()]


@pytest.mark.parametrize("J", [1, 3, 64, 257, 1024, 4096])
def test_multinomial_bitexact_vs_oracle(J):
    cuda()
    rng = np.random.default_rng(200 + J)
    for trial in range(4):
        if trial == 0:
            w = np.full(J, 1.0 / J)
        elif trial == 1:
            w = np.zeros(J)
            w[J // 3] = 1.0
        else:
            lw, _ = smc.normalise(3.0 * rng.standard_normal(J))
            w = np.exp(lw)
        u = rng.random(J)
        if trial == 0:
            u[0], u[-1] = 0.0, 1.0 - 2 ** -53
        print_case("multinomial", J=J, trial=trial)
        anc, pl = _multi_case(w, u)
        ref = smc.multinomial_ancestors(w, u)
        assert np.array_equal(anc, ref)
        assert np.array_equal(pl, smc.placement(ref))


def test_multinomial_inside_the_sampler_matches_the_oracle():
    """Blobs trajectory with multinomial resampling at every iteration (host-given uniforms)."""
    cuda()
    P = lib()
    widths, J, N, h = [2, 16, 2], 64, 512, 1e-3
    X, y = smc_inputs.blobs(N, seed=30)
    D = mlp.n_params(widths)
    th0 = smc_inputs.prior_draw(31, J, D, 1.0)
    print_case("multinomial-trajectory", J=J)
    o = smc.Sampler(X, y, widths, "tanh", step_size=h)
    o.init(th0, 128, N / 128)
    cfg = P.SMCConfig(widths=widths, n_particles=J, activation="tanh", step_size=h)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=128, lambda0=N / 128, theta0=to_dev(th0))
    sizes = [128, 192, 256, 320, 384, 448, 512, 512]
    for k in range(1, len(sizes)):
        xi = smc_inputs.momenta(40 + k, (J, D))
        g.set_noise(to_dev(xi))
        g.step(sizes[k], N / sizes[k])
        o.step(sizes[k], N / sizes[k], xi)
        u = smc_inputs.uniforms(50 + k, J)
        res_g, anc_g = g.resample("always", want=True, scheme="multinomial", uniforms=to_dev(u))
        res_o = o.resample(u, mode="always", scheme="multinomial")
        assert res_g and res_o
        assert anc_g == o.ancestors.tolist(), k
        st = g.state()
        th = st["theta"].cpu().numpy()
        assert np.max(np.abs(th - o.theta)) < 1e-5 * np.max(np.abs(o.theta)), k
        assert np.allclose(st["logw"].cpu().numpy(), -np.log(J))
    g.close()


def test_device_drawn_uniforms_are_reproducible_and_binomial():
    """Philox-drawn uniforms: the same seed gives the same ancestors; over 300 resamplings of
    a fixed weight vector the mean count of particle j is J w_j within 5 standard errors."""
    cuda()
    P = lib()
    widths, J, N = [2, 4, 2], 16, 64
    X, y = smc_inputs.blobs(N, seed=32)
    D = mlp.n_params(widths)
    th0 = smc_inputs.prior_draw(33, J, D, 1.0)
    print_case("multinomial-device", J=J)
    runs = []
    for rep in range(2):
        cfg = P.SMCConfig(widths=widths, n_particles=J, activation="tanh", seed=99)
        g = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=N, lambda0=1.0, theta0=to_dev(th0))
        w = np.random.default_rng(34).dirichlet(np.full(J, 2.0))
        lw0 = to_dev(np.log(w))
        counts, ancs = np.zeros(J), []
        for r in range(300):
            g.set_state(to_dev(th0), logw=lw0, rng_counter=r)  # the same weights every time
            _, anc = g.resample("always", want=True, scheme="multinomial")
            ancs.append(anc)
            counts += np.bincount(anc, minlength=J)
        runs.append(ancs)
        g.close()
    assert runs[0] == runs[1]
    assert len({tuple(a) for a in runs[0]}) > 250  # a new draw at every generator position
    mean = counts / 300
    se = np.sqrt(J * w * (1 - w) / 300)
    assert np.all(np.abs(mean - J * w) <= 5 * se + 1e-9), (mean, J * w)


def test_all_nonfinite_population_is_not_resampled():
    """Every particle's parameters non-finite: the step without statistics leaves every log-weight
    at -inf; resampling must report SMC_ERR_NONFINITE instead of turning the population into
    copies of one particle with uniform weights (Section 2: the normalised weights of Eq.
    normalise do not exist), and the population stays as it was."""
    cuda()
    P = lib()
    widths, J, N = [2, 4, 2], 8, 64
    X, y = smc_inputs.blobs(N, seed=40)
    D = mlp.n_params(widths)
    th0 = smc_inputs.prior_draw(41, J, D, 1.0)
    print_case("resample-all-nonfinite", J=J)
    cfg = P.SMCConfig(widths=widths, n_particles=J, activation="tanh", seed=5, step_size=0.01)
    g = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=N, lambda0=1.0, theta0=to_dev(th0))
    bad = np.full((J, D), np.nan, np.float32)
    g.set_state(to_dev(bad))
    g.step(N, 1.0, info=False)  # returns no statistics, so it does not check
    for scheme in ("systematic", "multinomial"):
        for mode in ("if_needed", "always"):
            with pytest.raises(P.SMCError) as e:
                g.resample(mode, scheme=scheme)
            assert e.value.status == 5  # SMC_ERR_NONFINITE
    st = g.state()
    assert np.all(np.isneginf(st["logw"].cpu().numpy()) | np.isnan(st["logw"].cpu().numpy()))
    g.close()
