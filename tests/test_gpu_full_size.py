"""GPU parity at the benchmark's full size, in the configuration the benchmark times: the
784-100-10 ReLU network with J = 256 particles over all 60,000 MNIST-shaped samples in split
BF16 (the fused layer-1 + output-layer kernel and the layer-1 weight-gradient GEMM, one
chunk), checked on particles the oracle evaluates one by one (Eq. approx-grad, unscaled)."""
import numpy as np
import pytest

from gpu_helpers import bf16_round, cuda, lib, print_case, to_dev, torch
from oracle import mlp
import smc_inputs

pytestmark = pytest.mark.gpu


def test_full_size_loglik_and_gradient_on_sampled_particles():
    cuda()
    P = lib()
    widths, J, M = [784, 100, 10], 256, 60000
    X, y = smc_inputs.templates28(M, seed=0)
    D = mlp.n_params(widths)
    theta = smc_inputs.prior_draw(3, J, D, 0.05)
    print_case("full-size", J=J, M=M, prec="bf16x3")
    cfg = P.SMCConfig(widths=widths, n_particles=J, precision="bf16x3", step_size=0.002)
    td = to_dev(theta)
    s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=M, lambda0=1.0, theta0=td)
    assert s.chunk_samples() >= M
    ll, g = s.nn_backward(td, M)
    torch.cuda.synchronize()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    s.close()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
    Xo = bf16_round(X)
    for j in (0, 137, 255):
        ll_o, g_o = mlp.loglik_grad(theta[j:j + 1].astype(np.float64), Xo, y, widths, "relu")
        e_ll = abs(ll[j] - ll_o[0]) / abs(ll_o[0])
        e_g = np.max(np.abs(g[j] - g_o[0])) / np.max(np.abs(g_o[0]))
        print(f"particle {j}: ll {e_ll:.3g}, grad {e_g:.3g}", flush=True)
        assert e_ll < 1e-4, (j, e_ll)
        assert e_g < 5e-3, (j, e_g)


def test_lenet5_full_size_chunking_and_sampled_predictive():
    """LeNet-5 at the batching-scheme study's size (J = 32, 60,000 images): the gradient over
    the whole set does not depend on how it is chunked (the per-sample terms are the same, only
    the FP32 summation order differs), and the posterior predictive of sampled images matches
    the oracle's."""
    cuda()
    P = lib()
    from oracle import lenet, smc
    dims, J, M = list(lenet.LENET5_MNIST), 32, 60000
    sh = lenet.LeNetShape(*dims)
    X, y = smc_inputs.templates28(M, seed=0)
    theta = smc_inputs.prior_draw(5, J, sh.D, 0.05)
    td = to_dev(theta)
    print_case("lenet-full-size", J=J, M=M)
    out = []
    for budget in (0, 256 << 20):  # chunks of the default budget, then of 256 MB
        cfg = P.SMCConfig(widths=dims, n_particles=J, model="lenet", activation="tanh", act_budget_bytes=budget)
        s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=M, lambda0=1.0, theta0=td)
        ll, g = s.nn_backward(td, M)
        torch.cuda.synchronize()
        out.append((s.chunk_samples(), ll.cpu().numpy(), g.cpu().numpy()))
        if budget == 0:
            r = s.predict(to_dev(X), to_dev(y.astype(np.int32)), probs=True)
            probs = r["probs"].cpu().numpy()
            lw = s.state()["logw"].cpu().numpy()
        s.close()
    (mc0, ll0, g0), (mc1, ll1, g1) = out
    assert mc0 != mc1, (mc0, mc1)
    assert np.all(np.isfinite(g0)) and np.all(np.isfinite(ll0))
    d = np.max(np.abs(g0 - g1) / np.max(np.abs(g1), axis=1, keepdims=True))
    print(f"chunks of {mc0} vs {mc1}: gradient {d:.3g}", flush=True)
    assert d < 1e-4, d
    assert np.max(np.abs(ll0 - ll1) / np.abs(ll1)) < 1e-6
    idx = np.array([0, 12345, 33333, 59999])
    p_o, _, _ = smc.predictive(theta.astype(np.float64), lw, X[idx], y[idx], None, "tanh", lenet.Model(sh, "tanh"))
    np.testing.assert_allclose(probs[idx], p_o, rtol=1e-4, atol=1e-6)


def test_cnn_bench_size_on_sampled_particles():
    """The convolutional network at the size its benchmark leg runs (J = 128, 1,000-image
    subsets of the 32x32x3 textures, BF16 operands), checked on particles the oracle evaluates
    one by one, at the BF16 tolerances of the small cases."""
    cuda()
    P = lib()
    from oracle import cnn
    dims, J, M = (32, 32, 3, 16, 32, 10), 128, 1000
    sh = cnn.CNNShape(*dims)
    X, y = smc_inputs.textures32(M, seed=0)
    X = X.reshape(M, -1)
    theta = smc_inputs.prior_draw(6, J, sh.D, 0.05)
    td = to_dev(theta)
    print_case("cnn-bench-size", J=J, M=M, prec="bf16")
    cfg = P.SMCConfig(widths=list(dims), n_particles=J, model="cnn", precision="bf16")
    s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=M, lambda0=1.0, theta0=td)
    ll, g = s.nn_backward(td, M)
    torch.cuda.synchronize()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    s.close()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
    for j in (0, 127):
        ll_o, g_o = cnn.loglik_grad(theta[j:j + 1].astype(np.float64), X, y, sh)
        e_ll = abs(ll[j] - ll_o[0]) / abs(ll_o[0])
        e_g = np.max(np.abs(g[j] - g_o[0])) / np.max(np.abs(g_o[0]))
        print(f"particle {j}: ll {e_ll:.3g}, grad {e_g:.3g}", flush=True)
        assert e_ll < 2e-2, (j, e_ll)
        assert e_g < 1e-1, (j, e_g)


def test_deep_network_full_size_on_sampled_particles():
    """The 784-256-256-10 network with J = 1024 particles over all 60,000 samples (BF16 operands,
    the activation budget splitting the set into chunks with recomputation), checked on
    particles the oracle evaluates one by one, at the BF16 tolerances of the small cases."""
    cuda()
    P = lib()
    widths, J, M = [784, 256, 256, 10], 1024, 60000
    X, y = smc_inputs.templates28(M, seed=0)
    D = mlp.n_params(widths)
    theta = smc_inputs.prior_draw(8, J, D, 0.05)
    td = to_dev(theta)
    print_case("deep-full-size", J=J, M=M, prec="bf16")
    cfg = P.SMCConfig(widths=widths, n_particles=J, precision="bf16")
    s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=M, lambda0=1.0, theta0=td)
    assert s.chunk_samples() < M
    ll, g = s.nn_backward(td, M)
    torch.cuda.synchronize()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    s.close()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
    for j in (0, 1023):
        ll_o, g_o = mlp.loglik_grad(theta[j:j + 1].astype(np.float64), X, y, widths, "relu")
        e_ll = abs(ll[j] - ll_o[0]) / abs(ll_o[0])
        e_g = np.max(np.abs(g[j] - g_o[0])) / np.max(np.abs(g_o[0]))
        print(f"particle {j}: ll {e_ll:.3g}, grad {e_g:.3g}", flush=True)
        assert e_ll < 2e-2, (j, e_ll)
        assert e_g < 3e-2, (j, e_g)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_weight_gradient_tiles_with_ragged_edges(precision):
    """The large weight-gradient tiles (sixteen waves of 64x32 for 256x128, in BF16 and FP32) at
    a ragged size: J = 257 particles give 25,700 unit rows (the last 256-row tile holds one
    particle's 100 rows and 156 of clamped padding), 785 gradient columns (the last 128-wide
    tile 17), and 3,001 samples (a ragged last K step); sampled particles, including the one in
    the last row tile, against the oracle (Eq. approx-grad, unscaled)."""
    cuda()
    P = lib()
    widths, J, M = [784, 100, 10], 257, 3001
    X, y = smc_inputs.templates28(M, seed=4)
    D = mlp.n_params(widths)
    theta = smc_inputs.prior_draw(8, J, D, 0.05)
    print_case("ragged-weight-gradient", J=J, M=M, prec=precision)
    cfg = P.SMCConfig(widths=widths, n_particles=J, precision=precision, step_size=0.002)
    td = to_dev(theta)
    s = P.SMCSampler(cfg, to_dev(X), to_dev(y.astype(np.int32)), m0=M, lambda0=1.0, theta0=td)
    ll, g = s.nn_backward(td, M)
    torch.cuda.synchronize()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    s.close()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
    Xo = X.astype(np.float64) if precision == "fp32" else bf16_round(X)
    tol_g = 2e-4 if precision == "fp32" else 5e-3
    for j in (0, 131, 255, 256):
        ll_o, g_o = mlp.loglik_grad(theta[j:j + 1].astype(np.float64), Xo, y, widths, "relu")
        e_ll = abs(ll[j] - ll_o[0]) / abs(ll_o[0])
        e_g = np.max(np.abs(g[j] - g_o[0])) / np.max(np.abs(g_o[0]))
        print(f"particle {j}: ll {e_ll:.3g}, grad {e_g:.3g}", flush=True)
        assert e_ll < 1e-4, (j, e_ll)
        assert e_g < tol_g, (j, e_g)
