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
