"""The allocation-free proposal-network trainer (smc_mlp_train_noalloc) against the
allocating one (smc_mlp_train): the same kernels in the same order over the same inputs,
so parameters, Adam moments and the loss must agree bit for bit.  Two calls in a row, the
second on fewer rows than the first, check that the shared device scratch carries nothing
from one call into the next."""
import numpy as np
import pytest

from gpu_helpers import cuda, lib, print_case, to_dev, torch
from oracle import learned as olearned

pytestmark = pytest.mark.gpu

G = 4


def _inputs(R, seed):
    rng = np.random.default_rng(seed)
    feat = rng.normal(size=(R, 4)) * [2.0, 0.7, 0.3, 0.3] + [1.0, -0.5, 0.3, 0.4]
    tgt = rng.normal(size=(R, 1 + G))
    return to_dev(feat.astype(np.float32)), to_dev(tgt.astype(np.float32))


def test_noalloc_training_matches_the_allocating_call():
    cuda()
    P = lib()
    blob = olearned.init_blob(G, 5, mu=[1.0, -0.5, 0.3, 0.4], sd=[2.0, 0.7, 0.3, 0.3]).astype(np.float32)
    Pn = P._lib.smc_mlp_n_params(G)
    assert blob.shape[0] == Pn
    # a: allocating call, b: allocation-free call, each on its own copy of the state
    pa, pb = to_dev(blob), to_dev(blob)
    aa = torch.zeros(2 * Pn, dtype=torch.float32, device="cuda")
    ab = torch.zeros(2 * Pn, dtype=torch.float32, device="cuda")
    loss_b = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    first = 1
    for call, (R, steps, seed) in enumerate([(20000, 3, 11), (700, 2, 12)]):
        feat, tgt = _inputs(R, seed)
        print_case("mlp-train-noalloc", call=call, R=R, steps=steps, seed=seed)
        loss_a = P._lib.smc_mlp_train(pa.data_ptr(), aa.data_ptr(), feat.data_ptr(), tgt.data_ptr(), R, G, first,
                                      steps, 1e-2, stream)
        P._lib.smc_mlp_train_noalloc(pb.data_ptr(), ab.data_ptr(), feat.data_ptr(), tgt.data_ptr(), R, G, first,
                                     steps, 1e-2, loss_b.data_ptr(), stream)
        torch.cuda.synchronize()
        first += steps
        assert torch.equal(pa, pb), f"parameters differ after call {call}"
        assert torch.equal(aa, ab), f"Adam moments differ after call {call}"
        lb = float(loss_b.item())
        assert np.isfinite(loss_a) and lb == loss_a, (call, loss_a, lb)
    assert not torch.equal(pa, to_dev(blob)), "training moved no parameter"


def test_noalloc_training_rejects_sizes_beyond_its_scratch():
    cuda()
    P = lib()
    Pn = P._lib.smc_mlp_n_params(G)
    par = torch.zeros(Pn, dtype=torch.float32, device="cuda")
    adam = torch.zeros(2 * Pn, dtype=torch.float32, device="cuda")
    feat, tgt = _inputs(64, 3)
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(P._lib.SMCError, match="32768"):
        P._lib.smc_mlp_train_noalloc(par.data_ptr(), adam.data_ptr(), feat.data_ptr(), tgt.data_ptr(), 32769, G, 1,
                                     1, 1e-2, None, stream)
    with pytest.raises(P._lib.SMCError, match="n_groups"):
        P._lib.smc_mlp_train_noalloc(par.data_ptr(), adam.data_ptr(), feat.data_ptr(), tgt.data_ptr(), 64, 9, 1, 1,
                                     1e-2, None, stream)
