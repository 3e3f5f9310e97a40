"""Writes e2e_mnist_shaped.json: the FP64 oracle sampler (oracle/ only) on the MNIST-shaped
workload at its full data size, for the end-to-end accuracy parity test of the GPU sampler.

Workload: 28x28 class-template images (60,000 train in one annealing order, 10,000 test),
MLP 784-100-10 ReLU, N(0, 1) prior, Langevin moves (S = 1) with h = 0.002, the Linear
schedule C = kappa = 1000 over K = 60 iterations (Section 3.1, clamped at N), lambda_k =
N / M_k, systematic resampling when ESS < J/2 (Section 2).  J = 16 particles (the oracle's
cost grows with J; the benchmark runs J = 256).  Every random draw is an input: theta_0, the
momenta of iteration k and the resampling offset of iteration k come from the seeded
generators in smc_inputs with the seeds recorded in the file, so the GPU run can replay them.

    python tests/golden/make_e2e_mnist_shaped.py      (about two minutes on 8 host cores)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import smc_inputs  # noqa: E402
from oracle import mlp, schedules, smc  # noqa: E402

RECIPE = {"widths": [784, 100, 10], "activation": "relu", "J": 16, "N": 60000, "N_test": 10000, "K": 60,
          "C": 1000, "kappa": 1000, "step_size": 0.002, "prior_std": 1.0, "ess_frac": 0.5,
          "seed_train": 0, "seed_test": 1, "seed_order": 2, "seed_theta0": 31, "seed_momenta_base": 5000,
          "seed_offsets": 77, "checkpoints": [1, 5, 10, 20, 30, 40, 50, 60]}


def main():
    r = RECIPE
    X, y = smc_inputs.templates28(r["N"], seed=r["seed_train"])
    Xt, yt = smc_inputs.templates28(r["N_test"], seed=r["seed_test"])
    perm = smc_inputs.annealing_permutation(r["N"], seed=r["seed_order"])
    X, y = X[perm], y[perm]
    D = mlp.n_params(r["widths"])
    th0 = smc_inputs.prior_draw(r["seed_theta0"], r["J"], D, r["prior_std"])
    u = smc_inputs.uniforms(r["seed_offsets"], r["K"] + 1)
    sizes = schedules.sizes("linear", r["K"], r["N"], r["C"], r["kappa"])
    o = smc.Sampler(X, y, r["widths"], r["activation"], prior_std=r["prior_std"], step_size=r["step_size"],
                    ess_frac=r["ess_frac"])
    t0 = time.perf_counter()
    o.init(th0, sizes[0], r["N"] / sizes[0])
    resampled = [bool(o.resample(u[0]))]
    trace = []
    for k in range(1, r["K"] + 1):
        xi = smc_inputs.momenta(r["seed_momenta_base"] + k, (r["J"], D))
        o.step(sizes[k], r["N"] / sizes[k], xi)
        ess = float(o.ess)
        resampled.append(bool(o.resample(u[k])))
        if k in r["checkpoints"]:
            _, acc, mlpd = o.predictive(Xt, yt)
            trace.append({"k": k, "M_k": int(sizes[k]), "ess": ess, "accuracy": acc, "mean_log_pred": mlpd})
            print(f"k={k} M={sizes[k]} ess={ess:.2f} acc={acc:.4f} mlpd={mlpd:.5f} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)
    out = {"recipe": r, "schedule": [int(s) for s in sizes], "resampled": resampled, "trace": trace,
           "written_by": "tests/golden/make_e2e_mnist_shaped.py (oracle/ only)"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "e2e_mnist_shaped.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
