"""The package's host-side annealing schedules agree with the oracle's and with the
hand-worked values of the schedule equations (Section 3.1)."""
import importlib.util
import os

import numpy as np

from oracle import schedules as oracle_schedules
from oracle import schedules

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _product():
    spec = importlib.util.spec_from_file_location(
        "smc_schedules", os.path.join(ROOT, "paper_2601_21983_amd", "schedules.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_product_schedules_match_oracle():
    m = _product()
    for name in m.NAMES:
        for K, N, C, kap in [(60, 60000, 1000, 1000), (200, 60000, 500, 500), (10, 1024, 128, 128),
                             (7, 100, 3, 5), (1, 10, 10, 1), (33, 5000, 17, 250)]:
            assert m.sizes(name, K, N, C, kap) == oracle_schedules.sizes(name, K, N, C, kap), (name, K, N, C, kap)


def test_product_schedules_golden():
    m = _product()
    for line in open(os.path.join(ROOT, "tests", "golden", "schedules.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, K, N, C, kap, k, mk = line.split()
        assert m.subset_size(name, int(k), int(K), int(N), int(C), int(kap)) == int(mk), line


def test_posterior_mean_and_change():
    theta = np.array([[1.0, 2.0, 3.0], [3.0, 2.0, 1.0], [5.0, -1.0, 0.5]])
    # equal weights: the arithmetic mean; a one-hot weight picks that particle
    np.testing.assert_allclose(schedules.posterior_mean(theta, np.zeros(3)), theta.mean(axis=0), rtol=1e-15)
    np.testing.assert_array_equal(schedules.posterior_mean(theta, [-np.inf, 0.0, -np.inf]), theta[1])
    # weights 1/4, 1/4, 1/2 from log-weights shifted by an arbitrary constant
    lw = np.log([1.0, 1.0, 2.0]) + 123.0
    np.testing.assert_allclose(schedules.posterior_mean(theta, lw), [3.5, 0.5, 1.25], rtol=1e-14)
    # |(0.3, 0.4)| / |(3, 4)| = 0.5 / 5
    assert abs(schedules.mean_change([3.0, 4.0], [3.3, 4.4]) - 0.1) < 1e-15
    assert schedules.mean_change([0.0, 0.0], [0.0, 0.0]) == 0.0
    assert schedules.mean_change([0.0, 0.0], [1.0, 0.0]) == float("inf")


def test_adaptive_growth_rule():
    assert schedules.adaptive_next(1000, 0.005, 1e-2, 1000, 50000) == 2000
    assert schedules.adaptive_next(1000, 0.02, 1e-2, 1000, 50000) == 1000
    assert schedules.adaptive_next(1000, 1e-2, 1e-2, 1000, 50000) == 1000  # strict comparison
    assert schedules.adaptive_next(49500, 0.0, 1e-2, 1000, 50000) == 50000  # clamped to N
