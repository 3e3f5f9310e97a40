"""The package's host-side annealing schedules agree with the oracle's and with the
hand-worked values of the schedule equations (Section 3.1)."""
import importlib.util
import os

from oracle import schedules as oracle_schedules

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
