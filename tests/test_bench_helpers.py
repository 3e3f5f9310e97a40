"""Host logic of bench.py: the launch list that its traffic model averages over (the fused
kernel's gradient passes of the timed iterations, each with its operand mode)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    argv = sys.argv
    sys.argv = ["bench.py"]
    try:
        import bench as b
    finally:
        sys.argv = argv
    return b


def test_fused_launches_follow_the_schedule(bench):
    from paper_2601_21983_amd import schedules
    sizes = schedules.sizes("linear", 60, 60000, 1000, 1000)
    grown = [k for k in range(1, 61) if sizes[k] != sizes[k - 1]]
    for through in (0, 4, 60):
        L = bench.fused_launches(sizes, 60, through)
        # one pass per move plus one gradient-only pass per grown subset
        assert len(L) == 60 + len(grown)
        # gradient-only passes run the plain forward once the fixed-step move takes over
        assert sum(1 for mode, _ in L if mode == "plain") == sum(1 for k in grown if k > through)
        assert all(m % 256 == 0 and m >= 256 for _, m in L)
    # the first iterations' samples, padded to 256
    L = bench.fused_launches(sizes, 2, 0)
    assert L[0] == ("plain", (sizes[1] + 255) // 256 * 256) and L[1] == ("split", (sizes[1] + 255) // 256 * 256)


def test_traffic_needs_every_mode(bench):
    assert bench.measured_traffic("gemm_fwd1", []) is None
    assert bench.measured_traffic("gemm_fwd1", [("other-mode", 1024)]) is None
