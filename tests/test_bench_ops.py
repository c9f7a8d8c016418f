"""bench.py's algorithmic operation counts (host logic, no GPU)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))
import bench  # noqa: E402


def cdiv(a, b):
    return -(-a // b)


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_r3_live_word_count(p):
    """9 ops per live word of each pair and divstep: the first step has every
    f, g word and one v, r word live, the last one f, g word and every v, r
    word; the total lies between the ideal and the full-width count, and under
    the one-lane kernel's 96-step segment schedule."""
    W = cdiv(p + 1, 32)
    n = 2 * p - 1
    live = bench.r3_kernel_ops(p, 1) / 9
    full = n * 2 * W
    assert live < full
    assert 0.70 * full < live < 0.80 * full
    seg = 0
    for a in range(0, n, 96):
        b = min(n, a + 96)
        seg += (b - a) * (cdiv(min(p + 1, n - a), 32) + min(W, cdiv(b + 1, 32)))
    assert live <= seg
    assert bench.r3_kernel_ops(p, 3) == 3 * bench.r3_kernel_ops(p, 1)


def test_r3_live_count_at_761():
    """The figure quoted with the roofline: 0.498 M lane-ops per key."""
    assert round(bench.r3_kernel_ops(761, 1) / 1e6, 3) == 0.498


def test_group_ops_split_moves_work_only():
    """The eager split (back-substitution beside the R/3 stage, h after it)
    moves the c_i and t_i products from group_back to group_prefix; the total
    is the same."""
    for p, n, G, W in [(761, 65536, 32, 8), (761, 1000, 7, 2), (1277, 300, 64, 4)]:
        a = bench.group_kernel_ops(p, n, G, W)
        b = bench.group_kernel_ops(p, n, G, W, split=True)
        assert a["group_prefix"] + a["group_back"] == b["group_prefix"] + b["group_back"]
        assert b["group_back"] == 2 * 2 * n * p * p      # h_i: 2 limb pairs, 2 ops per multiply-add
