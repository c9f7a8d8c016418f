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


def _mf_pairs(p):
    """(tile, K-step) pairs of one matrix-core product in R/q (ntrup_mfma.h)."""
    nd = (p + 14) // 16 + 1
    nks = cdiv(nd, 4)
    nt = cdiv(cdiv(p, 16), 16)
    return nt * nks


def _jump_mfmas(p, n=48):
    """MFMAs of one jump-divstep reciprocal in R/q (n divsteps per jump): per
    full jump, four output polynomials of two products each, four MFMAs
    (limb pairs) per output tile of 256 coefficients; f' and g' (shifted
    down by n) need the tiles up to coefficient p + n, v' and r' those up to
    p (the compiler drops the MFMAs of a tile none of whose outputs is
    stored); the last jump computes v' alone."""
    nt_fg = cdiv(p + 1 + n, 256)
    nt_vr = cdiv(p + 1, 256)
    nj = cdiv(2 * p - 1, n)
    return (nj - 1) * (2 * 2 * nt_fg + 2 * 2 * nt_vr) * 4 + 2 * nt_vr * 4


def expected_group_mfmas(p, n, G, W, jump, jump_steps=48):
    """MFMA instructions per launch of the prefix, back-substitution and h
    kernels of the eager split path, counting 3g - 3 R/q products per group of
    g keys (Section 2.2's batchInv): g - 1 prefix products (small x big, two
    limb MFMAs per pair), g - 1 back products c_i (big x big, four) and g - 1
    t updates (small x big, two); 3 (W - 1) big products per W groups sharing
    one reciprocal; one small x big product h_i per key."""
    pairs = _mf_pairs(p)
    groups = [min(G, n - s) for s in range(0, n, G)]
    blocks = cdiv(len(groups), W)
    prefix = sum((g - 1) * 2 * pairs for g in groups) + blocks * (3 * (W - 1) * 4 * pairs
                                                                   + (_jump_mfmas(p, jump_steps) if jump & 1 else 0))
    back = sum((g - 1) * 6 * pairs for g in groups)
    return prefix, back, n * 2 * pairs


def test_batchinv_products_per_group_from_counters():
    """Section 2.2 / Section 1: batchInv of n elements takes 3n - 3
    multiplications and one inversion (93 for n = 32).  The committed
    hardware counters of the benchmark's group kernels (SQ_INSTS_MFMA per
    launch, profiles/kernel_counters.json) equal exactly the MFMA count of
    3G - 3 products per group (plus the shared reciprocals and h)."""
    import json
    facts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
    bic = facts["batchinv_counts"]
    assert bic["mults_per_n"] == "3n-3" and 3 * 32 - 3 == bic["n32_mults"]
    path = os.path.join(os.path.dirname(__file__), "..", "profiles", "kernel_counters.json")
    data = json.load(open(path))
    cfg = data["config"]
    p, n, G, W = cfg["p"], cfg["n_keys"], cfg["group_size"], cfg["inverse_share"]
    prefix, back, h = expected_group_mfmas(p, n, G, W, cfg["recip_jump"], cfg.get("jump_steps", 48))
    k = data["kernels"]
    assert k["keygen_prefix_kernel<%d,%d,%s>" % (p, W, "true" if cfg["recip_jump"] & 1 else "false")]["mfma_insts"] \
        == prefix
    assert k["keygen_cinv_kernel<%d>" % p]["mfma_insts"] == back
    assert k["keygen_h_kernel<%d>" % p]["mfma_insts"] == h
    # per group of G keys: (G-1) small + (G-1) (big + small) = 3G - 3 products
    pairs = _mf_pairs(p)
    per_group = ((G - 1) * 2 * pairs + (G - 1) * 6 * pairs) // (2 * pairs)   # in small-product units
    assert per_group == 4 * (G - 1)   # 3G - 3 products, the G - 1 big ones at twice the MFMAs
