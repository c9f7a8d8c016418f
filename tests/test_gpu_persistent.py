"""The persistent fused form (one kernel per call; config persistent=1):
encoded pk and sk bytes equal the oracle's for every parameter set, group
size, shared-reciprocal width, R/3 lane layout, retry setting, for mixed
parameter sets in one launch, under graph replay, and at the benchmark size
(where every key is compared with the stage pipeline and sampled keys with the
oracle).  Every call also checks the context's error word, which records a
dependency wait that ran out (bit 4) as well as key-level failures.
"""
import numpy as np
import pytest

from paper_2106_08759_amd import workloads as wl
import oracle_pool

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2106_08759_amd as nk
    c = nk.Context(0)
    yield c
    c.close()


def host(t):
    return t.cpu().numpy()


def run(ctx, p, first, n, **cfg):
    base = ctx.get_config(p)
    try:
        ctx.set_config(p, persistent=1, product_engine=1, **cfg)
        pk, sk = ctx.batch_keygen(p, wl.SEED, first, n)
        assert ctx.status() == 0
        return host(pk), host(sk)
    finally:
        ctx.set_config(p, **base)


def test_small_761(ctx):
    n = 200
    ref = oracle_pool.oracle_keys(wl.SEED, 761, range(n))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(n))
    pk, sk = run(ctx, 761, 0, n, group_size=32, inverse_share=4, lanes_per_key=2)
    assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk)


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_bit_exact_layouts(ctx, p):
    """Group sizes with ragged last groups and blocks of W groups, both R/3
    lane layouts of the fused kernel."""
    n = 200
    ref = oracle_pool.oracle_keys(wl.SEED, p, range(n))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(n))
    for G, W, L in [(1, 1, 2), (7, 4, 4), (32, 8 if p != 1277 else 4, 2), (64, 2, 4), (13, 8 if p != 1277 else 2, 4)]:
        pk, sk = run(ctx, p, 0, n, group_size=G, inverse_share=W, lanes_per_key=L)
        assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk), (p, G, W, L)


@pytest.mark.parametrize("p", [653, 1277])
def test_resampling(ctx, p):
    """Keys whose first g is not a unit go through the retry items (several
    draws side by side); the accepted g is the first unit."""
    n = 300
    ref = oracle_pool.oracle_keys(wl.SEED, p, range(n))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(n))
    assert sum(ref[i][5] > 1 for i in range(n)) >= 5
    for spec in (1, 4, 8):
        pk, sk = run(ctx, p, 0, n, group_size=32, inverse_share=2, lanes_per_key=4,
                     retry_parallel_attempts=spec)
        assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk), (p, spec)


def test_offset_range(ctx):
    ref = oracle_pool.oracle_keys(wl.SEED, 857, range(1000, 1077))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(1000, 1077))
    pk, sk = run(ctx, 857, 1000, 77, group_size=16, inverse_share=2, lanes_per_key=2)
    assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk)


def test_mixed_one_launch(ctx):
    """Four parameter sets of uneven sizes as one persistent launch."""
    jobs = [(653, 100, 140), (761, 7, 233), (857, 0, 17), (1277, 3, 121)]
    base = {p: ctx.get_config(p) for p, _, _ in jobs}
    try:
        for p, _, _ in jobs:
            ctx.set_config(p, persistent=1, product_engine=1, lanes_per_key=2, group_size=16, inverse_share=2)
        outs = ctx.batch_keygen_mixed(wl.SEED, jobs)
        assert ctx.status() == 0
    finally:
        for p, c in base.items():
            ctx.set_config(p, **c)
    for (p, first, n), (pk, sk) in zip(jobs, outs):
        ref = oracle_pool.oracle_keys(wl.SEED, p, range(first, first + n))
        rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(first, first + n))
        assert np.array_equal(host(pk), rpk) and np.array_equal(host(sk), rsk), p


def test_graph_replay(ctx):
    """The persistent launch captured once and replayed, with eager work and
    synchronizations between replays; each replay gives the same bytes."""
    import torch
    n = 256
    ref = oracle_pool.oracle_keys(wl.SEED, 761, range(300, 300 + n))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(300, 300 + n))
    base = ctx.get_config(761)
    try:
        ctx.set_config(761, persistent=1, product_engine=1, use_graph=1, group_size=32, inverse_share=4,
                       lanes_per_key=4)
        for rep in range(3):
            pk, sk = ctx.batch_keygen(761, wl.SEED, 300, n)
            torch.cuda.synchronize()
            assert ctx.status() == 0
            assert np.array_equal(host(pk), rpk) and np.array_equal(host(sk), rsk), rep
            _ = torch.ones(1 << 20, device="cuda").sum().item()
    finally:
        ctx.set_config(761, **base)


def test_full_size_matches_pipeline(ctx):
    """N = 65536 sntrup761: every key of the fused form equals the stage
    pipeline's; 128 spread keys equal the oracle's."""
    n = 65536
    base = ctx.get_config(761)
    try:
        ctx.set_config(761, persistent=0, product_engine=1, use_graph=0, group_size=32, inverse_share=8,
                       lanes_per_key=4)
        pk0, sk0 = ctx.batch_keygen(761, wl.SEED, 0, n)
        assert ctx.status() == 0
        a_pk, a_sk = host(pk0), host(sk0)
        del pk0, sk0
        ctx.set_config(761, persistent=1)
        pk1, sk1 = ctx.batch_keygen(761, wl.SEED, 0, n)
        assert ctx.status() == 0
        b_pk, b_sk = host(pk1), host(sk1)
    finally:
        ctx.set_config(761, **base)
    assert np.array_equal(a_pk, b_pk) and np.array_equal(a_sk, b_sk)
    idx = list(np.linspace(0, n - 1, 128).astype(int))
    ref = oracle_pool.oracle_keys(wl.SEED, 761, idx)
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, idx)
    assert np.array_equal(b_pk[idx], rpk) and np.array_equal(b_sk[idx], rsk)
