"""Batched R/3 reciprocals (config r3_batch; Section 3.1, Algorithm 1:
batchInv over R/3 after an invertibility check of each g).  The R/3 product
on the matrix cores equals the oracle's product mod 3; the keys equal the
oracle's for every parameter set and group size, also when the screen is off
and groups holding a non-unit g take the per-key fallback."""
import numpy as np
import pytest

from paper_2106_08759_amd import workloads as wl
import oracle
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


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_mul_r3_matches_oracle(ctx, p):
    import torch
    rng = np.random.default_rng(p)
    n = 24
    a = rng.integers(-1, 2, (n, p)).astype(np.int8)
    b = rng.integers(-1, 2, (n, p)).astype(np.int8)
    a[0] = 0
    a[0, p - 1] = 1                  # x^{p-1}: exercises the wrap of the reduction
    b[0] = 0
    b[0, p - 1] = -1
    a[1] = 1                          # all-ones rows: the largest sums
    b[1] = 1
    c = host(ctx.mul_r3(p, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()))
    for i in range(n):
        want = oracle.mul_mod(a[i].astype(np.int64), b[i].astype(np.int64), p, 3)
        want = np.where(want == 2, -1, want)         # centered, as the library returns it
        assert np.array_equal(c[i].astype(np.int64), want), (p, i)


def run(ctx, p, first, n, **cfg):
    base = ctx.get_config(p)
    try:
        ctx.set_config(p, product_engine=1, persistent=0, **cfg)
        pk, sk = ctx.batch_keygen(p, wl.SEED, first, n)
        assert ctx.status() == 0
        return host(pk), host(sk)
    finally:
        ctx.set_config(p, **base)


@pytest.mark.parametrize("jump", [1, 3])
@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_keys_bit_exact(ctx, p, jump):
    """Group reciprocals in R/3 by bitsliced divsteps (recip_jump bit 1
    clear) or by jump divsteps on the matrix cores (set)."""
    n = 200
    ref = oracle_pool.oracle_keys(wl.SEED, p, range(n))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(n))
    for G in (1, 7, 32, 64):
        pk, sk = run(ctx, p, 0, n, r3_batch=1, group_size=G, recip_jump=jump)
        assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk), (p, G)


@pytest.mark.parametrize("jump", [1, 3])
@pytest.mark.parametrize("p", [653, 1277])
def test_fallback_path(ctx, p, jump):
    """Screen off: about a quarter to a half of the groups of 8 hold a g that
    is not a unit; the group reciprocal (either form) reports the product as
    no unit and those groups take the per-key divstep pass from their first
    draw."""
    n = 300
    ref = oracle_pool.oracle_keys(wl.SEED, p, range(n))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(n))
    assert sum(ref[i][5] > 1 for i in range(n)) >= 5
    for G, spec in ((8, 4), (32, 1), (3, 8)):
        pk, sk = run(ctx, p, 0, n, r3_batch=2, group_size=G, retry_parallel_attempts=spec, recip_jump=jump)
        assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk), (p, G, spec)


def test_offset_range_and_graph(ctx):
    import torch
    ref = oracle_pool.oracle_keys(wl.SEED, 761, range(4000, 4100))
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(4000, 4100))
    for ug in (0, 1, 1):
        pk, sk = run(ctx, 761, 4000, 100, r3_batch=1, group_size=16, use_graph=ug)
        torch.cuda.synchronize()
        assert np.array_equal(pk, rpk) and np.array_equal(sk, rsk), ug


def test_full_size_matches_per_key(ctx):
    """N = 65536 sntrup761: every key equals the per-key divstep pipeline's."""
    n = 65536
    a = run(ctx, 761, 0, n, r3_batch=0, group_size=32, inverse_share=8, lanes_per_key=4, use_graph=0)
    b = run(ctx, 761, 0, n, r3_batch=1, group_size=32, inverse_share=8, lanes_per_key=4, use_graph=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
