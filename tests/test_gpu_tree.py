"""The tree form of the R/q batch inversion (group_form = 1: Montgomery's
3G - 3 products of Section 2.2 over a product tree shared by the waves of a
workgroup): keys equal the oracle's for every parameter set, group sizes
2..256 with ragged last groups, both reciprocal forms, per-key and batched
R/3, eager and graph launches, raw outputs included."""
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


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_tree_keys_bit_exact(ctx, p):
    n, first = 300, 5
    idx = list(range(first, first + n))
    ref = oracle_pool.oracle_keys(wl.SEED, p, idx)
    rpk, rsk = oracle_pool.pk_sk_arrays(ref, idx)
    base = ctx.get_config(p)
    try:
        for G, jump, r3b, graph in ((2, 1, 0, 0), (4, 0, 1, 0), (16, 1, 1, 1), (64, 1, 0, 0), (256, 1, 1, 0),
                                    (128, 0, 0, 1), (32, 3, 1, 0)):
            ctx.set_config(p, product_engine=1, persistent=0, group_form=1, group_size=G, inverse_share=1,
                           recip_jump=jump, r3_batch=r3b, use_graph=graph)
            pk, sk, h, f, ginv = ctx.batch_keygen(p, wl.SEED, first, n, raw=True)
            assert ctx.status() == 0
            assert np.array_equal(host(pk), rpk) and np.array_equal(host(sk), rsk), (G, jump, r3b, graph)
            hh = host(h)
            assert all(np.array_equal(hh[j], ref[i][2]) for j, i in enumerate(idx)), (G, jump, r3b, graph)
    finally:
        ctx.set_config(p, **base)


def test_tree_config_validation(ctx):
    import paper_2106_08759_amd as nk
    for bad in (dict(group_size=48), dict(group_size=512), dict(group_size=1), dict(persistent=1, lanes_per_key=2)):
        with pytest.raises(nk.NtrupError):
            ctx.set_config(761, group_form=1, **dict(dict(group_size=64, persistent=0), **bad))
    ctx.set_config(761, group_form=0)


def test_tree_full_size_equals_chain(ctx):
    """N = 65536 sntrup761: every key of the tree form (G = 64, batched R/3)
    equals the chain form's."""
    n = 65536
    base = ctx.get_config(761)
    try:
        ctx.set_config(761, product_engine=1, persistent=0, use_graph=0, r3_batch=1, group_form=0, group_size=64,
                       inverse_share=4, lanes_per_key=1)
        a_pk, a_sk = (host(t) for t in ctx.batch_keygen(761, wl.SEED, 0, n))
        ctx.set_config(761, group_form=1)
        b_pk, b_sk = (host(t) for t in ctx.batch_keygen(761, wl.SEED, 0, n))
    finally:
        ctx.set_config(761, **base)
    assert np.array_equal(a_pk, b_pk) and np.array_equal(a_sk, b_sk)
