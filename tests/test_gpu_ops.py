"""Kernel-level parity: each single operation of the GPU library against the
oracle on the same seeded inputs, bit-exact (all results are integers).

Sizes span several wave tiles and ragged tails; the extremes +-(q-1)/2 give
the largest int32 partial sums.
"""
import numpy as np
import pytest

import oracle
from paper_2106_08759_amd import workloads as wl

pytestmark = pytest.mark.gpu

P_ALL = [653, 761, 857, 1277]


@pytest.fixture(scope="module")
def ctx():
    import paper_2106_08759_amd as nk
    c = nk.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def centered(v, m):
    v = np.asarray(v, dtype=np.int64) % m
    return np.where(v > (m - 1) // 2, v - m, v)


@pytest.mark.parametrize("p", P_ALL)
def test_sample_matches_oracle(ctx, p):
    _, q, w = wl.PQW[p]
    n = 37  # ragged: not a multiple of the 4 keys per block
    for attempt in (0, 5):
        f, g = ctx.sample(p, wl.SEED, 1000, n, attempt=attempt)
        f, g = host(f), host(g)
        for i in range(n):
            assert np.array_equal(f[i], oracle.sample_short(wl.SEED, 1000 + i, p, w)), (p, i)
            assert np.array_equal(g[i], oracle.sample_small(wl.SEED, 1000 + i, p, attempt)), (p, i, attempt)


@pytest.mark.parametrize("p", [761, 1277])
def test_sample_short_unaligned_rows(ctx, p):
    """f rows at an odd device address (encapsulation's r may be any int8
    array): the sampler's word stores fall back to bytes, the rows equal the
    oracle's and the bytes around them are untouched."""
    import torch
    import paper_2106_08759_amd as nk
    _, q, w = wl.PQW[p]
    n, off = 13, 3
    buf = torch.full((n * p + 8,), 0x55, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc = nk.lib().ntrup_op_sample(ctx._h, p, nk._seed_bytes(wl.SEED), 7, n, 0, buf.data_ptr() + off, None,
                                  torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    b = host(buf)
    assert (b[:off] == 0x55).all() and (b[off + n * p:] == 0x55).all()
    f = b[off:off + n * p].view(np.int8).reshape(n, p)
    for i in range(n):
        assert np.array_equal(f[i], oracle.sample_short(wl.SEED, 7 + i, p, w)), (p, i)


ENGINES = [0, 1]  # vector dot2 Toeplitz, int8 matrix cores


def _with_engine(ctx, p, engine):
    ctx.set_config(p, product_engine=engine)


DEFAULT_ENGINE = 1


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("p", P_ALL)
def test_mul_big_matches_oracle(ctx, p, engine):
    _, q, _ = wl.PQW[p]
    a = np.concatenate([wl.random_rq(p, 6, tag=1), wl.extreme_rq(p)])
    b = np.concatenate([wl.random_rq(p, 6, tag=2), wl.extreme_rq(p)[::-1]])
    _with_engine(ctx, p, engine)
    try:
        c = host(ctx.mul_rq(p, dev(a), dev(b)))
    finally:
        _with_engine(ctx, p, DEFAULT_ENGINE)
    for i in range(len(a)):
        ref = centered(oracle.mul_mod(a[i], b[i], p, q), q)
        assert np.array_equal(c[i], ref), (p, engine, i)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("p", P_ALL)
def test_mul_small_matches_oracle(ctx, p, engine):
    _, q, _ = wl.PQW[p]
    a = wl.random_small(p, 6, tag=3, bound=3).astype(np.int16)
    a[0] = 3
    a[1] = -3
    b = np.concatenate([wl.random_rq(p, 4, tag=4), wl.extreme_rq(p)[:2]])
    _with_engine(ctx, p, engine)
    try:
        c = host(ctx.mul_rq(p, dev(a), dev(b), small_a=True))
    finally:
        _with_engine(ctx, p, DEFAULT_ENGINE)
    for i in range(len(a)):
        assert np.array_equal(c[i], centered(oracle.mul_mod(a[i], b[i], p, q), q)), (p, engine, i)


@pytest.mark.parametrize("p", P_ALL)
def test_mul_engines_agree_on_many(ctx, p):
    """2048 random products per engine (several thousand MFMA tiles, every
    lane position): the matrix-core product equals the vector product, which
    the tests above pin to the oracle."""
    import torch
    _, q, _ = wl.PQW[p]
    a = dev(wl.random_rq(p, 2048, tag=11))
    s = dev(wl.random_small(p, 2048, tag=12, bound=3).astype(np.int16))
    b = dev(wl.random_rq(p, 2048, tag=13))
    outs = []
    for engine in ENGINES:
        _with_engine(ctx, p, engine)
        outs.append((host(ctx.mul_rq(p, a, b)), host(ctx.mul_rq(p, s, b, small_a=True))))
    _with_engine(ctx, p, DEFAULT_ENGINE)
    torch.cuda.synchronize()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("jump", [0, 1])
@pytest.mark.parametrize("p", P_ALL)
def test_recip_rq_matches_oracle(ctx, p, jump):
    """The plain divstep loop (jump = 0) and jump divsteps on the matrix cores
    (jump = 1): random units, 1, x, 0 (not a unit), the extreme elements."""
    _, q, _ = wl.PQW[p]
    a = wl.random_rq(p, 5, tag=5)
    a[3] = 0
    a[3, 0] = 1          # 1
    a[4] = 0
    a[4, 1] = 1          # x
    z = np.zeros((1, p), dtype=np.int16)  # 0 is not a unit
    a = np.concatenate([a, z, wl.extreme_rq(p)])
    base = ctx.get_config(p)
    try:
        ctx.set_config(p, recip_jump=jump)
        out, ok = ctx.recip_rq(p, dev(a))
        out, ok = host(out), host(ok)
    finally:
        ctx.set_config(p, **base)
    for i in range(len(a)):
        ref = oracle.inv_mod(a[i], p, q)
        assert ok[i] == (ref is not None), (p, i)
        if ref is not None:
            assert np.array_equal(out[i], centered(ref, q)), (p, i)


def _f3_factor(p, d):
    import ringmath as rm
    fac = rm.gf_factor_of_degree(p, d)
    a = np.zeros(p, dtype=np.int8)
    a[: len(fac)] = centered(fac, 3)
    return a


@pytest.mark.parametrize("p", P_ALL)
@pytest.mark.parametrize("lpk", [1, 2, 4, 8, 16, 32, 64])
def test_recip_r3_matches_oracle(ctx, p, lpk):
    ctx.set_config(p, lanes_per_key=lpk)
    try:
        n = 70  # more than one wave of keys, ragged
        a = wl.random_small(p, n, tag=6)
        a[0] = 0                       # not a unit
        a[1] = 0
        a[1, 0] = 1                    # 1
        a[2] = -a[2]
        small_factor = {653: 3, 761: 19, 857: 25, 1277: 3}[p]
        a[3] = _f3_factor(p, small_factor)   # a factor of x^p - x - 1: not a unit
        out, ok = ctx.recip_r3(p, dev(a))
        out, ok = host(out), host(ok)
        for i in range(n):
            ref = oracle.inv_mod(a[i], p, 3)
            assert ok[i] == (ref is not None), (p, lpk, i)
            if ref is not None:
                assert np.array_equal(out[i], centered(ref, 3)), (p, lpk, i)
    finally:
        ctx.set_config(p, lanes_per_key=2)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("p,G,n", [(761, 1, 3), (761, 5, 23), (761, 32, 70), (653, 7, 15),
                                   (857, 4, 9), (1277, 3, 7)])
def test_batch_inverse_matches_oracle(ctx, p, G, n, engine):
    """Montgomery's trick (Section 2.2) over groups of G: every output is the
    unique inverse, whatever the grouping and the ragged last group."""
    _, q, _ = wl.PQW[p]
    a = wl.random_rq(p, n, tag=7 + G)
    _with_engine(ctx, p, engine)
    try:
        out = host(ctx.batch_inv_rq(p, dev(a), G))
    finally:
        _with_engine(ctx, p, DEFAULT_ENGINE)
    assert ctx.status() == 0
    for i in range(n):
        assert np.array_equal(out[i], centered(oracle.inv_mod(a[i], p, q), q)), (p, G, i)
