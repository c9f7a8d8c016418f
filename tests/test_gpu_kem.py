"""Encapsulation / decapsulation core on the GPU (ntrup_batch_encap/decap,
the KEM of Section 1) against the oracle, element by element: ciphertexts
and r of encapsulation, r' and the accept flag of decapsulation, with valid,
tampered and zero ciphertexts, with and without the re-encryption check; and
at N = 65536 sntrup761 keys, decap(encap) = r for every key plus the oracle
on sampled keys."""
import numpy as np
import pytest

from paper_2106_08759_amd import workloads as wl
import oracle
import oracle_pool

pytestmark = pytest.mark.gpu

SEED_E = bytes(range(100, 132))


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


def oracle_pairs(p, idx):
    keys = oracle_pool.oracle_keys(wl.SEED, p, idx)
    h = np.stack([keys[i][2] for i in idx]).astype(np.int16)
    f = np.stack([keys[i][3] for i in idx]).astype(np.int8)
    gi = np.stack([keys[i][4] for i in idx]).astype(np.int8)
    return h, f, gi


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_encap_decap_match_oracle(ctx, p):
    """37 keys (not a multiple of the 8 XCD slices): encapsulation of oracle
    key pairs, then decapsulation of valid, tampered (c + 3 x^k), zero and
    random ciphertexts, with and without h."""
    _, q, w = oracle.PARAMS[p]
    n, first = 37, 5
    idx = list(range(n))
    h, f, gi = oracle_pairs(p, idx)
    c_d, r_d = ctx.batch_encap(p, SEED_E, first, dev(h))
    c_g, r_g = host(c_d), host(r_d)
    for j in range(n):
        c_o, r_o = oracle.encap(SEED_E, p, first + j, h[j])
        assert np.array_equal(c_g[j], c_o), ("c", j)
        assert np.array_equal(r_g[j], r_o), ("r", j)
    # ciphertexts: 0..19 valid, 20..27 tampered at one coefficient, 28 zero,
    # 29..36 uniform multiples of 3
    rng = np.random.default_rng(p)
    ct = c_g.copy()
    for j in range(20, 28):
        k = int(rng.integers(0, p))
        ct[j, k] = ct[j, k] + 3 if ct[j, k] + 3 <= (q - 1) // 2 else ct[j, k] - 3
    ct[28] = 0
    ct[29:] = 3 * rng.integers(-((q - 1) // 6), (q - 1) // 6 + 1, size=(8, p))
    for with_h in (True, False):
        r_d, ok_d = ctx.batch_decap(p, dev(ct), dev(f), dev(gi), dev(h) if with_h else None)
        r_g2, ok_g = host(r_d), host(ok_d)
        for j in range(n):
            r_o, ok_o = oracle.decap(ct[j], f[j], gi[j], p, h[j] if with_h else None)
            assert np.array_equal(r_g2[j], r_o), ("r'", j, with_h)
            assert bool(ok_g[j]) == ok_o, ("ok", j, with_h)
        if with_h:
            assert ok_g[:20].all() and not ok_g[20:].any()
            assert np.array_equal(r_g2[:20], r_g[:20])


def test_kem_full_batch_761(ctx):
    """N = 65536 sntrup761 keys from ntrup_batch_keygen's raw outputs:
    decap(encap) gives r back with ok = 1 for every key; 64 spread keys'
    ciphertexts and r equal the oracle's (its own key pairs)."""
    p, n = 761, 65536
    _, q, w = oracle.PARAMS[p]
    _, _, h, f, gi = ctx.batch_keygen(p, wl.SEED, 0, n, raw=True)
    c, r = ctx.batch_encap(p, SEED_E, 0, h)
    r2, ok = ctx.batch_decap(p, c, f, gi, h)
    assert bool((r2 == r).all()) and bool((ok == 1).all())
    rn = host(r)
    assert (np.count_nonzero(rn, axis=1) == w).all()
    idx = sorted(set(np.linspace(0, n - 1, 64).astype(int).tolist()))
    hk, _, _ = oracle_pairs(p, idx)
    cg = host(c)
    for j, i in enumerate(idx):
        c_o, r_o = oracle.encap(SEED_E, p, i, hk[j])
        assert np.array_equal(cg[i], c_o) and np.array_equal(rn[i], r_o), i


def test_kem_sizes_and_errors(ctx):
    import paper_2106_08759_amd as nk
    L = nk.lib()
    assert L.ntrup_batch_encap(ctx._h, 761, SEED_E, 0, 0, None, None, None, None) == 0
    assert L.ntrup_batch_decap(ctx._h, 761, 0, None, None, None, None, None, None, None) == 0
    assert L.ntrup_batch_encap(ctx._h, 760, SEED_E, 0, 1, None, None, None, None) == nk.NTRUP_EINVAL
    assert L.ntrup_batch_encap(ctx._h, 761, SEED_E, 0, 1, None, None, None, None) == nk.NTRUP_EINVAL
    assert L.ntrup_batch_decap(ctx._h, 761, 1 << 24, None, None, None, None, None, None, None) == nk.NTRUP_EINVAL
    # one key, no h and no ok array
    import torch
    h, f, gi = oracle_pairs(857, [3])
    c, r = ctx.batch_encap(857, SEED_E, 3, dev(h))
    fd, gd = dev(f), dev(gi)
    r2 = torch.zeros_like(r)
    torch.cuda.synchronize()
    assert L.ntrup_batch_decap(ctx._h, 857, 1, c.data_ptr(), fd.data_ptr(), gd.data_ptr(), None, r2.data_ptr(),
                               None, torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    assert np.array_equal(host(r2), host(r))
    assert np.array_equal(host(r)[0], oracle.encap(SEED_E, 857, 3, h[0])[1])
