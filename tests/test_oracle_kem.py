"""Pins of the oracle's encapsulation / decapsulation core (the KEM of
Section 1; Streamlined NTRU Prime's published encryption, restated in
oracle/ntrup_oracle.c) against what the mathematics fixes:

* Round is its definition: every output is the multiple of 3 nearest the
  input, checked over every residue mod q for the four parameter sets;
* encrypt is Round of the ring product, the product computed independently
  (numpy convolution and the x^p = x + 1 fold);
* decryption inverts encryption for key pairs and every r tried, and the
  reason holds exactly: the centered 3 f c equals g r + 3 f (c - h r) over Z,
  with every coefficient below q / 2;
* the weight check and the re-encryption check catch what they must: c = 0
  gives the fixed element, a ciphertext changed by 3 decrypts to the same r
  but fails the re-encryption check.
"""
import numpy as np
import pytest

import oracle
import ringmath as rm

SEED = bytes(range(32))
SEED_E = bytes(range(100, 132))


def centered(v, m):
    v = np.asarray(v, dtype=np.int64) % m
    return np.where(v > (m - 1) // 2, v - m, v)


@pytest.mark.parametrize("p", sorted(oracle.PARAMS))
def test_round_is_nearest_multiple_of_three(p):
    """encrypt(h, 1) = Round(h): over every centered residue of q."""
    _, q, _ = oracle.PARAMS[p]
    one = np.zeros(p, dtype=np.int8)
    one[0] = 1
    vals = np.arange(-(q - 1) // 2, (q - 1) // 2 + 1, dtype=np.int64)
    for s in range(0, vals.size, p):
        h = np.zeros(p, dtype=np.int16)
        chunk = vals[s:s + p]
        h[:chunk.size] = chunk
        c = oracle.encrypt(h, one, p).astype(np.int64)
        x = h.astype(np.int64)
        assert (c % 3 == 0).all()
        assert (np.abs(c - x) <= 1).all()
        assert (np.abs(c) <= (q - 1) // 2).all()


@pytest.mark.parametrize("p", [653, 761])
def test_encrypt_is_round_of_product(p):
    _, q, w = oracle.PARAMS[p]
    rng = np.random.default_rng(p)
    for k in range(3):
        h = centered(rng.integers(0, q, size=p), q).astype(np.int16)
        r = oracle.sample_short(SEED_E, k, p, w, oracle.ENCAP_STREAM)
        c = oracle.encrypt(h, r, p).astype(np.int64)
        hr = centered(rm.mul_mod(h, r, p, q).astype(np.int64), q)
        assert (c % 3 == 0).all() and (np.abs(c - hr) <= 1).all()


@pytest.mark.parametrize("p", sorted(oracle.PARAMS))
def test_decrypt_inverts_encrypt(p):
    """For oracle key pairs and encapsulations: decap(encap) recovers r, and
    the centered 3 f c is exactly g r + 3 f e over Z (e = c - h r, entries
    in {-1, 0, 1}) with every coefficient below q / 2 -- the reason reducing
    mod 3 and multiplying by 1/g gives r back."""
    _, q, w = oracle.PARAMS[p]
    assert q > 16 * w + 1
    for idx in range(2):
        kp = oracle.keygen(SEED, p, idx)
        for j in range(2):
            c, r = oracle.encap(SEED_E, p, 10 * idx + j, kp["h"])
            assert np.count_nonzero(r) == w
            hr = centered(rm.mul_mod(kp["h"], r, p, q).astype(np.int64), q)
            e = c.astype(np.int64) - hr
            assert set(np.unique(e)) <= {-1, 0, 1}
            lhs = centered(rm.mul_mod(3 * kp["f"].astype(np.int64), c, p, q).astype(np.int64), q)
            rhs = rm.mul_z(kp["g"], r, p) + rm.mul_z(3 * kp["f"].astype(np.int64), e, p)
            assert np.array_equal(lhs, rhs)
            assert np.abs(rhs).max() < q / 2
            r2, ok = oracle.decap(c, kp["f"], kp["ginv"], p, kp["h"])
            assert ok and np.array_equal(r2, r)
            r3, wok = oracle.decrypt(c, kp["f"], kp["ginv"], p)
            assert wok and np.array_equal(r3, r)


@pytest.mark.parametrize("p", [653, 1277])
def test_weight_fallback_and_reencryption_check(p):
    _, q, w = oracle.PARAMS[p]
    kp = oracle.keygen(SEED, p, 3)
    default = np.array([1] * w + [0] * (p - w), dtype=np.int8)
    # c = 0: e = 0, r' = 0 of weight 0 -> the fixed element; it does not
    # encrypt to 0
    zero = np.zeros(p, dtype=np.int16)
    r, wok = oracle.decrypt(zero, kp["f"], kp["ginv"], p)
    assert not wok and np.array_equal(r, default)
    r, ok = oracle.decap(zero, kp["f"], kp["ginv"], p, kp["h"])
    assert not ok and np.array_equal(r, default)
    r, ok = oracle.decap(zero, kp["f"], kp["ginv"], p)
    assert not ok
    # c + 3 x^k: 3 f c changes by 9 f x^k, nothing mod 3 (no coefficient
    # crosses q / 2), so r' = r, but encrypt(r') = c != c + 3 x^k
    c, r0 = oracle.encap(SEED_E, p, 5, kp["h"])
    for k in (0, 1, p // 2, p - 1):
        ct = c.copy()
        ct[k] = ct[k] + 3 if ct[k] + 3 <= (q - 1) // 2 else ct[k] - 3
        r, ok = oracle.decap(ct, kp["f"], kp["ginv"], p, kp["h"])
        assert not ok and np.array_equal(r, r0)
        r, wok = oracle.decap(ct, kp["f"], kp["ginv"], p)
        assert wok and np.array_equal(r, r0)


def test_encap_stream_is_a_short_sample():
    """r comes from the Short sampler on its own stream: weight w, values in
    {-1, 0, 1}, and different from the KeyGen f of the same index."""
    for p, (_, q, w) in oracle.PARAMS.items():
        for idx in range(3):
            c, r = oracle.encap(SEED, p, idx, np.zeros(p, dtype=np.int16))
            assert np.count_nonzero(r) == w and set(np.unique(r)) <= {-1, 0, 1}
            assert np.array_equal(r, oracle.sample_short(SEED, idx, p, w, oracle.ENCAP_STREAM))
            assert not np.array_equal(r, oracle.sample_short(SEED, idx, p, w))
            assert not c.any()
