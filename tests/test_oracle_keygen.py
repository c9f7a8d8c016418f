"""Pin the oracle's KeyGen, samplers and encodings.

KeyGen (OpenSSLNTRU paper, Section 3.1): g small and invertible in R/3,
ginv = 1/g in R/3, f in Short, h = g/(3f) in R/q.  Pins:
  * the defining identities g * ginv = 1 (R/3) and h * 3f = g (R/q), with the
    sympy-pinned numpy product of ringmath, on every parameter set;
  * Short has exactly w nonzeros in {-1, 1} (Section 2.1); small is in {-1,0,1};
  * sampling statistics (positions, signs and g values uniform: chi-square);
  * rejected g attempts are really non-units (gcd with x^p - x - 1 over F_3);
  * the non-unit rate for p=653 equals 1 - prod(1 - 3^-d) over the F_3 factor
    degrees d of x^653 - x - 1, found by distinct-degree factorization;
  * the byte encodings decode (independent numpy bit unpacking) to the arrays.
"""
import json
import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle
import ringmath as rm

SEED = bytes(range(32))
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_param_table_matches_paper():
    for k, v in GOLDEN["params"].items():
        if k.startswith("_"):
            continue
        assert oracle.PARAMS[int(k)] == tuple(v)


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_keygen_identities(p):
    _, q, w = oracle.PARAMS[p]
    for index in (0, 1, 977):
        k = oracle.keygen(SEED, p, index)
        f, g, gi, h = (k[n].astype(np.int64) for n in ("f", "g", "ginv", "h"))
        assert set(np.unique(f)) <= {-1, 0, 1} and np.count_nonzero(f) == w
        assert set(np.unique(g)) <= {-1, 0, 1}
        assert set(np.unique(gi)) <= {-1, 0, 1}
        assert np.abs(h).max() <= (q - 1) // 2
        assert np.array_equal(rm.mul_mod(g, gi, p, 3), rm.one(p))
        assert np.array_equal(rm.mul_mod(h, 3 * f, p, q), g % q)
        # the outputs are the ones the samplers give for the accepted attempt
        assert np.array_equal(k["f"], oracle.sample_short(SEED, index, p, w))
        assert np.array_equal(k["g"], oracle.sample_small(SEED, index, p, k["attempts"] - 1))


def test_keygen_deterministic_and_index_dependent():
    a = oracle.keygen(SEED, 761, 5)
    b = oracle.keygen(SEED, 761, 5)
    c = oracle.keygen(SEED, 761, 6)
    d = oracle.keygen(bytes(32), 761, 5)
    assert all(np.array_equal(a[n], b[n]) for n in ("f", "g", "ginv", "h"))
    assert not np.array_equal(a["h"], c["h"]) and not np.array_equal(a["h"], d["h"])


def _rejected_attempts(args):
    p, lo, hi = args
    _, q, w = oracle.PARAMS[p]
    out = []
    for i in range(lo, hi):
        k = oracle.keygen(SEED, p, i)
        out.append((i, k["attempts"]))
    return out


@pytest.mark.slow
def test_rejection_rate_653_matches_factor_degrees():
    """Fraction of small g that are not units in R/3 for p=653."""
    p = 653
    # distinct-degree factorization of x^653 - x - 1 over F_3 up to degree 30;
    # factors of larger degree change the rate by less than p * 3^-31 < 1e-12
    degs, d = [], 1
    for d in range(1, 31):
        deg = len(rm.gf_factor_of_degree(p, d)) - 1
        new = deg - sum(x for x in degs if d % x == 0)
        assert new >= 0 and new % d == 0
        degs += [d] * (new // d)
    rate = 1.0 - np.prod([1.0 - 3.0 ** (-x) for x in degs])
    n = 2400
    with mp.get_context("fork").Pool(8) as pool:
        res = sum(pool.map(_rejected_attempts, [(p, i, i + n // 8) for i in range(0, n, n // 8)]), [])
    draws = sum(a for _, a in res)
    rejects = draws - n
    # rejects among `draws` Bernoulli(rate) samples; 5 sigma binomial band
    mean = draws * rate
    sd = np.sqrt(draws * rate * (1 - rate))
    assert abs(rejects - mean) < 5 * sd + 1, (rejects, mean, sd, degs)
    assert degs == [3, 16, 23] and 0.037 < rate < 0.03705


def test_rejected_attempts_are_non_units():
    """For keys that needed more than one g, each rejected g shares a factor
    with x^p - x - 1 over F_3 (sympy gcd), and the accepted one does not."""
    p = 653
    found = 0
    for index in range(200):
        k = oracle.keygen(SEED, p, index)
        for att in range(k["attempts"] - 1):
            g = oracle.sample_small(SEED, index, p, att)
            assert rm.gf3_gcd_degree(g) > 0
            found += 1
        if k["attempts"] > 1:
            assert rm.gf3_gcd_degree(k["g"]) == 0
        if found >= 3:
            break
    assert found >= 1


def test_sampler_statistics():
    """Positions of nonzeros of f uniform over [0,p), signs balanced, g values
    uniform on {-1,0,1}: chi-square tests at a loose threshold."""
    from scipy import stats
    p, q, w = oracle.PARAMS[761]
    nkeys = 400
    pos = np.zeros(p)
    signs = np.zeros(2)
    gvals = np.zeros(3)
    for i in range(nkeys):
        f = oracle.sample_short(SEED, i, p, w)
        pos += f != 0
        signs += [np.count_nonzero(f == -1), np.count_nonzero(f == 1)]
        g = oracle.sample_small(SEED, i, p, 0)
        gvals += [np.count_nonzero(g == v) for v in (-1, 0, 1)]
    # positions: each key contributes exactly w hits spread over p bins
    chi_pos = ((pos - nkeys * w / p) ** 2 / (nkeys * w / p)).sum()
    assert stats.chi2.sf(chi_pos, p - 1) > 1e-4
    assert stats.chisquare(signs).pvalue > 1e-4
    assert stats.chisquare(gvals).pvalue > 1e-4


def _decode_pk(pk: bytes, p: int, q: int) -> np.ndarray:
    bits = np.unpackbits(np.frombuffer(pk, dtype=np.uint8), bitorder="little")
    vals = bits[: 13 * p].reshape(p, 13) @ (1 << np.arange(13))
    return vals.astype(np.int64) - (q - 1) // 2


def _decode_trits(b: bytes, p: int) -> np.ndarray:
    bits = np.unpackbits(np.frombuffer(b, dtype=np.uint8), bitorder="little")
    vals = bits[: 2 * p].reshape(p, 2) @ np.array([1, 2])
    return vals.astype(np.int64) - 1


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_encodings_roundtrip(p):
    _, q, w = oracle.PARAMS[p]
    k = oracle.keygen(SEED, p, 3)
    pk = oracle.encode_pk(k["h"], p, q)
    sk = oracle.encode_sk(k["f"], k["ginv"], p)
    assert len(pk) == (13 * p + 7) // 8 and len(sk) == 2 * ((p + 3) // 4)
    assert np.array_equal(_decode_pk(pk, p, q), k["h"])
    half = (p + 3) // 4
    assert np.array_equal(_decode_trits(sk[:half], p), k["f"])
    assert np.array_equal(_decode_trits(sk[half:], p), k["ginv"])
    # extremes of h
    h = np.array([-(q - 1) // 2, (q - 1) // 2] * (p // 2) + [0] * (p % 2), dtype=np.int16)
    assert np.array_equal(_decode_pk(oracle.encode_pk(h, p, q), p, q), h)


def test_pk_size_761_matches_storage_order():
    """13-bit packing gives 1237 B for p=761; with the 382-B sk the pair is
    1619 B, below the paper's 2921 B per sntrup761 pair (Appendix D), whose
    byte format the paper does not define."""
    assert oracle.pk_bytes(761) == 1237 and oracle.sk_bytes(761) == 382
