"""Pin the oracle's ring arithmetic (products and reciprocals in R/3, R/q).

Rings: R/m = F_m[x]/(x^p - x - 1) (OpenSSLNTRU paper, Section 2.1).  Pins:
  * products against sympy's polynomial remainder over GF(m);
  * the reduction x^(p-1) * x = x + 1;
  * reciprocals by brute force over every element of a toy field
    (p=5, m=3: 243 elements), by sympy's invert at full size, and by the
    closed-form unit count of a toy ring that is not a field;
  * non-units built from the F_3 factors of x^761 - x - 1 whose degrees the
    paper prints (Section 3.1.1: 19, 60, 682).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import ringmath as rm

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


@pytest.mark.parametrize("p,m", [(5, 3), (7, 5), (761, 3), (761, 4591), (1277, 7879)])
def test_mul_matches_sympy(p, m):
    rng = np.random.default_rng(p * 7 + m)
    for _ in range(2):
        a = rng.integers(-(m - 1) // 2, (m - 1) // 2 + 1, p)
        b = rng.integers(-(m - 1) // 2, (m - 1) // 2 + 1, p)
        ref = rm.mul_mod_sympy(a, b, p, m)
        assert np.array_equal(oracle.mul_mod(a, b, p, m), ref)
        # the numpy helper used by later invariant checks is pinned here too
        assert np.array_equal(rm.mul_mod(a, b, p, m), ref)


@pytest.mark.parametrize("p,m", [(761, 4591), (653, 3)])
def test_mul_extremes(p, m):
    h = (m - 1) // 2
    for va, vb in [(h, h), (-h, h), (-h, -h)]:
        a = np.full(p, va)
        b = np.full(p, vb)
        assert np.array_equal(oracle.mul_mod(a, b, p, m), rm.mul_mod_sympy(a, b, p, m))


@pytest.mark.parametrize("p", [5, 761])
def test_fold_identity(p):
    """x^(p-1) * x = x^p = x + 1 in R (Section 2.1)."""
    a = np.zeros(p, dtype=np.int64); a[p - 1] = 1
    b = np.zeros(p, dtype=np.int64); b[1] = 1
    want = np.zeros(p, dtype=np.int64); want[0] = 1; want[1] = 1
    assert np.array_equal(oracle.mul_mod(a, b, p, 4591), want)


def _all_elements(p, m):
    return itertools.product(range(m), repeat=p)


def _all_products(p, m):
    """Every product a*b in F_m[x]/(x^p - x - 1) for small p, m, vectorised:
    the convolution by outer products, then x^k = x^(k-p+1) + x^(k-p) for k >= p."""
    E = np.array(list(_all_elements(p, m)), dtype=np.int64)
    outer = E[:, None, :, None] * E[None, :, None, :]          # [a, b, i, j]
    conv = np.zeros(E.shape[:1] * 2 + (2 * p - 1,), dtype=np.int64)
    for i in range(p):
        conv[:, :, i:i + p] += outer[:, :, i, :]
    for k in range(2 * p - 2, p - 1, -1):
        conv[:, :, k - p] += conv[:, :, k]
        conv[:, :, k - p + 1] += conv[:, :, k]
    return E, conv[:, :, :p] % m


def test_inverse_brute_force_toy_field():
    """F_3[x]/(x^5 - x - 1) is a field of 243 elements: every nonzero element
    has exactly one inverse, found by exhaustive search over all products."""
    p, m = 5, 3
    E, prod = _all_products(p, m)
    is_one = (prod == rm.one(p)).all(axis=2)                  # [a, b]
    for ai, a in enumerate(E):
        got = oracle.inv_mod(a, p, m)
        partners = np.nonzero(is_one[ai])[0]
        if not a.any():
            assert got is None and partners.size == 0
            continue
        assert partners.size == 1
        assert np.array_equal(got, E[partners[0]])


@pytest.mark.parametrize("p,m", [(7, 3), (5, 7)])
def test_unit_count_toy_non_field(p, m):
    """x^7 - x - 1 over F_3 and x^5 - x - 1 over F_7 are squarefree but
    reducible (checked by sympy).  For squarefree M = prod f_i the ring
    F_m[x]/(M) has prod (m^deg f_i - 1) units.  The oracle must report exactly
    that many, every reported inverse must be one, and every element sharing a
    factor with M must be refused."""
    import sympy as sp
    x = sp.symbols("x")
    _, facs = sp.factor_list(x**p - x - 1, modulus=m)
    assert len(facs) >= 2 and all(e == 1 for _, e in facs)
    expected = 1
    for f, _ in facs:
        expected *= m ** sp.degree(f, x) - 1
    Mp = sp.Poly(x**p - x - 1, x, modulus=m)
    units = 0
    for e in _all_elements(p, m):
        a = np.array(e, dtype=np.int64)
        inv = oracle.inv_mod(a, p, m)
        if inv is not None:
            units += 1
            assert np.array_equal(rm.mul_mod(a, inv, p, m), rm.one(p))
        elif a.any() and units % 7 == 0:
            A = sp.Poly(list(reversed([int(v) for v in a])), x, modulus=m)
            assert sp.gcd(A, Mp).degree() > 0
    assert units == expected


@pytest.mark.parametrize("p,q", [(4, 5), (5, 5), (5, 11)])
def test_inverse_small_fields(p, q):
    """x^4 - x - 1 over F_5, x^5 - x - 1 over F_5 (Artin-Schreier) and over
    F_11 are irreducible (checked by sympy), so every nonzero element is a
    unit: the oracle's inverse must satisfy a * (1/a) = 1."""
    import sympy as sp
    x = sp.symbols("x")
    assert sp.Poly(x**p - x - 1, x, modulus=q).is_irreducible
    rng = np.random.default_rng(q)
    elems = list(_all_elements(p, q)) if q ** p <= 3200 else [tuple(rng.integers(0, q, p)) for _ in range(600)]
    for e in elems:
        a = np.array(e, dtype=np.int64)
        inv = oracle.inv_mod(a, p, q)
        if not a.any():
            assert inv is None
        else:
            assert np.array_equal(rm.mul_mod(a, inv, p, q), rm.one(p))


@pytest.mark.parametrize("p,m", [(761, 3), (761, 4591), (653, 4621), (857, 3)])
def test_inverse_matches_sympy_full_size(p, m):
    rng = np.random.default_rng(p + m)
    a = rng.integers(0, m, p)
    ref = rm.inv_mod_sympy(a, p, m)
    got = oracle.inv_mod(a, p, m)
    assert ref is not None and got is not None
    assert np.array_equal(got, ref)


def test_paper_factor_degrees_761_and_non_units():
    """Section 3.1.1: x^761 - x - 1 over F_3 factors with degrees 19, 60, 682.
    The degree-19 and degree-60 factors (extracted by gcd with x^(3^d) - x)
    and multiples of them are not units; the oracle must say so."""
    degs = GOLDEN["f3_factor_degrees_761"]["degrees"]
    p = 761
    f19 = rm.gf_factor_of_degree(p, 19)
    f60 = rm.gf_factor_of_degree(p, 60)
    assert len(f19) - 1 == degs[0] and len(f60) - 1 == degs[1]
    assert p - degs[0] - degs[1] == degs[2]
    rng = np.random.default_rng(19)
    for fac in (f19, f60):
        a = np.zeros(p, dtype=np.int64); a[:len(fac)] = fac
        assert oracle.inv_mod(a, p, 3) is None
        r = rng.integers(0, 3, p)
        assert oracle.inv_mod(rm.mul_mod(a, r, p, 3), p, 3) is None
    assert oracle.inv_mod(np.zeros(p, dtype=np.int64), p, 3) is None


def test_inverse_of_units_and_one():
    p, q = 761, 4591
    assert np.array_equal(oracle.inv_mod(rm.one(p), p, q), rm.one(p))
    # x is a unit: x * (x^(p-1) - 1) = x^p - x = 1
    a = np.zeros(p, dtype=np.int64); a[1] = 1
    want = np.zeros(p, dtype=np.int64); want[p - 1] = 1; want[0] = q - 1
    assert np.array_equal(oracle.inv_mod(a, p, q), want)


@pytest.mark.slow
@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_rq_is_a_field(p):
    """Section 2.1: p, q are chosen so that R/q is a field, i.e. x^p - x - 1 is
    irreducible mod q (Rabin's test; for 1277 with the round-3 q = 7879).
    Montgomery's trick relies on it: every nonzero 3f is a unit."""
    _, q, _ = oracle.PARAMS[p]
    assert rm.is_irreducible_prime_degree(p, q)


def test_rabin_helper_detects_reducible():
    assert not rm.is_irreducible_prime_degree(5, 7)
    assert not rm.is_irreducible_prime_degree(7, 3)
    assert rm.is_irreducible_prime_degree(5, 11)
