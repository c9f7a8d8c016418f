"""The factor table of the batched R/3 invertibility screen
(csrc/ntrup_r3_factors.h): every stored factor divides x^p - x - 1 over F_3
and is irreducible, and together the screened factors account for the g
rejection rate of each parameter set."""
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2106_08759_amd", "csrc", "ntrup_r3_factors.h")


def table():
    txt = open(HDR).read()
    out = {}
    for p, body in re.findall(r"struct R3Factors<(\d+)> \{(.*?)\};", txt, re.S):
        ents = re.findall(r"\{(\d+), 0x([0-9A-F]+)u, 0x([0-9A-F]+)u\}", body)
        degs = re.search(r"factor degrees ([0-9, ]+)", txt[:txt.index("struct R3Factors<%s>" % p)].split("// p =")[-1])
        out[int(p)] = ([(int(d), int(m, 16), int(s, 16)) for d, m, s in ents],
                       [int(x) for x in degs.group(1).split(",")])
    return out


def poly_of(d, m, s):
    """Coefficients (low first) of x^d + sum c_j x^j, mod 3 in {0, 1, 2}."""
    c = np.zeros(d + 1, dtype=np.int64)
    for j in range(d):
        if (m >> j) & 1:
            c[j] = 2 if (s >> j) & 1 else 1
    c[d] = 1
    return c


def polymod(a, f):
    """a mod f over F_3 (f monic), coefficient arrays low first."""
    a = a.copy() % 3
    d = len(f) - 1
    for k in range(len(a) - 1, d - 1, -1):
        c = a[k] % 3
        if c:
            a[k - d:k + 1] = (a[k - d:k + 1] - c * f) % 3
    return a[:d] % 3


def polymulmod(a, b, f):
    return polymod(np.convolve(a, b) % 3, f)


def frob(a, f):
    """a^3 mod f over F_3: the Frobenius x^j -> x^(3j)."""
    out = np.zeros(3 * (len(a) - 1) + 1, dtype=np.int64)
    out[::3] = a
    return polymod(out, f)


def polygcd(a, b):
    a, b = np.trim_zeros(a % 3, "b"), np.trim_zeros(b % 3, "b")
    while len(b):
        inv = 1 if b[-1] == 1 else 2
        bm = (b * inv) % 3
        a = np.trim_zeros(polymod(a, bm) if len(a) >= len(bm) else a, "b")
        a, b = b, a
    return a


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_factors_divide_and_are_irreducible(p):
    small, degrees = table()[p]
    assert sorted(degrees) == degrees and sum(degrees) == p
    assert [d for d, _, _ in small] == [d for d in degrees if d <= 32]
    mod = np.zeros(p + 1, dtype=np.int64)
    mod[p], mod[1], mod[0] = 1, 2, 2          # x^p - x - 1
    for d, m, s in small:
        f = poly_of(d, m, s)
        assert not polymod(mod, f).any(), (p, d)
        # Rabin: x^(3^d) = x mod f, and gcd(x^(3^(d/r)) - x, f) = 1 for primes r | d
        x = np.zeros(2, dtype=np.int64)
        x[1] = 1
        powers = [polymod(x, f)]
        for _ in range(d):
            powers.append(frob(powers[-1], f))
        xd = powers[d]
        assert np.array_equal(np.trim_zeros(xd, "b"), np.trim_zeros(polymod(x, f), "b")), (p, d)
        for r in [r for r in range(2, d + 1) if d % r == 0 and all(r % q for q in range(2, r))]:
            t = powers[d // r].copy()
            t = np.pad(t, (0, max(0, 2 - len(t))))
            t[1] = (t[1] - 1) % 3
            g = polygcd(f, t)
            assert len(g) == 1, (p, d, r)


def test_rejection_rates_match_factor_degrees():
    """P(g not a unit) = 1 - prod(1 - 3^-d) over all factors; the survey of
    the paper's parameter sets quotes 3.704% (653) and 4.951% (1277)."""
    t = table()
    rate = {p: 1 - np.prod([1 - 3.0 ** -d for d in degs]) for p, (_, degs) in t.items()}
    assert abs(rate[653] - 0.03704) < 1e-4
    assert abs(rate[1277] - 0.04951) < 1e-4
    assert rate[761] < 1e-9 and rate[857] < 1e-11


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_screen_groups_are_products_of_members(p):
    """Each Horner pass of the screen reduces by a product of small factors
    (degree <= 32); every small factor is a member of exactly one product."""
    txt = open(HDR).read()
    body = re.search(r"struct R3Factors<%d> \{(.*?)\n\};" % p, txt, re.S).group(1)
    small, _ = table()[p]
    groups = re.findall(r"\{(\d+), 0x([0-9A-F]+)u, 0x([0-9A-F]+)u, (\d+), \{([0-9, ]+)\}\}", body)
    assert groups
    seen = []
    for d, m, s, nmem, mem in groups:
        d, nmem = int(d), int(nmem)
        mem = [int(x) for x in mem.split(",")][:nmem]
        assert d <= 32
        prod = np.array([1], dtype=np.int64)
        for i in mem:
            prod = np.convolve(prod, poly_of(*small[i])) % 3
        assert np.array_equal(prod, poly_of(d, int(m, 16), int(s, 16)) % 3), (p, d, mem)
        seen += mem
    assert sorted(seen) == list(range(len(small)))
