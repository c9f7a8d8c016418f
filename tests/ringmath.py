"""Independent ring arithmetic used to pin the oracle and to check invariants.

Nothing here imports the oracle or the GPU library.  The helpers are written
from the definitions of R/m = F_m[x]/(x^p - x - 1) (OpenSSLNTRU paper,
Section 2.1) and are themselves checked against sympy in the tests.
"""
from __future__ import annotations

import numpy as np


def reduce_mod_ring(c, p: int, m: int) -> np.ndarray:
    """Reduce a coefficient list of any length modulo (m, x^p - x - 1).

    Repeatedly replaces the top term c_k x^k (k >= p) by c_k (x^(k-p+1) + x^(k-p)),
    which is x^p = x + 1 applied to the leading power.
    """
    c = [int(v) for v in c]
    for k in range(len(c) - 1, p - 1, -1):
        v = c[k]
        if v:
            c[k - p] += v
            c[k - p + 1] += v
            c[k] = 0
    c = (c + [0] * p)[:p]
    return np.array([v % m for v in c], dtype=np.int64)


def mul_mod(a, b, p: int, m: int) -> np.ndarray:
    """Product in R/m with numpy's integer convolution (object dtype: exact)."""
    full = np.convolve(np.asarray(a, dtype=object) % m, np.asarray(b, dtype=object) % m)
    return reduce_mod_ring(full, p, m)


def mul_z(a, b, p: int) -> np.ndarray:
    """Product in Z[x]/(x^p - x - 1), exact (no coefficient reduction)."""
    full = np.convolve(np.asarray(a, dtype=object), np.asarray(b, dtype=object))
    c = [int(v) for v in full]
    for k in range(len(c) - 1, p - 1, -1):
        v = c[k]
        if v:
            c[k - p] += v
            c[k - p + 1] += v
            c[k] = 0
    return np.array((c + [0] * p)[:p], dtype=np.int64)


def mul_mod_sympy(a, b, p: int, m: int) -> np.ndarray:
    """Product in R/m computed by sympy's polynomial remainder over GF(m)."""
    import sympy as sp

    x = sp.symbols("x")
    A = sp.Poly(list(reversed([int(v) % m for v in a])), x, modulus=m)
    B = sp.Poly(list(reversed([int(v) % m for v in b])), x, modulus=m)
    M = sp.Poly(x**p - x - 1, x, modulus=m)
    R = (A * B).rem(M)
    coeffs = [int(c) % m for c in reversed(R.all_coeffs())]
    coeffs = (coeffs + [0] * p)[:p]
    return np.array(coeffs, dtype=np.int64)


def inv_mod_sympy(a, p: int, m: int):
    """1/a in R/m by sympy's invert over GF(m); None if not a unit."""
    import sympy as sp

    x = sp.symbols("x")
    A = sp.Poly(list(reversed([int(v) % m for v in a])), x, modulus=m)
    M = sp.Poly(x**p - x - 1, x, modulus=m)
    try:
        R = sp.invert(A, M)
    except (sp.polys.polyerrors.NotInvertible, ZeroDivisionError):
        return None
    coeffs = [int(c) % m for c in reversed(sp.Poly(R, x, modulus=m).all_coeffs())]
    coeffs = (coeffs + [0] * p)[:p]
    return np.array(coeffs, dtype=np.int64)


def one(p: int) -> np.ndarray:
    e = np.zeros(p, dtype=np.int64)
    e[0] = 1
    return e


def centered(v, m: int) -> np.ndarray:
    v = np.asarray(v, dtype=np.int64) % m
    return np.where(v > (m - 1) // 2, v - m, v)


# ---- F_3 distinct-degree information about x^p - x - 1 -------------------

def frobenius_f3(p: int, dmax: int):
    """x^(3^d) mod (3, x^p - x - 1) for d = 1..dmax.

    In characteristic 3, (sum a_i x^i)^3 = sum a_i x^(3i) because a^3 = a in
    F_3, so each power is the previous one with exponents tripled, reduced.
    """
    cur = np.zeros(p, dtype=np.int64)
    cur[1] = 1  # x
    out = []
    for _ in range(dmax):
        spread = np.zeros(3 * p, dtype=object)
        spread[0:3 * p:3] = cur
        cur = reduce_mod_ring(spread, p, 3)
        out.append(cur.copy())
    return out


def gf3_gcd_degree(a) -> int:
    """Degree of gcd(a, x^p - x - 1) over F_3 given a (length p list) and p=len(a)."""
    import sympy as sp
    from sympy.polys.domains import ZZ
    from sympy.polys.galoistools import gf_gcd

    p = len(a)
    M = [1] + [0] * (p - 2) + [2, 2]  # x^p - x - 1 = x^p + 2x + 2 over F_3
    A = [int(v) % 3 for v in reversed(list(a))]
    while A and A[0] == 0:
        A.pop(0)
    g = gf_gcd(M, A, 3, ZZ)
    return len(g) - 1


def gf_factor_of_degree(p: int, d: int):
    """The product of the irreducible factors of x^p - x - 1 over F_3 whose
    degree divides d, as a coefficient list (constant term first), from
    gcd(x^(3^d) - x, x^p - x - 1)."""
    from sympy.polys.domains import ZZ
    from sympy.polys.galoistools import gf_gcd, gf_monic

    fr = frobenius_f3(p, d)[-1].copy()
    fr[1] = (fr[1] - 1) % 3
    M = [1] + [0] * (p - 2) + [2, 2]
    A = [int(v) for v in reversed(list(fr))]
    while A and A[0] == 0:
        A.pop(0)
    g = gf_monic(gf_gcd(M, A, 3, ZZ), 3, ZZ)[1]
    return [int(v) for v in reversed(g)]


def is_irreducible_prime_degree(p: int, q: int) -> bool:
    """Rabin's test for x^p - x - 1 over F_q when p is prime: irreducible iff
    x^(q^p) = x mod M and gcd(x^q - x, M) = 1.  Frobenius y -> y^q is F_q-linear
    on F_q[x]/(M), so x^(q^p) is p products with the Frobenius matrix, done in
    float64 (entries < q^2 p < 2^53, exact)."""
    from sympy.polys.domains import ZZ
    from sympy.polys.galoistools import gf_gcd

    for d in range(2, int(p ** 0.5) + 1):
        assert p % d, "p must be prime"

    def mul(a, b):
        return reduce_mod_ring(np.convolve(a.astype(object), b.astype(object)), p, q)

    # x^q mod M by square-and-multiply
    xq = np.zeros(p, dtype=np.int64); xq[0] = 1
    base = np.zeros(p, dtype=np.int64); base[1] = 1
    e = q
    while e:
        if e & 1:
            xq = mul(xq, base)
        base = mul(base, base)
        e >>= 1
    # Frobenius matrix: column j = x^(jq) mod M
    Q = np.zeros((p, p), dtype=np.float64)
    col = np.zeros(p, dtype=np.int64); col[0] = 1
    for j in range(p):
        Q[:, j] = col
        col = mul(col, xq)
    y = np.zeros(p, dtype=np.float64); y[1] = 1
    for _ in range(p):
        y = np.mod(Q @ y, q)
    x_ = np.zeros(p); x_[1] = 1
    if not np.array_equal(y, x_):
        return False
    t = xq.copy(); t[1] = (t[1] - 1) % q
    M = [1] + [0] * (p - 2) + [q - 1, q - 1]
    T = [int(v) for v in reversed(t)]
    while T and T[0] == 0:
        T.pop(0)
    return len(gf_gcd(M, T, q, ZZ)) == 1
