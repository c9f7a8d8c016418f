"""CPU model of the jump-divstep R/q reciprocal (the recursive form of the
Bernstein-Yang divsteps that the paper's jump-div-step note refers to, one
level deep), step for step as the GPU kernel schedules it, checked against the
oracle's extended-Euclid reciprocal and against the plain divstep loop.

The divstep on (delta, f, g, v, r), with f0, g0 the constant terms of f, g:
  swap = delta > 0 and g0 != 0;  delta <- (swap ? -delta : delta) + 1
  (f, g) <- (swap ? g : f, (f0 g - g0 f) / x)
  (v, r) <- (x (swap ? r : v), f0 r - g0 v)
i.e. both pairs move by the matrix A = [[1-s, s], [-g0, f0]], the (f, g)
pair then scaled by diag(1, 1/x) and the (v, r) pair by diag(x, 1).  n steps
therefore multiply (v, r) by U = prod diag(x, 1) A_j (polynomial entries of
degree <= n) and (f, g) by U / x^n, and the n steps' controls (swap, f0, g0)
depend only on the low n coefficients of f and g.  The kernel runs n = 48
steps at a time on the low 64 coefficients (one per lane) while building U,
then applies U to the full f, g, v, r with matrix-core products (the last,
shorter jump only to v: the constant term of f comes from the inner steps).

Start (as the plain kernel): f = 1 - x^(p-1) - x^p (x^p - x - 1 reversed),
g = the input reversed as a degree-(p-1) polynomial, v = 0, r = 1, delta = 1;
after 2p - 1 steps the input is a unit iff delta = 0, and its reciprocal has
coefficient i = v_{p-i} / f0.
"""
import numpy as np
import pytest

import oracle

CHUNK = 48    # divsteps per jump (U of degree <= 48: 49 coefficients, four 16-blocks)
LOW = 64      # coefficients of f and g the inner steps run on (one per lane)
PQ = {653: 4621, 761: 4591, 857: 5167, 1277: 7879}


def start_state(a, p, q):
    f = np.zeros(p + 1, dtype=np.int64)
    f[0], f[p - 1], f[p] = 1, q - 1, q - 1
    g = np.zeros(p + 1, dtype=np.int64)
    g[:p] = np.asarray(a, dtype=np.int64)[::-1] % q
    v = np.zeros(p + 1, dtype=np.int64)
    r = np.zeros(p + 1, dtype=np.int64)
    r[0] = 1
    return 1, f, g, v, r


def finish(delta, f, v, p, q):
    if delta != 0:
        return None
    inv0 = pow(int(f[0]) % q, q - 2, q)
    return np.array([inv0 * int(v[p - i]) % q for i in range(p)], dtype=np.int64)


def recip_plain(a, p, q):
    """2p - 1 single divsteps on the full polynomials."""
    delta, f, g, v, r = start_state(a, p, q)
    for _ in range(2 * p - 1):
        f0, g0 = int(f[0]), int(g[0])
        s = delta > 0 and g0 % q != 0
        delta = (-delta if s else delta) + 1
        ng = (f0 * g - g0 * f) % q
        nr = (f0 * r - g0 * v) % q
        f, v = (g, r) if s else (f, v)
        g = np.concatenate([ng[1:], [0]])
        r = nr
        v = np.concatenate([[0], v[:-1]])
    return finish(delta, f, v, p, q)


def inner_steps(delta, f_low, g_low, n, q):
    """n divsteps on the low coefficients; returns delta, U as four
    coefficient arrays of length n + 1 (u00, u01, u10, u11) and the truncated
    f after the steps (its low len - n coefficients are exact)."""
    f, g = f_low.copy(), g_low.copy()
    u = [np.zeros(n + 1, dtype=np.int64) for _ in range(4)]
    u[0][0] = u[3][0] = 1
    for _ in range(n):
        f0, g0 = int(f[0]), int(g[0])
        s = delta > 0 and g0 % q != 0
        delta = (-delta if s else delta) + 1
        ng = (f0 * g - g0 * f) % q
        f = g if s else f
        g = np.concatenate([ng[1:], [0]])           # truncated: the top coefficient becomes 0
        n10 = (f0 * u[2] - g0 * u[0]) % q
        n11 = (f0 * u[3] - g0 * u[1]) % q
        r0 = (u[2], u[3]) if s else (u[0], u[1])
        u = [np.concatenate([[0], r0[0][:-1]]), np.concatenate([[0], r0[1][:-1]]), n10, n11]
    return delta, u, f


def recip_jump(a, p, q, chunk=CHUNK, low=LOW, check=None):
    delta, f, g, v, r = start_state(a, p, q)
    total = 2 * p - 1
    done = 0
    while done < total:
        n = min(chunk, total - done)
        fl = np.zeros(low, dtype=np.int64)
        gl = np.zeros(low, dtype=np.int64)
        fl[:min(low, f.size)] = f[:low]
        gl[:min(low, g.size)] = g[:low]
        delta, u, f_inner = inner_steps(delta, fl, gl, n, q)
        nv = (np.convolve(u[0], v) + np.convolve(u[1], r)) % q
        if done + n == total:
            # the last jump (any n): v' alone, and f's constant term from
            # the inner steps, which hold the low coefficients of f' exactly
            f = f_inner
            v = nv[:p + 1]
            done += n
            break
        nf = (np.convolve(u[0], f) + np.convolve(u[1], g)) % q
        ng = (np.convolve(u[2], f) + np.convolve(u[3], g)) % q
        nr = (np.convolve(u[2], v) + np.convolve(u[3], r)) % q
        if check is not None:
            check(n, nf, ng, nv, nr)
            assert np.array_equal(nf[n:n + low - n], f_inner[:low - n])
        f, g = nf[n:n + p + 1], ng[n:n + p + 1]
        v, r = nv[:p + 1], nr[:p + 1]
        done += n
    return finish(delta, f, v, p, q)


def toy_elements(p, q, count, rng):
    out = [rng.integers(0, q, size=p) for _ in range(count)]
    e = np.zeros(p, dtype=np.int64)
    e[0] = 1
    out.append(e)                                    # 1
    x = np.zeros(p, dtype=np.int64)
    x[1] = 1
    out.append(x)                                    # x
    out.append(np.full(p, q - 1, dtype=np.int64))    # -(1 + x + ... + x^(p-1))
    return out


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_jump_in_r3_equals_oracle(p):
    """The same schedule over F_3 (the batched R/3 stage's group reciprocals):
    random elements of R/3, and for p = 761 the degree-19 factor of
    x^761 - x - 1 mod 3 (Section 3.1.1), a non-unit."""
    rng = np.random.default_rng(3 * p)
    elems = [rng.integers(0, 3, size=p) for _ in range(4)]
    for a in elems:
        want = oracle.inv_mod(a, p, 3)
        got = recip_jump(a, p, 3)
        if want is None:
            assert got is None
        else:
            assert np.array_equal(got, want)
    if p == 761:
        import ringmath as rm
        fac = rm.gf_factor_of_degree(761, 19)
        a = np.zeros(p, dtype=np.int64)
        a[:len(fac)] = np.asarray(fac) % 3
        assert oracle.inv_mod(a, p, 3) is None and recip_jump(a, p, 3) is None


@pytest.mark.parametrize("p", [653, 761, 857, 1277])
def test_jump_equals_oracle_reciprocal(p):
    """The jump schedule's reciprocal equals the oracle's extended-Euclid
    reciprocal, and the low n coefficients of U (f, g) vanish (the division
    by x^n is exact), v and r never exceed degree p."""
    q = PQ[p]
    rng = np.random.default_rng(p)

    def check(n, nf, ng, nv, nr):
        assert not nf[:n].any() and not ng[:n].any()
        assert not nv[p + 1:].any() and not nr[p + 1:].any()

    for a in toy_elements(p, q, 3, rng):
        want = oracle.inv_mod(a, p, q)
        got = recip_jump(a, p, q, check=check)
        assert want is not None and got is not None
        assert np.array_equal(got, want)


# a factor of x^p - x - 1 modulo q for three non-field toy rings (lowest
# coefficient first): x - 11 mod 29, x - 2 mod 5, x^3 - x - 2 mod 7
TOY_FACTORS = {(7, 29): [-11, 1], (11, 5): [-2, 1], (13, 7): [-2, -1, 0, 1]}


def test_jump_equals_plain_divsteps_and_flags_nonunits():
    """On three non-field rings Z_q[x]/(x^p - x - 1): the jump and plain loops
    agree with the oracle element by element, including the verdict for
    non-units (zero, a factor of x^p - x - 1 and its multiples)."""
    rng = np.random.default_rng(7)
    for (p, q), fac in TOY_FACTORS.items():
        fa = np.zeros(p, dtype=np.int64)
        fa[:len(fac)] = np.asarray(fac) % q
        mult = [oracle.mul_mod(fa, rng.integers(0, q, size=p), p, q) for _ in range(4)]
        elems = [rng.integers(0, q, size=p) for _ in range(60)] + [np.zeros(p, dtype=np.int64), fa] + mult
        nonunits = 0
        for a in elems:
            a = np.asarray(a, dtype=np.int64)
            want = oracle.inv_mod(a, p, q)
            plain = recip_plain(a, p, q)
            for chunk in (1, 3, 5, 48, 60):
                got = recip_jump(a, p, q, chunk=chunk, low=max(chunk + 1, 16))
                if want is None:
                    assert got is None and plain is None
                else:
                    assert np.array_equal(got, want) and np.array_equal(plain, want)
            nonunits += want is None
        assert nonunits >= 6


def test_chunk_schedule_covers_2p_minus_1():
    for p in PQ:
        steps = [min(CHUNK, 2 * p - 1 - d) for d in range(0, 2 * p - 1, CHUNK)]
        assert sum(steps) == 2 * p - 1 and all(0 < s <= CHUNK for s in steps)
        assert CHUNK + 1 <= LOW and CHUNK % 12 == 0   # U's 49 coefficients and the truncated f, g fit
        # one wave; whole three-step trips, dword-aligned shifts
