"""The live-word argument of the one-lane R/3 divsteps, on a bit-level model
(no GPU): at divstep j of 2p-1 only the words of f and g holding the
min(p+1, 2p-1-j) coefficients the remaining steps read are updated, and only
the words of v and r holding degree <= j+1.  The model updates f, g, v, r as
32-coefficient (nonzero, sign) word pairs like the kernel, in segments of a
fixed number of steps with each segment's worst-case live counts; the dead
f, g words are overwritten with junk at every segment start, and the dead v, r
words must stay zero.  The result (1/g and whether g is a unit) must equal the
full-width loop's and the oracle's."""
import numpy as np
import pytest

import oracle

M32 = 0xFFFFFFFF


def cdiv(a, b):
    return -(-a // b)


def divsteps(p, g, seg=None):
    """Bitsliced divsteps on reversed f = x^p - x - 1 and reversed g; seg=None
    updates every word at every step.  Returns (delta, 1/g centered or None)."""
    W = cdiv(p + 1, 32)
    rev = [int(g[p - 1 - i]) if i < p else 0 for i in range(32 * W)]   # reversed g, degree p-1
    gm = [sum(1 << b for b in range(32) if rev[32 * k + b] != 0) for k in range(W)]
    gs = [sum(1 << b for b in range(32) if rev[32 * k + b] == -1) for k in range(W)]
    fm, fs = [0] * W, [0] * W
    fm[0] |= 1
    for e in (p - 1, p):
        fm[e // 32] |= 1 << (e % 32)
        fs[e // 32] |= 1 << (e % 32)
    vm, vs, rm, rs = [0] * W, [0] * W, [0] * W, [0] * W
    rm[0] = 1
    delta = 1
    n = 2 * p - 1
    bounds = [(0, n, W, W)] if seg is None else [
        (a, min(n, a + seg), cdiv(min(p + 1, n - a), 32), min(W, cdiv(min(n, a + seg) + 1, 32)))
        for a in range(0, n, seg)]
    for a, b, nfg, nvr in bounds:
        for k in range(nfg, W):      # stale words: junk that must never reach a read position
            gm[k] ^= 0xA5A5A5A5
            gs[k] ^= 0x5A5A5A5A
            fm[k] ^= 0x3C3C3C3C
            fs[k] ^= 0xC3C3C3C3
        for _ in range(a, b):
            nz = M32 if gm[0] & 1 else 0
            neg = nz & (M32 if ((fs[0] ^ gs[0]) & 1) == 0 else 0)      # s = -g(0)/f(0) = -1
            sw = nz if delta > 0 else 0
            delta = (1 - delta) if sw else (1 + delta)
            for k in range(nfg):
                mbf = fm[k] & nz
                xg, ug = gs[k] ^ neg ^ fs[k], gs[k] ^ neg ^ mbf
                ngm = (gm[k] ^ mbf) | (gm[k] & mbf & ~xg & M32)
                ngs = (ug & gm[k]) | (fs[k] & ~gm[k] & M32)
                fm[k] = (gm[k] & sw) | (fm[k] & ~sw & M32)
                fs[k] = (gs[k] & sw) | (fs[k] & ~sw & M32)
                gm[k], gs[k] = ngm, ngs
            for k in range(nvr):
                mbv = vm[k] & nz
                xr, ur = rs[k] ^ neg ^ vs[k], rs[k] ^ neg ^ mbv
                nrm = (rm[k] ^ mbv) | (rm[k] & mbv & ~xr & M32)
                nrs = (ur & rm[k]) | (vs[k] & ~rm[k] & M32)
                nvm = (rm[k] & sw) | (vm[k] & ~sw & M32)
                nvs = (rs[k] & sw) | (vs[k] & ~sw & M32)
                rm[k], rs[k], vm[k], vs[k] = nrm, nrs, nvm, nvs
            for x in (gm, gs):   # g <- g / x over the live words
                for k in range(nfg - 1):
                    x[k] = ((x[k] >> 1) | (x[k + 1] << 31)) & M32
                x[nfg - 1] >>= 1
            for x in (vm, vs):   # v <- x v over the live words; nothing live drops out
                assert nvr == W or (x[nvr - 1] >> 31) == 0
                for k in range(nvr - 1, 0, -1):
                    x[k] = ((x[k] << 1) | (x[k - 1] >> 31)) & M32
                x[0] = (x[0] << 1) & M32
            for k in range(nvr, W):
                assert vm[k] == vs[k] == rm[k] == rs[k] == 0
    if delta != 0:
        return delta, None
    flip = fs[0] & 1                 # scale v by f(0)^-1 = f(0)
    coef = []
    for i in range(1, p + 1):        # (1/g)_j = f(0)^-1 v[p - j]
        m, s_ = (vm[i // 32] >> (i % 32)) & 1, (vs[i // 32] >> (i % 32)) & 1
        coef.append(0 if not m else (-1 if s_ ^ flip else 1))
    return delta, np.array(coef[::-1], dtype=np.int64)


@pytest.mark.parametrize("p", [653, 761])
def test_live_words_equal_full_width_and_oracle(p):
    seed = bytes(range(32))
    cases = [oracle.sample_small(seed, i, p, 0) for i in range(2)]
    if p == 653:
        z = np.zeros(p, dtype=np.int64)
        z[:4] = [-1, -1, 0, 1]           # x^3 - x - 1, a factor of x^653 - x - 1 over F_3
        cases.append(z)
    for g in cases:
        ref = oracle.inv_mod(g, p, 3)
        full = divsteps(p, g)
        for seg in (96, 33):
            live = divsteps(p, g, seg)
            assert live[0] == full[0]
            assert (live[1] is None) == (full[1] is None) == (ref is None)
            if ref is not None:
                assert np.array_equal(live[1] % 3, full[1] % 3)
                assert np.array_equal(live[1] % 3, np.asarray(ref) % 3)
