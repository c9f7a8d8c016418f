// Exhaustive host check of the exact int32 reduction helpers of
// paper_2106_08759_amd/csrc/ntrup_params.h (built with g++, which takes the
// header's host path: mul24 emulates the signed 24-bit multiply).
//
// For each modulus q of the four parameter sets (Section 2.1, plus 7879):
//   reduce_rough<q>(x): x - r divisible by q; r in (-q/2, 3q/2) for every
//     |x| < 2^31; r in (-q/16, 17q/16) for |x| < 2^28;
//   freeze<q>(x): x - r divisible by q; r in [-(q-1)/2, (q-1)/2];
//   mul24(a, b) = a * b for every pair of rough residues a, b in
//     (-q/2, 3q/2) (the divstep's row update multiplies such pairs) and for
//     every quotient estimate t of reduce_rough against q (low 32 bits);
//   mac_chunk<q>(): that many products of two centered residues on top of a
//     value below 2q in magnitude stay below 2^31, and one more would not.
// Prints one line per modulus and exits nonzero at the first violation.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../paper_2106_08759_amd/csrc/ntrup_params.h"

using namespace ntrup;

// d divisible by the odd modulus q <=> d * q^-1 (mod 2^64) is a quotient
// that fits in int32 (exact division by multiplication with the inverse).
static uint64_t inv64(uint64_t q) {
    uint64_t v = q;                       // correct to 3 bits for odd q
    for (int i = 0; i < 6; i++) v *= 2 - q * v;
    return v;
}
static bool divisible(int64_t d, uint64_t qinv) {
    const int64_t k = (int64_t)((uint64_t)d * qinv);
    return k > -(1LL << 32) && k < (1LL << 32);
}

template <int Q>
static int check() {
    long bad = 0;
    const uint64_t qi = inv64(Q);
    if ((uint64_t)Q * qi != 1) return 1;
    // every int32 except INT32_MIN (|x| < 2^31)
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (int64_t hi = -32768; hi < 32768; hi++) {
        for (int64_t lo = 0; lo < 65536; lo++) {
            const int64_t x64 = hi * 65536 + lo;
            if (x64 == INT32_MIN) continue;
            const int32_t x = (int32_t)x64;
            const int32_t r = reduce_rough<Q>(x);
            if (!divisible((int64_t)x - r, qi) || 2 * (int64_t)r <= -Q || 2 * (int64_t)r >= 3 * (int64_t)Q) bad++;
            if (x64 > -(1LL << 28) && x64 < (1LL << 28) &&
                (16 * (int64_t)r <= -Q || 16 * (int64_t)r >= 17 * (int64_t)Q))
                bad++;
            const int32_t f = freeze<Q>(x);
            if (!divisible((int64_t)x - f, qi) || f < -(Q - 1) / 2 || f > (Q - 1) / 2) bad++;
        }
    }
    if (bad) {
        printf("q=%d reduce_rough/freeze: %ld violations\n", Q, bad);
        return 1;
    }
    // mul24 on every pair of rough residues
    long bad24 = 0;
    const int lo = -(Q / 2), hi = (3 * Q) / 2;
#pragma omp parallel for reduction(+ : bad24) schedule(static)
    for (int a = lo; a <= hi; a++)
        for (int b = lo; b <= hi; b++)
            if ((int64_t)mul24(a, b) != (int64_t)a * b) bad24++;
    // quotient estimates of reduce_rough: t = floor(x m / 2^32) over |x| < 2^31
    const int64_t m = barrett_m(Q);
    const int64_t tmax = (INT32_MAX * m) >> 32, tmin = (-(int64_t)INT32_MAX * m) >> 32;
    if (tmax >= (1 << 23) || tmin < -(1 << 23)) bad24++;
    // (near x = -2^31, t q drops below -2^31 for q = 4621 and 7879: mul24
    // gives the low 32 bits, and x - t q, which fits, is exact modulo 2^32)
    for (int64_t t = tmin; t <= tmax; t++)
        if (mul24((int32_t)t, Q) != (int32_t)(uint32_t)(uint64_t)(t * Q)) bad24++;
    if (bad24) {
        printf("q=%d mul24: %ld violations\n", Q, bad24);
        return 1;
    }
    // mac_chunk: k products of centered residues on top of |v| < 2q
    const int64_t k = mac_chunk<Q>(), hq = (Q - 1) / 2;
    if (k < 1 || k * hq * hq + 2 * Q > INT32_MAX || (k + 1) * hq * hq + 2 * Q <= INT32_MAX) {
        printf("q=%d mac_chunk=%lld bound violated\n", Q, (long long)k);
        return 1;
    }
    printf("q=%d ok (mac_chunk=%lld, t in [%lld, %lld])\n", Q, (long long)k, (long long)tmin, (long long)tmax);
    return 0;
}

int main() {
    int rc = check<4621>() | check<4591>() | check<5167>() | check<7879>();
    return rc;
}
