// Parameter sets and exact int32 reduction helpers shared by every kernel.
//
// Rings (OpenSSLNTRU paper, Section 2.1): R/3 = (Z/3)[x]/(x^p - x - 1) and
// R/q = (Z/q)[x]/(x^p - x - 1), with (p, q) chosen so that R/q is a field.
// (p, q, w) = (653, 4621, 288), (761, 4591, 286), (857, 5167, 322) are the
// paper's; sntrup1277 uses the round-3 values (1277, 7879, 492).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define NTRUP_HD __host__ __device__ __forceinline__
#else
#define NTRUP_HD static inline
#endif

namespace ntrup {

constexpr int kMaxAttempts = 64;  // g samples per key before giving up

template <int P> struct Param;
template <> struct Param<653>  { static constexpr int q = 4621, w = 288; };
template <> struct Param<761>  { static constexpr int q = 4591, w = 286; };
template <> struct Param<857>  { static constexpr int q = 5167, w = 322; };
template <> struct Param<1277> { static constexpr int q = 7879, w = 492; };

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }
constexpr int pk_bytes(int p) { return ceil_div(13 * p, 8); }
constexpr int sk_half_bytes(int p) { return ceil_div(p, 4); }
constexpr int sk_bytes(int p) { return 2 * sk_half_bytes(p); }

// Barrett constant floor(2^32 / q).
constexpr int32_t barrett_m(int q) { return (int32_t)(((uint64_t)1 << 32) / (uint64_t)q); }

// Signed 24-bit multiply (the low 24 bits of each operand, sign-extended),
// the semantics of v_mul_i32_i24; exact whenever |a|, |b| < 2^23.
NTRUP_HD int32_t mul24(int32_t a, int32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __mul24(a, b);
#else
    const int32_t a24 = (int32_t)((uint32_t)a << 8) >> 8, b24 = (int32_t)((uint32_t)b << 8) >> 8;
    return (int32_t)((int64_t)a24 * b24);
#endif
}

// x - q * floor(x * m / 2^32) with m = floor(2^32/q).  For |x| < 2^31 the
// result lies in (-q/2, 3q/2); for |x| < 2^28 in (-q/16, 17q/16).  The
// quotient estimate is below 2^23 in magnitude, so q * t is a 24-bit multiply.
// Checked exhaustively over all int32 inputs (and the 24-bit multiply over
// its operand ranges) by tests/reduce_check.cpp, built with g++ on the host.
template <int Q>
NTRUP_HD int32_t reduce_rough(int32_t x) {
    constexpr int32_t m = barrett_m(Q);
    int32_t t = (int32_t)(((int64_t)x * (int64_t)m) >> 32);
    return x - mul24(t, Q);
}

// Centered representative in [-(q-1)/2, (q-1)/2] of any |x| < 2^31.
template <int Q>
NTRUP_HD int32_t freeze(int32_t x) {
    int32_t r = reduce_rough<Q>(x);          // (-q/2, 3q/2)
    r -= (r > (Q - 1) / 2) ? Q : 0;          // (-q/2, q/2]
    return r;
}

// Number of products of two centered residues that an int32 accumulator can
// take on top of a rough-reduced value without overflow.
template <int Q>
constexpr int mac_chunk() {
    return (int)((2147483647LL - 2LL * Q) / ((int64_t)((Q - 1) / 2) * ((Q - 1) / 2)));
}

}  // namespace ntrup
