// Seed expansion: ChaCha20 block function (20 rounds, 32-bit block counter,
// 96-bit nonce, as published in RFC 8439), one block per call, in registers.
//
// The paper asks only for uniform random small g and f in Short (Section 3.1,
// Algorithm 1).  This library fixes the randomness so that every key is a
// pure function of (master seed, p, key index):
//   key   = 32-byte master seed (eight little-endian words, passed by value)
//   nonce = key index (u64 LE) || p (u16 LE) || stream id (u16 LE)
//   stream 0 feeds f; stream 1+k feeds the k-th attempt at g;
//   word i of a stream is the little-endian u32 at keystream offset 4i.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntrup {

struct Seed {
    uint32_t k[8];
};

__device__ __forceinline__ uint32_t rotl(uint32_t x, int n) {
    return __builtin_amdgcn_alignbit(x, x, 32 - n);
}

#define NTRUP_QR(a, b, c, d)                 \
    a += b; d ^= a; d = rotl(d, 16);         \
    c += d; b ^= c; b = rotl(b, 12);         \
    a += b; d ^= a; d = rotl(d, 8);          \
    c += d; b ^= c; b = rotl(b, 7);

// Sixteen keystream words of block `counter` for stream `stream` of key
// `index` under ring degree p.
__device__ __forceinline__ void chacha_block(const Seed& seed, uint64_t index, int p,
                                             int stream, uint32_t counter, uint32_t out[16]) {
    const uint32_t n0 = (uint32_t)index, n1 = (uint32_t)(index >> 32);
    const uint32_t n2 = (uint32_t)p | ((uint32_t)stream << 16);
    uint32_t x0 = 0x61707865u, x1 = 0x3320646eu, x2 = 0x79622d32u, x3 = 0x6b206574u;
    uint32_t x4 = seed.k[0], x5 = seed.k[1], x6 = seed.k[2], x7 = seed.k[3];
    uint32_t x8 = seed.k[4], x9 = seed.k[5], x10 = seed.k[6], x11 = seed.k[7];
    uint32_t x12 = counter, x13 = n0, x14 = n1, x15 = n2;
#pragma unroll 1
    for (int i = 0; i < 10; i++) {
        NTRUP_QR(x0, x4, x8, x12)
        NTRUP_QR(x1, x5, x9, x13)
        NTRUP_QR(x2, x6, x10, x14)
        NTRUP_QR(x3, x7, x11, x15)
        NTRUP_QR(x0, x5, x10, x15)
        NTRUP_QR(x1, x6, x11, x12)
        NTRUP_QR(x2, x7, x8, x13)
        NTRUP_QR(x3, x4, x9, x14)
    }
    out[0] = x0 + 0x61707865u;  out[1] = x1 + 0x3320646eu;
    out[2] = x2 + 0x79622d32u;  out[3] = x3 + 0x6b206574u;
    out[4] = x4 + seed.k[0];    out[5] = x5 + seed.k[1];
    out[6] = x6 + seed.k[2];    out[7] = x7 + seed.k[3];
    out[8] = x8 + seed.k[4];    out[9] = x9 + seed.k[5];
    out[10] = x10 + seed.k[6];  out[11] = x11 + seed.k[7];
    out[12] = x12 + counter;    out[13] = x13 + n0;
    out[14] = x14 + n1;         out[15] = x15 + n2;
}

#undef NTRUP_QR

}  // namespace ntrup
