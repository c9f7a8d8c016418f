// Encapsulation and decapsulation core on the batch keys.
//
// The paper uses sntrup as a key-encapsulation mechanism (Section 1: key
// generation; encapsulation with a public key, giving a ciphertext and a
// session key; decapsulation with the secret key) and prints only the KeyGen
// steps.  The arithmetic here is Streamlined NTRU Prime's published
// encryption core:
//   encapsulation: r in Short (the Short sampler on stream kEncapStream of
//     the key's index), c = Round(h r) in R/q, where Round replaces each
//     centered coefficient by the nearest multiple of 3;
//   decapsulation: e = 3 f c in R/q (centered), e mod 3, r' = e (1/g) in
//     R/3 (centered); r' is replaced by the fixed weight-w element
//     (1, ..., 1, 0, ..., 0) unless it has weight w; with the public key the
//     kernel also computes Round(h r') and reports whether it equals c.
// The hashes that turn r and c into a session key, and a byte format for c,
// are not defined in the paper and are left to the caller.
//
// One wave per key, every product on the matrix cores (mfma_mul): h r and
// 3 f c are small x big products in R/q (two limb pairs), e (1/g) a one-limb
// product in R/3.  The weight check and the choice of the fallback element
// are selects, not branches, and the re-encryption comparison is one ballot
// per 64 coefficients: the instruction stream does not depend on the secret.
// Workgroups are dealt to the eight XCDs in turn: block b takes key
// (b mod 8) per + b / 8, so each XCD reads a contiguous range of rows.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_keygen.h"
#include "ntrup_mfma.h"
#include "ntrup_params.h"

namespace ntrup {

constexpr int kEncapStream = 0x8000;   // KeyGen uses streams 0 .. 64

struct KemArgs {
    int n;
    int per;               // keys per XCD slice; grid = 8 per
    const int16_t* h;      // [n][p] public keys, centered (decap: nullptr = no re-encryption)
    const int8_t* f;       // [n][p] decap: f
    const int8_t* ginv;    // [n][p] decap: 1/g in R/3
    const int16_t* c_in;   // [n][p] decap: ciphertexts
    int16_t* c_out;        // [n][p] encap: ciphertexts
    int8_t* r;             // [n][p] encap: r (sampled before); decap: r'
    uint8_t* ok;           // [n] decap: 1 = accepted (nullptr = not written)
};

template <int P>
struct KemWave {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];   // Toeplitz limbs: h, c, or e mod 3
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HS[S::HLEN];   // folded small operand: r, 3f, 1/g, r'
    __attribute__((aligned(16))) int16_t Cb[RqShape<P>::JP];
};

// Nearest multiple of 3 to a centered x (|x| < 4096): 3 floor((x + 1) / 3),
// the floor taken on x + 1 + 12288 >= 0.
__device__ __forceinline__ int32_t kem_round3(int32_t x) {
    return 3 * (int32_t)((uint32_t)(x + 12289) / 3u) - 12288;
}

// Round(h r) for key `key`: h as the Toeplitz operand, r folded; c to the
// key's row.
template <int P>
__device__ __forceinline__ void kem_encrypt_row(const int16_t* h, const uint32_t (&rw)[KgShape<P>::NU], int key,
                                                KemWave<P>& L, int16_t* out_row, const int16_t* cmp_row,
                                                bool& same) {
    using S = MfShape<P>;
    KgRegs<P> rg;
    kg_load_b<P>(h, key, rg);
    kg_put_toeplitz16<P>(rg.b, L.TL, L.TH);
    put_folded8<P>(rw, L.HS);
    wave_sync();
    mfma_mul<P, false>(L.TL, L.TH, L.HS, nullptr, L.Cb, nullptr, nullptr, nullptr);
    wave_sync();
    bool diff = false;
    for (int i = lane_id(); i < P; i += 64) {
        const int16_t v = (int16_t)kem_round3(L.Cb[i]);
        if (out_row) out_row[i] = v;
        if (cmp_row) diff |= v != cmp_row[i];
    }
    same = __ballot(diff) == 0;
}

template <int P>
__global__ __launch_bounds__(64) void kem_encap_kernel(KemArgs a) {
    using S = MfShape<P>;
    __shared__ KemWave<P> L;
    const int key = (int)(blockIdx.x & 7u) * a.per + (int)(blockIdx.x >> 3);
    if (key >= a.n) return;
    KgRegs<P> rr;
    kg_load_f<P>(a.r, key, rr);
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.TH, S::TLEN);
    kg_zero<P>(L.HS, S::HLEN);
    wave_sync();
    bool same;
    kem_encrypt_row<P>(a.h, rr.f, key, L, a.c_out + (size_t)key * P, nullptr, same);
}

template <int P>
__global__ __launch_bounds__(64) void kem_decap_kernel(KemArgs a) {
    using S = MfShape<P>;
    constexpr int W = Param<P>::w;
    constexpr int NU = KgShape<P>::NU;
    __shared__ KemWave<P> L;
    const int key = (int)(blockIdx.x & 7u) * a.per + (int)(blockIdx.x >> 3);
    if (key >= a.n) return;
    const int lane = lane_id();
    KgRegs<P> rc, rf;
    kg_load_b<P>(a.c_in, key, rc);
    kg_load_f<P>(a.f, key, rc);
    kg_load_f<P>(a.ginv, key, rf);
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.TH, S::TLEN);
    kg_zero<P>(L.HS, S::HLEN);
    wave_sync();
    // e = 3 f c in R/q
    kg_put_toeplitz16<P>(rc.b, L.TL, L.TH);
    kg_put_3f<P>(rc, L.HS);
    wave_sync();
    mfma_mul<P, false>(L.TL, L.TH, L.HS, nullptr, L.Cb, nullptr, nullptr, nullptr);
    wave_sync();
    // e mod 3 (centered: x - Round(x)) as the one-limb Toeplitz operand,
    // 1/g folded
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        if (m0 >= P) continue;
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int32_t x = (m0 + t < P) ? (int32_t)L.Cb[m0 + t] : 0;
            w |= ((uint32_t)(x - kem_round3(x)) & 0xFFu) << (8 * (3 - t));
        }
        *(uint32_t*)(L.TL + S::Z0 - m0 - 3) = w;
    }
    put_folded8<P>(rf.f, L.HS);
    wave_sync();
    // r' = e (1/g) in R/3
    mfma_mul<P, false, false, 3>(L.TL, nullptr, L.HS, nullptr, L.Cb, nullptr, nullptr, nullptr);
    wave_sync();
    // weight check: one ballot per 64 coefficients
    int weight = 0;
    for (int i0 = 0; i0 < P; i0 += 64) {
        const int i = i0 + lane;
        weight += __popcll(__ballot(i < P && L.Cb[i] != 0));
    }
    const bool wok = weight == W;
    // r' or the fixed element (a mask select), as four bytes per lane word
    // (the layout of the folded operand)
    const uint32_t keep = 0u - (uint32_t)wok;
    uint32_t rw[NU];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int m = m0 + t;
            const uint32_t got = (m < P) ? (uint32_t)(int32_t)L.Cb[m] : 0u;
            const uint32_t fixed = (m < W) ? 1u : 0u;
            w |= (((got & keep) | (fixed & ~keep)) & 0xFFu) << (8 * t);
        }
        rw[u] = w;
    }
    int8_t* rrow = a.r + (size_t)key * P;
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (m0 + t < P) rrow[m0 + t] = (int8_t)(rw[u] >> (8 * t));
    }
    bool ok = wok;
    if (a.h) {
        // re-encryption: Round(h r') against c (TH still holds the high
        // limbs of c; kem_encrypt_row rewrites every entry of TL and TH in
        // [0, p), and the entries outside stay zero)
        wave_sync();
        kem_encrypt_row<P>(a.h, rw, key, L, nullptr, a.c_in + (size_t)key * P, ok);
    }
    if (a.ok && lane == 0) a.ok[key] = ok ? 1 : 0;
}

}  // namespace ntrup
