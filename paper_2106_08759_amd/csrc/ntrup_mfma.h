// Exact R/q product on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// The ring is R/q = (Z/q)[x]/(x^p - x - 1) (Section 2.1).  With 16-coefficient
// blocks, the schoolbook convolution conv = a*b (degree <= 2p-2) is one matrix
// product per 16-block w of conv:
//   conv_{16w + r} = sum_d sum_k a_{16d + r - k} * b_{16(w - d) + k},
//                    r, k in [0, 16), coefficients outside [0, p) being 0,
// i.e. R (16 x NW) = T (16 x 16 ND) * H (16 ND x NW) with the block Toeplitz
// T[r][(d,k)] = a_{16d + r - k} and the block Hankel H[(d,k)][w] = b_{16(w-d)+k};
// each pair (a_j, b_m) with j + m = 16w + r appears exactly once.  The
// reduction x^p = x + 1 then gives c_i = conv_i + conv_{i+p} + [i>=1] conv_{i+p-1}.
//
// Exactness.  A centered residue x (|x| <= (q-1)/2 < 4096) is split as
// x = 128 x_h + x_l with x_l in [-64, 64) and |x_h| <= 31; small operands
// (|x| <= 3) are one int8 limb.  Each MFMA accumulates at most 16 ND <= 1296
// products of int8 limbs in int32 (< 2^23 in magnitude), and the limb
// partial sums are reduced mod q before they are combined.
//
// Layouts on one wave (16x16x64 int8: A lane l = row l%16 with K-bytes
// 16(l/16) .. 16(l/16)+15; B lane l = column l%16 with the same K-bytes;
// accumulator v of lane l = row 4(l/16) + v, column l%16):
//   K-step kappa covers the Toeplitz blocks d = 4 kappa + g, g = lane/16;
//   A (Toeplitz): lane (r, g) needs a_{16d + r - e}, e = 0..15: 16 consecutive
//     bytes of the reversed limb array TL[z] = limb(a_{Z0 - z}) starting at
//     Z0 - 16d - r, assembled from 5 aligned dwords with v_alignbyte (the byte
//     offset (Z0 - r) mod 4 is fixed per lane);
//   B (Hankel): lane (c, g) of tile t needs b_{16j + e}, j = 16t + c - 4 kappa - g:
//     one aligned 16-byte read of the zero-padded limb array HL;
//   the accumulator of lane (c, g), tile t, holds conv_{16(16t+c) + 4g + v}.
// Only (tile, K-step) pairs whose blocks overlap the operands are issued;
// the loops are unrolled so that this selection happens at compile time.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_params.h"
#include "ntrup_rq.h"

namespace ntrup {

#ifndef NTRUP_MF_SCHED
#define NTRUP_MF_SCHED 1
#endif

constexpr int round_up(int a, int b) { return ceil_div(a, b) * b; }

template <int P>
struct MfShape {
    static constexpr int Q = Param<P>::q;
    static constexpr int ND = (P + 14) / 16 + 1;        // Toeplitz blocks: 16d - 15 <= p - 1
    static constexpr int NKS = ceil_div(ND, 4);         // K-steps
    static constexpr int NBH = (P - 1) / 16 + 1;        // blocks of the Hankel operand
    static constexpr int NW = ceil_div(2 * P - 1, 16);  // blocks of the convolution
    static constexpr int NT = ceil_div(NW, 16);         // 16-column tiles
    static constexpr int Z0 = 64 * NKS + 15;            // TL[z] = limb(a_{Z0 - z})
    static constexpr int TLEN = round_up(Z0 + 20, 16);
    static constexpr int klo(int t) {
        const int d = 16 * t - NBH + 1;
        return d > 0 ? d / 4 : 0;
    }
    static constexpr int khi(int t) {
        const int d = 16 * t + 15;
        return (d < ND - 1 ? d : ND - 1) / 4;
    }
    static constexpr int jmin() {
        int m = 0;
        for (int t = 0; t < NT; t++) m = (16 * t - 3 - 4 * khi(t) < m) ? 16 * t - 3 - 4 * khi(t) : m;
        return m;
    }
    static constexpr int jmax() {
        int m = 0;
        for (int t = 0; t < NT; t++) m = (16 * t + 15 - 4 * klo(t) > m) ? 16 * t + 15 - 4 * klo(t) : m;
        return m;
    }
    static constexpr int HOFF = -16 * jmin();           // HL[HOFF + m] = limb(b_m)
    static constexpr int HLEN = 16 * (jmax() - jmin() + 1);
    static constexpr int CLEN = 256 * NT;               // conv staging (int16)
    static_assert(256 * NT >= 2 * P, "tiles cover conv and conv_{2p-1} = 0");
    static_assert(HOFF + 16 * NBH <= HLEN, "padding covers the Hankel operand");
    static constexpr int pairs() {
        int s = 0;
        for (int t = 0; t < NT; t++) s += khi(t) - klo(t) + 1;
        return s;
    }
};

typedef int mf_v4i __attribute__((ext_vector_type(4)));

// x = 128 hi + lo, lo in [-64, 64), as two int8 values.
__device__ __forceinline__ void split_limb(int32_t x, uint32_t& lo, uint32_t& hi) {
    const int32_t h = (x + 64) >> 7;
    lo = (uint32_t)(uint8_t)(int8_t)(x - 128 * h);
    hi = (uint32_t)(uint8_t)(int8_t)h;
}

// Reversed Toeplitz limbs of X (int16, p centered entries):
// TL[z] = lo(X[Z0 - z]), TH[z] = hi(X[Z0 - z]), zero outside [0, p).
template <int P>
__device__ __forceinline__ void build_toeplitz(const int16_t* X, uint8_t* TL, uint8_t* TH) {
    using S = MfShape<P>;
    for (int i = lane_id(); i < S::TLEN / 4; i += 64) {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int m = S::Z0 - (4 * i + t);
            const int32_t v = (m >= 0 && m < P) ? (int32_t)X[m] : 0;
            uint32_t l, h;
            split_limb(v, l, h);
            lo |= l << (8 * t);
            hi |= h << (8 * t);
        }
        ((uint32_t*)TL)[i] = lo;
        ((uint32_t*)TH)[i] = hi;
    }
}

// Zero-padded Hankel limbs of X: HL[HOFF + m] = lo(X[m]), HH likewise; a
// small operand (|X_m| <= 3, hi = 0) needs HL only: pass HH = nullptr.
template <int P>
__device__ __forceinline__ void build_hankel(const int16_t* X, uint8_t* HL, uint8_t* HH) {
    using S = MfShape<P>;
    for (int i = lane_id(); i < S::HLEN / 4; i += 64) {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int m = 4 * i + t - S::HOFF;
            const int32_t v = (m >= 0 && m < P) ? (int32_t)X[m] : 0;
            uint32_t l, h;
            split_limb(v, l, h);
            lo |= l << (8 * t);
            hi |= h << (8 * t);
        }
        ((uint32_t*)HL)[i] = lo;
        if (HH) ((uint32_t*)HH)[i] = hi;
    }
}

// conv of T-operand (limbs TL, TH) and H-operand (limbs HL, and HH when
// H_BIG) over the tiles [T0, T1), written to CS as centered int16:
// CS[16w + r] = conv_{16w+r} mod q.  Software-pipelined: the fragments of
// K-step k+1 are read from LDS while the MFMAs of K-step k run.
template <int P, bool H_BIG, int T0, int T1>
__device__ __forceinline__ void mfma_conv(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                          const uint8_t* HH, int16_t* CS) {
    using S = MfShape<P>;
    constexpr int Q = S::Q;
    constexpr int NTC = T1 - T0;
    constexpr int KLO = S::klo(T0), KHI = S::khi(T1 - 1);
    const int lane = lane_id();
    const int rc = lane & 15, g = lane >> 4;
    // Toeplitz read position of K-step 0: bytes from Z0 - 16 g - rc
    const int s0 = S::Z0 - 16 * g - rc;
    const int sh = s0 & 3;
    const uint32_t* tl32 = (const uint32_t*)TL + (s0 >> 2);
    const uint32_t* th32 = (const uint32_t*)TH + (s0 >> 2);
    // Hankel read position of tile 0, K-step 0: block rc - g
    const uint8_t* hl = HL + S::HOFF + 16 * (rc - g);
    const uint8_t* hh = H_BIG ? HH + S::HOFF + 16 * (rc - g) : hl;
    mf_v4i acc0[NTC], acc1[NTC], acc2[NTC];   // (lo, hi) or (ll, mid, hh)
#pragma unroll
    for (int t = 0; t < NTC; t++) {
        acc0[t] = mf_v4i{0, 0, 0, 0};
        acc1[t] = mf_v4i{0, 0, 0, 0};
        acc2[t] = mf_v4i{0, 0, 0, 0};
    }
    // fragments of the next K-step
    uint32_t nDL[5], nDH[5];
    mf_v4i nBL[NTC], nBH[NTC];
    auto load_step = [&](int k) {
#pragma unroll
        for (int j = 0; j < 5; j++) {
            nDL[j] = tl32[j - 16 * k];
            nDH[j] = th32[j - 16 * k];
        }
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            if (k < S::klo(T0 + t) || k > S::khi(T0 + t)) continue;
            const int off = 16 * (16 * (T0 + t) - 4 * k);
            nBL[t] = *(const mf_v4i*)(hl + off);
            if (H_BIG) nBH[t] = *(const mf_v4i*)(hh + off);
        }
    };
    load_step(KLO);
#pragma unroll
    for (int k = KLO; k <= KHI; k++) {
        // one K-step of fragments in flight beyond the current one
        if (NTRUP_MF_SCHED) __builtin_amdgcn_sched_barrier(0);
        uint32_t DL[5], DH[5];
        mf_v4i BL[NTC], BH[NTC];
#pragma unroll
        for (int j = 0; j < 5; j++) {
            DL[j] = nDL[j];
            DH[j] = nDH[j];
        }
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            BL[t] = nBL[t];
            BH[t] = nBH[t];
        }
        if (k < KHI) load_step(k + 1);
        mf_v4i tl, th;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            tl[j] = (int)__builtin_amdgcn_alignbyte(DL[j + 1], DL[j], sh);
            th[j] = (int)__builtin_amdgcn_alignbyte(DH[j + 1], DH[j], sh);
        }
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            if (k < S::klo(T0 + t) || k > S::khi(T0 + t)) continue;
            if (H_BIG) {
                acc0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BL[t], acc0[t], 0, 0, 0);
                acc1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BH[t], acc1[t], 0, 0, 0);
                acc1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BL[t], acc1[t], 0, 0, 0);
                acc2[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BH[t], acc2[t], 0, 0, 0);
            } else {
                acc0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BL[t], acc0[t], 0, 0, 0);
                acc1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BL[t], acc1[t], 0, 0, 0);
            }
        }
    }
    // 2^14 mod q, centered
    constexpr int32_t C14 = ((16384 % Q) > Q / 2) ? (16384 % Q) - Q : (16384 % Q);
#pragma unroll
    for (int t = 0; t < NTC; t++) {
        int32_t v[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (H_BIG)
                v[e] = freeze<Q>(reduce_rough<Q>(acc0[t][e]) + 128 * reduce_rough<Q>(acc1[t][e]) +
                                 C14 * reduce_rough<Q>(acc2[t][e]));
            else
                v[e] = freeze<Q>(acc0[t][e] + 128 * acc1[t][e]);
        }
        const uint32_t w0 = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
        const uint32_t w1 = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
        *(uint2*)(CS + 16 * (16 * (T0 + t) + rc) + 4 * g) = make_uint2(w0, w1);
    }
}

// c = a * b in R/q from the staged convolution:
//   c_i = conv_i + conv_{i+p} + [i >= 1] conv_{i+p-1},
// four consecutive outputs i = 4 lane + 256 u + t per lane.  Any of
//   dst  (LDS int16, c_i at dst[i]),
//   TLo/THo (LDS, the reversed Toeplitz limbs of c for the next product:
//        TLo[Z0 - i] = lo(c_i), THo[Z0 - i] = hi(c_i)),
//   row  (global int16)
// may be nullptr.
template <int P>
__device__ __forceinline__ void mfma_fold(const int16_t* CS, int16_t* dst, uint8_t* TLo, uint8_t* THo,
                                          int16_t* row) {
    using S = MfShape<P>;
    constexpr int Q = S::Q;
    constexpr int NU = ceil_div(P, 256);
    static_assert(S::CLEN >= 2 * P + 4, "the last window read stays in the staging");
    static_assert((S::Z0 - 3) % 4 == 0, "reversed limb words are aligned");
    const int lane = lane_id();
    uint32_t A[NU][2], E[NU][3];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int i = 4 * lane + 256 * u;
        if (i < P) {
            const uint2 a = *(const uint2*)(CS + i);
            const uint32_t* e = (const uint32_t*)(CS + i + P - 1);   // i + p - 1 is even
            A[u][0] = a.x;
            A[u][1] = a.y;
            E[u][0] = e[0];
            E[u][1] = e[1];
            E[u][2] = e[2];
        }
    }
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int i = 4 * lane + 256 * u;
        if (i >= P) continue;
        int32_t c[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int32_t cs = (int16_t)(A[u][t >> 1] >> (16 * (t & 1)));
            const int32_t e0 = (int16_t)(E[u][t >> 1] >> (16 * (t & 1)));               // conv_{i+p-1+t}
            const int32_t e1 = (int16_t)(E[u][(t + 1) >> 1] >> (16 * ((t + 1) & 1)));   // conv_{i+p+t}
            const int32_t v = cs + e1 + ((i + t >= 1) ? e0 : 0);
            c[t] = (i + t < P) ? freeze<Q>(v) : 0;
        }
        if (dst) {
            if (i + 3 < P) {
                *(uint2*)(dst + i) = make_uint2((uint32_t)(uint16_t)c[0] | ((uint32_t)(uint16_t)c[1] << 16),
                                                (uint32_t)(uint16_t)c[2] | ((uint32_t)(uint16_t)c[3] << 16));
            } else {
#pragma unroll
                for (int t = 0; t < 4; t++)
                    if (i + t < P) dst[i + t] = (int16_t)c[t];
            }
        }
        if (TLo) {
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                uint32_t l, h;
                split_limb(c[t], l, h);
                lo |= l << (8 * (3 - t));
                hi |= h << (8 * (3 - t));
            }
            *(uint32_t*)(TLo + S::Z0 - i - 3) = lo;
            *(uint32_t*)(THo + S::Z0 - i - 3) = hi;
        }
        if (row) {
#pragma unroll
            for (int t = 0; t < 4; t++)
                if (i + t < P) row[i + t] = (int16_t)c[t];
        }
    }
}

// Tile chunks of one product: at most MAXC tiles share one pass over the
// K-steps, so that the accumulators (2 or 3 sets of 4 registers per tile)
// stay in registers next to the Toeplitz fragments.
#ifndef NTRUP_MF_MAXC_SMALL
#define NTRUP_MF_MAXC_SMALL 6
#endif
#ifndef NTRUP_MF_MAXC_BIG
#define NTRUP_MF_MAXC_BIG 4
#endif
template <int P, bool H_BIG>
struct MfSplit {
    static constexpr int NT = MfShape<P>::NT;
    static constexpr int MAXC = H_BIG ? NTRUP_MF_MAXC_BIG : NTRUP_MF_MAXC_SMALL;
    static constexpr int NC = ceil_div(NT, MAXC);
    static constexpr int lo(int c) { return c * NT / NC; }
};

template <int P, bool H_BIG, int C>
__device__ __forceinline__ void mfma_conv_chunks(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                                 const uint8_t* HH, int16_t* CS) {
    using SP = MfSplit<P, H_BIG>;
    if constexpr (C < SP::NC) {
        mfma_conv<P, H_BIG, SP::lo(C), SP::lo(C + 1)>(TL, TH, HL, HH, CS);
        mfma_conv_chunks<P, H_BIG, C + 1>(TL, TH, HL, HH, CS);
    }
}

// c = a * b: T-operand limbs (TL, TH) and H-operand limbs (HL, HH) already
// built; CS = conv staging (CLEN int16).  Ends with the result in dst, the
// Toeplitz limbs (TLo, THo; may be TL, TH themselves) and / or row.
// Wave-local: the caller orders the inputs (wave_sync) before the call.
template <int P, bool H_BIG>
__device__ __forceinline__ void mfma_mul(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL, const uint8_t* HH,
                                         int16_t* CS, int16_t* dst, uint8_t* TLo, uint8_t* THo, int16_t* row) {
    mfma_conv_chunks<P, H_BIG, 0>(TL, TH, HL, HH, CS);
    wave_sync();
    mfma_fold<P>(CS, dst, TLo, THo, row);
}

}  // namespace ntrup
