// Exact R/q product on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// The ring is R/q = (Z/q)[x]/(x^p - x - 1) (Section 2.1).  Since x^p = x + 1
// and every product degree k in [p, 2p-2] reduces in one step to
// x^{k-p+1} + x^{k-p}, the product c = a b is
//   c_i = conv_i + conv_{i+p} + [i >= 1] conv_{i+p-1},   conv = a * b,
// which is one Toeplitz-by-vector product with the folded operand
//   E_m = b_m (1 <= m < p),  E_0 = b_0 + b_{p-1},
//   E_m = b_{m+p} + b_{m+p-1} (-(p-1) <= m <= -1),  0 elsewhere:
//   c_i = sum_j a_j E_{i-j} for i >= 1, and for i = 0 the same sum minus
//   conv_{p-1} = c_{p-1} - a_{p-1} b_{p-1} (the one pair (j, m) = (0, 0) whose
//   b_{p-1} term belongs to x^{p-1}, not to x^0 + x^p).
// With 16-coefficient blocks this is one matrix product per 16-block w of c:
//   c_{16w + r} = sum_d sum_k a_{16d + r - k} * E_{16(w - d) + k},
// R (16 x NWO) = T (16 x 16 ND) * H (16 ND x NWO) with the block Toeplitz
// T[r][(d,k)] = a_{16d + r - k} and the block Hankel H[(d,k)][w] = E_{16(w-d)+k}.
// Folding the reduction into H halves the output columns of the schoolbook
// product (p instead of 2p - 1) and leaves no convolution to stage and fold.
//
// Exactness.  A centered residue x (|x| <= (q-1)/2 < 2300) is split as
// x = 128 x_h + x_l with x_l in [-64, 64) and |x_h| <= 18; an entry of E is
// a sum of two residues (|x_h| <= 36 after the split).  Small operands
// (|x| <= 3, |E_m| <= 6) are one int8 limb.  Each output sums at most p
// nonzero products of int8 limbs in int32 (< 2^23 in magnitude), and the
// limb partial sums are reduced mod q before they are combined.
//
// Layouts on one wave (16x16x64 int8: A lane l = row l%16 with K-bytes
// 16(l/16) .. 16(l/16)+15; B lane l = column l%16 with the same K-bytes;
// accumulator v of lane l = row 4(l/16) + v, column l%16):
//   K-step kappa covers the Toeplitz blocks d = 4 kappa + g, g = lane/16;
//   A (Toeplitz): lane (r, g) needs a_{16d + r - e}, e = 0..15: 16 consecutive
//     bytes of the reversed limb array TL[z] = limb(a_{Z0 - z}) starting at
//     Z0 - 16d - r, assembled from 5 aligned dwords with v_alignbyte (the byte
//     offset (Z0 - r) mod 4 is fixed per lane);
//   B (Hankel): lane (c, g) of tile t needs E_{16j + e}, j = 16t + c - 4 kappa - g:
//     one aligned 16-byte read of the zero-padded limb array HL;
//   the accumulator of lane (c, g), tile t, holds c_{256t + 16c + 4g + v}.
// Every (tile, K-step) pair meets nonzero blocks of both operands; the loops
// are unrolled at compile time.
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
    static constexpr int NWO = ceil_div(P, 16);         // 16-blocks of the product
    static constexpr int NT = ceil_div(NWO, 16);        // 16-column tiles
    static constexpr int Z0 = 64 * NKS + 15;            // TL[z] = limb(a_{Z0 - z})
    static constexpr int TLEN = round_up(Z0 + 20, 16);
    static constexpr int HOFF = 64 * NKS - 16;          // HL[HOFF + m] = limb(E_m): lowest block read is -(4 NKS - 1)
    static constexpr int HLEN = HOFF + 256 * NT;        // highest block read is 16 NT - 1
    static constexpr int NEG = HOFF - (P - 1);          // first byte of E_{-(p-1)}
    static_assert(P % 4 == 1, "every parameter set has p = 1 mod 4: the folded words stay dword-aligned");
    static_assert(NEG >= 0 && NEG % 4 == 0, "E_{-(p-1)} starts on a dword inside the array");
    static_assert(HOFF % 16 == 0 && HLEN % 16 == 0, "16-byte Hankel reads are aligned");
    static_assert((Z0 - 3) % 4 == 0, "reversed limb words are aligned");
    static constexpr int pairs() { return NT * NKS; }
    // lane and tile holding c_{p-1} (accumulator element 0)
    static constexpr int TP = (P - 1) / 256;
    static constexpr int LP = ((P - 1) % 256) / 16 + 16 * (((P - 1) % 16) / 4);
    static_assert((P - 1) % 4 == 0, "c_{p-1} is accumulator element 0 of its lane");
};

typedef int mf_v4i __attribute__((ext_vector_type(4)));

// The Toeplitz fragment of a lane is 16 consecutive bytes of the reversed limb
// array at a byte offset fixed per lane (Z0 - 16 g - r, less 64 per K-step):
// five aligned dwords joined by v_alignbyte (four VALU operations per
// fragment).  NTRUP_MF_UNALIGNED = 1 reads it with one ds_read_b128 at the
// unaligned byte address instead (the LDS runs in unaligned mode on gfx950):
// correct, but the unaligned reads stall the LDS, and a batch took 1.90
// instead of 1.37 ms.
#ifndef NTRUP_MF_UNALIGNED
#define NTRUP_MF_UNALIGNED 0
#endif
__device__ __forceinline__ mf_v4i lds_read16(const uint8_t* p) {
    mf_v4i v;
    __builtin_memcpy(&v, p, 16);
    return v;
}

// Fragment reader for one reversed limb array: 16 bytes from byte
// s0 - 64 k at K-step k.
struct ToeplitzFrag {
    const uint8_t* base;   // array + s0
    const uint32_t* w32;   // aligned-dword form
    int sh;
    uint32_t d[5];
    mf_v4i v;
    __device__ __forceinline__ ToeplitzFrag(const uint8_t* arr, int s0)
        : base(arr + s0), w32((const uint32_t*)arr + (s0 >> 2)), sh(s0 & 3) {}
    __device__ __forceinline__ void load(int k) {
        if (NTRUP_MF_UNALIGNED) {
            v = lds_read16(base - 64 * k);
        } else {
#pragma unroll
            for (int j = 0; j < 5; j++) d[j] = w32[j - 16 * k];
        }
    }
    __device__ __forceinline__ mf_v4i get() const {
        if (NTRUP_MF_UNALIGNED) return v;
        mf_v4i t;
#pragma unroll
        for (int j = 0; j < 4; j++) t[j] = (int)__builtin_amdgcn_alignbyte(d[j + 1], d[j], sh);
        return t;
    }
};

// Combining the limb partial sums of a big x big product into a centered
// residue: s = a0 + 2^7 a1 + 2^14 a2 (mod q), where a0 sums lo x lo, a1
// lo x hi + hi x lo and a2 hi x hi over at most p pairs.  The Toeplitz
// operand is a centered residue (|lo| <= 64, |hi| <= AH) and the folded
// Hankel operand a sum of two (|lo| <= 64, |hi| <= EH), so
// |a0 + 2^7 a1| <= p (64^2 + 2^7 (64 EH + 64 AH)) and |a2| <= p AH EH.
// With C = |2^14 mod q| (centered) the raw sum fits int32 when
// p (64^2 + 2^7 (64 EH + 64 AH) + C AH EH) < 2^31 (p = 653, 761, 857): one
// reduction.  Otherwise (p = 1277) a2 is reduced first, |C rr(a2)| < 3Cq/2.
template <int P, int Q>
struct LimbSum {
    static constexpr int64_t C14 = ((16384 % Q) > Q / 2) ? (16384 % Q) - Q : (16384 % Q);
    static constexpr int64_t C = C14 < 0 ? -C14 : C14;
    static constexpr int64_t AH = ((Q - 1) / 2 + 64) / 128;
    static constexpr int64_t EH = ((Q - 1) + 64) / 128;
    static constexpr int64_t LOWER = (int64_t)P * (64 * 64 + 128 * (64 * EH + 64 * AH));
    static constexpr bool DIRECT = LOWER + (int64_t)P * C * AH * EH < 2147483647LL;
    static_assert(DIRECT || LOWER + C * (3 * Q / 2 + 1) < 2147483647LL, "a0 + 2^7 a1 + C rr(a2) fits int32");
};

template <int P, int Q>
__device__ __forceinline__ int32_t limb_sum(int32_t a0, int32_t a1, int32_t a2) {
    using B = LimbSum<P, Q>;
    constexpr int32_t C14 = (int32_t)B::C14;
    if constexpr (B::DIRECT) return freeze<Q>(a0 + 128 * a1 + C14 * a2);
    else return freeze<Q>(a0 + 128 * a1 + C14 * reduce_rough<Q>(a2));
}

// x = 128 hi + lo, lo in [-64, 64), as two int8 values.
__device__ __forceinline__ void split_limb(int32_t x, uint32_t& lo, uint32_t& hi) {
    const int32_t h = (x + 64) >> 7;
    lo = (uint32_t)(uint8_t)(int8_t)(x - 128 * h);
    hi = (uint32_t)(uint8_t)(int8_t)h;
}

// Byte-wise sum of two words of four int8 values (no carries between bytes).
__device__ __forceinline__ uint32_t add8x4(uint32_t a, uint32_t b) {
    return ((a & 0x7F7F7F7Fu) + (b & 0x7F7F7F7Fu)) ^ ((a ^ b) & 0x80808080u);
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

// Folded coefficient E_m of X (int16, p centered entries).
template <int P>
__device__ __forceinline__ int32_t folded_coef(const int16_t* X, int m) {
    if (m >= 1 && m < P) return X[m];
    if (m == 0) return (int32_t)X[0] + (int32_t)X[P - 1];
    if (m < 0 && m >= -(P - 1)) return (int32_t)X[m + P] + (int32_t)X[m + P - 1];
    return 0;
}

// Hankel limbs of X, folded and zero-padded: HL[HOFF + m] = lo(E_m), HH
// likewise; a small operand (|X_m| <= 3, hi = 0) needs HL only: pass
// HH = nullptr.  X may be in LDS or in global memory.
template <int P>
__device__ __forceinline__ void build_hankel(const int16_t* X, uint8_t* HL, uint8_t* HH) {
    using S = MfShape<P>;
    for (int i = lane_id(); i < S::HLEN / 4; i += 64) {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            uint32_t l, h;
            split_limb(folded_coef<P>(X, 4 * i + t - S::HOFF), l, h);
            lo |= l << (8 * t);
            hi |= h << (8 * t);
        }
        ((uint32_t*)HL)[i] = lo;
        if (HH) ((uint32_t*)HH)[i] = hi;
    }
}

// Folded Hankel bytes of a small operand held in registers: lane l holds
// x_m, m = 4l + 256u + t (t = 0..3), as the int8 bytes of w[u] (zero for
// m >= p).  Writes E_m for -(p-1) <= m < p at H[HOFF + m]; the padding
// around it is left as it is (zero).
template <int P, int NU>
__device__ __forceinline__ void put_folded8(const uint32_t (&w)[NU], uint8_t* H) {
    using S = MfShape<P>;
    constexpr int UP = (P - 1) / 256, LPB = ((P - 1) / 4) % 64;   // word and lane of x_{p-1} (byte 0)
    static_assert(NU * 256 >= P, "the words cover the operand");
    const int lane = lane_id();
    const uint32_t xp = (uint32_t)__builtin_amdgcn_readlane((int)w[UP], LPB) & 0xFFu;
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t nx = (uint32_t)__shfl_down((int)w[u], 1);   // word of m0 + 4
        if (u + 1 < NU) {
            const uint32_t n0 = (uint32_t)__builtin_amdgcn_readlane((int)w[u + 1 < NU ? u + 1 : u], 0);
            nx = (lane == 63) ? n0 : nx;
        }
        if (m0 < P) {
            // E_m = x_m (m >= 1), E_0 = x_0 + x_{p-1}
            const uint32_t pos = (u == 0 && lane == 0) ? add8x4(w[u], xp) : w[u];
            *(uint32_t*)(H + S::HOFF + m0) = pos;
            // E_{m0 - (p-1) + t} = x_{m0+t+1} + x_{m0+t}
            if (m0 + 4 < P) *(uint32_t*)(H + S::NEG + m0) = add8x4(w[u], (w[u] >> 8) | (nx << 24));
        }
    }
}

// The same for a big operand: lane l holds x_m (int16, centered) as two
// words per u, w[u][0] = (x_{m0}, x_{m0+1}), w[u][1] = (x_{m0+2}, x_{m0+3});
// writes the limbs of E_m to HL and HH.
template <int P, int NU>
__device__ __forceinline__ void put_folded16(const uint32_t (&w)[NU][2], uint8_t* HL, uint8_t* HH) {
    using S = MfShape<P>;
    constexpr int UP = (P - 1) / 256, LPB = ((P - 1) / 4) % 64;
    static_assert(NU * 256 >= P, "the words cover the operand");
    const int lane = lane_id();
    const int32_t xp = (int32_t)(int16_t)(__builtin_amdgcn_readlane((int)w[UP][0], LPB) & 0xFFFF);
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t nx = (uint32_t)__shfl_down((int)w[u][0], 1);
        if (u + 1 < NU) {
            const uint32_t n0 = (uint32_t)__builtin_amdgcn_readlane((int)w[u + 1 < NU ? u + 1 : u][0], 0);
            nx = (lane == 63) ? n0 : nx;
        }
        if (m0 < P) {
            int32_t x[5];
#pragma unroll
            for (int t = 0; t < 4; t++) x[t] = (int32_t)(int16_t)(w[u][t >> 1] >> (16 * (t & 1)));
            x[4] = (int32_t)(int16_t)(nx & 0xFFFFu);
            uint32_t pl = 0, ph = 0, nl = 0, nh = 0;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                uint32_t l, h;
                split_limb(x[t] + ((u == 0 && t == 0 && lane == 0) ? xp : 0), l, h);
                pl |= l << (8 * t);
                ph |= h << (8 * t);
                split_limb(x[t] + x[t + 1], l, h);
                nl |= l << (8 * t);
                nh |= h << (8 * t);
            }
            *(uint32_t*)(HL + S::HOFF + m0) = pl;
            *(uint32_t*)(HH + S::HOFF + m0) = ph;
            if (m0 + 4 < P) {
                *(uint32_t*)(HL + S::NEG + m0) = nl;
                *(uint32_t*)(HH + S::NEG + m0) = nh;
            }
        }
    }
}

// Output tiles [T0, T1) of c = a b (before the correction of c_0): T-operand
// limbs (TL, TH), folded H-operand limbs (HL, and HH when H_BIG).  Lane
// (c, g) returns c_{i+v}, i = 256t + 16c + 4g, in out[t] as centered int16
// pairs (zero for i + v >= p).  Software-pipelined: the fragments of K-step
// k+1 are read from LDS while the MFMAs of K-step k run.
template <int P, bool H_BIG, int T0, int T1, bool T_BIG, int MOD>
__device__ __forceinline__ void mfma_tiles(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                           const uint8_t* HH, uint32_t (&out)[MfShape<P>::NT][2]) {
    using S = MfShape<P>;
    constexpr int Q = MOD;
    static_assert(T_BIG || !H_BIG, "a one-limb Toeplitz operand goes with a one-limb Hankel operand");
    constexpr int NTC = T1 - T0;
    const int lane = lane_id();
    const int rc = lane & 15, g = lane >> 4;
    // Toeplitz read position of K-step 0: bytes from Z0 - 16 g - rc
    const int s0 = S::Z0 - 16 * g - rc;
    ToeplitzFrag nFL(TL, s0), nFH(T_BIG ? TH : TL, s0);
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
    mf_v4i nBL[NTC], nBH[NTC];
    auto load_step = [&](int k) {
        nFL.load(k);
        if (T_BIG) nFH.load(k);
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            const int off = 16 * (16 * (T0 + t) - 4 * k);
            nBL[t] = *(const mf_v4i*)(hl + off);
            if (H_BIG) nBH[t] = *(const mf_v4i*)(hh + off);
        }
    };
    load_step(0);
#pragma unroll
    for (int k = 0; k < S::NKS; k++) {
        // one K-step of fragments in flight beyond the current one
        if (NTRUP_MF_SCHED) __builtin_amdgcn_sched_barrier(0);
        const ToeplitzFrag FL = nFL, FH = nFH;
        mf_v4i BL[NTC], BH[NTC];
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            BL[t] = nBL[t];
            BH[t] = nBH[t];
        }
        if (k + 1 < S::NKS) load_step(k + 1);
        const mf_v4i tl = FL.get();
        const mf_v4i th = T_BIG ? FH.get() : tl;
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            if (H_BIG) {
                acc0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BL[t], acc0[t], 0, 0, 0);
                acc1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BH[t], acc1[t], 0, 0, 0);
                acc1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BL[t], acc1[t], 0, 0, 0);
                acc2[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BH[t], acc2[t], 0, 0, 0);
            } else {
                acc0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BL[t], acc0[t], 0, 0, 0);
                if (T_BIG) acc1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BL[t], acc1[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NTC; t++) {
        const int i = 256 * (T0 + t) + 16 * rc + 4 * g;
        int32_t v[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (H_BIG)
                v[e] = limb_sum<P, Q>(acc0[t][e], acc1[t][e], acc2[t][e]);
            else if (T_BIG)
                v[e] = freeze<Q>(acc0[t][e] + 128 * acc1[t][e]);
            else
                v[e] = freeze<Q>(acc0[t][e]);
            v[e] = (i + e < P) ? v[e] : 0;
        }
        out[T0 + t][0] = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
        out[T0 + t][1] = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
    }
}

// Tile chunks of one product: at most MAXC tiles share one pass over the
// K-steps, so that the accumulators (2 or 3 sets of 4 registers per tile)
// stay in registers next to the fragments.
#ifndef NTRUP_MF_MAXC_SMALL
#define NTRUP_MF_MAXC_SMALL 6
#endif
#ifndef NTRUP_MF_MAXC_BIG
#define NTRUP_MF_MAXC_BIG 5
#endif
template <int P, bool H_BIG>
struct MfSplit {
    static constexpr int NT = MfShape<P>::NT;
    static constexpr int MAXC = H_BIG ? NTRUP_MF_MAXC_BIG : NTRUP_MF_MAXC_SMALL;
    static constexpr int NC = ceil_div(NT, MAXC);
    static constexpr int lo(int c) { return c * NT / NC; }
};

template <int P, bool H_BIG, int C, bool T_BIG, int MOD>
__device__ __forceinline__ void mfma_chunks(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                            const uint8_t* HH, uint32_t (&out)[MfShape<P>::NT][2]) {
    using SP = MfSplit<P, H_BIG>;
    if constexpr (C < SP::NC) {
        mfma_tiles<P, H_BIG, SP::lo(C), SP::lo(C + 1), T_BIG, MOD>(TL, TH, HL, HH, out);
        mfma_chunks<P, H_BIG, C + 1, T_BIG, MOD>(TL, TH, HL, HH, out);
    }
}

// c = a b in R/q: T-operand limbs (TL, TH) of a and folded H-operand limbs
// (HL, HH) of b already built.  Any of
//   dst  (LDS int16, c_i at dst[i]),
//   TLo/THo (LDS, the reversed Toeplitz limbs of c for the next product:
//        TLo[Z0 - i] = lo(c_i), THo[Z0 - i] = hi(c_i); may be TL, TH),
//   row  (global int16), row8 (global int8, for |c_i| < 128)
// may be nullptr.  Wave-local: the caller orders the inputs (wave_sync)
// before the call and the outputs after it.
// T_BIG = false: a one-limb Toeplitz operand (TH unused; then THo is not
// written and H is one limb too); MOD: the coefficient modulus (q for R/q,
// 3 for R/3 with both operands in {-1, 0, 1}).
template <int P, bool H_BIG, bool T_BIG = true, int MOD = Param<P>::q>
__device__ __forceinline__ void mfma_mul(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL, const uint8_t* HH,
                                         int16_t* dst, uint8_t* TLo, uint8_t* THo, int16_t* row,
                                         int8_t* row8 = nullptr) {
    using S = MfShape<P>;
    constexpr int Q = MOD;
    // a_{p-1} b_{p-1} (b_{p-1} = E_{p-1}), read before TLo may replace TL
    const int32_t ap = (int32_t)(int8_t)TL[S::Z0 - (P - 1)] +
                       (T_BIG ? 128 * (int32_t)(int8_t)TH[S::Z0 - (P - 1)] : 0);
    const int32_t bp = (int32_t)(int8_t)HL[S::HOFF + P - 1] +
                       (H_BIG ? 128 * (int32_t)(int8_t)HH[S::HOFF + P - 1] : 0);
    uint32_t out[S::NT][2];
    mfma_chunks<P, H_BIG, 0, T_BIG, MOD>(TL, TH, HL, HH, out);
    // c_0 = (folded sum at 0) - conv_{p-1},  conv_{p-1} = c_{p-1} - a_{p-1} b_{p-1}
    const int lane = lane_id();
    const int32_t cp = (int32_t)(int16_t)(__builtin_amdgcn_readlane((int)out[S::TP][0], S::LP) & 0xFFFF);
    const int32_t c0 = freeze<Q>((int32_t)(int16_t)(out[0][0] & 0xFFFFu) - cp + ap * bp);
    if (lane == 0) out[0][0] = (out[0][0] & 0xFFFF0000u) | (uint32_t)(uint16_t)c0;
    wave_sync();
    const int rc = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < S::NT; t++) {
        const int i = 256 * t + 16 * rc + 4 * g;
        if (i >= P) continue;
        const uint32_t w0 = out[t][0], w1 = out[t][1];
        if (dst) {
            if (i + 3 < P) *(uint2*)(dst + i) = make_uint2(w0, w1);
            else dst[i] = (int16_t)(w0 & 0xFFFFu);   // p = 1 mod 4: c_{p-1} alone
        }
        if (TLo) {
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                uint32_t l, h;
                split_limb((int32_t)(int16_t)((e < 2 ? w0 : w1) >> (16 * (e & 1))), l, h);
                lo |= l << (8 * (3 - e));
                hi |= h << (8 * (3 - e));
            }
            *(uint32_t*)(TLo + S::Z0 - i - 3) = lo;
            if (T_BIG) *(uint32_t*)(THo + S::Z0 - i - 3) = hi;
        }
        if (row) {
#pragma unroll
            for (int e = 0; e < 4; e++)
                if (i + e < P) row[i + e] = (int16_t)((e < 2 ? w0 : w1) >> (16 * (e & 1)));
        }
        if (row8) {
#pragma unroll
            for (int e = 0; e < 4; e++)
                if (i + e < P) row8[i + e] = (int8_t)((e < 2 ? w0 : w1) >> (16 * (e & 1)));
        }
    }
}


// Two products sharing the Toeplitz operand a (limbs TL, TH): c1 = a b1 with
// a big folded operand b1 (HL, HH) and c2 = a b2 with a small one (HS), over
// the tiles [T0, T1), in one pass over the K-steps (the Toeplitz fragments are
// read once for both).  Returns both as mfma_tiles does.
template <int P, int T0, int T1>
__device__ __forceinline__ void mfma_tiles2(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                            const uint8_t* HH, const uint8_t* HS,
                                            uint32_t (&out1)[MfShape<P>::NT][2], uint32_t (&out2)[MfShape<P>::NT][2]) {
    using S = MfShape<P>;
    constexpr int Q = S::Q;
    constexpr int NTC = T1 - T0;
    const int lane = lane_id();
    const int rc = lane & 15, g = lane >> 4;
    const int s0 = S::Z0 - 16 * g - rc;
    ToeplitzFrag nFL(TL, s0), nFH(TH, s0);
    const int hoff = S::HOFF + 16 * (rc - g);
    mf_v4i a0[NTC], a1[NTC], a2[NTC], s0a[NTC], s1a[NTC];
#pragma unroll
    for (int t = 0; t < NTC; t++) {
        a0[t] = a1[t] = a2[t] = s0a[t] = s1a[t] = mf_v4i{0, 0, 0, 0};
    }
    mf_v4i nBL[NTC], nBH[NTC], nBS[NTC];
    auto load_step = [&](int k) {
        nFL.load(k);
        nFH.load(k);
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            const int off = hoff + 16 * (16 * (T0 + t) - 4 * k);
            nBL[t] = *(const mf_v4i*)(HL + off);
            nBH[t] = *(const mf_v4i*)(HH + off);
            nBS[t] = *(const mf_v4i*)(HS + off);
        }
    };
    load_step(0);
#pragma unroll
    for (int k = 0; k < S::NKS; k++) {
        if (NTRUP_MF_SCHED) __builtin_amdgcn_sched_barrier(0);
        const ToeplitzFrag FL = nFL, FH = nFH;
        mf_v4i BL[NTC], BH[NTC], BS[NTC];
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            BL[t] = nBL[t];
            BH[t] = nBH[t];
            BS[t] = nBS[t];
        }
        if (k + 1 < S::NKS) load_step(k + 1);
        const mf_v4i tl = FL.get(), th = FH.get();
#pragma unroll
        for (int t = 0; t < NTC; t++) {
            a0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BL[t], a0[t], 0, 0, 0);
            a1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BH[t], a1[t], 0, 0, 0);
            s0a[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, BS[t], s0a[t], 0, 0, 0);
            a1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BL[t], a1[t], 0, 0, 0);
            a2[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BH[t], a2[t], 0, 0, 0);
            s1a[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, BS[t], s1a[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NTC; t++) {
        const int i = 256 * (T0 + t) + 16 * rc + 4 * g;
        int32_t v[4], w[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            v[e] = limb_sum<P, Q>(a0[t][e], a1[t][e], a2[t][e]);
            w[e] = freeze<Q>(s0a[t][e] + 128 * s1a[t][e]);
            v[e] = (i + e < P) ? v[e] : 0;
            w[e] = (i + e < P) ? w[e] : 0;
        }
        out1[T0 + t][0] = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
        out1[T0 + t][1] = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
        out2[T0 + t][0] = (uint32_t)(uint16_t)w[0] | ((uint32_t)(uint16_t)w[1] << 16);
        out2[T0 + t][1] = (uint32_t)(uint16_t)w[2] | ((uint32_t)(uint16_t)w[3] << 16);
    }
}

#ifndef NTRUP_MF_MAXC_PAIR
#define NTRUP_MF_MAXC_PAIR 3
#endif
template <int P, int C>
__device__ __forceinline__ void mfma_chunks2(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                             const uint8_t* HH, const uint8_t* HS,
                                             uint32_t (&out1)[MfShape<P>::NT][2], uint32_t (&out2)[MfShape<P>::NT][2]) {
    constexpr int NT = MfShape<P>::NT, NC = ceil_div(NT, NTRUP_MF_MAXC_PAIR);
    if constexpr (C < NC) {
        mfma_tiles2<P, C * NT / NC, (C + 1) * NT / NC>(TL, TH, HL, HH, HS, out1, out2);
        mfma_chunks2<P, C + 1>(TL, TH, HL, HH, HS, out1, out2);
    }
}

// The reversed Toeplitz limbs of a product held as mfma_tiles returns it,
// after the correction of c_0 (see mfma_mul).
template <int P>
__device__ __forceinline__ void mfma_fix_store(uint32_t (&out)[MfShape<P>::NT][2], int32_t ap, int32_t bp, uint8_t* TLo,
                                               uint8_t* THo) {
    using S = MfShape<P>;
    constexpr int Q = S::Q;
    const int lane = lane_id();
    const int32_t cp = (int32_t)(int16_t)(__builtin_amdgcn_readlane((int)out[S::TP][0], S::LP) & 0xFFFF);
    const int32_t c0 = freeze<Q>((int32_t)(int16_t)(out[0][0] & 0xFFFFu) - cp + ap * bp);
    if (lane == 0) out[0][0] = (out[0][0] & 0xFFFF0000u) | (uint32_t)(uint16_t)c0;
    const int rc = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < S::NT; t++) {
        const int i = 256 * t + 16 * rc + 4 * g;
        if (i >= P) continue;
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            uint32_t l, h;
            split_limb((int32_t)(int16_t)((e < 2 ? out[t][0] : out[t][1]) >> (16 * (e & 1))), l, h);
            lo |= l << (8 * (3 - e));
            hi |= h << (8 * (3 - e));
        }
        *(uint32_t*)(TLo + S::Z0 - i - 3) = lo;
        *(uint32_t*)(THo + S::Z0 - i - 3) = hi;
    }
}

// The coefficients of a product held as mfma_tiles returns it, after the
// correction of c_0, to a global int16 row.
template <int P>
__device__ __forceinline__ void mfma_fix_row(uint32_t (&out)[MfShape<P>::NT][2], int32_t ap, int32_t bp, int16_t* row) {
    using S = MfShape<P>;
    constexpr int Q = S::Q;
    const int lane = lane_id();
    const int32_t cp = (int32_t)(int16_t)(__builtin_amdgcn_readlane((int)out[S::TP][0], S::LP) & 0xFFFF);
    const int32_t c0 = freeze<Q>((int32_t)(int16_t)(out[0][0] & 0xFFFFu) - cp + ap * bp);
    if (lane == 0) out[0][0] = (out[0][0] & 0xFFFF0000u) | (uint32_t)(uint16_t)c0;
    const int rc = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < S::NT; t++) {
        const int i = 256 * t + 16 * rc + 4 * g;
        if (i >= P) continue;
#pragma unroll
        for (int e = 0; e < 4; e++)
            if (i + e < P) row[i + e] = (int16_t)((e < 2 ? out[t][0] : out[t][1]) >> (16 * (e & 1)));
    }
}

// c1 = a b1 (big b1: HL, HH) to the global int16 row row1 and c2 = a b2
// (small b2: HS) to the Toeplitz limbs U2L/U2H (which may be TL/TH).
template <int P>
__device__ __forceinline__ void mfma_mul2_row(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL,
                                              const uint8_t* HH, const uint8_t* HS, int16_t* row1, uint8_t* U2L,
                                              uint8_t* U2H) {
    using S = MfShape<P>;
    const int32_t ap = (int32_t)(int8_t)TL[S::Z0 - (P - 1)] + 128 * (int32_t)(int8_t)TH[S::Z0 - (P - 1)];
    const int32_t bp1 = (int32_t)(int8_t)HL[S::HOFF + P - 1] + 128 * (int32_t)(int8_t)HH[S::HOFF + P - 1];
    const int32_t bp2 = (int32_t)(int8_t)HS[S::HOFF + P - 1];
    uint32_t out1[S::NT][2], out2[S::NT][2];
    mfma_chunks2<P, 0>(TL, TH, HL, HH, HS, out1, out2);
    wave_sync();
    mfma_fix_row<P>(out1, ap, bp1, row1);
    mfma_fix_store<P>(out2, ap, bp2, U2L, U2H);
}

// c1 = a b1 (big b1: HL, HH) to the Toeplitz limbs U1L/U1H and c2 = a b2
// (small b2: HS) to U2L/U2H, which may be TL/TH themselves (a replaced by
// c2).  Wave-local like mfma_mul.
template <int P>
__device__ __forceinline__ void mfma_mul2(const uint8_t* TL, const uint8_t* TH, const uint8_t* HL, const uint8_t* HH,
                                          const uint8_t* HS, uint8_t* U1L, uint8_t* U1H, uint8_t* U2L, uint8_t* U2H) {
    using S = MfShape<P>;
    const int32_t ap = (int32_t)(int8_t)TL[S::Z0 - (P - 1)] + 128 * (int32_t)(int8_t)TH[S::Z0 - (P - 1)];
    const int32_t bp1 = (int32_t)(int8_t)HL[S::HOFF + P - 1] + 128 * (int32_t)(int8_t)HH[S::HOFF + P - 1];
    const int32_t bp2 = (int32_t)(int8_t)HS[S::HOFF + P - 1];
    uint32_t out1[S::NT][2], out2[S::NT][2];
    mfma_chunks2<P, 0>(TL, TH, HL, HH, HS, out1, out2);
    wave_sync();
    mfma_fix_store<P>(out1, ap, bp1, U1L, U1H);
    mfma_fix_store<P>(out2, ap, bp2, U2L, U2H);
}

}  // namespace ntrup
