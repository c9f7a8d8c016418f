// Per-key reciprocal in R/3 = (Z/3)[x]/(x^p - x - 1) by constant-time
// divsteps, bitsliced, one key per lane or per group of 2, 4 or 8 lanes.
//
// KeyGen (OpenSSLNTRU paper, Section 3.1) needs 1/g in R/3 and needs g to be
// invertible; the paper notes that earlier NTRU Prime software obtained
// invertibility as a side effect of a constant-time extended-gcd (the
// Bernstein-Yang divstep algorithm it cites in Section 3.1).  This kernel is
// that per-key form: a fixed 2p-1 divsteps on (f, g) = (reversed x^p-x-1,
// reversed g), with secret-independent control flow and memory access.
//
// Divstep (delta, f, g), f(0) != 0:
//   if delta > 0 and g(0) != 0:  (1 - delta, g, (g(0) f - f(0) g) / x)
//   else                         (1 + delta, f, (f(0) g - g(0) f) / x)
// with (v, r) updated by the same matrix but multiplied by x instead of
// divided.  Starting from delta = 1, v = 0, r = 1, after 2p-1 steps g is a
// unit iff delta = 0, and then 1/g has coefficient i equal to f(0)^-1 v[p-i].
// Any unit multiple of the (g, r) row may be used at each step; over F_3 the
// row is taken as s*g + f with s = -g(0)/f(0) (s^2 = 1), so one F_3 add per
// coefficient suffices.
//
// Bitsliced representation: 32 coefficients per word pair (m, s) with
// m = (c != 0) and s = (c == -1); s is a don't-care where m = 0 inside the
// loop and canonical (s & m) in every stored output.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_chacha.h"
#include "ntrup_params.h"

namespace ntrup {

template <int P, int LPK>
struct R3Shape {
    static_assert(LPK == 1 || LPK == 2 || LPK == 4 || LPK == 8 || LPK == 16 || LPK == 32 || LPK == 64,
                  "1, 2, 4, 8, 16, 32 or 64 lanes per key");
    static constexpr int W = ceil_div(P + 1, 32);   // words holding p+1 coefficients
    static constexpr int W2 = ceil_div(W, LPK);     // words per lane
    static constexpr int WT = W2 * LPK;             // padded words per polynomial
    static constexpr int NT = 32 * WT;              // padded bit length
    static constexpr int D = NT - P;                // reversal offset (>= 1)
    static constexpr int WN = ceil_div(P, 32);      // words of a natural p-coefficient poly
    static constexpr int KPW = 64 / LPK;            // keys per wave
    using Words = uint32_t[W2];                     // one plane of one lane
    static_assert(D >= 1, "room for x^p");
};

// Lane-group helpers.  A key owns LPK consecutive lanes (a group of up to 16
// lies in one DPP row of 16 lanes, a group of 32 in two); group_first
// broadcasts the value of the group's first lane with DPP moves: a quad
// permute for LPK <= 4; for LPK = 8 the quad broadcast followed by row_shr:4
// written into banks 1 and 3 only (lanes 4-7 and 12-15 of each row take the
// broadcast of the quad below, lanes 0-3 and 8-11 keep their own); for 16,
// row_newbcast:0 (lane 0 of each row to its row); for 32, that followed by
// row_bcast:15 written into rows 1 and 3 only (each takes lane 15 of the row
// below, which by then holds that row's lane 0); for 64, the wave's first
// lane (v_readfirstlane: every lane is active in the divstep loop).
template <int LPK>
__device__ __forceinline__ uint32_t group_first(uint32_t x) {
    if (LPK == 1) return x;
    if (LPK == 64) return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
    if (LPK == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xA0, 0xF, 0xF, true);  // [0,0,2,2]
    if (LPK >= 16) {
        const int r = __builtin_amdgcn_mov_dpp((int)x, 0x150, 0xF, 0xF, true);             // row_newbcast:0
        if (LPK == 16) return (uint32_t)r;
        return (uint32_t)__builtin_amdgcn_update_dpp(r, r, 0x142, 0xA, 0xF, false);        // row_bcast:15
    }
    const int q = __builtin_amdgcn_mov_dpp((int)x, 0x00, 0xF, 0xF, true);                  // [0,0,0,0]
    if (LPK == 4) return (uint32_t)q;
    return (uint32_t)__builtin_amdgcn_update_dpp(q, q, 0x114, 0xF, 0xA, false);             // row_shr:4
}
// lane i reads lane i+1 / lane i-1: within its row of 16 (row_shl:1 /
// row_shr:1) when a group lies in one row, across the wave (wave_shl:1 /
// wave_shr:1) for groups of 32 or 64; the caller masks the lane that must
// read 0
template <int LPK>
__device__ __forceinline__ uint32_t group_next(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, LPK >= 32 ? 0x130 : 0x101, 0xF, 0xF, true);
}
template <int LPK>
__device__ __forceinline__ uint32_t group_prev(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, LPK >= 32 ? 0x138 : 0x111, 0xF, 0xF, true);
}

// Three-input boolean functions on gfx950 (v_bitop3_b32): the 8-bit table is
// the function evaluated on the operand patterns 0xF0, 0xCC, 0xAA.
constexpr uint32_t kSel = ((0xF0u & 0xCCu) | (~0xF0u & 0xAAu)) & 0xFFu;   // x ? y : z  (0xCA)
constexpr uint32_t kXor3 = (0xF0u ^ 0xCCu ^ 0xAAu) & 0xFFu;              // x ^ y ^ z  (0x96)
constexpr uint32_t kAddM = ((0xF0u ^ 0xCCu) | (0xF0u & 0xCCu & ~0xAAu)) & 0xFFu;  // (0x7C)
constexpr uint32_t kAndXnor = (0xF0u & ~(0xCCu ^ 0xAAu)) & 0xFFu;            // x & ~(y ^ z)  (0x90)
static_assert(kSel == 0xCA && kXor3 == 0x96 && kAddM == 0x7C && kAndXnor == 0x90, "bitop3 tables");

__device__ __forceinline__ uint32_t sel(uint32_t mask, uint32_t a, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(mask, a, b, kSel);
}
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, kXor3);
}
// nonzero plane of a + b in F_3 from the nonzero planes x, y and the sign
// difference z: (x ^ y) | (x & y & ~z)
__device__ __forceinline__ uint32_t addm(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, kAddM);
}

// Natural-order bitsliced words of a small polynomial c_0..c_{p-1} staged in
// LDS as [plane][WT] (plane 0 = m, plane 1 = s), zero beyond p.
//
// load_reversed: word k of (reversed c as a degree-(p-1) polynomial), i.e.
// bit i = c_{p-1-i} for i < p, 0 above.  With Rv = the bit-reversal of the
// NT-bit natural string, that is (Rv >> D).
template <int P, int LPK>
__device__ __forceinline__ uint32_t load_reversed(const uint32_t* nat, int k) {
    using S = R3Shape<P, LPK>;
    const int a = k + S::D / 32, o = S::D % 32;
    uint32_t lo = (a < S::WT) ? __builtin_bitreverse32(nat[S::WT - 1 - a]) : 0u;
    uint32_t hi = (a + 1 < S::WT) ? __builtin_bitreverse32(nat[S::WT - 2 - a]) : 0u;
    return o ? __builtin_amdgcn_alignbit(hi, lo, o) : lo;
}

// Word k of the natural-order output u with u_j = v[p - j] for j < p, taken
// from the NT-bit string v staged in LDS: u = bitreverse(v) >> (D - 1),
// masked to p bits.
template <int P, int LPK>
__device__ __forceinline__ uint32_t load_output(const uint32_t* vst, int k) {
    using S = R3Shape<P, LPK>;
    const int a = k + (S::D - 1) / 32, o = (S::D - 1) % 32;
    uint32_t lo = (a < S::WT) ? __builtin_bitreverse32(vst[S::WT - 1 - a]) : 0u;
    uint32_t hi = (a + 1 < S::WT) ? __builtin_bitreverse32(vst[S::WT - 2 - a]) : 0u;
    uint32_t w = o ? __builtin_amdgcn_alignbit(hi, lo, o) : lo;
    const int valid = P - 32 * k;
    if (valid < 32) w &= (valid <= 0) ? 0u : ((1u << valid) - 1u);
    return w;
}

// One-lane form (a whole key in one lane): only the live words are touched.
// At step j (0-based) of the 2p-1, the steps still to come read only
// coefficients [0, 2p-1-j) of f and g (each step's control reads coefficient
// 0, and the new g's coefficient i comes from coefficients i and i+1), and
// v, r have degree at most j, v at most j+1 after its shift.  So the words of
// f and g above ceil(min(p+1, 2p-1-j)/32) can be left stale (their bits only
// ever reach positions that are no longer read) and the words of v and r
// above ceil((j+2)/32) are still zero.  The 2p-1 steps run in segments of
// kR3Seg steps, each with the live word counts of its worst step as
// compile-time constants: about 79% of the word updates of the full loop.
#ifndef NTRUP_R3_SEG
#define NTRUP_R3_SEG 96
#endif
constexpr int kR3Seg = NTRUP_R3_SEG;
static_assert(kR3Seg % 3 == 0, "segments of whole three-step trips (2p-1 is a multiple of 3 for every p here)");

template <int W, int NFG, int NVR>
__device__ __forceinline__ void r3_step_live(uint32_t (&fm)[W], uint32_t (&fs)[W], uint32_t (&gm)[W],
                                             uint32_t (&gs)[W], uint32_t (&vm)[W], uint32_t (&vs)[W],
                                             uint32_t (&rm)[W], uint32_t (&rs)[W], int32_t& e) {
    const uint32_t NZ = (uint32_t)__builtin_amdgcn_sbfe((int)gm[0], 0, 1);
    const uint32_t NEG = (uint32_t)__builtin_amdgcn_sbfe((int)__builtin_amdgcn_bitop3_b32(gm[0], gs[0], fs[0], kAndXnor),
                                                         0, 1);
    const uint32_t SW = NZ & ~(uint32_t)(e >> 31);
    e = (int32_t)((uint32_t)e ^ SW) + (int32_t)SW + 1;
#pragma unroll
    for (int k = 0; k < NFG; k++) {
        const uint32_t mbf = fm[k] & NZ;
        const uint32_t xg = xor3(gs[k], NEG, fs[k]), ug = xor3(gs[k], NEG, mbf);
        const uint32_t ngm = addm(gm[k], mbf, xg), ngs = sel(gm[k], ug, fs[k]);
        fm[k] = sel(SW, gm[k], fm[k]);
        fs[k] = sel(SW, gs[k], fs[k]);
        gm[k] = ngm;
        gs[k] = ngs;
    }
#pragma unroll
    for (int k = 0; k < NVR; k++) {
        const uint32_t mbv = vm[k] & NZ;
        const uint32_t xr = xor3(rs[k], NEG, vs[k]), ur = xor3(rs[k], NEG, mbv);
        const uint32_t nrm = addm(rm[k], mbv, xr), nrs = sel(rm[k], ur, vs[k]);
        const uint32_t nvm = sel(SW, rm[k], vm[k]), nvs = sel(SW, rs[k], vs[k]);
        rm[k] = nrm;
        rs[k] = nrs;
        vm[k] = nvm;
        vs[k] = nvs;
    }
#pragma unroll
    for (int k = 0; k < NFG - 1; k++) {
        gm[k] = __builtin_amdgcn_alignbit(gm[k + 1], gm[k], 1);
        gs[k] = __builtin_amdgcn_alignbit(gs[k + 1], gs[k], 1);
    }
    gm[NFG - 1] >>= 1;
    gs[NFG - 1] >>= 1;
#pragma unroll
    for (int k = NVR - 1; k > 0; k--) {
        vm[k] = __builtin_amdgcn_alignbit(vm[k], vm[k - 1], 31);
        vs[k] = __builtin_amdgcn_alignbit(vs[k], vs[k - 1], 31);
    }
    vm[0] <<= 1;
    vs[0] <<= 1;
}

template <int P, int SEG, int W>
__device__ __forceinline__ void r3_live_segments(uint32_t (&fm)[W], uint32_t (&fs)[W], uint32_t (&gm)[W],
                                                 uint32_t (&gs)[W], uint32_t (&vm)[W], uint32_t (&vs)[W],
                                                 uint32_t (&rm)[W], uint32_t (&rs)[W], int32_t& e) {
    constexpr int N = 2 * P - 1, A = SEG * kR3Seg, B = A + kR3Seg < N ? A + kR3Seg : N;
    constexpr int LFG = P + 1 < N - A ? P + 1 : N - A;     // f, g coefficients read from step A on
    constexpr int NFG = ceil_div(LFG, 32);
    constexpr int NVR = ceil_div(B + 1, 32) < W ? ceil_div(B + 1, 32) : W;   // v, r words by step B-1
    static_assert((B - A) % 3 == 0, "whole trips");
#pragma unroll 3
    for (int j = A; j < B; j++) r3_step_live<W, NFG, NVR>(fm, fs, gm, gs, vm, vs, rm, rs, e);
    if constexpr (B < N) r3_live_segments<P, SEG + 1, W>(fm, fs, gm, gs, vm, vs, rm, rs, e);
}

// The divstep loop.  In: this lane's W2 words of reversed g (gm, gs).  Out:
// v words (vm, vs) scaled by f(0)^-1, and the final delta.  h = lane index
// inside the key (0 or 1); the even lane holds coefficient 0.
template <int P, int LPK>
__device__ __forceinline__ int r3_divsteps(typename R3Shape<P, LPK>::Words& gm,
                                           typename R3Shape<P, LPK>::Words& gs,
                                           typename R3Shape<P, LPK>::Words& vm,
                                           typename R3Shape<P, LPK>::Words& vs, int h) {
    using S = R3Shape<P, LPK>;
    constexpr int W2 = S::W2;
    uint32_t fm[W2], fs[W2], rm[W2], rs[W2];
    // f = reversal of x^p - x - 1 = 1 - x^(p-1) - x^p; r = 1; v = 0.
#pragma unroll
    for (int k = 0; k < W2; k++) {
        const int base = 32 * (h * W2 + k);
        uint32_t m = 0, s = 0;
        if (base == 0) m |= 1u;
#pragma unroll
        for (int e = P - 1; e <= P; e++)
            if (e >= base && e < base + 32) { m |= 1u << (e - base); s |= 1u << (e - base); }
        fm[k] = m;
        fs[k] = s;
        rm[k] = (base == 0) ? 1u : 0u;
        rs[k] = 0;
        vm[k] = 0;
        vs[k] = 0;
    }
    // e = delta - 1: delta > 0 iff the sign bit of e is clear
    int32_t e = 0;
    const uint32_t last = (h == LPK - 1) ? 0xFFFFFFFFu : 0u;   // top lane of the key's group
    const uint32_t first = (h == 0) ? 0xFFFFFFFFu : 0u;        // bottom lane
    if constexpr (LPK == 1) r3_live_segments<P, 0, W2>(fm, fs, gm, gs, vm, vs, rm, rs, e);
    // three steps per trip: the register renaming of the updates needs no moves
#pragma unroll 3
    for (int step = 0; step < (LPK == 1 ? 0 : 2 * P - 1); step++) {
        // coefficient 0 of f and g lives in bit 0 of word 0 of the group's first
        // lane; f(0) != 0, so only its sign matters
        const uint32_t fs0 = group_first<LPK>(fs[0]);
        const uint32_t gm0 = group_first<LPK>(gm[0]);
        const uint32_t gs0 = group_first<LPK>(gs[0]);
        const uint32_t NZ = (uint32_t)__builtin_amdgcn_sbfe((int)gm0, 0, 1);          // s != 0
        const uint32_t NEG = (uint32_t)__builtin_amdgcn_sbfe(
            (int)__builtin_amdgcn_bitop3_b32(gm0, gs0, fs0, kAndXnor), 0, 1);          // s == -1
        const uint32_t SW = NZ & ~(uint32_t)(e >> 31);                               // swap mask
        // delta' = swap ? 1 - delta : 1 + delta, i.e. e' = swap ? ~e : e + 1
        e = (int32_t)((uint32_t)e ^ SW) + (int32_t)SW + 1;
#pragma unroll
        for (int k = 0; k < W2; k++) {
            // g' = s*g + (s != 0 ? f : 0); r' = s*r + (s != 0 ? v : 0)   (F_3 adds)
            const uint32_t mbf = fm[k] & NZ, mbv = vm[k] & NZ;
            const uint32_t xg = xor3(gs[k], NEG, fs[k]), xr = xor3(rs[k], NEG, vs[k]);
            const uint32_t ug = xor3(gs[k], NEG, mbf), ur = xor3(rs[k], NEG, mbv);
            const uint32_t ngm = addm(gm[k], mbf, xg);
            const uint32_t ngs = sel(gm[k], ug, fs[k]);
            const uint32_t nrm = addm(rm[k], mbv, xr);
            const uint32_t nrs = sel(rm[k], ur, vs[k]);
            // (f, v) <- swap ? (g, r) : (f, v), from the values before the update
            fm[k] = sel(SW, gm[k], fm[k]);
            fs[k] = sel(SW, gs[k], fs[k]);
            const uint32_t nvm = sel(SW, rm[k], vm[k]);
            const uint32_t nvs = sel(SW, rs[k], vs[k]);
            gm[k] = ngm; gs[k] = ngs; rm[k] = nrm; rs[k] = nrs;
            vm[k] = nvm; vs[k] = nvs;
        }
        // g <- g / x (one bit down), v <- x v (one bit up)
        uint32_t gin_m = 0, gin_s = 0, vin_m = 0, vin_s = 0;
        if (LPK > 1) {
            // the next lane's word 0 feeds this lane's top word (0 for the top lane)
            gin_m = group_next<LPK>(gm[0]) & ~last;
            gin_s = group_next<LPK>(gs[0]) & ~last;
            // the previous lane's top word feeds this lane's word 0 (0 for the bottom lane)
            vin_m = group_prev<LPK>(vm[W2 - 1]) & ~first;
            vin_s = group_prev<LPK>(vs[W2 - 1]) & ~first;
        }
#pragma unroll
        for (int k = 0; k < W2 - 1; k++) {
            gm[k] = __builtin_amdgcn_alignbit(gm[k + 1], gm[k], 1);
            gs[k] = __builtin_amdgcn_alignbit(gs[k + 1], gs[k], 1);
        }
        gm[W2 - 1] = __builtin_amdgcn_alignbit(gin_m, gm[W2 - 1], 1);
        gs[W2 - 1] = __builtin_amdgcn_alignbit(gin_s, gs[W2 - 1], 1);
#pragma unroll
        for (int k = W2 - 1; k > 0; k--) {
            vm[k] = __builtin_amdgcn_alignbit(vm[k], vm[k - 1], 31);
            vs[k] = __builtin_amdgcn_alignbit(vs[k], vs[k - 1], 31);
        }
        vm[0] = __builtin_amdgcn_alignbit(vm[0], vin_m, 31);
        vs[0] = __builtin_amdgcn_alignbit(vs[0], vin_s, 31);
    }
    // scale v by f(0)^-1 = f(0) (f(0) = -1 flips the sign plane); canonical s
    uint32_t f0 = (fs[0] & 1u);
    f0 = group_first<LPK>(f0);
    const uint32_t FLIP = 0u - f0;
#pragma unroll
    for (int k = 0; k < W2; k++) vs[k] = (vs[k] ^ FLIP) & vm[k];
    return e + 1;
}

}  // namespace ntrup
