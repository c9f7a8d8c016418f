// Reciprocal in R/q (or R/3) by jump divsteps on one wave: the recursive form of the
// constant-time divsteps (Bernstein and Yang; the gcd that Section 3.1 uses,
// whose jump-div-step variant Appendix D times for n = 1), one level deep.
//
// The divstep on (delta, f, g, v, r), f0 and g0 the constant terms of f, g:
//   swap = delta > 0 and g0 != 0;  delta <- (swap ? -delta : delta) + 1;
//   (f, g) <- (swap ? g : f, (f0 g - g0 f) / x);
//   (v, r) <- (x (swap ? r : v), f0 r - g0 v).
// Both pairs move by A = [[1-s, s], [-g0, f0]], then (f, g) by diag(1, 1/x)
// and (v, r) by diag(x, 1).  So n steps multiply (v, r) by
// U = prod diag(x, 1) A_j, whose entries are polynomials of degree <= n, and
// (f, g) by U / x^n (an exact division); and the n steps' controls depend
// only on the low n coefficients of f and g.  Each jump here:
//   1. runs n = kJumpN steps on the low 64 coefficients of f and g (one per
//      lane), building U in registers (one coefficient of each entry per
//      lane);
//   2. applies U to the full f, g, v, r on the int8 matrix cores:
//      f' = (u00 f + u01 g) / x^n, g' = (u10 f + u11 g) / x^n,
//      v' = u00 v + u01 r, r' = u10 v + u11 r -- eight products of a
//      49-coefficient polynomial by a (p+1)-coefficient one, each a single
//      K-step of v_mfma_i32_16x16x64_i8 per 256 outputs (two 7-bit limbs per
//      residue: four MFMAs per pair of operands).
// 2p - 1 steps take ceil((2p-1)/48) jumps (32 at p = 761) against 2p - 1
// full-width steps of the plain loop (recip_wave), about a quarter of its
// vector instructions.  Start, finish and result are the plain loop's: f is
// x^p - x - 1 reversed, g the input reversed, v = 0, r = 1, delta = 1; the
// input is a unit iff delta = 0 at the end, and 1/a has coefficient i equal
// to v_{p-i} / f0.  tests/test_jump_divsteps.py models this schedule on the
// CPU against the oracle.  The same code inverts in R/3 (modulus 3, one
// int8 limb per coefficient, one MFMA per pair of operands): the group
// products of the batched R/3 stage.  (With modulus 3 every value the
// reduction helpers see stays below 2^8 in magnitude, so their 24-bit
// quotient bound holds there too.)
//
// Layouts (LDS, one wave): each polynomial X in {f, g, v, r} is kept as two
// zero-padded byte arrays, HL[kJumpHOff + m] = lo(X_m), HH = hi(X_m) for
// 0 <= m <= p (the Hankel operand: lane (c, gq) of output tile t reads the
// 16 bytes of X_{16 j + e}, j = 16 t + c - gq); two such sets alternate
// between jumps.  Each entry of U is a reversed byte array
// TL[kJumpZ0 - k] = lo(u_k) (the Toeplitz operand: lane (r, gq) reads the 16
// bytes of u_{16 gq + r - e}).  Output element v of lane (c, gq), tile t, is
// coefficient 256 t + 16 c + 4 gq + v of the product.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_mfma.h"
#include "ntrup_params.h"
#include "ntrup_rq.h"

namespace ntrup {

constexpr int kJumpN = 48;     // divsteps per jump: U has degree <= 48, four 16-blocks
constexpr int kJumpZ0 = 79;    // TL[kJumpZ0 - k] = limb(u_k); (kJumpZ0 - 3) % 4 == 0
constexpr int kJumpTLen = 112; // reads reach byte kJumpZ0 + 15 + 4 (five dwords per lane)
constexpr int kJumpHOff = 48;  // Hankel blocks j >= -3 read zeros below X_0

template <int P>
struct JumpShape {
    static constexpr int NT = ceil_div(P + 1 + kJumpN, 256);   // output tiles: f' needs outputs up to p + n
    static constexpr int HLEN = kJumpHOff + 256 * NT;
    static constexpr int NJUMP = ceil_div(2 * P - 1, kJumpN);
    static_assert(kJumpN + 1 <= 64, "U and the truncated f, g fit one coefficient per lane");
    // output row r of a block sums u_k for k in [r - 15, r + 48] (four
    // 16-blocks of one K-step), so every r sees all of u_0 .. u_n only for
    // n <= 48 (a 60-step jump misses u_49 .. u_60 in rows r < 12)
    static_assert(16 * 3 >= kJumpN && kJumpZ0 >= 63 && (kJumpZ0 - 3) % 4 == 0, "one K-step covers U");
    static_assert(kJumpN % 4 == 0, "f' = out shifted by n stays dword-aligned (full jumps only)");
    static_assert(kJumpN % 3 == 0 && (2 * P - 1) % 3 == 0, "every jump is whole three-step trips");
    static_assert(HLEN % 16 == 0, "16-byte Hankel reads stay aligned");
};

// LDS of one jump reciprocal.
template <int P>
struct JumpLds {
    using S = JumpShape<P>;
    __attribute__((aligned(16))) uint8_t H[2][4][2][S::HLEN];   // [set][f g v r][lo hi]
    __attribute__((aligned(16))) uint8_t T[4][2][kJumpTLen];    // [u00 u01 u10 u11][lo hi]
    __attribute__((aligned(16))) int32_t low[2][64];            // low coefficients of f, g
    __attribute__((aligned(16))) int16_t v[S::NT * 256];        // v after the last jump
};

// Writes the four limb bytes of x_m .. x_{m+3} (centered) at H + m.
__device__ __forceinline__ void jump_put4(uint8_t* HL, uint8_t* HH, int m, const int32_t (&x)[4]) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        uint32_t l, h;
        split_limb(x[e], l, h);
        lo |= l << (8 * e);
        hi |= h << (8 * e);
    }
    *(uint32_t*)(HL + m) = lo;
    *(uint32_t*)(HH + m) = hi;
}

// Accumulates the product of U entry `ue` (Toeplitz limbs TL, TH) with X
// (Hankel limbs XL, XH) into the per-tile accumulators (lo lo, lo hi + hi lo,
// hi hi); with one limb (LIMBS = 1, residues mod 3) only lo lo.
template <int P, int LIMBS>
__device__ __forceinline__ void jump_mac(const uint8_t* TL, const uint8_t* TH, const uint8_t* XL,
                                         const uint8_t* XH, mf_v4i (&a0)[JumpShape<P>::NT],
                                         mf_v4i (&a1)[JumpShape<P>::NT], mf_v4i (&a2)[JumpShape<P>::NT]) {
    using S = JumpShape<P>;
    const int lane = lane_id();
    const int rc = lane & 15, gq = lane >> 4;
    const int s0 = kJumpZ0 - 16 * gq - rc;   // first byte: u_{16 gq + rc}
    ToeplitzFrag FL(TL, s0), FH(TH, s0);
    FL.load(0);
    if (LIMBS == 2) FH.load(0);
    const mf_v4i tl = FL.get();
    const mf_v4i th = LIMBS == 2 ? FH.get() : tl;
    const uint8_t* xl = XL + kJumpHOff + 16 * (rc - gq);
    const uint8_t* xh = XH + kJumpHOff + 16 * (rc - gq);
#pragma unroll
    for (int t = 0; t < S::NT; t++) {
        const mf_v4i bl = *(const mf_v4i*)(xl + 256 * t);
        const mf_v4i bh = *(const mf_v4i*)(xh + 256 * t);
        a0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, bl, a0[t], 0, 0, 0);
        if (LIMBS == 2) {
            a1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tl, bh, a1[t], 0, 0, 0);
            a1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, bl, a1[t], 0, 0, 0);
            a2[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(th, bh, a2[t], 0, 0, 0);
        }
    }
}

// One output polynomial of a jump: Y = (U[ia] X0 + U[ib] X1) mod M, shifted
// down by `shift` coefficients (n for f and g, 0 for v and r); its
// coefficients 0..p go to the Hankel limbs YL, YH (the rest stay zero),
// coefficients below 64 also to `low` when given, and all of them to `vout`
// (int16) when given.
template <int P, int M>
__device__ __forceinline__ void jump_output(JumpLds<P>& L, int ia, int ib, const uint8_t* X0L, const uint8_t* X0H,
                                            const uint8_t* X1L, const uint8_t* X1H, int shift, uint8_t* YL,
                                            uint8_t* YH, int32_t* low, int16_t* vout) {
    using S = JumpShape<P>;
    constexpr int Q = M;
    constexpr int LIMBS = M == 3 ? 1 : 2;
    // 2^14 mod q, centered
    constexpr int32_t C14 = ((16384 % Q) > Q / 2) ? (16384 % Q) - Q : (16384 % Q);
    mf_v4i a0[S::NT], a1[S::NT], a2[S::NT];
#pragma unroll
    for (int t = 0; t < S::NT; t++) {
        a0[t] = mf_v4i{0, 0, 0, 0};
        a1[t] = mf_v4i{0, 0, 0, 0};
        a2[t] = mf_v4i{0, 0, 0, 0};
    }
    jump_mac<P, LIMBS>(L.T[ia][0], L.T[ia][1], X0L, X0H, a0, a1, a2);
    jump_mac<P, LIMBS>(L.T[ib][0], L.T[ib][1], X1L, X1H, a0, a1, a2);
    const int lane = lane_id();
    const int rc = lane & 15, gq = lane >> 4;
#pragma unroll
    for (int t = 0; t < S::NT; t++) {
        const int m = 256 * t + 16 * rc + 4 * gq - shift;   // coefficient of Y in element 0
        int32_t y[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            // |a0| + 128 |a1| + |C14| |a2| < 2^31: at most 98 limb products per output
            // (two products of 49 coefficients of U by residues)
            const int32_t s = LIMBS == 1 ? a0[t][e] : a0[t][e] + 128 * a1[t][e] + C14 * a2[t][e];
            y[e] = (m + e <= P) ? freeze<Q>(s) : 0;
        }
        if (m >= 0 && m <= P) {
            jump_put4(YL + kJumpHOff, YH + kJumpHOff, m, y);
            if (low && m < 64) {
#pragma unroll
                for (int e = 0; e < 4; e++) low[m + e] = y[e];
            }
            if (vout) {
#pragma unroll
                for (int e = 0; e < 4; e++) vout[m + e] = (int16_t)y[e];
            }
        }
    }
}

// Reciprocal of the centered element Bin (LDS, p entries) in R/M, M = q
// (R/q, residues as two 7-bit limbs) or M = 3 (R/3, one limb), by jump
// divsteps.  Writes the centered reciprocal to OUT (LDS, may alias Bin).
// Returns 1 iff Bin is a unit (on wave 0).
//
// COOP = false: one wave (wave 0, nw = 1) does everything; other waves of
// the block need not take part.  COOP = true: all nw waves of the block call
// it (block barriers): wave 0 runs each jump's inner steps, then the jump's
// four output products (f', g', v', r') are dealt to the waves, output o to
// wave o mod nw, so that they run side by side.
template <int P, int M, typename T, bool COOP>
__device__ int recip_jump_block(const T* Bin, T* OUT, JumpLds<P>& L, int wave, int nw) {
    using S = JumpShape<P>;
    constexpr int Q = M;
    const int lane = lane_id();
    auto sync = [&]() {
        if constexpr (COOP) __syncthreads();
        else wave_sync();
    };
    // both Hankel sets and the Toeplitz arrays start zeroed
    {
        uint32_t* z = (uint32_t*)&L.H[0][0][0][0];
        for (int i = lane + 64 * wave; i < 2 * 4 * 2 * S::HLEN / 4; i += 64 * nw) z[i] = 0u;
        uint32_t* zt = (uint32_t*)&L.T[0][0][0];
        for (int i = lane + 64 * wave; i < 4 * 2 * kJumpTLen / 4; i += 64 * nw) zt[i] = 0u;
    }
    sync();
    // set 0: f = 1 - x^(p-1) - x^p, g = Bin reversed, v = 0, r = 1
    if (wave == 0) {
        for (int m = 4 * lane; m <= P; m += 256) {
            int32_t fx[4], gx[4], rx[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = m + e;
                fx[e] = (i == 0) ? 1 : ((i == P - 1 || i == P) ? -1 : 0);
                gx[e] = (i < P) ? (int32_t)Bin[P - 1 - i] : 0;
                rx[e] = (i == 0) ? 1 : 0;
            }
            jump_put4(L.H[0][0][0] + kJumpHOff, L.H[0][0][1] + kJumpHOff, m, fx);
            jump_put4(L.H[0][1][0] + kJumpHOff, L.H[0][1][1] + kJumpHOff, m, gx);
            jump_put4(L.H[0][3][0] + kJumpHOff, L.H[0][3][1] + kJumpHOff, m, rx);
        }
        L.low[0][lane] = (lane == 0) ? 1 : 0;
        L.low[1][lane] = (lane < P) ? (int32_t)Bin[P - 1 - lane] : 0;
    }
    sync();

    int32_t delta = 1, fend = 1;
    constexpr int NSTEP = 2 * P - 1;
#pragma unroll 1
    for (int jmp = 0; jmp < S::NJUMP; jmp++) {
        const int cur = jmp & 1, nxt = cur ^ 1;
        const int n = min(kJumpN, NSTEP - jmp * kJumpN);
        int32_t F = 0;
        if (wave == 0) {
            // 1. n divsteps on the low 64 coefficients, building U
            F = L.low[0][lane];
            int32_t G = L.low[1][lane];
            int32_t u00 = (lane == 0) ? 1 : 0, u01 = 0, u10 = 0, u11 = (lane == 0) ? 1 : 0;
            // n is a multiple of 3 (2p - 1 is for every parameter set): three
            // steps per trip, so that the updated registers are renamed, not moved
#pragma unroll 1
            for (int j = 0; j < n; j += 3) {
#pragma unroll
            for (int jj = 0; jj < 3; jj++) {
                const int32_t f0 = __builtin_amdgcn_readfirstlane(F);
                const int32_t g0 = __builtin_amdgcn_readfirstlane(G);
                const int32_t sw = -((int32_t)(delta > 0) & (int32_t)(freeze<Q>(g0) != 0));
                delta = bsel(sw, -delta, delta) + 1;
                const int32_t ng0 = -g0;
                const int32_t ng = reduce_rough<Q>(mul24(ng0, F) + mul24(f0, G));
                const int32_t n10 = reduce_rough<Q>(mul24(ng0, u00) + mul24(f0, u10));
                const int32_t n11 = reduce_rough<Q>(mul24(ng0, u01) + mul24(f0, u11));
                F = bsel(sw, G, F);
                const int32_t r0a = bsel(sw, u10, u00), r0b = bsel(sw, u11, u01);
                G = from_next_lane(ng);
                u00 = from_prev_lane(r0a);
                u01 = from_prev_lane(r0b);
                u10 = n10;
                u11 = n11;
            }
            }
            // 2. U's limbs as reversed Toeplitz bytes (coefficients above n are zero)
            const int32_t ue[4] = {freeze<Q>(u00), freeze<Q>(u01), freeze<Q>(u10), freeze<Q>(u11)};
#pragma unroll
            for (int k = 0; k < 4; k++) {
                uint32_t l, h;
                split_limb(ue[k], l, h);
                L.T[k][0][kJumpZ0 - lane] = (uint8_t)l;
                L.T[k][1][kJumpZ0 - lane] = (uint8_t)h;
            }
        }
        sync();
        // 3. apply U: f', g' shifted down by n (= 48, a multiple of 4, so
        // the shifted outputs stay dword-aligned); v', r' as they are.  The
        // last jump (n = (2p-1) mod 48 steps, any residue mod 4) needs only
        // v' and the constant term of f', which the inner steps hold exactly
        // (lane 0 of F on wave 0: its low 64 - n coefficients are f''s).
        uint8_t(*Hc)[2][S::HLEN] = L.H[cur];
        uint8_t(*Hn)[2][S::HLEN] = L.H[nxt];
        if (jmp + 1 < S::NJUMP) {
            if (0 % nw == wave)
                jump_output<P, M>(L, 0, 1, Hc[0][0], Hc[0][1], Hc[1][0], Hc[1][1], kJumpN, Hn[0][0], Hn[0][1],
                                  L.low[0], nullptr);
            if (1 % nw == wave)
                jump_output<P, M>(L, 2, 3, Hc[0][0], Hc[0][1], Hc[1][0], Hc[1][1], kJumpN, Hn[1][0], Hn[1][1],
                                  L.low[1], nullptr);
            if (2 % nw == wave)
                jump_output<P, M>(L, 0, 1, Hc[2][0], Hc[2][1], Hc[3][0], Hc[3][1], 0, Hn[2][0], Hn[2][1], nullptr,
                                  nullptr);
            if (3 % nw == wave)
                jump_output<P, M>(L, 2, 3, Hc[2][0], Hc[2][1], Hc[3][0], Hc[3][1], 0, Hn[3][0], Hn[3][1], nullptr,
                                  nullptr);
        } else {
            if (2 % nw == wave)
                jump_output<P, M>(L, 0, 1, Hc[2][0], Hc[2][1], Hc[3][0], Hc[3][1], 0, Hn[2][0], Hn[2][1], nullptr,
                                  L.v);
            if (wave == 0) fend = __builtin_amdgcn_readfirstlane(F);
        }
        sync();
    }
    if (wave != 0) return 0;
    // f0^-1 by Fermat's little theorem (uniform scalar work)
    const int32_t f0 = freeze<Q>(fend);
    int32_t inv = 1, base = f0;
#pragma unroll
    for (int e = Q - 2; e > 0; e >>= 1) {
        if (e & 1) inv = freeze<Q>(inv * base);
        base = freeze<Q>(base * base);
    }
    int32_t res[ceil_div(P, 64)];
#pragma unroll
    for (int k = 0; k < ceil_div(P, 64); k++) {
        const int i = lane + 64 * k;
        res[k] = (i < P) ? freeze<Q>(mul24(inv, (int32_t)L.v[P - i])) : 0;
    }
    wave_sync();   // OUT may alias Bin, which no later step reads
#pragma unroll
    for (int k = 0; k < ceil_div(P, 64); k++) {
        const int i = lane + 64 * k;
        if (i < P) OUT[i] = (T)res[k];
    }
    wave_sync();
    return delta == 0;
}

// One wave alone (see recip_jump_block).
template <int P, int M = Param<P>::q, typename T = int16_t>
__device__ int recip_jump_wave(const T* Bin, T* OUT, JumpLds<P>& L) {
    return recip_jump_block<P, M, T, false>(Bin, OUT, L, 0, 1);
}

}  // namespace ntrup
