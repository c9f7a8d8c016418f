// Arithmetic in R/q = (Z/q)[x]/(x^p - x - 1) on one 64-lane wave: the product
// engine used by Montgomery's batch inversion and by h = g/(3f), and the
// constant-time divstep reciprocal used once per Montgomery group.
//
// Product.  The paper's own R/q multiplier (Section 3.3) is an NTT design for
// Haswell; here the product is an exact int32 Toeplitz product for 64-wide
// SIMD.  For c = a*b mod x^p - x - 1 (Section 2.1), the schoolbook
// convolution conv_k = sum_j a_j b_{k-j} folds by x^p = x + 1 as
//   c_i = conv_i + conv_{i+p} + [i >= 1] conv_{i+p-1},
// so with E_d = b_d + b_{d+p} + b_{d+p-1} (b_m = 0 outside [0, p)),
//   c_i = sum_j a_j E_{i-j}            for 1 <= i < p,
//   c_0 = sum_j a_j E_{-j} - conv_{p-1}.
// Every output is one length-p dot product of a with a window of E: a lane
// owns R consecutive outputs and slides a register window over E (in LDS)
// while a_j is broadcast from LDS -- exactly p*R multiply-adds per lane, no
// triangular waste, no divergence.
//
// Exactness: operands are centered residues; products are accumulated in
// int32 and Barrett-reduced every mac_chunk<q>() terms when both operands are
// big; a small operand (|a_j| <= 3) never needs an intermediate reduction.
//
// Reciprocal.  Constant-time divsteps (the Bernstein-Yang algorithm the
// paper cites in Section 3.1) over F_q on (f, g) = (reversed x^p - x - 1,
// reversed a), 2p-1 steps, delta = 0 at the end iff a is a unit, and then
// 1/a has coefficient i equal to f(0)^-1 v[p - i].  Coefficients are spread
// over the wave in blocks of RI per lane; the per-step shifts g/x and x*v are
// register renamings plus one DPP lane shift each.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_params.h"

namespace ntrup {

template <int P>
struct RqShape {
    static constexpr int Q = Param<P>::q;
    static constexpr int R = ceil_div(P, 64);             // product outputs per lane
    static constexpr int NCH = ceil_div(P, R);            // chunks of R terms
    static constexpr int JP = NCH * R;                    // padded broadcast length
    static constexpr int EOFF = ceil_div(JP - 1, 4) * 4;  // E index of d = 0
    static constexpr int ELEN = EOFF + 64 * R;            // d in [-EOFF, 64R)
    static constexpr int RI = ceil_div(P + 1, 64);        // divstep coefficients per lane
    static constexpr int CH = mac_chunk<Q>() / R;         // chunks between reductions
    static_assert(CH >= 1, "chunk too long for exact int32 accumulation");
    static_assert(64 * R >= P && 64 * RI >= P + 1, "wave covers the ring");
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Select without a branch: mask is all-ones or all-zeros.
__device__ __forceinline__ int32_t bsel(int32_t mask, int32_t a, int32_t b) {
    return (a & mask) | (b & ~mask);
}

// Lane l receives lane l+1's value (lane 63 receives 0) / lane l-1's value
// (lane 0 receives 0): DPP wave shifts, one VALU op each.
__device__ __forceinline__ int32_t from_next_lane(int32_t x) {
    return __builtin_amdgcn_update_dpp(0, x, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
}
__device__ __forceinline__ int32_t from_prev_lane(int32_t x) {
    return __builtin_amdgcn_update_dpp(0, x, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}

// E_d = b_d + b_{d+p} + b_{d+p-1} for d in [-(p-1), p-1], centered; 0 elsewhere.
template <int P>
__device__ __forceinline__ void build_E(const int32_t* B, int32_t* E) {
    using S = RqShape<P>;
    for (int idx = lane_id(); idx < S::ELEN; idx += 64) {
        const int d = idx - S::EOFF;
        int32_t v = 0;
        if (d > -P && d < P) {
            if (d >= 0) v += B[d];
            if (d < 0) v += B[d + P];
            if (d <= 0) v += B[d + P - 1];
        }
        E[idx] = freeze<S::Q>(v);
    }
}

// acc[t] = c_{R*lane + t} of A * B, centered, where E = build_E(B).  A has JP
// entries (zero beyond p).  BIG = false requires |A_j| <= 3.
template <int P, bool BIG>
__device__ __forceinline__ void mul_wave(const int32_t* A, const int32_t* B, const int32_t* E,
                                         int32_t (&acc)[RqShape<P>::R]) {
    using S = RqShape<P>;
    constexpr int R = S::R;
    const int lane = lane_id();
    const int32_t* Eb = E + S::EOFF + R * lane;  // Eb[t - j]
    int32_t X[2 * R - 1];
#pragma unroll
    for (int u = 0; u < 2 * R - 1; u++) X[u] = Eb[u - (R - 1)];
#pragma unroll
    for (int t = 0; t < R; t++) acc[t] = 0;
#pragma unroll 1
    for (int c = 0; c < S::NCH; c++) {
        const int j0 = c * R;
        int32_t a[R];
#pragma unroll
        for (int jj = 0; jj < R; jj++) a[jj] = A[j0 + jj];
#pragma unroll
        for (int jj = 0; jj < R; jj++)
#pragma unroll
            for (int t = 0; t < R; t++) acc[t] = __mul24(a[jj], X[t - jj + R - 1]) + acc[t];
        if (BIG && (c + 1) % S::CH == 0) {
#pragma unroll
            for (int t = 0; t < R; t++) acc[t] = reduce_rough<S::Q>(acc[t]);
        }
#pragma unroll
        for (int u = 2 * R - 2; u >= R; u--) X[u] = X[u - R];
        if (c + 1 < S::NCH) {
#pragma unroll
            for (int u = 0; u < R; u++) X[u] = Eb[u - (R - 1) - j0 - R];
        }
    }
    // c_0 correction: conv_{p-1} = sum_j A_j B_{p-1-j}, summed over the wave
    int32_t part = 0;
    for (int j = lane; j < P; j += 64) part = __mul24(A[j], B[P - 1 - j]) + part;
    part = reduce_rough<S::Q>(part);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
#pragma unroll
    for (int t = 0; t < R; t++) {
        int32_t v = reduce_rough<S::Q>(acc[t]);
        if (t == 0) v -= (lane == 0) ? part : 0;
        acc[t] = freeze<S::Q>(v);
    }
}

// One divstep; s = step index modulo RI fixes the register naming:
// logical g[t] = G[(t+s) % RI], logical v[t] = V[(t-s) mod RI].
template <int P, int s>
__device__ __forceinline__ void rq_divstep(int32_t (&F)[RqShape<P>::RI], int32_t (&G)[RqShape<P>::RI],
                                          int32_t (&V)[RqShape<P>::RI], int32_t (&Rr)[RqShape<P>::RI],
                                          int32_t& delta) {
    using S = RqShape<P>;
    constexpr int RI = S::RI;
    constexpr int Q = S::Q;
    const int32_t f0 = __builtin_amdgcn_readfirstlane(F[0]);
    const int32_t g0 = __builtin_amdgcn_readfirstlane(G[s % RI]);
    const int32_t g0nz = (freeze<Q>(g0) != 0) ? 1 : 0;
    const int32_t sw = -((int32_t)(delta > 0) & g0nz);  // all-ones when swapping
    delta = bsel(sw, -delta, delta) + 1;
    const int32_t ng0 = -g0;
#pragma unroll
    for (int t = 0; t < RI; t++) {
        int32_t& g = G[(t + s) % RI];
        int32_t& v = V[((t - s) % RI + RI) % RI];
        const int32_t f = F[t], r = Rr[t];
        const int32_t ng = reduce_rough<Q>(__mul24(ng0, f) + __mul24(f0, g));
        const int32_t nr = reduce_rough<Q>(__mul24(ng0, v) + __mul24(f0, r));
        F[t] = bsel(sw, g, f);
        const int32_t nv = bsel(sw, r, v);
        g = ng;
        Rr[t] = nr;
        v = nv;
    }
    G[s % RI] = from_next_lane(G[s % RI]);
    V[(RI - 1 - s % RI + RI) % RI] = from_prev_lane(V[(RI - 1 - s % RI + RI) % RI]);
}

template <int P, int... Ss>
__device__ __forceinline__ void rq_divsteps_seq(int32_t (&F)[RqShape<P>::RI], int32_t (&G)[RqShape<P>::RI],
                                                int32_t (&V)[RqShape<P>::RI], int32_t (&Rr)[RqShape<P>::RI],
                                                int32_t& delta, std::integer_sequence<int, Ss...>) {
    (rq_divstep<P, Ss>(F, G, V, Rr, delta), ...);
}

// Reciprocal of the centered element Bin (LDS, p entries) in R/q.  Writes
// the centered reciprocal to OUT (LDS, may alias Bin) using STG (LDS, at
// least 64*RI entries) as staging.  Returns 1 iff Bin is a unit.
template <int P>
__device__ int recip_wave(const int32_t* Bin, int32_t* OUT, int32_t* STG) {
    using S = RqShape<P>;
    constexpr int RI = S::RI;
    constexpr int Q = S::Q;
    const int lane = lane_id();
    int32_t F[RI], G[RI], V[RI], Rr[RI];
#pragma unroll
    for (int t = 0; t < RI; t++) {
        const int i = RI * lane + t;
        F[t] = (i == 0) ? 1 : ((i == P - 1 || i == P) ? -1 : 0);
        G[t] = (i < P) ? Bin[P - 1 - i] : 0;
        V[t] = 0;
        Rr[t] = (i == 0) ? 1 : 0;
    }
    int32_t delta = 1;
    constexpr int NSTEP = 2 * P - 1;
#pragma unroll 1
    for (int blk = 0; blk < NSTEP / RI; blk++)
        rq_divsteps_seq<P>(F, G, V, Rr, delta, std::make_integer_sequence<int, RI>{});
    rq_divsteps_seq<P>(F, G, V, Rr, delta, std::make_integer_sequence<int, NSTEP % RI>{});
    constexpr int SR = NSTEP % RI;  // final naming offset of V
    // f(0)^-1 by Fermat's little theorem (uniform scalar work)
    const int32_t f0 = freeze<Q>(__builtin_amdgcn_readfirstlane(F[0]));
    int32_t inv = 1, base = f0;
#pragma unroll
    for (int e = Q - 2; e > 0; e >>= 1) {
        if (e & 1) inv = freeze<Q>(inv * base);
        base = freeze<Q>(base * base);
    }
#pragma unroll
    for (int t = 0; t < RI; t++) STG[RI * lane + t] = freeze<Q>(__mul24(inv, V[((t - SR) % RI + RI) % RI]));
    __syncthreads();
    for (int i = lane; i < P; i += 64) OUT[i] = STG[P - i];
    __syncthreads();
    return delta == 0;
}

}  // namespace ntrup
