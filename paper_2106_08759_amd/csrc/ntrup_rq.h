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
    static constexpr int M = ceil_div(R, 2);              // coefficient pairs per chunk
    static constexpr int NPAIR = ceil_div(P, 2);          // pairs of the broadcast operand
    static constexpr int NCH = ceil_div(NPAIR, M);        // chunks
    static constexpr int JP = 2 * NCH * M;                // padded broadcast length (int16)
    // packed-window index of d = 0: >= JP - 2 + 2M (the last chunk's look-ahead
    // loads stay inside the window), and = 2M - 2 (mod 4) so that the window
    // loads of lanes with R = 0 (mod 4) are 16-byte aligned
    static constexpr int POFF = (JP - 2 + 2 * M) + ((2 * M - 2 - (JP - 2 + 2 * M)) % 4 + 4) % 4;
    static constexpr int JPA = JP + 2 * M;                // broadcast array length incl. look-ahead
    static constexpr int PLEN = POFF + 64 * R;            // d in [-POFF, 64R)
    static constexpr int XW = R + 2 * M - 2;              // live window length
    static constexpr int NPH = 3;                         // window phases (chunks per cycle)
    static constexpr int XB = NPH * 2 * M;                // circular window registers
    static constexpr int RI = ceil_div(P + 1, 64);        // divstep coefficients per lane
    static constexpr int CH = mac_chunk<Q>() / (2 * M);   // chunks between reductions
    static_assert(CH >= 1, "chunk too long for exact int32 accumulation");
    static_assert(XW + 2 * M <= XB, "look-ahead slots never overlap the live window");
    static_assert(64 * R >= P && 64 * RI >= P + 1, "wave covers the ring");
    static_assert(PLEN >= 64 * RI, "packed window doubles as divstep staging");
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Orders the LDS traffic of one wave (lanes exchanging data through LDS):
// the LDS executes a wave's instructions in order, so a compiler fence and a
// wait for the wave's own outstanding LDS operations suffice -- no workgroup
// barrier, and global loads in flight stay in flight.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unconstrained
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

typedef short short2_t __attribute__((ext_vector_type(2)));

// a.lo * b.lo + a.hi * b.hi + c on signed 16-bit halves, exact in int32
// (v_dot2_i32_i16, two multiply-adds per lane per instruction).
__device__ __forceinline__ int32_t dot2(int32_t a, int32_t b, int32_t c) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, a), __builtin_bit_cast(short2_t, b), c, false);
}

// E_d = b_d + b_{d+p} + b_{d+p-1}, centered, for d in [-(p-1), p-1]; 0 elsewhere.
template <int P>
__device__ __forceinline__ int32_t e_coef(const int16_t* B, int d) {
    int32_t v = 0;
    if (d > -P && d < P) {
        if (d >= 0) v += B[d];
        if (d < 0) v += B[d + P];
        if (d <= 0) v += B[d + P - 1];
    }
    return freeze<Param<P>::q>(v);
}

// Packed Toeplitz window of the big operand B (int16, p entries, centered):
// Pk[POFF + d] = (E_d, E_{d-1}) as two int16 halves (low = E_d).  Two passes
// through Et (int16, PLEN + 1 entries: Et[i] = E_{i - POFF - 1}).
template <int P>
__device__ __forceinline__ void build_window(const int16_t* B, int16_t* Et, int32_t* Pk) {
    using S = RqShape<P>;
    for (int i = lane_id(); i <= S::PLEN; i += 64) Et[i] = (int16_t)e_coef<P>(B, i - S::POFF - 1);
    __syncthreads();
    for (int i = lane_id(); i < S::PLEN; i += 64)
        Pk[i] = (int32_t)((uint32_t)(uint16_t)Et[i + 1] | ((uint32_t)(uint16_t)Et[i] << 16));
}

// One chunk of M coefficient pairs at window phase PH.  The live window slot u
// of phase PH sits in register Xp[(u + off(PH)) % XB], off(PH) = -2M*PH mod XB,
// so sliding by 2M between chunks is a renaming; the 2M new slots of the next
// chunk are disjoint from the live ones and are loaded here (the look-ahead
// after the last chunk reads the zero padding below d = -(JP-2)).
template <int P, int PH>
__device__ __forceinline__ constexpr int win_off() {
    return ((RqShape<P>::NPH - PH) % RqShape<P>::NPH) * 2 * RqShape<P>::M;
}

template <int P, int NA, int PH>
__device__ __forceinline__ void mul_chunk(int32_t (&Xp)[RqShape<P>::XB], const int32_t (&a)[NA][RqShape<P>::M],
                                          int32_t (&acc)[NA][RqShape<P>::R], const int32_t* Pb, int m0) {
    using S = RqShape<P>;
    constexpr int R = S::R, M = S::M, XB = S::XB;
    constexpr int OFF = win_off<P, PH>(), NOFF = win_off<P, (PH + 1) % S::NPH>();
    // keep each chunk's look-ahead loads inside the chunk: hoisted further they
    // would land in registers that an earlier chunk still reads
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 2 * M; u++) Xp[(u + NOFF) % XB] = Pb[u - 2 * (m0 + M)];
#pragma unroll
    for (int mm = 0; mm < M; mm++)
#pragma unroll
        for (int k = 0; k < NA; k++)
#pragma unroll
            for (int t = 0; t < R; t++)
                acc[k][t] = dot2(a[k][mm], Xp[(t - 2 * mm + 2 * M - 2 + OFF) % XB], acc[k][t]);
}

template <int P, int NA>
__device__ __forceinline__ void load_pairs(int32_t (&a)[NA][RqShape<P>::M], const int32_t* const (&Ap)[2], int m0) {
#pragma unroll
    for (int k = 0; k < NA; k++)
#pragma unroll
        for (int mm = 0; mm < RqShape<P>::M; mm++) a[k][mm] = Ap[k][m0 + mm];
}

template <int P, int NA, bool BIG0, bool BIG1>
__device__ __forceinline__ void reduce_acc(int32_t (&acc)[NA][RqShape<P>::R]) {
#pragma unroll
    for (int k = 0; k < NA; k++)
        if (k == 0 ? BIG0 : BIG1)
#pragma unroll
            for (int t = 0; t < RqShape<P>::R; t++) acc[k][t] = reduce_rough<RqShape<P>::Q>(acc[k][t]);
}

// NA products sharing the big operand B: acc[k][t] = c_{R*lane + t} of
// A_k * B, centered.  A_k are int16 arrays of JPA entries (zero from p to JP;
// the look-ahead tail beyond JP is read but never used) read as coefficient
// pairs; BIGk = false requires |A_k| <= 3 (no intermediate reduction needed).
// Pk = build_window(B).
template <int P, int NA, bool BIG0, bool BIG1>
__device__ __forceinline__ void mul_wave(const int16_t* A0, const int16_t* A1, const int16_t* B,
                                         const int32_t* Pk, int32_t (&acc)[NA][RqShape<P>::R]) {
    using S = RqShape<P>;
    constexpr int R = S::R, M = S::M, Q = S::Q;
    const int lane = lane_id();
    const int32_t* Pb = Pk + S::POFF + R * lane - (2 * M - 2);  // live slot u of chunk 0 = Pb[u]
    const int32_t* const Ap[2] = {(const int32_t*)A0, (const int32_t*)A1};
    int32_t Xp[S::XB];
#pragma unroll
    for (int u = 0; u < S::XW; u++) Xp[u] = Pb[u];
#pragma unroll
    for (int k = 0; k < NA; k++)
#pragma unroll
        for (int t = 0; t < R; t++) acc[k][t] = 0;
    int32_t a0[NA][M], a1[NA][M], a2[NA][M];  // broadcast pairs of the three phases
    load_pairs<P, NA>(a0, Ap, 0);
    // NIT iterations of three chunks, in segments of SEG iterations between
    // Barrett reductions (branch-free inner loop), then NCH % 3 chunks
    constexpr bool BIG = BIG0 || (NA > 1 && BIG1);
    constexpr int NIT = S::NCH / 3;
    constexpr int SEG = BIG ? (S::CH / 3 > 0 ? S::CH / 3 : 1) : (NIT > 0 ? NIT : 1);
    static_assert(!BIG || S::CH >= 3, "a reduction segment holds at least one iteration");
    int c = 0;
#pragma unroll 1
    for (int seg = 0; seg < NIT; seg += SEG) {
        const int end = min(seg + SEG, NIT);
#pragma unroll 1
        for (int it = seg; it < end; it++, c += 3) {
            load_pairs<P, NA>(a1, Ap, (c + 1) * M);
            mul_chunk<P, NA, 0>(Xp, a0, acc, Pb, c * M);
            load_pairs<P, NA>(a2, Ap, (c + 2) * M);
            mul_chunk<P, NA, 1>(Xp, a1, acc, Pb, (c + 1) * M);
            load_pairs<P, NA>(a0, Ap, (c + 3) * M);
            mul_chunk<P, NA, 2>(Xp, a2, acc, Pb, (c + 2) * M);
        }
        if (BIG) reduce_acc<P, NA, BIG0, BIG1>(acc);
    }
    if (S::NCH % 3 >= 1) {
        if (S::NCH % 3 == 2) load_pairs<P, NA>(a1, Ap, (c + 1) * M);
        mul_chunk<P, NA, 0>(Xp, a0, acc, Pb, c * M);
        if (S::NCH % 3 == 2) mul_chunk<P, NA, 1>(Xp, a1, acc, Pb, (c + 1) * M);
    }
    // c_0 correction: conv_{p-1} = sum_j A_j B_{p-1-j}, summed over the wave
    const int16_t* As[2] = {A0, A1};
#pragma unroll
    for (int k = 0; k < NA; k++) {
        int32_t part = 0;
        for (int j = lane; j < P; j += 64) part = mul24(As[k][j], B[P - 1 - j]) + part;
        part = reduce_rough<Q>(part);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
#pragma unroll
        for (int t = 0; t < R; t++) {
            int32_t v = reduce_rough<Q>(acc[k][t]);
            if (t == 0) v -= (lane == 0) ? part : 0;
            acc[k][t] = freeze<Q>(v);
        }
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
        const int32_t ng = reduce_rough<Q>(mul24(ng0, f) + mul24(f0, g));
        const int32_t nr = reduce_rough<Q>(mul24(ng0, v) + mul24(f0, r));
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

// Reciprocal of the centered element Bin (LDS, p int16 entries) in R/q.
// Writes the centered reciprocal to OUT (LDS, may alias Bin) using STG (LDS,
// at least 64*RI int32 entries) as staging.  Returns 1 iff Bin is a unit.
template <int P>
__device__ int recip_wave(const int16_t* Bin, int16_t* OUT, int32_t* STG) {
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
    for (int t = 0; t < RI; t++) STG[RI * lane + t] = freeze<Q>(mul24(inv, V[((t - SR) % RI + RI) % RI]));
    wave_sync();
    for (int i = lane; i < P; i += 64) OUT[i] = (int16_t)STG[P - i];
    wave_sync();
    return delta == 0;
}

}  // namespace ntrup
