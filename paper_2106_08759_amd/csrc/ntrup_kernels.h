// Kernels of the batched KeyGen pipeline (OpenSSLNTRU paper, Section 3.1,
// Algorithm 1 BatchKeyGen with the R/q reciprocals batched by Montgomery's
// trick of Section 2.2 and the R/3 reciprocal taken per key):
//
//   sample_short_kernel  f in Short, one wave per key (ChaCha20 + bitonic sort)
//   r3_kernel            g small, resampled until invertible; 1/g in R/3;
//                        one key per lane (or lane pair), bitsliced divsteps
//   group_kernel         per Montgomery group of G keys, one wave:
//                        prefix products b_i = a_i b_{i-1} of a_i = 3 f_i,
//                        one divstep reciprocal t_G = 1/b_G, back-substitution
//                        c_i = t_i b_{i-1}, t_{i-1} = t_i a_i, then
//                        h_i = g_i c_i and the encoded pk / sk bytes
//
// Workspace layouts (n keys):
//   f_rows  int8   [n][p]         f, centered
//   gbits   uint32 [WN][2][n]     accepted g, bitsliced (plane 0: c != 0,
//   ibits   uint32 [WN][2][n]     1/g          plane 1: c == -1), natural order
//   bscr    int16  [n][p]         prefix products of each group
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "ntrup_chacha.h"
#include "ntrup_jump.h"
#include "ntrup_mfma.h"
#include "ntrup_params.h"
#include "ntrup_r3.h"
#include "ntrup_rq.h"

namespace ntrup {

// ----------------------------------------------------------------------------
// Short sampler: L_i = (r_i & ~3) | v_i, v_i = 2(r_i & 1) for i < w, else 1;
// sort L ascending as u32; f_i = (L_i & 3) - 1.  The sort key is the top 30
// bits of each word, so the w nonzeros land on uniformly random positions
// with independent random signs (the definition of Short, Section 2.1).
// ----------------------------------------------------------------------------
template <int P>
struct ShortShape {
    static constexpr int NS = P <= 1024 ? 1024 : 2048;  // sorting network size
    static constexpr int EPL = NS / 64;                 // elements per lane
};

// med3(a, b, 0) = min(a, b) and med3(a, b, ~0) = max(a, b) for unsigned
// words: one v_med3_u32 does a compare-exchange half whose direction is a
// per-lane value.
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Bitonic sort of 64*EPL words held across the wave, ascending.  Branch-free:
// every compare-exchange half is a med3 against 0 (keep the smaller) or ~0
// (keep the larger).  A slot's rank in the network is e + EPL sort_lane(lane)
// (slot e of lane `lane`): the network's lane bits are a permutation of the
// physical ones, chosen so that the lane exchange that costs the most (lane
// ^ 4: two row shifts and a select) carries the network's highest lane bit,
// which one stage uses, and every other lane bit costs one instruction per
// word and stage:
//   network bit 0, 1, 2  <->  lane ^ 1, ^ 2 (quad permutes), ^ 8 (row rotate):
//     the partner's word by one DPP move, then one med3;
//   network bit 3, 4     <->  lane ^ 16, ^ 32: v_permlane16_swap /
//     v_permlane32_swap of two slots (e, e+1) exchanges the rows, so that
//     each lane holds both words of one pair (the lower row's in the first
//     result, the upper row's in the second, whichever slot they came from),
//     two med3, and the same swap again (an involution) puts them back;
//   network bit 5        <->  lane ^ 4.
// The input order is free (any order sorts); ranks are used on output.
__device__ __forceinline__ int sort_lane(int lane) {
    return (lane & 3) | (((lane >> 3) & 1) << 2) | (((lane >> 4) & 3) << 3) | (((lane >> 2) & 1) << 5);
}

// The value of lane lane ^ lj, lj in {1, 2, 4, 8}, by DPP: quad permutes for
// 1 and 2, row shifts for 4 (row_shl:4 gives lane i+4, row_shr:4 lane i-4),
// a row rotate for 8.
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, int lj, int lane) {
    switch (lj) {
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);   // quad [1,0,3,2]
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);   // quad [2,3,0,1]
        case 4: {
            const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x104, 0xF, 0xF, true);   // row_shl:4
            const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
            return (lane & 4) ? dn : up;
        }
        default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_rotate:8
    }
}

// Rows exchanged between two slots: v_permlane16_swap (R = 16) or
// v_permlane32_swap (R = 32) of (a, b), in place.
template <int R>
__device__ __forceinline__ void row_swap(uint32_t& a, uint32_t& b) {
    if constexpr (R == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = (uint32_t)r[0];
        b = (uint32_t)r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = (uint32_t)r[0];
        b = (uint32_t)r[1];
    }
}

// One stage (merge size K, partner distance J) of the network; K and J are
// template arguments, so that every slot index is a constant (a loop over
// stages left to the unroller was expanded only in part for 32 slots per
// lane, with indexed register access in its place).
template <int EPL, int K, int J>
__device__ __forceinline__ void bitonic_stage(uint32_t (&L)[EPL], int lane, int i0) {
    if constexpr (J >= EPL) {
        // network lane bit JB; the direction depends on the lane only
        constexpr int JB = __builtin_ctz(J / EPL);
        const uint32_t c = ((i0 & K) == 0) ? 0u : 0xFFFFFFFFu;   // 0: ascending pair
        if constexpr (JB == 3 || JB == 4) {
#pragma unroll
            for (int e = 0; e < EPL; e += 2) {
                uint32_t lo = L[e], hi = L[e + 1];
                row_swap<JB == 3 ? 16 : 32>(lo, hi);
                const uint32_t x = med3_u32(lo, hi, c), y = med3_u32(lo, hi, ~c);
                lo = x;
                hi = y;
                row_swap<JB == 3 ? 16 : 32>(lo, hi);
                L[e] = lo;
                L[e + 1] = hi;
            }
        } else {
            // partner in lane ^ LJ, same slot: keep the smaller iff this lane
            // is the lower side of an ascending pair
            constexpr int LJ = JB == 5 ? 4 : (JB == 2 ? 8 : 1 << JB);
            const uint32_t cc = ((i0 & J) == 0) ? c : ~c;
#pragma unroll
            for (int e = 0; e < EPL; e++) {
                const uint32_t o = lane_xor(L[e], LJ, lane);
                L[e] = med3_u32(L[e], o, cc);
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < EPL; e++) {
            if ((e & J) == 0) {
                const int e2 = e | J;
                const bool up = ((i0 + e) & K) == 0;
                const uint32_t c = up ? 0u : 0xFFFFFFFFu;
                const uint32_t x = L[e], y = L[e2];
                L[e] = med3_u32(x, y, c);
                L[e2] = med3_u32(x, y, ~c);
            }
        }
    }
}

// The stages J = J0, J0/2, .., 1 of the merge of size K.
template <int EPL, int K, int J>
__device__ __forceinline__ void bitonic_merge(uint32_t (&L)[EPL], int lane, int i0) {
    if constexpr (J > 0) {
        bitonic_stage<EPL, K, J>(L, lane, i0);
        bitonic_merge<EPL, K, J / 2>(L, lane, i0);
    }
}

// The merges of size K, 2K, .., 64 EPL.
template <int EPL, int K>
__device__ __forceinline__ void bitonic_merges_from(uint32_t (&L)[EPL], int lane, int i0) {
    if constexpr (K <= 64 * EPL) {
        bitonic_merge<EPL, K, K / 2>(L, lane, i0);
        bitonic_merges_from<EPL, 2 * K>(L, lane, i0);
    }
}

template <int EPL>
__device__ __forceinline__ void bitonic_sort_wave(uint32_t (&L)[EPL], int lane) {
    static_assert(EPL % 2 == 0, "row swaps pair the slots");
    const int i0 = sort_lane(lane) * EPL;   // rank of slot 0
    bitonic_merges_from<EPL, 2>(L, lane, i0);
}

// f of one key (key index `index`), written to `row`; one wave.
template <int P>
__device__ __forceinline__ void sample_short_key(const Seed& seed, uint64_t index, int8_t* __restrict__ row) {
    constexpr int W = Param<P>::w;
    constexpr int EPL = ShortShape<P>::EPL;
    const int lane = lane_id();
    uint32_t L[EPL];
#pragma unroll
    for (int b = 0; b < EPL / 16; b++) {
        uint32_t r[16];
        chacha_block(seed, index, P, 0, (uint32_t)(lane * (EPL / 16) + b), r);
#pragma unroll
        for (int e = 0; e < 16; e++) L[16 * b + e] = r[e];
    }
#pragma unroll
    for (int e = 0; e < EPL; e++) {
        const int i = lane * EPL + e;
        const uint32_t v = (i < W) ? 2u * (L[e] & 1u) : 1u;
        L[e] = (i < P) ? ((L[e] & ~3u) | v) : 0xFFFFFFFFu;
    }
    bitonic_sort_wave<EPL>(L, lane);
    const int i0 = sort_lane(lane) * EPL;
#pragma unroll
    for (int e = 0; e < EPL; e++) {
        const int i = i0 + e;
        if (i < P) row[i] = (int8_t)((int)(L[e] & 3u) - 1);
    }
}

// An element of Short (KeyGen's f: stream 0; encapsulation's r: its own
// stream) for four keys per 256-thread block.  A key needs only NB = ceil(p/16)
// ChaCha20 blocks (48 at p = 761, against the 64 that one block per lane of a
// sorting wave would compute), so the block's threads compute the 4 NB blocks
// first -- one per thread, the threads past them (a whole wave at
// p = 761) skip -- and pass the words through LDS to the sorting wave of
// their key.  LDS rows are EPL + 1 words per lane slot, so that both the
// writes (one ChaCha block per thread) and the reads (one slot per lane) hit
// 64 different banks.  The sorted coefficients go back through LDS, so that
// the four keys' rows (one contiguous range of 4p bytes) are stored as whole
// words by all threads instead of one scattered byte per lane and slot.
template <int P>
__global__ __launch_bounds__(256) void sample_short_kernel(Seed seed, uint64_t first_index, int n, int stream,
                                                           int8_t* __restrict__ f_rows) {
    constexpr int W = Param<P>::w;
    constexpr int EPL = ShortShape<P>::EPL;
    constexpr int SL = EPL + 1;                 // words per lane slot in LDS
    constexpr int NB = ceil_div(P, 16);         // ChaCha20 blocks per key
    constexpr int KPB = 4;                      // keys per workgroup (one wave each)
    static_assert(16 * NB <= 64 * EPL && EPL % 16 == 0, "a key's words fit its sorting network");
    __shared__ __attribute__((aligned(16))) uint32_t words[KPB][64 * SL];
    // then the sorted rows of the workgroup's keys (stride RS bytes, over the
    // words once every wave has read its own), written out as the one
    // contiguous byte range [key0 P, (key0 + KPB) P) of f_rows
    constexpr int RS = 64 * EPL;
    static_assert(KPB * RS <= (int)sizeof(words), "the rows fit over the words");
    uint8_t (*rows)[RS] = (uint8_t (*)[RS])&words[0][0];
    // KeyGen's f heads the launch stream's chain of kernels while the R/3
    // stage's sampler runs beside it: its waves take issue priority
    __builtin_amdgcn_s_setprio(2);
    const int key0 = blockIdx.x * KPB;
    const int tid = threadIdx.x;
    for (int b = tid; b < KPB * NB; b += 64 * KPB) {
        const int k = b / NB, blk = b - k * NB;
        if (key0 + k < n) {
            uint32_t r[16];
            chacha_block(seed, first_index + (uint64_t)(key0 + k), P, stream, (uint32_t)blk, r);
            // element i = 16 blk + e sits in lane slot i / EPL at offset i % EPL
            uint32_t* dst = &words[k][(16 * blk / EPL) * SL + (16 * blk) % EPL];
#pragma unroll
            for (int e = 0; e < 16; e++) dst[e] = r[e];
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int key = key0 + wave;
    uint32_t L[EPL];
#pragma unroll
    for (int e = 0; e < EPL; e++) {
        const int i = lane * EPL + e;
        const uint32_t x = (i < P) ? words[wave][lane * SL + e] : 0u;
        const uint32_t v = (i < W) ? 2u * (x & 1u) : 1u;
        L[e] = (i < P) ? ((x & ~3u) | v) : 0xFFFFFFFFu;
    }
    __syncthreads();
    if (key < n) {  // whole wave
        bitonic_sort_wave<EPL>(L, lane);
        // coefficient L & 3 - 1 as a byte, four to a word, ranks i0 .. i0+EPL-1
        const int i0 = sort_lane(lane) * EPL;
#pragma unroll
        for (int q = 0; q < EPL / 16; q++) {
            uint32_t w4[4];
#pragma unroll
            for (int d = 0; d < 4; d++) {
                uint32_t x = 0;
#pragma unroll
                for (int t = 0; t < 4; t++) x |= (((L[16 * q + 4 * d + t] & 3u) - 1u) & 0xFFu) << (8 * t);
                w4[d] = x;
            }
            *(uint4*)&rows[wave][i0 + 16 * q] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
        }
    }
    __syncthreads();
    // P KPB is a multiple of 4 (P = 1 mod 4, KPB = 4): on a word-aligned
    // f_rows the range starts and ends on a word.  Words past the last key's
    // end (a partial last workgroup) and every word of an unaligned f_rows
    // are written byte by byte.
    constexpr int NW = P * KPB / 4;
    static_assert(P * KPB % 4 == 0, "the workgroup's byte range is whole words");
    const int live = min(KPB, n - key0) * P;   // bytes of this workgroup's keys
    const bool aligned = ((uintptr_t)f_rows & 3u) == 0;
    uint32_t* out = (uint32_t*)(f_rows + (size_t)key0 * P);
    for (int d = tid; d < NW; d += 64 * KPB) {
        uint32_t x = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int b = 4 * d + t, k = b / P;
            x |= (uint32_t)rows[k][b - k * P] << (8 * t);
        }
        if (aligned && 4 * d + 4 <= live) {
            out[d] = x;
        } else {
#pragma unroll
            for (int t = 0; t < 4; t++)
                if (4 * d + t < live) ((uint8_t*)out)[4 * d + t] = (uint8_t)(x >> (8 * t));
        }
    }
}

// ----------------------------------------------------------------------------
// Small sampler: g_i = floor(3 r_i / 2^32) - 1 from stream 1 + attempt.
// Natural-order bitsliced word k (coefficients 32k .. 32k+31).
// ----------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void sample_small_word(const Seed& seed, uint64_t index, int attempt, int k,
                                                  uint32_t& mw, uint32_t& sw) {
    mw = 0;
    sw = 0;
#pragma unroll
    for (int half = 0; half < 2; half++) {
        const int blk = 2 * k + half;
        if (16 * blk < P) {
            uint32_t r[16];
            chacha_block(seed, index, P, 1 + attempt, (uint32_t)blk, r);
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int i = 16 * blk + e;
                const uint32_t u = __umulhi(r[e], 3u);  // 0, 1, 2 -> -1, 0, 1
                const uint32_t live = (i < P) ? 1u : 0u;
                mw |= ((u != 1u) & live) << (16 * half + e);
                sw |= ((u == 0u) & live) << (16 * half + e);
            }
        }
    }
}

// ----------------------------------------------------------------------------
// R/3 stage.  Main pass: slot -> key.  Retry pass: keys from list_in.  Each
// round draws a fresh g for the keys not yet done; keys still pending after
// max_rounds go to list_out (wave-aggregated atomics), or, without list_out,
// count as exhausted.
// ----------------------------------------------------------------------------
struct R3Args {
    Seed seed;
    uint64_t first_index;
    int n;
    int max_rounds;
    int spec;               // attempts tried side by side per key (1, 2, 4 or 8)
    const int* list_in;     // null in the main pass
    const int* count_in;
    int* list_out;          // null: no further pass
    int* count_out;
    uint8_t* attempts;      // [n] g samples drawn
    uint32_t* gbits;        // [WN][2][n]
    uint32_t* ibits;        // [WN][2][n]
    int* err;               // |= 1 when a key exhausts kMaxAttempts
    const int8_t* g_in;     // test entry: explicit g rows [n][p], one round, no sampling
    int* kfinal;            // optional: kfinal[key / G] += 1 once a key's result is final
    int G;
};

// A wave holds 64/LPK lane groups; with spec = A, consecutive runs of A
// groups work on one key and try attempts base, base+1, ..., base+A-1 at
// once.  The key takes the lowest attempt whose g is a unit -- exactly the
// g a one-at-a-time resampling loop would accept -- so the outputs do not
// depend on A.  Keys whose A attempts all fail move on by A attempts.
template <int P, int LPK>
struct R3Lds {
    using S = R3Shape<P, LPK>;
    uint32_t nat[S::KPW][2][S::WT];   // natural-order g words of each lane group
    uint32_t vst[S::KPW][2][S::WT];   // divstep outputs, for the reversal
};

// One wave's keys (wave slot ws: keys or list entries ws * KPW/A ...); a
// wave-sized block (the barriers are wave barriers).
template <int P, int LPK>
__device__ __forceinline__ void r3_wave(const R3Args& args, int ws, R3Lds<P, LPK>& lds) {
    using S = R3Shape<P, LPK>;
    constexpr int W2 = S::W2;
    auto& nat = lds.nat;
    auto& vst = lds.vst;
    const int lane = lane_id();
    const int A = args.spec;
    const int gi = lane / LPK;            // lane group
    const int a = gi % A;                 // which of the key's side-by-side attempts
    const int h = lane & (LPK - 1);
    const int kw = gi / A;                // key slot in the wave
    const int slot = ws * (S::KPW / A) + kw;
    int key = -1, base = 0;
    if (args.list_in) {
        if (slot < *args.count_in) {
            key = args.list_in[slot];
            base = args.attempts[key];
        }
    } else if (slot < args.n) {
        key = slot;
    }
    if (__ballot(key >= 0) == 0) return;  // whole wave idle
    const uint64_t index = args.first_index + (uint64_t)(key < 0 ? 0 : key);
    bool done = key < 0;
    uint32_t* nm = nat[gi][0];
    uint32_t* ns = nat[gi][1];
    for (int round = 0; round < args.max_rounds; round++) {
        if (__all(done)) break;
        const int attempt = base + a;
        for (int k = h; k < S::WT; k += LPK) {
            uint32_t mw = 0, sw = 0;
            if (k < S::WN) {
                if (args.g_in) {
                    const int8_t* row = args.g_in + (size_t)(key < 0 ? 0 : key) * P;
#pragma unroll 4
                    for (int e = 0; e < 32; e++) {
                        const int i = 32 * k + e;
                        const int c = (i < P) ? row[i] : 0;
                        mw |= (uint32_t)(c != 0) << e;
                        sw |= (uint32_t)(c < 0) << e;
                    }
                } else {
                    sample_small_word<P>(args.seed, index, attempt < kMaxAttempts ? attempt : 0, k, mw, sw);
                }
            }
            nm[k] = mw;
            ns[k] = sw;
        }
        __syncthreads();
        uint32_t gm[W2], gs[W2], vm[W2], vs[W2];
#pragma unroll
        for (int k = 0; k < W2; k++) {
            gm[k] = load_reversed<P, LPK>(nm, h * W2 + k);
            gs[k] = load_reversed<P, LPK>(ns, h * W2 + k);
        }
        const int delta = r3_divsteps<P, LPK>(gm, gs, vm, vs, h);
#pragma unroll
        for (int k = 0; k < W2; k++) {
            vst[gi][0][h * W2 + k] = vm[k];
            vst[gi][1][h * W2 + k] = vs[k];
        }
        __syncthreads();
        // lowest successful attempt of each key, from the group leaders' votes
        const unsigned long long votes = __ballot(h == 0 && !done && delta == 0 && attempt < kMaxAttempts);
        uint32_t mine = 0;
        for (int b = 0; b < A; b++) mine |= (uint32_t)((votes >> ((kw * A + b) * LPK)) & 1ull) << b;
        if (!done && mine) {
            const int win = __builtin_ctz(mine);
            if (a == win) {
                for (int k = h; k < S::WN; k += LPK) {
                    const size_t n = (size_t)args.n;
                    args.gbits[(size_t)(2 * k) * n + key] = nm[k];
                    args.gbits[(size_t)(2 * k + 1) * n + key] = ns[k] & nm[k];
                    args.ibits[(size_t)(2 * k) * n + key] = load_output<P, LPK>(vst[gi][0], k);
                    args.ibits[(size_t)(2 * k + 1) * n + key] = load_output<P, LPK>(vst[gi][1], k);
                }
                if (h == 0) args.attempts[key] = (uint8_t)(base + win + 1);
            }
            done = true;
        } else if (!done) {
            base += A;
            if (base >= kMaxAttempts || args.g_in) {
                if (h == 0 && a == 0) {
                    args.attempts[key] = args.g_in ? (uint8_t)0 : (uint8_t)kMaxAttempts;
                    if (!args.g_in) atomicOr(args.err, 1);
                }
                done = true;
            }
        }
        __syncthreads();
    }
    const bool pend = !done && h == 0 && a == 0;
    if (args.list_out) {
        if (pend) args.attempts[key] = (uint8_t)base;
        const unsigned long long m = __ballot(pend);
        if (m) {
            int b0 = 0;
            if (lane == 0) b0 = atomicAdd(args.count_out, __popcll(m));
            b0 = __shfl(b0, 0);
            if (pend) args.list_out[b0 + __popcll(m & ((1ull << lane) - 1ull))] = key;
        }
    } else if (pend) {
        atomicOr(args.err, 1);
    }
    if (args.kfinal) {
        // every lane's outputs visible before the group counters move
        __threadfence();
        if (key >= 0 && done && h == 0 && a == 0) atomicAdd(&args.kfinal[key / args.G], 1);
    }
}

template <int P, int LPK>
__global__ __launch_bounds__(64) void r3_kernel(R3Args args) {
    __shared__ R3Lds<P, LPK> lds;
    r3_wave<P, LPK>(args, (int)blockIdx.x, lds);
}

// ----------------------------------------------------------------------------
// Montgomery group stage.
// ----------------------------------------------------------------------------
struct GroupArgs {
    int n;
    int G;
    const int8_t* f_rows;
    const uint32_t* gbits;
    const uint32_t* ibits;
    int16_t* bscr;
    uint8_t* pk;
    uint8_t* sk;
    int* err;               // |= 2 when a group product is not a unit
    const int16_t* a_in;    // batch-inverse entry: invert these rows (centered) ...
    int16_t* c_out;         // ... and write the reciprocals here
};

template <int P>
struct GroupLds {
    using S = RqShape<P>;
    __attribute__((aligned(16))) int16_t A0[S::JPA];  // broadcast operands
    __attribute__((aligned(16))) int16_t A1[S::JPA];
    __attribute__((aligned(16))) int16_t Bb[S::JP];   // big operands (natural order)
    __attribute__((aligned(16))) int16_t Cb[S::JP];
    __attribute__((aligned(16))) int32_t Pk[S::PLEN]; // packed Toeplitz window / staging
    __attribute__((aligned(16))) int16_t Et[S::PLEN + 2];  // window build scratch
};

template <int P>
__device__ __forceinline__ void store_lds(const int32_t (&acc)[RqShape<P>::R], int16_t* dst) {
    constexpr int R = RqShape<P>::R;
    const int lane = lane_id();
#pragma unroll
    for (int t = 0; t < R; t++)
        if (R * lane + t < P) dst[R * lane + t] = (int16_t)acc[t];
}

template <int P>
__device__ __forceinline__ void store_row(const int32_t (&acc)[RqShape<P>::R], int16_t* row) {
    constexpr int R = RqShape<P>::R;
    const int lane = lane_id();
#pragma unroll
    for (int t = 0; t < R; t++)
        if (R * lane + t < P) row[R * lane + t] = (int16_t)acc[t];
}

// dst[j] = 3 f_j (j < p), 0 up to JP
template <int P>
__device__ __forceinline__ void load_3f(const int8_t* row, int16_t* dst) {
    for (int j = lane_id(); j < RqShape<P>::JP; j += 64) dst[j] = (j < P) ? (int16_t)(3 * (int32_t)row[j]) : 0;
}

template <int P>
__device__ __forceinline__ void load_row16(const int16_t* row, int16_t* dst) {
    for (int j = lane_id(); j < RqShape<P>::JP; j += 64) dst[j] = (j < P) ? row[j] : 0;
}

// dst[j] = g_j from the bitsliced words of key `key`
template <int P>
__device__ __forceinline__ void load_g(const uint32_t* gbits, int n, int key, int16_t* dst) {
    constexpr int WN = ceil_div(P, 32);
    constexpr int JP = RqShape<P>::JP;
    const int lane = lane_id();
    for (int j = P + lane; j < JP; j += 64) dst[j] = 0;
    if (lane < WN) {
        const uint32_t m = gbits[(size_t)(2 * lane) * n + key];
        const uint32_t s = gbits[(size_t)(2 * lane + 1) * n + key];
#pragma unroll 8
        for (int e = 0; e < 32; e++) {
            const int j = 32 * lane + e;
            if (j < P) dst[j] = (int16_t)((int32_t)((m >> e) & 1u) * (1 - 2 * (int32_t)((s >> e) & 1u)));
        }
    }
}

// pk: h_i + (q-1)/2 as 13-bit little-endian fields; sk: f then 1/g as 2-bit
// fields c + 1, four per byte, least significant first.
template <int P>
__device__ __forceinline__ void encode_key(int key, const int16_t* H, uint8_t* pk_out, uint8_t* sk_out,
                                           const int8_t* f_rows, const uint32_t* ibits, int n) {
    constexpr int Q = Param<P>::q;
    constexpr int PKB = pk_bytes(P), SKH = sk_half_bytes(P);
    const int lane = lane_id();
    uint8_t* pk = pk_out + (size_t)key * PKB;
    for (int b = lane; b < PKB; b += 64) {
        const int bit = 8 * b, i0 = bit / 13, o = bit - 13 * i0;
        const uint32_t v0 = (uint32_t)(H[i0] + (Q - 1) / 2);
        const uint32_t v1 = (i0 + 1 < P) ? (uint32_t)(H[i0 + 1] + (Q - 1) / 2) : 0u;
        pk[b] = (uint8_t)((v0 | (v1 << 13)) >> o);
    }
    uint8_t* sk = sk_out + (size_t)key * 2 * SKH;
    const int8_t* f = f_rows + (size_t)key * P;
    for (int b = lane; b < SKH; b += 64) {
        uint32_t bf = 0, bi = 0;
        const int w = b >> 3, sh = (4 * b) & 31;
        const uint32_t m = ibits[(size_t)(2 * w) * n + key] >> sh;
        const uint32_t s = ibits[(size_t)(2 * w + 1) * n + key] >> sh;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int i = 4 * b + e;
            if (i < P) {
                bf |= (uint32_t)(f[i] + 1) << (2 * e);
                const uint32_t mb = (m >> e) & 1u, sb = (s >> e) & 1u;
                bi |= (mb ? (sb ? 0u : 2u) : 1u) << (2 * e);
            }
        }
        sk[b] = (uint8_t)bf;
        sk[SKH + b] = (uint8_t)bi;
    }
}

// KEYGEN = true: a_i = 3 f_i (small), outputs encoded keys.
// KEYGEN = false: a_i = a_in rows (big), outputs c_i = 1/a_i to c_out.
template <int P, bool KEYGEN>
__global__ __launch_bounds__(64) void group_kernel(GroupArgs args) {
    constexpr int R = RqShape<P>::R;
    __shared__ GroupLds<P> L;
    const int lane = lane_id();
    const int n = args.n;
    const int k0 = blockIdx.x * args.G;
    const int gsz = min(args.G, n - k0);
    if (gsz <= 0) return;
    const int8_t* f_rows = args.f_rows;
    const int16_t* a_in = args.a_in;
    int16_t* bscr = args.bscr;
    int32_t acc1[1][R], acc2[2][R];

    // prefix products: b_1 = a_1, b_i = a_i b_{i-1}
    if (KEYGEN) load_3f<P>(f_rows + (size_t)k0 * P, L.Bb);
    else load_row16<P>(a_in + (size_t)k0 * P, L.Bb);
    __syncthreads();
    for (int j = lane; j < P; j += 64) bscr[(size_t)k0 * P + j] = L.Bb[j];
    for (int i = 1; i < gsz; i++) {
        if (KEYGEN) load_3f<P>(f_rows + (size_t)(k0 + i) * P, L.A0);
        else load_row16<P>(a_in + (size_t)(k0 + i) * P, L.A0);
        build_window<P>(L.Bb, L.Et, L.Pk);
        __syncthreads();
        mul_wave<P, 1, !KEYGEN, false>(L.A0, nullptr, L.Bb, L.Pk, acc1);
        __syncthreads();
        store_lds<P>(acc1[0], L.Bb);
        store_row<P>(acc1[0], bscr + (size_t)(k0 + i) * P);
        __syncthreads();
    }
    // one reciprocal per group: t = 1/b_gsz
    const int ok = recip_wave<P>(L.Bb, L.Bb, L.Pk);
    if (!ok && lane == 0) atomicOr(args.err, 2);

    // back-substitution: c_i = t_i b_{i-1} and t_{i-1} = t_i a_i share the
    // window of t_i (in Bb); then c_i is consumed (h_i = g_i c_i or output)
    for (int i = gsz; i >= 1; i--) {
        const int16_t* C = L.Bb;  // i == 1: c_1 = t_1
        if (i > 1) {
            load_row16<P>(bscr + (size_t)(k0 + i - 2) * P, L.A0);
            if (KEYGEN) load_3f<P>(f_rows + (size_t)(k0 + i - 1) * P, L.A1);
            else load_row16<P>(a_in + (size_t)(k0 + i - 1) * P, L.A1);
            build_window<P>(L.Bb, L.Et, L.Pk);
            __syncthreads();
            mul_wave<P, 2, true, !KEYGEN>(L.A0, L.A1, L.Bb, L.Pk, acc2);
            __syncthreads();
            store_lds<P>(acc2[0], L.Cb);
            store_lds<P>(acc2[1], L.Bb);
            __syncthreads();
            C = L.Cb;
        }
        const int key = k0 + i - 1;
        if (KEYGEN) {
            load_g<P>(args.gbits, n, key, L.A0);
            build_window<P>(C, L.Et, L.Pk);
            __syncthreads();
            mul_wave<P, 1, false, false>(L.A0, nullptr, C, L.Pk, acc1);   // h = g c
            __syncthreads();
            store_lds<P>(acc1[0], L.A1);
            __syncthreads();
            encode_key<P>(key, L.A1, args.pk, args.sk, f_rows, args.ibits, n);
        } else {
            for (int j = lane; j < P; j += 64) args.c_out[(size_t)key * P + j] = C[j];
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// Batch inversion (Section 2.2) on the int8 matrix cores: the Montgomery group
// of group_kernel with every product done by mfma_mul, the big running value
// (b_i, t_i) as the Toeplitz operand and the input rows as folded Hankel
// operands.
// ----------------------------------------------------------------------------
template <int P>
struct GroupMfLds {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];     // Toeplitz limbs of the running value
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HL[S::HLEN];     // Hankel limbs of an input or prefix row
    __attribute__((aligned(16))) uint8_t HH[S::HLEN];
    __attribute__((aligned(16))) int32_t ST[64 * RqShape<P>::RI];   // divstep staging
    __attribute__((aligned(16))) int16_t Bb[RqShape<P>::JP];  // running value (natural order)
    __attribute__((aligned(16))) int16_t Cb[RqShape<P>::JP];  // c_i
};

#ifndef NTRUP_GM_WAVES
#define NTRUP_GM_WAVES 1
#endif
template <int P>
__global__ __launch_bounds__(64, NTRUP_GM_WAVES) void group_mfma_kernel(GroupArgs args) {
    __shared__ GroupMfLds<P> L;
    const int lane = lane_id();
    const int n = args.n;
    const int k0 = blockIdx.x * args.G;
    const int gsz = min(args.G, n - k0);
    if (gsz <= 0) return;
    const int16_t* a_in = args.a_in;
    int16_t* bscr = args.bscr;

    // prefix products: b_1 = a_1, b_i = a_i b_{i-1} (Toeplitz operand b_{i-1})
    load_row16<P>(a_in + (size_t)k0 * P, L.Bb);
    __syncthreads();
    for (int j = lane; j < P; j += 64) bscr[(size_t)k0 * P + j] = L.Bb[j];
    for (int i = 1; i < gsz; i++) {
        build_toeplitz<P>(L.Bb, L.TL, L.TH);
        build_hankel<P>(a_in + (size_t)(k0 + i) * P, L.HL, L.HH);
        __syncthreads();
        mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, L.Bb, nullptr, nullptr, bscr + (size_t)(k0 + i) * P);
        __syncthreads();
    }
    // one reciprocal per group: t = 1/b_gsz
    const int ok = recip_wave<P>(L.Bb, L.Bb, L.ST);
    if (!ok && lane == 0) atomicOr(args.err, 2);
    __syncthreads();

    // back-substitution: c_i = t_i b_{i-1}, t_{i-1} = t_i a_i (Toeplitz operand t_i)
    for (int i = gsz; i >= 1; i--) {
        const int16_t* C = L.Bb;  // i == 1: c_1 = t_1
        if (i > 1) {
            build_toeplitz<P>(L.Bb, L.TL, L.TH);
            build_hankel<P>(bscr + (size_t)(k0 + i - 2) * P, L.HL, L.HH);
            __syncthreads();
            mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, L.Cb, nullptr, nullptr, nullptr);
            __syncthreads();
            build_hankel<P>(a_in + (size_t)(k0 + i - 1) * P, L.HL, L.HH);
            __syncthreads();
            mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, L.Bb, nullptr, nullptr, nullptr);
            __syncthreads();
            C = L.Cb;
        }
        const int key = k0 + i - 1;
        for (int j = lane; j < P; j += 64) args.c_out[(size_t)key * P + j] = C[j];
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// Single-operation entry points (used by the kernel-level tests).
// ----------------------------------------------------------------------------
template <int P, bool BIG>
__global__ __launch_bounds__(64) void mul_kernel(int n, const int16_t* a, const int16_t* b, int16_t* c) {
    __shared__ GroupLds<P> L;
    const int e = blockIdx.x;
    if (e >= n) return;
    int32_t acc[1][RqShape<P>::R];
    load_row16<P>(a + (size_t)e * P, L.A0);
    load_row16<P>(b + (size_t)e * P, L.Bb);
    __syncthreads();
    build_window<P>(L.Bb, L.Et, L.Pk);
    __syncthreads();
    mul_wave<P, 1, BIG, false>(L.A0, nullptr, L.Bb, L.Pk, acc);
    store_row<P>(acc[0], c + (size_t)e * P);
}

// LDS of one product on the matrix cores: operand rows and limb arrays.
template <int P>
struct MfLds {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HL[S::HLEN];
    __attribute__((aligned(16))) uint8_t HH[S::HLEN];
    __attribute__((aligned(16))) int16_t X[RqShape<P>::JP];
    __attribute__((aligned(16))) int16_t Y[RqShape<P>::JP];
};

// c = a * b with the matrix-core product: b is the Toeplitz operand (two
// limbs), a the Hankel operand (one limb when small, two when BIG).
template <int P, bool BIG>
__global__ __launch_bounds__(64) void mulm_kernel(int n, const int16_t* a, const int16_t* b, int16_t* c) {
    __shared__ MfLds<P> L;
    const int e = blockIdx.x;
    if (e >= n) return;
    load_row16<P>(a + (size_t)e * P, L.X);
    load_row16<P>(b + (size_t)e * P, L.Y);
    __syncthreads();
    build_toeplitz<P>(L.Y, L.TL, L.TH);
    build_hankel<P>(L.X, L.HL, BIG ? L.HH : nullptr);
    __syncthreads();
    mfma_mul<P, BIG>(L.TL, L.TH, L.HL, L.HH, nullptr, nullptr, nullptr, c + (size_t)e * P);
}

// R/q reciprocals of n rows: by the plain divstep loop on one wave
// (J = false) or by jump divsteps on the matrix cores (J = true), the four
// products of each jump on the block's 1 to kRecipJumpWaves waves side by
// side (the host launches four waves per row for up to 512 rows).
constexpr int kRecipJumpWaves = 4;
template <int P, bool J>
__global__ __launch_bounds__(J ? 64 * kRecipJumpWaves : 64) void recip_q_kernel(int n, const int16_t* a,
                                                                                int16_t* out, int32_t* ok) {
    __shared__ GroupLds<P> L;
    __shared__ typename std::conditional<J, JumpLds<P>, char>::type JL;
    const int e = blockIdx.x;
    if (e >= n) return;
    const int wave = (int)(threadIdx.x >> 6);
    if (wave == 0) load_row16<P>(a + (size_t)e * P, L.Bb);
    __syncthreads();
    int r;
    if constexpr (J) {
        r = recip_jump_block<P, Param<P>::q, int16_t, true>(L.Bb, L.Bb, JL, wave, (int)(blockDim.x >> 6));
        if (wave != 0) return;
    } else {
        r = recip_wave<P>(L.Bb, L.Bb, L.Pk);
    }
    for (int j = lane_id(); j < P; j += 64) out[(size_t)e * P + j] = L.Bb[j];
    if (lane_id() == 0) ok[e] = r;
}

// int8 rows [n][p] from bitsliced words [WN][2][n]
template <int P>
__global__ __launch_bounds__(256) void unpack_bits_kernel(int n, const uint32_t* bits, int8_t* rows) {
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= n) return;
    for (int k = 0; k < ceil_div(P, 32); k++) {
        const uint32_t m = bits[(size_t)(2 * k) * n + key], s = bits[(size_t)(2 * k + 1) * n + key];
        for (int e = 0; e < 32 && 32 * k + e < P; e++)
            rows[(size_t)key * P + 32 * k + e] = (int8_t)(((m >> e) & 1u) * (1 - 2 * ((s >> e) & 1u)));
    }
}

template <int P>
__global__ __launch_bounds__(256) void sample_small_kernel(Seed seed, uint64_t first_index, int n, int attempt,
                                                           int8_t* rows) {
    constexpr int WN = ceil_div(P, 32);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * WN) return;
    const int key = t / WN, k = t % WN;
    uint32_t m, s;
    sample_small_word<P>(seed, first_index + (uint64_t)key, attempt, k, m, s);
    for (int e = 0; e < 32 && 32 * k + e < P; e++)
        rows[(size_t)key * P + 32 * k + e] = (int8_t)(((m >> e) & 1u) * (1 - 2 * ((s >> e) & 1u)));
}

// Optional raw outputs of KeyGen from its encoded key pair: h (int16), f and
// 1/g (int8), centered, [n][p] each; one thread per coefficient, any pointer
// may be null.  The inverse of the pk / sk encodings of kg_encode.
template <int P>
__global__ __launch_bounds__(256) void decode_raw_kernel(int n, const uint8_t* pk, const uint8_t* sk, int16_t* h,
                                                         int8_t* f, int8_t* ginv) {
    constexpr int Q = Param<P>::q, PKB = pk_bytes(P), SKH = sk_half_bytes(P);
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)n * P) return;
    const size_t key = t / P;
    const int i = (int)(t - key * P);
    if (h) {
        const uint8_t* b = pk + key * PKB;
        const int bit = 13 * i, by = bit >> 3;
        uint32_t v = b[by] | ((uint32_t)b[by + 1] << 8);   // 13 * i + 12 < 13 p: by + 1 < PKB
        if (by + 2 < PKB) v |= (uint32_t)b[by + 2] << 16;
        h[t] = (int16_t)((int32_t)((v >> (bit & 7)) & 0x1FFFu) - (Q - 1) / 2);
    }
    const uint8_t* s = sk + key * 2 * SKH;
    if (f) f[t] = (int8_t)((int32_t)((s[i >> 2] >> (2 * (i & 3))) & 3u) - 1);
    if (ginv) ginv[t] = (int8_t)((int32_t)((s[SKH + (i >> 2)] >> (2 * (i & 3))) & 3u) - 1);
}

// (static: every object of the library that launches them holds its own copy)
static __global__ __attribute__((unused)) void copy_flags_kernel(int n, const uint8_t* src, int32_t* dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

static __global__ __attribute__((unused)) void zero_ints_kernel(int* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

}  // namespace ntrup
