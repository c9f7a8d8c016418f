// Montgomery's batch inversion (Section 2.2) over a product tree: one
// workgroup of kTreeWaves waves per group of G = 2^k keys.
//
// Section 2.2 chains the prefix products b_i = a_i b_{i-1}, inverts b_G and
// walks back, 3G - 3 products in a sequence of about 3G dependent steps.  The
// same 3G - 3 products arranged as a binary tree need only 2k dependent
// levels, and the products of a level are independent, so the workgroup's
// waves share them:
//   up:    node j (heap order: root 1, children 2j and 2j+1, leaves G..2G-1 =
//          a_i = 3 f_i of keys kw0 .. kw0+G-1) holds the product of its
//          leaves: b_j = b_{2j} b_{2j+1};                        G - 1 products
//   root:  t_1 = 1/b_1 by one reciprocal (jump or plain divsteps);
//   down:  t_{2j} = t_j b_{2j+1}, t_{2j+1} = t_j b_{2j}: t_j is the product
//          of the reciprocals of node j's leaves, so at the leaves t = 1/a_i
//          = c_i;                                                 2G - 2 products.
// Leaf pairs multiply two small operands (one int8 limb each), inner nodes two
// residues (two limbs each), the last level t_j by a small a_i.  Leaves past
// the last key of a ragged group are 1.
//
// Rows (global int16 [rows][p], rows kw0 + j of the group): b_j in `brow`,
// t_j in `trow` (j in [1, G)), c_i in `crow` (the key rows).  Three kernels:
// the up-sweep, the roots' reciprocals (one wave per group), the down-sweep.
// Within a sweep, levels are ordered by workgroup barriers; a wave owns the
// nodes j = first + w, first + w + kTreeWaves, ... of a level, so that the
// two children of a down-sweep node are written by the wave that read them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ntrup_jump.h"
#include "ntrup_keygen.h"
#include "ntrup_mfma.h"

namespace ntrup {

constexpr int kTreeWaves = 8;     // waves per workgroup (one group of G keys)
constexpr int kTreeMaxG = 256;    // G = 2^k, 2 <= G <= kTreeMaxG
// Waves per SIMD the up- and down-sweep kernels are compiled for: four (two
// 8-wave groups per CU, at most 128 VGPRs) where the operands fit with a few
// spilled registers, two for p = 1277, whose wider operands would spill more.
constexpr int tree_min_waves(int p) { return p < 1000 ? 4 : 2; }

template <int P>
struct TreeWaveLds {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HL[S::HLEN];
    __attribute__((aligned(16))) uint8_t HH[S::HLEN];
};

// The root reciprocal's LDS.
template <int P, bool J>
struct TreeRootLds {
    __attribute__((aligned(16))) int16_t R[RqShape<P>::JP];
    __attribute__((aligned(16))) int32_t STG[64 * RqShape<P>::RI];
    typename std::conditional<J, JumpLds<P>, char>::type JL;
};

// Reversed Toeplitz limb of a small operand s a_m (a an int8 row; scale 3
// gives 3 f): TL[Z0 - m] = s a_m, zero outside [0, p).  a = nullptr: the
// element 1.
template <int P>
__device__ __forceinline__ void tree_toeplitz_small(const int8_t* a, int scale, uint8_t* TL) {
    using S = MfShape<P>;
    for (int i = lane_id(); i < S::TLEN / 4; i += 64) {
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int m = S::Z0 - (4 * i + t);
            const int32_t v = (m >= 0 && m < P) ? (a ? scale * (int32_t)a[m] : (int32_t)(m == 0)) : 0;
            w |= (uint32_t)(uint8_t)(int8_t)v << (8 * t);
        }
        ((uint32_t*)TL)[i] = w;
    }
}

// Folded Hankel limb of a small operand s a (|E_m| <= 2 s): HL[HOFF + m] =
// E_m.  a = nullptr: the element 1 (E_0 = 1).
template <int P>
__device__ __forceinline__ void tree_hankel_small(const int8_t* a, int scale, uint8_t* HL) {
    using S = MfShape<P>;
    for (int i = lane_id(); i < S::HLEN / 4; i += 64) {
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int m = 4 * i + t - S::HOFF;
            int32_t v = 0;
            if (a) {
                if (m >= 1 && m < P) v = a[m];
                else if (m == 0) v = (int32_t)a[0] + (int32_t)a[P - 1];
                else if (m < 0 && m >= -(P - 1)) v = (int32_t)a[m + P] + (int32_t)a[m + P - 1];
                v *= scale;
            } else {
                v = (m == 0);
            }
            w |= (uint32_t)(uint8_t)(int8_t)v << (8 * t);
        }
        ((uint32_t*)HL)[i] = w;
    }
}

// Reversed Toeplitz limb of 3 f from the f bytes in registers (KgRegs
// layout): TL[Z0 - m] = 3 f_m for m < p (bytes 0x00, 0x01, 0xFF -> 0x00,
// 0x03, 0xFD, byte-reversed per word); the padding stays as it is.
template <int P>
__device__ __forceinline__ void tree_put_toeplitz_3f(const KgRegs<P>& r, uint8_t* TL) {
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        if (m0 < P) {
            const uint32_t f3 = r.f[u] ^ ((r.f[u] & 0x01010101u) << 1);
            *(uint32_t*)(TL + MfShape<P>::Z0 - m0 - 3) = __builtin_amdgcn_perm(0u, f3, 0x00010203u);
        }
    }
}

// Shared set-up of the up- and down-sweep kernels: one workgroup of
// kTreeWaves waves per group (blockIdx.x).  Operands go through registers
// (one row load, then the limb arrays written from the registers, as in the
// chain kernels); the limb arrays' padding is zeroed once.
template <int P>
struct TreeWave {
    using S = MfShape<P>;
    const GroupArgs& args;
    TreeWaveLds<P>& L;
    int G, kw0, gsz;
    int16_t* brow;   // row j: b_j
    int16_t* tr;     // row j: t_j
    KgRegs<P> ra;
    __device__ TreeWave(const GroupArgs& a, TreeWaveLds<P>& l, int16_t* trow)
        : args(a), L(l), G(a.G), kw0((int)blockIdx.x * a.G), gsz(min(a.G, a.n - (int)blockIdx.x * a.G)),
          brow(a.bscr + (size_t)blockIdx.x * a.G * P), tr(trow + (size_t)blockIdx.x * a.G * P) {
        kg_zero<P>(L.TL, S::TLEN);
        kg_zero<P>(L.TH, S::TLEN);
        kg_zero<P>(L.HL, S::HLEN);
        kg_zero<P>(L.HH, S::HLEN);
        wave_sync();
    }
    // a_i = 3 f_i of leaf `node` as a Toeplitz (T) or Hankel (H) limb; the
    // element 1 past the last key (whole arrays rewritten)
    __device__ void leaf_t(int node) {
        const int i = node - G;
        if (i < gsz) {
            kg_load_f<P>(args.f_rows, kw0 + i, ra);
            tree_put_toeplitz_3f<P>(ra, L.TL);
        } else {
            tree_toeplitz_small<P>(nullptr, 1, L.TL);
        }
    }
    __device__ void leaf_h(int node) {
        const int i = node - G;
        if (i < gsz) {
            kg_load_f<P>(args.f_rows, kw0 + i, ra);
            kg_put_3f<P>(ra, L.HL);
        } else {
            tree_hankel_small<P>(nullptr, 1, L.HL);
        }
    }
    __device__ void big_t(const int16_t* rows, int j) {
        kg_load_b<P>(rows, j, ra);
        kg_put_toeplitz16<P>(ra.b, L.TL, L.TH);
    }
    __device__ void big_h(const int16_t* rows, int j) {
        kg_load_b<P>(rows, j, ra);
        put_folded16<P>(ra.b, L.HL, L.HH);
    }
};

// Up-sweep of group blockIdx.x: b_j for every inner node j (rows of bscr),
// the leaves' parents first.
template <int P>
__global__ __launch_bounds__(64 * kTreeWaves, tree_min_waves(P)) void keygen_tree_up_kernel(GroupArgs args, int16_t* trow) {
    __shared__ TreeWaveLds<P> LW[kTreeWaves];
    const int wave = (int)(threadIdx.x >> 6);
    TreeWave<P> T(args, LW[wave], trow);
    for (int first = T.G / 2; first >= 1; first >>= 1) {
        for (int j = first + wave; j < 2 * first; j += kTreeWaves) {
            if (first == T.G / 2) {   // two leaves: small x small
                T.leaf_t(2 * j);
                T.leaf_h(2 * j + 1);
                wave_sync();
                mfma_mul<P, false, false>(T.L.TL, nullptr, T.L.HL, nullptr, nullptr, nullptr, nullptr,
                                          T.brow + (size_t)j * P);
            } else {
                T.big_t(T.brow, 2 * j);
                T.big_h(T.brow, 2 * j + 1);
                wave_sync();
                mfma_mul<P, true>(T.L.TL, T.L.TH, T.L.HL, T.L.HH, nullptr, nullptr, nullptr, T.brow + (size_t)j * P);
            }
            wave_sync();
        }
        __threadfence_block();
        __syncthreads();
    }
}

// Root of every group: t_1 = 1/b_1 (b_1 != 0: a product of nonzero elements
// of a field), one workgroup per group (a kernel of its own, so that the
// reciprocal's registers do not limit the sweeps' occupancy).  With jump
// divsteps the workgroup has 1 to kTreeRootWaves waves (blockDim.x / 64),
// which compute the four products of each jump side by side: the host
// launches four for few groups (latency) and one when the groups fill the
// chip (throughput: 1024 groups took 0.44 ms on four waves each against
// 0.28 on one).  The plain divstep loop runs on one wave.
constexpr int kTreeRootWaves = 4;
template <int P, bool J>
__global__ __launch_bounds__(J ? 64 * kTreeRootWaves : 64) void keygen_tree_root_kernel(GroupArgs args, int16_t* trow) {
    __shared__ TreeRootLds<P, J> Rt;
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const size_t row = (size_t)blockIdx.x * args.G + 1;
    if (wave == 0)
        for (int i = lane; i < P; i += 64) Rt.R[i] = args.bscr[row * P + i];
    int ok;
    if constexpr (J) {
        __syncthreads();
        ok = recip_jump_block<P, Param<P>::q, int16_t, true>(Rt.R, Rt.R, Rt.JL, wave, (int)(blockDim.x >> 6));
        if (wave != 0) return;
    } else {
        wave_sync();
        ok = recip_wave<P>(Rt.R, Rt.R, Rt.STG);
    }
    if (!ok && lane == 0) atomicOr(args.err, 2);
    for (int i = lane; i < P; i += 64) trow[row * P + i] = Rt.R[i];
}

// Down-sweep of group blockIdx.x from the root's children: t_j of the inner
// nodes (rows of trow), c_i = 1/(3 f_i) of the keys (rows of crow).
template <int P>
__global__ __launch_bounds__(64 * kTreeWaves, tree_min_waves(P)) void keygen_tree_down_kernel(GroupArgs args, int16_t* trow,
                                                                           int16_t* crow) {
    __shared__ TreeWaveLds<P> LW[kTreeWaves];
    const int wave = (int)(threadIdx.x >> 6);
    TreeWave<P> T(args, LW[wave], trow);
    const int G = T.G, kw0 = T.kw0, gsz = T.gsz;
    for (int first = 1; first < G; first <<= 1) {
        for (int j = first + wave; j < 2 * first; j += kTreeWaves) {
            T.big_t(T.tr, j);
            if (2 * first == G) {   // children are leaves: c_i = t_j a_sibling
                const int i0 = 2 * j - G, i1 = i0 + 1;
                T.leaf_h(2 * j + 1);
                wave_sync();
                mfma_mul<P, false>(T.L.TL, T.L.TH, T.L.HL, nullptr, nullptr, nullptr, nullptr,
                                   i0 < gsz ? crow + (size_t)(kw0 + i0) * P : nullptr);
                wave_sync();
                if (i1 < gsz) {
                    T.leaf_h(2 * j);
                    wave_sync();
                    mfma_mul<P, false>(T.L.TL, T.L.TH, T.L.HL, nullptr, nullptr, nullptr, nullptr,
                                       crow + (size_t)(kw0 + i1) * P);
                }
            } else {
                T.big_h(T.brow, 2 * j + 1);
                wave_sync();
                mfma_mul<P, true>(T.L.TL, T.L.TH, T.L.HL, T.L.HH, nullptr, nullptr, nullptr,
                                  T.tr + (size_t)(2 * j) * P);
                wave_sync();
                T.big_h(T.brow, 2 * j);
                wave_sync();
                mfma_mul<P, true>(T.L.TL, T.L.TH, T.L.HL, T.L.HH, nullptr, nullptr, nullptr,
                                  T.tr + (size_t)(2 * j + 1) * P);
            }
            wave_sync();
        }
        __threadfence_block();
        __syncthreads();
    }
}

}  // namespace ntrup
