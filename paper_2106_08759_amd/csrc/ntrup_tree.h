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
// t_j in `trow` (j in [1, G)), c_i in `crow` (the key rows).  Levels are
// ordered by workgroup barriers; a wave owns the nodes j = first + w,
// first + w + kTreeWaves, ... of a level, so that the two children of a
// down-sweep node are written by the wave that read them.
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

template <int P>
struct TreeWaveLds {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HL[S::HLEN];
    __attribute__((aligned(16))) uint8_t HH[S::HLEN];
};

// The root reciprocal's LDS (wave 0 alone, while the other waves wait at a
// barrier, so it shares the space of the product operands).
template <int P, bool J>
struct TreeRootLds {
    __attribute__((aligned(16))) int16_t R[RqShape<P>::JP];
    __attribute__((aligned(16))) int32_t STG[64 * RqShape<P>::RI];
    typename std::conditional<J, JumpLds<P>, char>::type JL;
};

template <int P, bool J>
union TreeLds {
    TreeWaveLds<P> w[kTreeWaves];
    TreeRootLds<P, J> root;
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

// The tree for group blockIdx.x.  args: n, G, f_rows, err; brow = args.bscr.
template <int P, bool J>
__global__ __launch_bounds__(64 * kTreeWaves) void keygen_tree_kernel(GroupArgs args, int16_t* trow, int16_t* crow) {
    __shared__ TreeLds<P, J> LDS;
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();
    const int n = args.n, G = args.G;
    const int kw0 = blockIdx.x * G;
    const int gsz = min(G, n - kw0);
    int16_t* brow = args.bscr + (size_t)kw0 * P;   // row j: b_j
    int16_t* tr = trow + (size_t)kw0 * P;          // row j: t_j
    const int8_t* f0 = args.f_rows + (size_t)kw0 * P;
    TreeWaveLds<P>& L = LDS.w[wave];
    // the operand a_i = 3 f_i of leaf G + i (nullptr: 1, past the last key)
    auto leaf = [&](int node) -> const int8_t* {
        const int i = node - G;
        return i < gsz ? f0 + (size_t)i * P : nullptr;
    };

    // up-sweep, the leaves' parents first
    for (int first = G / 2; first >= 1; first >>= 1) {
        for (int j = first + wave; j < 2 * first; j += kTreeWaves) {
            if (first == G / 2) {   // two leaves: small x small
                tree_toeplitz_small<P>(leaf(2 * j), 3, L.TL);
                tree_hankel_small<P>(leaf(2 * j + 1), 3, L.HL);
                wave_sync();
                mfma_mul<P, false, false>(L.TL, nullptr, L.HL, nullptr, nullptr, nullptr, nullptr,
                                          brow + (size_t)j * P);
            } else {
                build_toeplitz<P>(brow + (size_t)(2 * j) * P, L.TL, L.TH);
                build_hankel<P>(brow + (size_t)(2 * j + 1) * P, L.HL, L.HH);
                wave_sync();
                mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, nullptr, nullptr, nullptr, brow + (size_t)j * P);
            }
            wave_sync();
        }
        __threadfence_block();
        __syncthreads();
    }
    // root: t_1 = 1/b_1 (b_1 != 0: a product of nonzero elements of a field)
    if (wave == 0) {
        TreeRootLds<P, J>& Rt = LDS.root;
        for (int i = lane; i < P; i += 64) Rt.R[i] = brow[(size_t)P + i];
        wave_sync();
        int ok;
        if constexpr (J) ok = recip_jump_wave<P>(Rt.R, Rt.R, Rt.JL);
        else ok = recip_wave<P>(Rt.R, Rt.R, Rt.STG);
        if (!ok && lane == 0) atomicOr(args.err, 2);
        for (int i = lane; i < P; i += 64) tr[(size_t)P + i] = Rt.R[i];
    }
    __threadfence_block();
    __syncthreads();
    // down-sweep, from the root's children
    for (int first = 1; first < G; first <<= 1) {
        for (int j = first + wave; j < 2 * first; j += kTreeWaves) {
            build_toeplitz<P>(tr + (size_t)j * P, L.TL, L.TH);
            if (2 * first == G) {   // children are leaves: c_i = t_j a_sibling
                const int i0 = 2 * j - G, i1 = i0 + 1;
                tree_hankel_small<P>(leaf(2 * j + 1), 3, L.HL);
                wave_sync();
                mfma_mul<P, false>(L.TL, L.TH, L.HL, nullptr, nullptr, nullptr, nullptr,
                                   i0 < gsz ? crow + (size_t)(kw0 + i0) * P : nullptr);
                wave_sync();
                if (i1 < gsz) {
                    tree_hankel_small<P>(leaf(2 * j), 3, L.HL);
                    wave_sync();
                    mfma_mul<P, false>(L.TL, L.TH, L.HL, nullptr, nullptr, nullptr, nullptr,
                                       crow + (size_t)(kw0 + i1) * P);
                }
            } else {
                build_hankel<P>(brow + (size_t)(2 * j + 1) * P, L.HL, L.HH);
                wave_sync();
                mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, nullptr, nullptr, nullptr, tr + (size_t)(2 * j) * P);
                wave_sync();
                build_hankel<P>(brow + (size_t)(2 * j) * P, L.HL, L.HH);
                wave_sync();
                mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, nullptr, nullptr, nullptr,
                                  tr + (size_t)(2 * j + 1) * P);
            }
            wave_sync();
        }
        __threadfence_block();
        __syncthreads();
    }
}

}  // namespace ntrup
