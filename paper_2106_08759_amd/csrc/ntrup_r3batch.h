// Batched R/3 reciprocals (Section 3.1, Algorithm 1: batchInv over R/3 with
// the isInvertible check of each g), on the int8 matrix cores.
//
// r3b_screen_kernel   one lane per key: draw g (stream 1 + attempt) until g
//                     mod f_i != 0 for every irreducible factor f_i of
//                     x^p - x - 1 over F_3 of degree <= 32 (Horner, one
//                     bitsliced word per factor); writes g's bitsliced words
//                     and the accepted attempt.  The factors left unscreened
//                     have degree >= 60, so a non-unit g passes with
//                     probability below 3^-60 per draw.
// r3b_prefix_kernel   one wave per Montgomery group: b_1 = g_1, b_i = g_i
//                     b_{i-1} in R/3 (int8 rows), the group product to pj.
// (group reciprocals: the per-key divstep kernel on the rows of pj)
// r3b_back_kernel     one wave per group: from t = 1/b_G, 1/g_i = t b_{i-1},
//                     t <- t g_i, written as bitsliced words.  A group whose
//                     product is not a unit (one of its g failed on an
//                     unscreened factor) instead lists its keys for the
//                     per-key divstep pass, which resumes each key at its
//                     screened attempt; outputs are the same either way.
// Products are mfma_mul with one int8 limb per operand, reduced mod 3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_jump.h"
#include "ntrup_keygen.h"
#include "ntrup_mfma.h"
#include "ntrup_r3_factors.h"

namespace ntrup {

template <int P>
struct R3bArgs {
    Seed seed;
    uint64_t first_index;
    int n, G;
    uint32_t* gbits;        // [WN][2][n] bitsliced g (nonzero, negative)
    uint32_t* ibits;        // [WN][2][n] bitsliced 1/g
    uint8_t* attempts;      // [n] accepted attempt of each key
    int8_t* rows;           // [n][p] prefix products b_i
    int8_t* pj;             // [groups][p] group products
    const uint32_t* pinv;   // [WN][2][groups] their reciprocals (bitsliced)
    const uint8_t* pok;     // [groups] 1 iff the group product is a unit
    int* fb_list;           // keys of groups whose product is not a unit
    int* fb_count;
    int* err;               // |= 1 when a key finds no screened g in 64 draws
    int screen;             // 0: accept the first draw (tests of the fallback path)
    int* rt_list;           // keys whose first draw failed the screen
    int* rt_count;
    uint32_t* rt_scratch;   // their next draws: [draw][word][plane][rt_cap]
    int rt_cap;
};

// One Horner step r <- r x + c mod f over F_3 (bitsliced, f = x^d + sum c_j
// x^j monic with d <= 32): the coefficient leaving degree d - 1 is folded
// back with x^d = -(c_0 + ... + c_{d-1} x^{d-1}).
__device__ __forceinline__ void r3_horner_step(uint32_t& rm, uint32_t& rs, uint32_t cm, uint32_t cs, int d,
                                               uint32_t fm, uint32_t fs) {
    const uint32_t mask = d == 32 ? 0xFFFFFFFFu : ((1u << d) - 1u);
    const uint32_t tm = (rm >> (d - 1)) & 1u, ts = (rs >> (d - 1)) & 1u;
    const uint32_t am = ((rm << 1) | cm) & mask, as = ((rs << 1) | cs) & mask;
    // add (-t) (c_0 .. c_{d-1}): nonzero where c is and t != 0, negative
    // where c and -t differ in sign
    const uint32_t bm = fm & (0u - tm);
    const uint32_t bs = fs ^ (ts - 1u);
    rm = (am ^ bm) | (am & bm & ~(as ^ bs));
    rs = (am & (as ^ bm)) | (~am & bs);
}

// g mod F for each product F of small factors (one Horner pass over g, words
// fed from the highest), then that remainder mod each member factor.
template <int P>
struct R3Screen {
    using F = R3Factors<P>;
    uint32_t rm[F::ngroups], rs[F::ngroups];
    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int j = 0; j < F::ngroups; j++) rm[j] = rs[j] = 0u;
    }
    __device__ __forceinline__ void feed_word(uint32_t m, uint32_t s) {
#pragma unroll
        for (int b = 31; b >= 0; b--) {
            const uint32_t cm = (m >> b) & 1u, cs = (s >> b) & 1u;
#pragma unroll
            for (int j = 0; j < F::ngroups; j++) r3_horner_step(rm[j], rs[j], cm, cs, F::g[j].d, F::g[j].m, F::g[j].s);
        }
    }
    // Words k = WN-1 .. 0 of a bitsliced g whose nonzero plane of word k is
    // at w[k * stride] and sign plane at w[k * stride + plane]: the loads of
    // eight words are issued before their serial Horner steps.
    __device__ __forceinline__ void feed_words(const uint32_t* w, size_t plane, size_t stride) {
        constexpr int WN = ceil_div(P, 32), CH = 8;
        for (int c = WN; c > 0; c -= CH) {
            uint32_t wm[CH], ws[CH];
#pragma unroll
            for (int t = 0; t < CH; t++) {
                const int k = c - 1 - t;
                wm[t] = k >= 0 ? w[(size_t)k * stride] : 0u;
                ws[t] = k >= 0 ? w[(size_t)k * stride + plane] : 0u;
            }
#pragma unroll
            for (int t = 0; t < CH; t++)
                if (c - 1 - t >= 0) feed_word(wm[t], ws[t]);
        }
    }
    // true iff g mod f != 0 for every small factor f
    __device__ __forceinline__ bool passes() const {
        bool ok = true;
#pragma unroll
        for (int j = 0; j < F::ngroups; j++) {
            if (F::g[j].nmem == 1) {
                ok = ok && rm[j] != 0u;
                continue;
            }
#pragma unroll
            for (int e = 0; e < F::g[j].nmem; e++) {
                const R3Factor f = F::f[F::g[j].mem[e]];
                uint32_t tm = 0, ts = 0;
                for (int b = F::g[j].d - 1; b >= 0; b--)
                    r3_horner_step(tm, ts, (rm[j] >> b) & 1u, (rs[j] >> b) & 1u, f.d, f.m, f.s);
                ok = ok && tm != 0u;
            }
        }
        return ok;
    }
};

// First draw of every key's g: one thread per (key, 32-coefficient word).
template <int P>
__global__ __launch_bounds__(256) void r3b_sample_kernel(R3bArgs<P> a) {
    constexpr int WN = ceil_div(P, 32);
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)a.n * WN) return;
    const int key = (int)(t % (size_t)a.n), k = (int)(t / (size_t)a.n);
    uint32_t mw, sw;
    sample_small_word<P>(a.seed, a.first_index + (uint64_t)key, 0, k, mw, sw);
    a.gbits[(size_t)(2 * k) * a.n + key] = mw;
    a.gbits[(size_t)(2 * k + 1) * a.n + key] = sw & mw;
}

constexpr int kR3bRetryDraws = 4;   // draws tried side by side per listed key

// The screen of every key's first draw, one lane per key; keys whose draw
// fails go to a list.
template <int P>
__global__ __launch_bounds__(256) void r3b_screen_kernel(R3bArgs<P> a) {
    constexpr int WN = ceil_div(P, 32);
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)a.n;
    bool fail = false;
    if (key < a.n) {
        if (a.screen) {
            R3Screen<P> sc;
            sc.reset();
            sc.feed_words(a.gbits + key, n, 2 * n);
            fail = !sc.passes();
        }
        a.attempts[key] = 0;
    }
    const unsigned long long m = __ballot(fail);
    if (m) {
        const int lane = lane_id();
        int b0 = 0;
        if (lane == 0) b0 = atomicAdd(a.rt_count, __popcll(m));
        b0 = __shfl(b0, 0);
        if (fail) a.rt_list[b0 + __popcll(m & ((1ull << lane) - 1ull))] = key;
    }
}

// Draws 1 .. kR3bRetryDraws of every listed key (as many keys as the scratch
// holds), one thread per (key, draw, word).
template <int P>
__global__ __launch_bounds__(256) void r3b_retry_sample_kernel(R3bArgs<P> a) {
    constexpr int WN = ceil_div(P, 32);
    const int count = min(*(volatile int*)a.rt_count, a.rt_cap);
    const size_t total = (size_t)count * kR3bRetryDraws * WN;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % (size_t)count);
        const int rest = (int)(t / (size_t)count);
        const int d = rest % kR3bRetryDraws, k = rest / kR3bRetryDraws;
        const int key = a.rt_list[i];
        uint32_t mw, sw;
        sample_small_word<P>(a.seed, a.first_index + (uint64_t)key, 1 + d, k, mw, sw);
        const size_t base = ((size_t)(d * WN + k) * 2) * a.rt_cap;
        a.rt_scratch[base + i] = mw;
        a.rt_scratch[base + a.rt_cap + i] = sw & mw;
    }
}

// The lowest passing draw of every listed key; keys beyond the scratch, or
// whose kR3bRetryDraws draws all fail, draw on one by one.
template <int P>
__global__ __launch_bounds__(256) void r3b_retry_screen_kernel(R3bArgs<P> a) {
    constexpr int WN = ceil_div(P, 32);
    static_assert(kR3bRetryDraws * 64 == 256, "one wave per draw");
    // 64 listed keys per round of the workgroup; wave d screens draw 1 + d of
    // each (the serial Horner passes of the four draws side by side), then
    // wave 0 takes, per key, the lowest draw that passed
    __shared__ uint8_t pass[kR3bRetryDraws][64];
    const int count = *(volatile int*)a.rt_count;   // the same for every thread
    const size_t n = (size_t)a.n;
    const int d = (int)(threadIdx.x >> 6), j = (int)(threadIdx.x & 63);
    for (int i0 = blockIdx.x * 64; i0 < count; i0 += gridDim.x * 64) {
        const int i = i0 + j;
        bool ok = false;
        if (i < count && i < a.rt_cap) {
            R3Screen<P> sc;
            sc.reset();
            sc.feed_words(a.rt_scratch + ((size_t)(d * WN) * 2) * a.rt_cap + i, (size_t)a.rt_cap,
                          2 * (size_t)a.rt_cap);
            ok = sc.passes();
        }
        pass[d][j] = ok ? 1 : 0;
        __syncthreads();
        if (d == 0 && i < count) {
            const int key = a.rt_list[i];
            const uint64_t index = a.first_index + (uint64_t)key;
            int att = 1;
            bool done = false;
            if (i < a.rt_cap) {
                int win = -1;
#pragma unroll
                for (int dd = kR3bRetryDraws - 1; dd >= 0; dd--)
                    if (pass[dd][j]) win = dd;
                if (win >= 0) {
                    for (int k = 0; k < WN; k++) {
                        const size_t base = ((size_t)(win * WN + k) * 2) * a.rt_cap;
                        a.gbits[(size_t)(2 * k) * n + key] = a.rt_scratch[base + i];
                        a.gbits[(size_t)(2 * k + 1) * n + key] = a.rt_scratch[base + a.rt_cap + i];
                    }
                    att = 1 + win;
                    done = true;
                } else {
                    att = 1 + kR3bRetryDraws;
                }
            }
            for (; !done && att < kMaxAttempts; att++) {
                R3Screen<P> sc;
                sc.reset();
                for (int k = WN - 1; k >= 0; k--) {
                    uint32_t mw, sw;
                    sample_small_word<P>(a.seed, index, att, k, mw, sw);
                    sw &= mw;
                    a.gbits[(size_t)(2 * k) * n + key] = mw;
                    a.gbits[(size_t)(2 * k + 1) * n + key] = sw;
                    sc.feed_word(mw, sw);
                }
                if (sc.passes()) {
                    done = true;
                    break;
                }
            }
            if (!done) atomicOr(a.err, 1);
            a.attempts[key] = (uint8_t)(done ? att : kMaxAttempts);
        }
        __syncthreads();
    }
}

// Reversed Toeplitz bytes of a ternary polynomial from its bitsliced words
// (four coefficients per lane word, as kg_load_bits loads them).
template <int P>
__device__ __forceinline__ void r3b_put_toeplitz(const uint32_t (&m)[KgShape<P>::NU], const uint32_t (&s)[KgShape<P>::NU],
                                                 uint8_t* TL) {
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        if (m0 >= P) continue;
        const uint32_t w = spread4(m[u]) | (spread4(s[u]) * 0xFEu);
        *(uint32_t*)(TL + MfShape<P>::Z0 - m0 - 3) = __builtin_amdgcn_perm(0u, w, 0x00010203u);   // byte reverse
    }
}

template <int P>
struct R3bLds {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];   // Toeplitz bytes of the running value
    __attribute__((aligned(16))) uint8_t HB[S::HLEN];   // folded Hankel bytes of b_{i-1}
    __attribute__((aligned(16))) uint8_t HG[S::HLEN];   // folded Hankel bytes of g_i
    __attribute__((aligned(16))) int16_t C[RqShape<P>::JP];   // 1/g_i
};

// Two products in R/3 sharing the one-limb Toeplitz operand t (bytes TL):
// c1 = t y1 (folded bytes H1) to dst (int16) and c2 = t y2 (H2) to the
// Toeplitz bytes TLo (which may be TL itself), in one pass over the K-steps:
// t's fragments are read once for both.  Wave-local like mfma_mul.
template <int P>
__device__ __forceinline__ void r3_mul2(const uint8_t* TL, const uint8_t* H1, const uint8_t* H2, int16_t* dst,
                                        uint8_t* TLo) {
    using S = MfShape<P>;
    constexpr int NT = S::NT;
    static_assert(NT <= NTRUP_MF_MAXC_SMALL, "one chunk of tiles");
    const int lane = lane_id();
    const int rc = lane & 15, g = lane >> 4;
    const int32_t ap = (int32_t)(int8_t)TL[S::Z0 - (P - 1)];
    const int32_t bp1 = (int32_t)(int8_t)H1[S::HOFF + P - 1];
    const int32_t bp2 = (int32_t)(int8_t)H2[S::HOFF + P - 1];
    ToeplitzFrag nF(TL, S::Z0 - 16 * g - rc);
    const uint8_t* h1 = H1 + S::HOFF + 16 * (rc - g);
    const uint8_t* h2 = H2 + S::HOFF + 16 * (rc - g);
    mf_v4i a1[NT], a2[NT], nB1[NT], nB2[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) a1[t] = a2[t] = mf_v4i{0, 0, 0, 0};
    auto load_step = [&](int k) {
        nF.load(k);
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int off = 16 * (16 * t - 4 * k);
            nB1[t] = *(const mf_v4i*)(h1 + off);
            nB2[t] = *(const mf_v4i*)(h2 + off);
        }
    };
    load_step(0);
#pragma unroll
    for (int k = 0; k < S::NKS; k++) {
        if (NTRUP_MF_SCHED) __builtin_amdgcn_sched_barrier(0);
        const ToeplitzFrag F = nF;
        mf_v4i B1[NT], B2[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) {
            B1[t] = nB1[t];
            B2[t] = nB2[t];
        }
        if (k + 1 < S::NKS) load_step(k + 1);
        const mf_v4i tf = F.get();
#pragma unroll
        for (int t = 0; t < NT; t++) {
            a1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tf, B1[t], a1[t], 0, 0, 0);
            a2[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(tf, B2[t], a2[t], 0, 0, 0);
        }
    }
    // reduce mod 3 (centered), then c_0 -= conv_{p-1} = c_{p-1} - t_{p-1} y_{p-1}
    int32_t v1[NT][4], v2[NT][4];
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int i = 256 * t + 16 * rc + 4 * g;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            v1[t][e] = (i + e < P) ? freeze<3>(a1[t][e]) : 0;
            v2[t][e] = (i + e < P) ? freeze<3>(a2[t][e]) : 0;
        }
    }
    const int32_t cp1 = __builtin_amdgcn_readlane(v1[S::TP][0], S::LP);
    const int32_t cp2 = __builtin_amdgcn_readlane(v2[S::TP][0], S::LP);
    if (lane == 0) {
        v1[0][0] = freeze<3>(v1[0][0] - cp1 + ap * bp1);
        v2[0][0] = freeze<3>(v2[0][0] - cp2 + ap * bp2);
    }
    wave_sync();   // TLo may be TL, which the K-steps read
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int i = 256 * t + 16 * rc + 4 * g;
        if (i >= P) continue;
        if (i + 3 < P) {
            *(uint2*)(dst + i) = make_uint2((uint32_t)(uint16_t)v1[t][0] | ((uint32_t)(uint16_t)v1[t][1] << 16),
                                            (uint32_t)(uint16_t)v1[t][2] | ((uint32_t)(uint16_t)v1[t][3] << 16));
        } else {
            dst[i] = (int16_t)v1[t][0];   // p = 1 mod 4: c_{p-1} alone
        }
        uint32_t lo = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) lo |= ((uint32_t)v2[t][e] & 0xFFu) << (8 * (3 - e));
        *(uint32_t*)(TLo + S::Z0 - i - 3) = lo;
    }
}

template <int P>
__device__ __forceinline__ void r3b_load_g(const R3bArgs<P>& a, int key, uint32_t (&m)[KgShape<P>::NU],
                                           uint32_t (&s)[KgShape<P>::NU]) {
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t gm = 0, gs = 0;
        if (m0 < P) {
            const int wd = m0 >> 5, sh = m0 & 31;
            const uint32_t live = live4<P>(m0);
            gm = (a.gbits[(size_t)(2 * wd) * a.n + key] >> sh) & live;
            gs = (a.gbits[(size_t)(2 * wd + 1) * a.n + key] >> sh) & live;
        }
        m[u] = gm;
        s[u] = gs;
    }
}

// Prefix products of one group per wave.
template <int P>
__global__ __launch_bounds__(64) void r3b_prefix_kernel(R3bArgs<P> a) {
    using S = MfShape<P>;
    constexpr int NU = KgShape<P>::NU;
    __shared__ R3bLds<P> L;
    const int group = blockIdx.x;
    const int kw0 = group * a.G;
    const int gsz = min(a.G, a.n - kw0);
    if (gsz <= 0) return;
    const int lane = lane_id();
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.HG, S::HLEN);
    wave_sync();
    uint32_t m[NU], s[NU], w[NU];
    r3b_load_g<P>(a, kw0, m, s);
    r3b_put_toeplitz<P>(m, s, L.TL);                          // b_1 = g_1
    int8_t* row0 = a.rows + (size_t)kw0 * P;
    int8_t* prow = a.pj + (size_t)group * P;
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        const uint32_t bytes = spread4(m[u]) | (spread4(s[u]) * 0xFEu);
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (m0 + t < P) {
                row0[m0 + t] = (int8_t)(bytes >> (8 * t));
                if (gsz == 1) prow[m0 + t] = (int8_t)(bytes >> (8 * t));
            }
    }
    if (gsz == 1) return;
    for (int i = 1; i < gsz; i++) {
        r3b_load_g<P>(a, kw0 + i, m, s);
#pragma unroll
        for (int u = 0; u < NU; u++) w[u] = spread4(m[u]) | (spread4(s[u]) * 0xFEu);
        put_folded8<P>(w, L.HG);
        wave_sync();
        mfma_mul<P, false, false, 3>(L.TL, nullptr, L.HG, nullptr, nullptr, L.TL, nullptr, nullptr,
                                     a.rows + (size_t)(kw0 + i) * P);                    // b_{i+1}
        if (i + 1 == gsz) {
            wave_sync();
            // the group product from the reversed Toeplitz bytes
            for (int j = lane; j < P; j += 64) prow[j] = (int8_t)L.TL[S::Z0 - j];
        }
        wave_sync();
    }
}

// Back-substitution of one group per wave.
template <int P>
__global__ __launch_bounds__(64) void r3b_back_kernel(R3bArgs<P> a) {
    using S = MfShape<P>;
    constexpr int NU = KgShape<P>::NU;
    constexpr int WN = ceil_div(P, 32);
    __shared__ R3bLds<P> L;
    const int group = blockIdx.x;
    const int kw0 = group * a.G;
    const int gsz = min(a.G, a.n - kw0);
    if (gsz <= 0) return;
    const int lane = lane_id();
    const int ngroups = ceil_div(a.n, a.G);
    if (a.pok[group] != 1) {
        // some g of this group is not a unit: per-key divsteps for all of them
        int b0 = 0;
        if (lane == 0) b0 = atomicAdd(a.fb_count, gsz);
        b0 = __shfl(b0, 0);
        for (int i = lane; i < gsz; i += 64) a.fb_list[b0 + i] = kw0 + i;
        return;
    }
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.HB, S::HLEN);
    kg_zero<P>(L.HG, S::HLEN);
    wave_sync();
    uint32_t m[NU], s[NU], w[NU];
    // t = 1/b_G from the group reciprocal's bitsliced words
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t gm = 0, gs = 0;
        if (m0 < P) {
            const int wd = m0 >> 5, sh = m0 & 31;
            const uint32_t live = live4<P>(m0);
            gm = (a.pinv[(size_t)(2 * wd) * ngroups + group] >> sh) & live;
            gs = (a.pinv[(size_t)(2 * wd + 1) * ngroups + group] >> sh) & live;
        }
        m[u] = gm;
        s[u] = gs;
    }
    r3b_put_toeplitz<P>(m, s, L.TL);
    for (int i = gsz; i >= 1; i--) {
        const int key = kw0 + i - 1;
        wave_sync();
        if (i > 1) {
            // c_i = t b_{i-1}
            const int8_t* brow = a.rows + (size_t)(key - 1) * P;
#pragma unroll
            for (int u = 0; u < NU; u++) {
                const int m0 = 4 * lane + 256 * u;
                uint32_t v = 0;
#pragma unroll
                for (int t = 0; t < 4; t++)
                    if (m0 + t < P) v |= (uint32_t)(uint8_t)brow[m0 + t] << (8 * t);
                w[u] = v;
            }
            put_folded8<P>(w, L.HB);
            // and t <- t g_i, in the same pass over the K-steps
            r3b_load_g<P>(a, key, m, s);
#pragma unroll
            for (int u = 0; u < NU; u++) w[u] = spread4(m[u]) | (spread4(s[u]) * 0xFEu);
            put_folded8<P>(w, L.HG);
            wave_sync();
            r3_mul2<P>(L.TL, L.HB, L.HG, L.C, L.TL);
        } else {
            for (int j = lane; j < P; j += 64) L.C[j] = (int16_t)(int8_t)L.TL[S::Z0 - j];   // c_1 = t
        }
        wave_sync();
        // 1/g of key as bitsliced words: one ballot per 64 coefficients and plane
#pragma unroll
        for (int r = 0; r < ceil_div(WN, 2); r++) {
            const int i2 = 64 * r + lane;
            const int v = i2 < P ? L.C[i2] : 0;
            const unsigned long long bm = __ballot(v != 0), bs = __ballot(v < 0);
            if (lane < 2 && 2 * r + lane < WN) {
                const int k = 2 * r + lane;
                a.ibits[(size_t)(2 * k) * a.n + key] = (uint32_t)(bm >> (32 * lane));
                a.ibits[(size_t)(2 * k + 1) * a.n + key] = (uint32_t)(bs >> (32 * lane));
            }
        }
    }
}

// The group products' reciprocals shared by up to kR3Share groups: one
// workgroup of kR3Share waves per kR3Share consecutive group products
// P_0 .. P_{k-1} (rows, int8): Q_0 = P_0, Q_w = Q_{w-1} P_w (wave 0), one
// reciprocal T = 1/Q_{k-1} by jump divsteps over F_3 with the four products of
// each jump on the waves side by side, then 1/P_w = T Q_{w-1} and T <- T P_w
// (wave 0) -- Montgomery's trick again, as on the R/q side.  Writes each 1/P_w
// as bitsliced words to ibits ([WN][2][n]) and ok = 1; if Q_{k-1} is not a
// unit (some P_w is not) every group of the workgroup gets ok = 0, and their
// keys take the per-key pass.
constexpr int kR3Share = 4;

template <int P>
struct R3ShareLds {
    using S = MfShape<P>;
    static constexpr int PR = round_up(P, 64);
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];
    __attribute__((aligned(16))) uint8_t HB[S::HLEN];
    __attribute__((aligned(16))) int16_t C[RqShape<P>::JP];
    __attribute__((aligned(16))) int8_t Q[kR3Share][PR];   // Q_w, then 1/P_w
    __attribute__((aligned(16))) int8_t X[PR];             // T
    JumpLds<P> JL;
};

// dst = x y in R/3 for int8 rows in LDS (one wave): x as the Toeplitz operand,
// y folded; TL and HB keep their zero padding.
template <int P>
__device__ __forceinline__ void r3_share_mul(const int8_t* x, const int8_t* y, int8_t* dst, R3ShareLds<P>& L) {
    using S = MfShape<P>;
    const int lane = lane_id();
    for (int m = lane; m < P; m += 64) {
        L.TL[S::Z0 - m] = (uint8_t)x[m];
        // folded E: E_m = y_m (1 <= m < p), E_0 = y_0 + y_{p-1},
        // E_{m-p} = y_m + y_{m-1} (1 <= m < p)
        L.HB[S::HOFF + m] = (uint8_t)(m == 0 ? (int8_t)(y[0] + y[P - 1]) : y[m]);
        if (m >= 1) L.HB[S::HOFF + m - P] = (uint8_t)(int8_t)(y[m] + y[m - 1]);
    }
    wave_sync();
    mfma_mul<P, false, false, 3>(L.TL, nullptr, L.HB, nullptr, L.C, nullptr, nullptr, nullptr);
    wave_sync();
    for (int m = lane; m < P; m += 64) dst[m] = (int8_t)L.C[m];
    wave_sync();
}

// 1/P_w as bitsliced words (one wave).
template <int P>
__device__ __forceinline__ void r3_share_store(const int8_t* x, uint32_t* ibits, int n, int e) {
    constexpr int WN = ceil_div(P, 32);
    const int lane = lane_id();
    for (int base = 0; base < P; base += 64) {
        const int i = base + lane;
        const int c = (i < P) ? (int)x[i] : 0;
        const uint64_t nz = __ballot(c != 0), neg = __ballot(c < 0);
        if (lane == 0) {
            const int k = base / 32;
            ibits[(size_t)(2 * k) * n + e] = (uint32_t)nz;
            ibits[(size_t)(2 * k + 1) * n + e] = (uint32_t)neg;
            if (k + 1 < WN) {
                ibits[(size_t)(2 * k + 2) * n + e] = (uint32_t)(nz >> 32);
                ibits[(size_t)(2 * k + 3) * n + e] = (uint32_t)(neg >> 32);
            }
        }
    }
}

template <int P>
__global__ __launch_bounds__(64 * kR3Share) void r3_share_recip_kernel(int n, const int8_t* rows, uint32_t* ibits,
                                                                       uint8_t* ok) {
    using S = MfShape<P>;
    __shared__ R3ShareLds<P> L;
    const int wave = (int)(threadIdx.x >> 6), lane = lane_id();
    const int g0 = (int)blockIdx.x * kR3Share;
    const int k = min(kR3Share, n - g0);   // groups of this workgroup, >= 1
    // the Toeplitz and Hankel padding stays zero
    for (int i = threadIdx.x; i < S::TLEN; i += 64 * kR3Share) L.TL[i] = 0;
    for (int i = threadIdx.x; i < S::HLEN; i += 64 * kR3Share) L.HB[i] = 0;
    __syncthreads();
    if (wave == 0) {
        // Q_0 = P_0, Q_w = Q_{w-1} P_w; the last one to X
        for (int m = lane; m < P; m += 64) L.Q[0][m] = rows[(size_t)g0 * P + m];
        wave_sync();
        for (int w = 1; w < k; w++) r3_share_mul<P>(L.Q[w - 1], rows + (size_t)(g0 + w) * P, L.Q[w], L);
        for (int m = lane; m < P; m += 64) L.X[m] = L.Q[k - 1][m];
    }
    __syncthreads();
    const int unit = recip_jump_block<P, 3, int8_t, true>(L.X, L.X, L.JL, wave, kR3Share);
    if (wave != 0) return;
    if (!unit) {
        if (lane < k) ok[g0 + lane] = 0;
        return;
    }
    // 1/P_w = T Q_{w-1}, T <- T P_w (w = k-1 .. 1), 1/P_0 = T
    for (int w = k - 1; w >= 1; w--) {
        r3_share_mul<P>(L.X, L.Q[w - 1], L.Q[w], L);                          // 1/P_w over Q_w
        r3_share_mul<P>(L.X, rows + (size_t)(g0 + w) * P, L.X, L);            // T <- T P_w
        r3_share_store<P>(L.Q[w], ibits, n, g0 + w);
    }
    r3_share_store<P>(L.X, ibits, n, g0);
    if (lane < k) ok[g0 + lane] = 1;
}

// c = a b in R/3 (int8 rows, centered), for the kernel tests.
template <int P>
__global__ __launch_bounds__(64) void mul3_kernel(int n, const int8_t* x, const int8_t* y, int8_t* z) {
    using S = MfShape<P>;
    constexpr int NU = KgShape<P>::NU;
    __shared__ R3bLds<P> L;
    const int e = blockIdx.x;
    if (e >= n) return;
    const int lane = lane_id();
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.HG, S::HLEN);
    wave_sync();
    uint32_t w[NU];
    for (int j = lane; j < P; j += 64) L.TL[S::Z0 - j] = (uint8_t)y[(size_t)e * P + j];
#pragma unroll
    for (int u = 0; u < NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t v = 0;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (m0 + t < P) v |= (uint32_t)(uint8_t)x[(size_t)e * P + m0 + t] << (8 * t);
        w[u] = v;
    }
    put_folded8<P>(w, L.HG);
    wave_sync();
    mfma_mul<P, false, false, 3>(L.TL, nullptr, L.HG, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 z + (size_t)e * P);
}

}  // namespace ntrup
