// Batched KeyGen group stage on the matrix cores (Section 3.1 KeyGen with the
// batch inversion of Section 2.2): for each key h = g / (3f) in R/q, encoded
// with f and 1/g into (pk, sk).  Two kernels:
//
// keygen_prefix_kernel<P, W>: one workgroup = W waves; wave w owns a
//   Montgomery group of G keys.
//   1. prefix (every wave): b_1 = 3f_1, b_i = 3f_i b_{i-1}; rows b_i kept in
//      HBM, P_w = b_G stays in the wave's LDS;
//   2. shared reciprocal (wave 0; the others have ended, or, with jump
//      divsteps, compute the products of each jump beside it): Q_0 = P_0,
//      Q_w = Q_{w-1} P_w, one constant-time divstep reciprocal
//      T = 1/Q_{W-1}, then for w = W-1..1: 1/P_w = T Q_{w-1} and T <- T P_w;
//      1/P_0 = T -- the same trick one level up; each 1/P_w goes to HBM.
//   This kernel needs only f, so it runs beside the R/3 stage.
// keygen_back_kernel<P>: one wave per group:
//   3. back-substitution from t = 1/P: c_i = t b_{i-1} (= 1/(3f_i)),
//      t <- t 3f_i, h_i = g_i c_i, then encoding.
// Or step 3 in two kernels, so that the part that needs only f runs beside
// the R/3 stage too:
// keygen_cinv_kernel<P>: one wave per group: c_i and t as above, each c_i
//   written to HBM over the prefix row b_i (already consumed);
// keygen_h_kernel<P>: one wave per key: h_i = g_i c_i and encoding.
// Every product is mfma_mul with the running value as Toeplitz operand.
//
// Latency: the next key's operands (the f row, the stored prefix row, the
// bitsliced g and 1/g words) are loaded into registers one step ahead and
// written to LDS at the start of the step; waves order their own LDS traffic
// with wave_sync.
//
// Register layout of the per-key operands: lane l holds coefficients
// m = 4l + 256u + t (t = 0..3, u < NU), four per 32-bit word, which is also the
// layout of sk (byte b = l + 64u covers coefficients 4b..4b+3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ntrup_kernels.h"
#include "ntrup_mfma.h"
#include "ntrup_params.h"
#include "ntrup_rq.h"

namespace ntrup {

template <int P>
struct KgShape {
    static constexpr int NU = ceil_div(P, 256);   // 4-coefficient words per lane
    static constexpr int WN = ceil_div(P, 32);    // bitsliced words per plane
};

// Per-wave LDS of the KeyGen group kernel.
template <int P>
struct KgWave {
    using S = MfShape<P>;
    static constexpr int STG = 64 * RqShape<P>::RI;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];   // Toeplitz limbs of the running value
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t UL[S::TLEN];   // Toeplitz limbs of c_i
    __attribute__((aligned(16))) uint8_t UH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HL[S::HLEN];   // Hankel limbs of a big operand
    __attribute__((aligned(16))) uint8_t HH[S::HLEN];
    __attribute__((aligned(16))) uint8_t HS[S::HLEN];   // 3 f of the current key
    __attribute__((aligned(16))) uint8_t HG[S::HLEN];   // g of the current key
    __attribute__((aligned(16))) int32_t ST[STG];       // divstep staging
    __attribute__((aligned(16))) int16_t Bb[RqShape<P>::JP];  // running value
    __attribute__((aligned(16))) int16_t Cb[RqShape<P>::JP];  // c_i, h_i, chain values
};

// Operands of one key, in registers.
template <int P>
struct KgRegs {
    static constexpr int NU = KgShape<P>::NU;
    uint32_t f[NU];       // f bytes (int8), four coefficients per word
    uint32_t b[NU][2];    // stored prefix row b_{i-1}: four int16
    uint32_t gm[NU], gs[NU];   // g: nonzero / negative bits (4 per word, low bits)
    uint32_t im[NU], is[NU];   // 1/g in R/3, same form
};

// Coefficient mask of the 4-coefficient word starting at m0.
template <int P>
__device__ __forceinline__ uint32_t live4(int m0) {
    return m0 >= P ? 0u : (P - m0 >= 4 ? 0xFu : ((1u << (P - m0)) - 1u));
}

template <int P>
__device__ __forceinline__ void kg_load_f(const int8_t* f_rows, int key, KgRegs<P>& r) {
    const int lane = lane_id();
    const uint8_t* row = (const uint8_t*)f_rows + (size_t)key * P;
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (m0 + t < P) w |= (uint32_t)row[m0 + t] << (8 * t);
        r.f[u] = w;
    }
}

template <int P>
__device__ __forceinline__ void kg_load_b(const int16_t* bscr, int row_index, KgRegs<P>& r) {
    const int lane = lane_id();
    const uint16_t* row = (const uint16_t*)bscr + (size_t)row_index * P;
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t v[4];
#pragma unroll
        for (int t = 0; t < 4; t++) v[t] = (m0 + t < P) ? (uint32_t)row[m0 + t] : 0u;
        r.b[u][0] = v[0] | (v[1] << 16);
        r.b[u][1] = v[2] | (v[3] << 16);
    }
}

template <int P>
__device__ __forceinline__ void kg_load_bits(const uint32_t* gbits, const uint32_t* ibits, int n, int key,
                                             KgRegs<P>& r) {
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        uint32_t gm = 0, gs = 0, im = 0, is = 0;
        if (m0 < P) {
            const int wd = m0 >> 5, sh = m0 & 31;
            const uint32_t live = live4<P>(m0);
            gm = (gbits[(size_t)(2 * wd) * n + key] >> sh) & live;
            gs = (gbits[(size_t)(2 * wd + 1) * n + key] >> sh) & live;
            im = (ibits[(size_t)(2 * wd) * n + key] >> sh) & live;
            is = (ibits[(size_t)(2 * wd + 1) * n + key] >> sh) & live;
        }
        r.gm[u] = gm;
        r.gs[u] = gs;
        r.im[u] = im;
        r.is[u] = is;
    }
}

// Four bits -> four bytes (bit t to the low bit of byte t).
__device__ __forceinline__ uint32_t spread4(uint32_t x) { return ((x & 0xFu) * 0x00204081u) & 0x01010101u; }
// Four bits -> four 2-bit fields (bit t to bit 2t).
__device__ __forceinline__ uint32_t spread2(uint32_t x) {
    return (x & 1u) | ((x & 2u) << 1) | ((x & 4u) << 2) | ((x & 8u) << 3);
}

// Folded Hankel bytes of 3 f (bytes 0x00, 0x01, 0xFF -> 0x00, 0x03, 0xFD).
template <int P>
__device__ __forceinline__ void kg_put_3f(const KgRegs<P>& r, uint8_t* HS) {
    uint32_t w[KgShape<P>::NU];
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) w[u] = r.f[u] ^ ((r.f[u] & 0x01010101u) << 1);
    put_folded8<P>(w, HS);
}

// Folded Hankel bytes of g (byte 0x01 for g = 1, 0xFF for g = -1).
template <int P>
__device__ __forceinline__ void kg_put_g(const KgRegs<P>& r, uint8_t* HG) {
    uint32_t w[KgShape<P>::NU];
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) w[u] = spread4(r.gm[u]) | (spread4(r.gs[u]) * 0xFEu);
    put_folded8<P>(w, HG);
}

// Folded Hankel limbs of the stored row b.
template <int P>
__device__ __forceinline__ void kg_put_b(const KgRegs<P>& r, uint8_t* HL, uint8_t* HH) {
    put_folded16<P>(r.b, HL, HH);
}

// The first prefix value b_1 = 3 f: X[m] = 3 f_m (int16), the same row to
// HBM, and its reversed Toeplitz limbs TL[Z0 - m] = 3 f_m (the high limbs of
// |3 f_m| <= 3 are 0: TH must hold zeros).
template <int P>
__device__ __forceinline__ void kg_put_3f16(const KgRegs<P>& r, int16_t* X, uint8_t* TL, int16_t* row) {
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        if (m0 >= P) continue;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (m0 + t < P) {
                const int16_t v = (int16_t)(3 * (int32_t)(int8_t)(r.f[u] >> (8 * t)));
                X[m0 + t] = v;
                row[m0 + t] = v;
            }
        }
        const uint32_t f3 = r.f[u] ^ ((r.f[u] & 0x01010101u) << 1);
        *(uint32_t*)(TL + MfShape<P>::Z0 - m0 - 3) = __builtin_amdgcn_perm(0u, f3, 0x00010203u);   // byte reverse
    }
}

// sk = (f, 1/g) as 2-bit fields c + 1, four per byte; pk = h_i + (q-1)/2 as
// 13-bit fields (h in LDS).
template <int P>
__device__ __forceinline__ void kg_encode(int key, const int16_t* H, const KgRegs<P>& r, uint8_t* pk_out,
                                          uint8_t* sk_out) {
    constexpr int Q = Param<P>::q;
    constexpr int PKB = pk_bytes(P), SKH = sk_half_bytes(P);
    constexpr int NO = ceil_div(P, 8);   // octets of coefficients: 8 fields of 13 bits = 13 bytes
    static_assert(8 * NO <= RqShape<P>::JP, "octet reads stay inside the LDS row");
    const int lane = lane_id();
    uint8_t* pk = pk_out + (size_t)key * PKB;
    for (int k = lane; k < NO; k += 64) {
        const uint4 hv = *(const uint4*)(H + 8 * k);
        const uint32_t hw[4] = {hv.x, hv.y, hv.z, hv.w};
        const int c = min(8, P - 8 * k);   // live coefficients of the octet
        uint32_t u[8];
#pragma unroll
        for (int e = 0; e < 8; e++)
            u[e] = (e < c) ? (uint32_t)((int32_t)(int16_t)(hw[e >> 1] >> (16 * (e & 1))) + (Q - 1) / 2) : 0u;
        // field e at bits [13e, 13e + 13) of the octet's 104-bit little-endian string
        const uint32_t w[4] = {u[0] | (u[1] << 13) | (u[2] << 26), (u[2] >> 6) | (u[3] << 7) | (u[4] << 20),
                               (u[4] >> 12) | (u[5] << 1) | (u[6] << 14) | (u[7] << 27), u[7] >> 5};
        const int nb = (13 * c + 7) / 8;
        uint8_t* dst = pk + 13 * k;
#pragma unroll
        for (int b = 0; b < 13; b++)
            if (b < nb) dst[b] = (uint8_t)(w[b >> 2] >> (8 * (b & 3)));
    }
    uint8_t* sk = sk_out + (size_t)key * 2 * SKH;
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int b = lane + 64 * u;
        if (b < SKH) {
            const uint32_t live = live4<P>(4 * b);
            // f + 1 per byte without carries between bytes
            const uint32_t x = ((r.f[u] & 0x7F7F7F7Fu) + 0x01010101u) ^ (r.f[u] & 0x80808080u);
            uint32_t bf = (x & 3u) | ((x >> 6) & 0xCu) | ((x >> 12) & 0x30u) | ((x >> 18) & 0xC0u);
            bf &= spread2(live) * 3u;
            const uint32_t bi = (spread2(~r.im[u] & live)) | (spread2(r.im[u] & ~r.is[u] & live) << 1);
            sk[b] = (uint8_t)bf;
            sk[SKH + b] = (uint8_t)bi;
        }
    }
}

template <int P>
__device__ __forceinline__ void kg_zero(uint8_t* p, int bytes) {
    for (int i = lane_id(); i < bytes / 4; i += 64) ((uint32_t*)p)[i] = 0u;
}

template <int P>
__device__ __forceinline__ void kg_set_one(int16_t* X) {
    for (int i = lane_id(); i < P; i += 64) X[i] = (int16_t)(i == 0);
}

template <int P>
__device__ __forceinline__ void kg_copy(const int16_t* src, int16_t* dst) {
    for (int i = lane_id(); i < P; i += 64) dst[i] = src[i];
}

// One back-substitution step for key kw0 + i - 1 (i >= 1): operands in cur,
// the next step's operands loaded into nxt.  On entry TL/TH hold the limbs
// of t = 1/b_i; on exit those of t 3f_i.
template <int P>
__device__ __forceinline__ void kg_back_step(const GroupArgs& args, KgWave<P>& L, int kw0, int i, KgRegs<P>& cur,
                                             KgRegs<P>& nxt) {
    const int key = kw0 + i - 1;
    kg_put_3f<P>(cur, L.HS);
    kg_put_g<P>(cur, L.HG);
    if (i > 1) {
        kg_put_b<P>(cur, L.HL, L.HH);
        kg_load_f<P>(args.f_rows, key - 1, nxt);
        if (i > 2) kg_load_b<P>(args.bscr, key - 2, nxt);
        kg_load_bits<P>(args.gbits, args.ibits, args.n, key - 1, nxt);
    }
    wave_sync();
    const uint8_t* CL = L.TL;   // i == 1: c_1 = t_1
    const uint8_t* CH = L.TH;
    if (i > 1) {
        // c_i = t b_{i-1} and t <- t 3f_i in one pass over the K-steps
        mfma_mul2<P>(L.TL, L.TH, L.HL, L.HH, L.HS, L.UL, L.UH, L.TL, L.TH);
        wave_sync();
        CL = L.UL;
        CH = L.UH;
    }
    mfma_mul<P, false>(CL, CH, L.HG, nullptr, L.Cb, nullptr, nullptr, nullptr);     // h = g c_i
    wave_sync();
    kg_encode<P>(key, L.Cb, cur, args.pk, args.sk);
}

// Reversed Toeplitz limbs of a big operand held in registers (the layout of
// KgRegs::b): TL[Z0 - m] = lo(x_m), TH likewise.  Entries outside [0, p) are
// left as they are (zero).
template <int P>
__device__ __forceinline__ void kg_put_toeplitz16(const uint32_t (&w)[KgShape<P>::NU][2], uint8_t* TL, uint8_t* TH) {
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < KgShape<P>::NU; u++) {
        const int m0 = 4 * lane + 256 * u;
        if (m0 >= P) continue;
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            uint32_t l, h;
            split_limb((int32_t)(int16_t)(w[u][e >> 1] >> (16 * (e & 1))), l, h);
            lo |= l << (8 * (3 - e));
            hi |= h << (8 * (3 - e));
        }
        *(uint32_t*)(TL + MfShape<P>::Z0 - m0 - 3) = lo;
        *(uint32_t*)(TH + MfShape<P>::Z0 - m0 - 3) = hi;
    }
}

// One step of the back-substitution alone, for key kw0 + i - 1 (i >= 1):
// c_i to the key's row of bscr (which held b_i, read one step earlier),
// t <- t 3f_i.  On entry TL/TH hold the limbs of t = 1/b_i.
template <int P>
__device__ __forceinline__ void kg_cinv_step(const GroupArgs& args, KgWave<P>& L, int kw0, int i, KgRegs<P>& cur,
                                             KgRegs<P>& nxt) {
    using S = MfShape<P>;
    const int key = kw0 + i - 1;
    int16_t* row = args.bscr + (size_t)key * P;
    if (i > 1) {
        kg_put_3f<P>(cur, L.HS);
        kg_put_b<P>(cur, L.HL, L.HH);
        kg_load_f<P>(args.f_rows, key - 1, nxt);
        if (i > 2) kg_load_b<P>(args.bscr, key - 2, nxt);
        wave_sync();
        // c_i = t b_{i-1} to HBM and t <- t 3f_i in one pass over the K-steps
        mfma_mul2_row<P>(L.TL, L.TH, L.HL, L.HH, L.HS, row, L.TL, L.TH);
        wave_sync();
    } else {
        // c_1 = t
        for (int m = lane_id(); m < P; m += 64)
            row[m] = (int16_t)((int32_t)(int8_t)L.TL[S::Z0 - m] + 128 * (int32_t)(int8_t)L.TH[S::Z0 - m]);
    }
}

// The back-substitution of group `group` from t = 1/P (row trow): every
// c_i = 1/(3 f_i) of the group to HBM.  One wave.
template <int P>
__device__ __forceinline__ void kg_cinv_group(const GroupArgs& args, int group, const int16_t* trow, KgWave<P>& L) {
    using S = MfShape<P>;
    const int kw0 = group * args.G;
    const int gsz = max(0, min(args.G, args.n - kw0));
    if (gsz <= 0) return;
    kg_zero<P>(L.HL, S::HLEN);
    kg_zero<P>(L.HH, S::HLEN);
    kg_zero<P>(L.HS, S::HLEN);
    KgRegs<P> ra, rb;
    kg_load_f<P>(args.f_rows, kw0 + gsz - 1, ra);
    if (gsz >= 2) kg_load_b<P>(args.bscr, kw0 + gsz - 2, ra);
    for (int j = lane_id(); j < P; j += 64) L.Bb[j] = trow[j];
    wave_sync();
    build_toeplitz<P>(L.Bb, L.TL, L.TH);
    wave_sync();
    for (int i = gsz; i >= 1; i -= 2) {
        kg_cinv_step<P>(args, L, kw0, i, ra, rb);
        if (i >= 2) kg_cinv_step<P>(args, L, kw0, i - 1, rb, ra);
    }
}

template <int P>
__global__ __launch_bounds__(64, (P < 800 ? 2 : 1)) void keygen_cinv_kernel(GroupArgs args, const int16_t* tinv) {
    __shared__ KgWave<P> L;
    // on the side stream beside the R/3 stage, like the prefix kernel
    __builtin_amdgcn_s_setprio(3);
    kg_cinv_group<P>(args, (int)blockIdx.x, tinv + (size_t)blockIdx.x * P, L);
}

// Per-wave LDS of the h kernel.
template <int P>
struct KgHWave {
    using S = MfShape<P>;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];   // Toeplitz limbs of c
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HG[S::HLEN];   // g
    __attribute__((aligned(16))) int16_t Cb[RqShape<P>::JP];  // h
};

// h = g c for one key per wave (c = 1/(3f) from the key's row of bscr), then
// the encoding of pk and sk.  Workgroups go to the eight XCDs in turn, and
// the g and 1/g words of 32 consecutive keys share a cache line (key-minor
// planes), so XCD x takes the contiguous key range [x per, (x+1) per): grid
// 8 per, block b -> key (b mod 8) per + b / 8.
template <int P>
__global__ __launch_bounds__(64) void keygen_h_kernel(GroupArgs args, int per) {
    using S = MfShape<P>;
    __shared__ KgHWave<P> L;
    const int key = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    if (key >= args.n) return;
    KgRegs<P> r;
    kg_load_b<P>(args.bscr, key, r);
    kg_load_f<P>(args.f_rows, key, r);
    kg_load_bits<P>(args.gbits, args.ibits, args.n, key, r);
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.TH, S::TLEN);
    kg_zero<P>(L.HG, S::HLEN);
    wave_sync();
    kg_put_toeplitz16<P>(r.b, L.TL, L.TH);
    kg_put_g<P>(r, L.HG);
    wave_sync();
    mfma_mul<P, false>(L.TL, L.TH, L.HG, nullptr, L.Cb, nullptr, nullptr, nullptr);
    wave_sync();
    kg_encode<P>(key, L.Cb, r, args.pk, args.sk);
}

// Per-wave LDS of the prefix kernel (no c_i or g operands).
template <int P>
struct KgPrefixWave {
    using S = MfShape<P>;
    static constexpr int STG = KgWave<P>::STG;
    __attribute__((aligned(16))) uint8_t TL[S::TLEN];
    __attribute__((aligned(16))) uint8_t TH[S::TLEN];
    __attribute__((aligned(16))) uint8_t HL[S::HLEN];
    __attribute__((aligned(16))) uint8_t HH[S::HLEN];
    __attribute__((aligned(16))) uint8_t HS[S::HLEN];
    __attribute__((aligned(16))) int32_t ST[STG];
    __attribute__((aligned(16))) int16_t Bb[RqShape<P>::JP];
    __attribute__((aligned(16))) int16_t Cb[RqShape<P>::JP];
};

// Step 1 for one group (keys kw0 .. kw0+gsz-1): prefix rows b_i to HBM, the
// group product b_gsz left in L.Bb (1 for an empty group).  One wave.
template <int P>
__device__ __forceinline__ void kg_prefix_chain(const GroupArgs& args, int kw0, int gsz, KgPrefixWave<P>& L) {
    using S = MfShape<P>;
    int16_t* bscr = args.bscr;
    kg_zero<P>(L.TL, S::TLEN);
    kg_zero<P>(L.TH, S::TLEN);
    kg_zero<P>(L.HS, S::HLEN);
    wave_sync();
    KgRegs<P> ra;
    if (gsz >= 1) {
        kg_load_f<P>(args.f_rows, kw0, ra);
        kg_put_3f16<P>(ra, L.Bb, L.TL, bscr + (size_t)kw0 * P);
        if (gsz > 1) kg_load_f<P>(args.f_rows, kw0 + 1, ra);
        for (int i = 1; i < gsz; i++) {
            kg_put_3f<P>(ra, L.HS);
            if (i + 1 < gsz) kg_load_f<P>(args.f_rows, kw0 + i + 1, ra);
            wave_sync();
            mfma_mul<P, false>(L.TL, L.TH, L.HS, nullptr, i + 1 == gsz ? L.Bb : nullptr, L.TL, L.TH,
                               bscr + (size_t)(kw0 + i) * P);
            wave_sync();
        }
    } else {
        kg_set_one<P>(L.Bb);
    }
}

// Steps 1 and 2: prefix products of each wave's group (rows b_i to HBM), then
// wave 0 alone inverts the W group products with one reciprocal and writes
// t = 1/P_w of every group to tinv (int16 [groups][p]).  The other waves end
// after the prefix barrier, so their registers serve other work (the R/3
// stage runs beside this kernel) while wave 0 runs the reciprocal.
//
// J: the shared reciprocal by jump divsteps on the matrix cores
// (recip_jump_wave) instead of the plain divstep loop (recip_wave).
template <int P, int W, bool J>
__global__ __launch_bounds__(64 * W, (P < 800 ? 2 : 1)) void keygen_prefix_kernel(GroupArgs args, int16_t* tinv) {
    __shared__ KgPrefixWave<P> LW[W];
    __shared__ typename std::conditional<J, JumpLds<P>, char>::type JL;
    const int wave = (int)(threadIdx.x >> 6);
    KgPrefixWave<P>& L = LW[wave];
    const int n = args.n;
    const int G = args.G;
    const int group = blockIdx.x * W + wave;
    const int kw0 = group * G;
    const int gsz = max(0, min(G, n - kw0));
    // this kernel's latency (a chain of products, then one long divstep
    // reciprocal on one wave) bounds the pipeline while the R/3 stage runs
    // beside it: its waves take issue priority over the R/3 waves
    __builtin_amdgcn_s_setprio(3);

    kg_prefix_chain<P>(args, kw0, gsz, L);
    __syncthreads();
    // with jump divsteps and W = 2 or 4 every wave of the block takes part in
    // the reciprocal (the four products of each jump side by side);
    // otherwise wave 0 finishes alone, and no barrier follows.  (With W = 8
    // the waves kept for the reciprocal would hold registers that the R/3
    // stage beside this kernel needs: 1.62 against 1.41 ms per batch.)
    constexpr bool COOP = J && (W == 2 || W == 4);
    if (!COOP && wave != 0) return;

    if (W == 1) {
        int ok;
        if constexpr (J) ok = recip_jump_wave<P>(L.Bb, L.Bb, JL);
        else ok = recip_wave<P>(L.Bb, L.Bb, L.ST);
        if (!ok && lane_id() == 0) atomicOr(args.err, 2);
    } else {
        // Q_{w-1} -> LW[w].Cb, Q_{W-1} -> LW[0].Cb; the Hankel arrays are
        // written whole by build_hankel (zero padding included)
        if (wave == 0) {
            kg_copy<P>(LW[0].Bb, LW[1].Cb);
            for (int w = 1; w < W; w++) {
                wave_sync();
                build_toeplitz<P>(LW[w].Cb, L.TL, L.TH);
                build_hankel<P>(LW[w].Bb, L.HL, L.HH);
                wave_sync();
                mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, w + 1 < W ? LW[w + 1].Cb : LW[0].Cb, nullptr, nullptr,
                                  nullptr);
            }
            wave_sync();
        }
        int ok;
        if constexpr (COOP) {
            __syncthreads();
            ok = recip_jump_block<P, Param<P>::q, int16_t, true>(LW[0].Cb, LW[0].Cb, JL, wave, W);
            if (wave != 0) return;
        } else if constexpr (J) {
            ok = recip_jump_wave<P>(LW[0].Cb, LW[0].Cb, JL);
        } else {
            ok = recip_wave<P>(LW[0].Cb, LW[0].Cb, L.ST);
        }
        if (!ok && lane_id() == 0) atomicOr(args.err, 2);
        for (int w = W - 1; w >= 1; w--) {
            wave_sync();
            build_toeplitz<P>(LW[0].Cb, L.TL, L.TH);   // T = 1/Q_w
            build_hankel<P>(LW[w].Bb, L.HL, L.HH);      // P_w
            wave_sync();
            mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, LW[0].Cb, nullptr, nullptr, nullptr);  // T <- T P_w
            wave_sync();
            build_hankel<P>(LW[w].Cb, L.HL, L.HH);      // Q_{w-1}
            wave_sync();
            mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, LW[w].Bb, nullptr, nullptr, nullptr);  // 1/P_w
        }
        wave_sync();
        kg_copy<P>(LW[0].Cb, LW[0].Bb);
    }
    wave_sync();
    for (int w = 0; w < W; w++) {
        const int grp = blockIdx.x * W + w;
        if ((size_t)grp * G >= (size_t)n) break;
        for (int j = lane_id(); j < P; j += 64) tinv[(size_t)grp * P + j] = LW[w].Bb[j];
    }
}

// Step 2 with the group products in HBM: groups grp0 .. grp0+wn-1 hold P_w
// in rows of tinv ([groups][p]); on exit those rows hold 1/P_w.  qrow
// ([groups][p]) keeps the partial products Q_0 .. Q_{wn-2}.  One wave.
template <int P>
__device__ __forceinline__ void kg_shared_recip_rows(const GroupArgs& args, int grp0, int wn, int16_t* tinv, int16_t* qrow,
                                     KgPrefixWave<P>& L) {
    const int lane = lane_id();
    int16_t* P0 = tinv + (size_t)grp0 * P;
    for (int j = lane; j < P; j += 64) {
        const int16_t v = P0[j];
        L.Cb[j] = v;                                   // Q_0 = P_0
        qrow[(size_t)grp0 * P + j] = v;
    }
    for (int w = 1; w < wn; w++) {
        wave_sync();
        build_toeplitz<P>(L.Cb, L.TL, L.TH);                            // Q_{w-1}
        build_hankel<P>(tinv + (size_t)(grp0 + w) * P, L.HL, L.HH);     // P_w
        wave_sync();
        mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, L.Cb, nullptr, nullptr,
                          w + 1 < wn ? qrow + (size_t)(grp0 + w) * P : nullptr);   // Q_w
    }
    wave_sync();
    const int ok = recip_wave<P>(L.Cb, L.Bb, L.ST);                      // T = 1/Q_{wn-1}
    if (!ok && lane == 0) atomicOr(args.err, 2);
    __threadfence();   // the qrow rows this wave wrote are read back below
    for (int w = wn - 1; w >= 1; w--) {
        wave_sync();
        build_toeplitz<P>(L.Bb, L.TL, L.TH);                            // T
        build_hankel<P>(tinv + (size_t)(grp0 + w) * P, L.HL, L.HH);     // P_w
        wave_sync();
        mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, L.Cb, nullptr, nullptr, nullptr);   // T P_w
        wave_sync();
        build_hankel<P>(qrow + (size_t)(grp0 + w - 1) * P, L.HL, L.HH); // Q_{w-1}
        wave_sync();
        mfma_mul<P, true>(L.TL, L.TH, L.HL, L.HH, nullptr, nullptr, nullptr,
                          tinv + (size_t)(grp0 + w) * P);                // 1/P_w over P_w
        wave_sync();
        kg_copy<P>(L.Cb, L.Bb);                                          // T <- T P_w
    }
    wave_sync();
    for (int j = lane; j < P; j += 64) P0[j] = L.Bb[j];                  // 1/P_0 = T
}

// Step 3: back-substitution from t = 1/P (row trow of the group's
// reciprocal), h = g c and encoding, for group `group`.  One wave.
template <int P>
__device__ __forceinline__ void kg_back_group(const GroupArgs& args, int group, const int16_t* trow, KgWave<P>& L) {
    using S = MfShape<P>;
    const int n = args.n;
    const int G = args.G;
    const int kw0 = group * G;
    const int gsz = max(0, min(G, n - kw0));
    if (gsz <= 0) return;
    kg_zero<P>(L.UL, S::TLEN);
    kg_zero<P>(L.UH, S::TLEN);
    kg_zero<P>(L.HL, S::HLEN);
    kg_zero<P>(L.HH, S::HLEN);
    kg_zero<P>(L.HS, S::HLEN);
    kg_zero<P>(L.HG, S::HLEN);
    KgRegs<P> ra, rb;
    kg_load_f<P>(args.f_rows, kw0 + gsz - 1, ra);
    if (gsz >= 2) kg_load_b<P>(args.bscr, kw0 + gsz - 2, ra);
    kg_load_bits<P>(args.gbits, args.ibits, n, kw0 + gsz - 1, ra);
    for (int j = lane_id(); j < P; j += 64) L.Bb[j] = trow[j];
    wave_sync();
    build_toeplitz<P>(L.Bb, L.TL, L.TH);
    // two steps per trip so that the operand register sets alternate at
    // compile time
    for (int i = gsz; i >= 1; i -= 2) {
        kg_back_step<P>(args, L, kw0, i, ra, rb);
        if (i >= 2) kg_back_step<P>(args, L, kw0, i - 1, rb, ra);
    }
}

// Step 3 as a kernel: one wave per group.
template <int P>
__global__ __launch_bounds__(64, (P < 800 ? 2 : 1)) void keygen_back_kernel(GroupArgs args, const int16_t* tinv) {
    __shared__ KgWave<P> L;
    kg_back_group<P>(args, (int)blockIdx.x, tinv + (size_t)blockIdx.x * P, L);
}

}  // namespace ntrup
