// Issue-rate probes for the int32 vector ALU (measurement only; not part of
// the KeyGen library).  Each probe runs 8 independent two-register chains per
// lane in which every step's operations depend on the previous step's
// results and no algebraic rewrite removes one (nonlinear mixes, or funnel
// shifts of two different registers); the hardware counters (SQ_INSTS_VALU)
// confirm the instruction count.  Kinds:
//   0 arx     add, xor, rotate (the ChaCha20 quarter-round pattern)
//   1 add     v_add_u32 pairs in a Fibonacci pattern (a += b; b += a)
//   2 bitop3  v_bitop3_b32 with the majority function (a = maj(a, b, c) ...)
//   3 align   v_alignbit_b32 of two registers (a = alignbit(a, b, s) ...)
//   4 mad24   v_mad_u32_u24 (a = a * b + c on 24-bit operands)
//   5 perm    v_perm_b32 byte permutes of two registers (a = perm(a, b, s))
//   6 xor     v_xor_b32 and v_add_u32 (a ^= b'; b ^= a + 1)
//   7 med3    v_med3_u32 of three registers of different chains
//   8 minmax  v_min_u32 and v_max_u32 of registers of different chains
//   9 dpp     v_mov_b32 with a DPP row rotation, then v_xor_b32
// Timed over grids of 1, 2, 4 or 8 waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <int R>
__device__ __forceinline__ uint32_t rotl(uint32_t x) {
    return __builtin_amdgcn_alignbit(x, x, 32 - R);
}

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xe8" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

template <int KIND>
__global__ __launch_bounds__(64) void valu_chain_kernel(uint32_t* out, int iters) {
    const uint32_t t = blockIdx.x * 64u + threadIdx.x;
    uint32_t a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        a[k] = t * (2u * k + 1u) + 0x9E3779B9u * k;
        b[k] = (t ^ (0x7F4A7C15u * (k + 1))) | 1u;
    }
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if constexpr (KIND == 0) {
                a[k] += b[k];
                b[k] = rotl<7>(b[k] ^ a[k]);
            } else if constexpr (KIND == 1) {
                a[k] += b[k];
                b[k] += a[k];
            } else if constexpr (KIND == 2) {
                a[k] = maj3(a[k], b[k], a[(k + 1) & 7]);
                b[k] = maj3(b[k], a[k], b[(k + 3) & 7]);
            } else if constexpr (KIND == 3) {
                a[k] = __builtin_amdgcn_alignbit(a[k], b[k], 3 + 2 * k);
                b[k] = __builtin_amdgcn_alignbit(b[k], a[k], 29 - 2 * k);
            } else if constexpr (KIND == 4) {
                a[k] = __umul24(a[k], b[k]) + 0x5bd1e995u;
                b[k] = __umul24(b[k], a[k]) + 0x1b873593u;
            } else if constexpr (KIND == 5) {
                a[k] = __builtin_amdgcn_perm(a[k], b[k], 0x05040302u + 0x01010101u * (k & 1));
                b[k] = __builtin_amdgcn_perm(b[k], a[k], 0x02010007u);
            } else if constexpr (KIND == 6) {
                a[k] ^= b[(k + 1) & 7];
                b[k] ^= a[k] + 1u;
            } else if constexpr (KIND == 7) {
                a[k] = med3u(a[k], b[k], a[(k + 1) & 7]);
                b[k] = med3u(b[k], a[k], b[(k + 3) & 7]);
            } else if constexpr (KIND == 8) {
                a[k] = min(a[k], b[(k + 1) & 7]);
                b[k] = max(b[k], a[(k + 2) & 7]);
            } else {
                a[k] = (uint32_t)__builtin_amdgcn_mov_dpp((int)b[k], 0x128, 0xF, 0xF, true);
                b[k] ^= a[k];
            }
        }
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) x ^= a[k] ^ b[k];
    out[t] = x;
}

}  // namespace

extern "C" {

// Launch probe `kind` (0..9) over `blocks` one-wave blocks of `iters` steps
// each on `stream`; out: device, blocks * 64 words.  Returns a hipError_t.
int calib_valu(int kind, int blocks, int iters, uint32_t* out, void* stream) {
    if (blocks <= 0 || iters <= 0 || !out || kind < 0 || kind > 9) return (int)hipErrorInvalidValue;
    const hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case 0: hipLaunchKernelGGL(valu_chain_kernel<0>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 1: hipLaunchKernelGGL(valu_chain_kernel<1>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 2: hipLaunchKernelGGL(valu_chain_kernel<2>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 3: hipLaunchKernelGGL(valu_chain_kernel<3>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 4: hipLaunchKernelGGL(valu_chain_kernel<4>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 5: hipLaunchKernelGGL(valu_chain_kernel<5>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 6: hipLaunchKernelGGL(valu_chain_kernel<6>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 7: hipLaunchKernelGGL(valu_chain_kernel<7>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        case 8: hipLaunchKernelGGL(valu_chain_kernel<8>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
        default: hipLaunchKernelGGL(valu_chain_kernel<9>, dim3((unsigned)blocks), dim3(64), 0, st, out, iters); break;
    }
    return (int)hipGetLastError();
}

// VALU instructions per lane and step of probe `kind` (8 chains x 3 for the
// add-xor-rotate mix and the xor kind, 8 x 2 otherwise).
int calib_valu_ops_per_step(int kind) { return (kind == 0 || kind == 6) ? 24 : 16; }

}
