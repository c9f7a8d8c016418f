// Issue-rate probe for the int32 vector ALU (measurement only; not part of
// the KeyGen library).  Every lane runs 8 independent add-xor-rotate chains
// (the ChaCha20 quarter-round pattern): each step's three operations depend
// on the previous step's results in a way no algebraic rewrite folds away
// (additions mod 2^32 and xors do not commute, the rotate amounts differ per
// chain), so the instruction count the hardware counters report (SQ_INSTS_VALU)
// is what actually issued.  Timed over grids of 1, 2, 4 or 8 waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <int R>
__device__ __forceinline__ uint32_t rotl(uint32_t x) {
    return __builtin_amdgcn_alignbit(x, x, 32 - R);
}

__global__ __launch_bounds__(64) void valu_chain_kernel(uint32_t* out, int iters) {
    const uint32_t t = blockIdx.x * 64u + threadIdx.x;
    uint32_t a0 = t, a1 = t ^ 0x9E3779B9u, a2 = t * 3u, a3 = t + 7u, a4 = ~t, a5 = t ^ 0x7F4A7C15u, a6 = t << 3,
             a7 = t + 0x6A09E667u;
    uint32_t b0 = 1u, b1 = 2u, b2 = 3u, b3 = 5u, b4 = 7u, b5 = 11u, b6 = 13u, b7 = 17u;
    for (int i = 0; i < iters; i++) {
#define NTRUP_STEP(A, B, R) \
    A += B;                 \
    B = rotl<R>(B ^ A);
        NTRUP_STEP(a0, b0, 7) NTRUP_STEP(a1, b1, 8) NTRUP_STEP(a2, b2, 9) NTRUP_STEP(a3, b3, 11)
        NTRUP_STEP(a4, b4, 12) NTRUP_STEP(a5, b5, 13) NTRUP_STEP(a6, b6, 16) NTRUP_STEP(a7, b7, 5)
#undef NTRUP_STEP
    }
    out[t] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^ b0 ^ b1 ^ b2 ^ b3 ^ b4 ^ b5 ^ b6 ^ b7;
}

}  // namespace

extern "C" {

// Launch `blocks` one-wave blocks of `iters` chain steps each on `stream`;
// out: device, blocks * 64 words.  Returns a hipError_t.
int calib_valu(int blocks, int iters, uint32_t* out, void* stream) {
    if (blocks <= 0 || iters <= 0 || !out) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(valu_chain_kernel, dim3((unsigned)blocks), dim3(64), 0, (hipStream_t)stream, out, iters);
    return (int)hipGetLastError();
}

// Source-level VALU operations per lane and chain step (add, xor, rotate).
int calib_valu_ops_per_step(void) { return 3 * 8; }

}
