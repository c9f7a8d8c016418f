// Persistent fused KeyGen: one launch runs every stage of one or more jobs
// (a job = one parameter set and key range; Section 3.1 KeyGen with the batch
// inversion of Section 2.2) as items of a single work list.
//
// Items, one wave each, in the order the list hands them out:
//   S  Short sampling of 16 keys                            (no input)
//   R  R/3 main pass of one wave's keys (64 / L of them)      (no input)
//   C  prefix chain of one Montgomery group                   (S of its keys)
//   Q  shared R/q reciprocal of W groups                      (C of the groups)
//   T  retry draws for keys whose first g was not a unit      (every R of the job)
//   B  back-substitution, h and encoding of one group         (Q of the group,
//                                                              final R/3 of its keys)
// The host orders the list S | R and C interleaved | Q | T | B, job by job
// within each stage.  Resident waves take the next item with one atomic
// add; an item waits only for items handed out before it, each of which a
// running wave holds, so the list always drains, and every wave leaves when
// the list is empty.  Dependencies are counters in the job's workspace,
// raised with agent-scope release after the item's stores and polled with
// agent-scope acquire (the eight XCDs' L2s are not coherent with each other
// for ordinary device memory).  A poll gives up after kPSpinMax attempts
// and marks the job's error word (bit 4) instead of hanging.
//
// The LDS of a block is one union of the per-stage layouts, so the kernel
// holds the largest of them, not their sum.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntrup_kernels.h"
#include "ntrup_keygen.h"

namespace ntrup {

constexpr int kPKeysPerS = 16;        // keys per sampling item
constexpr int kPMaxJobs = 4;
constexpr int kPMaxSegs = 96;
constexpr int kPSpinMax = 1 << 17;    // polls (~1 us each) of one dependency before giving up
constexpr int kPRetryLanes = 8;       // lanes per key of the retry items

enum PStage : int { PS_SAMPLE = 0, PS_R3 = 1, PS_CHAIN = 2, PS_RECIP = 3, PS_RETRY = 4, PS_BACK = 5 };

struct PJob {
    int p;
    int n, G, W;
    int ns, nr, ngroups, nq, nt;      // items per stage (B has ngroups)
    int retry_spec;                   // g draws side by side per key in T items
    uint64_t first_index;
    GroupArgs g;                      // n, G, f_rows, gbits, ibits, bscr, pk, sk, err
    int16_t* tinv;                    // group products, then their reciprocals
    int16_t* qrow;                    // partial products of the shared reciprocals
    uint8_t* attempts;
    int* list;                        // keys whose first g was not a unit
    int* list_count;
    int* sdone;                       // [ns]
    int* cdone;                       // [ngroups]
    int* qdone;                       // [nq]
    int* kfinal;                      // [ngroups] keys with a final R/3 result
    int* rcount;                      // R items done
};

struct PSeg {
    int first;      // list index of the segment's first item
    int local0;     // its index within the job's stage
    int count;
    int jobstage;   // job * 8 + stage
};

struct PLaunch {
    Seed seed;
    int njobs, nsegs, total;
    int* next;                        // the list's next index (zero at launch)
    PJob jobs[kPMaxJobs];
    PSeg segs[kPMaxSegs];
};

__device__ __forceinline__ int p_load(const int* a) {
    return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *a >= target.  Lane 0 polls; false (and error bit 4) when the
// bound runs out.
__device__ __forceinline__ bool p_wait(const int* a, int target, int* err) {
    int ok = 1;
    if (lane_id() == 0) {
        int it = 0;
        while (p_load(a) < target) {
            if (++it >= kPSpinMax) {
                ok = 0;
                atomicOr(err, 4);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
    }
    ok = __shfl(ok, 0);
    __threadfence();   // every lane's later loads see what the producer stored
    return ok != 0;
}

// Raise *a by v after every lane's stores.
__device__ __forceinline__ void p_signal(int* a, int v) {
    __threadfence();
    if (lane_id() == 0) __hip_atomic_fetch_add(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int P, int LPK>
struct PLdsBytes {
    static constexpr size_t a = sizeof(KgWave<P>), b = sizeof(KgPrefixWave<P>);
    static constexpr size_t c = sizeof(R3Lds<P, LPK>), d = sizeof(R3Lds<P, kPRetryLanes>);
    static constexpr size_t ab = a > b ? a : b, cd = c > d ? c : d;
    static constexpr size_t value = ab > cd ? ab : cd;
};

template <int LPK, int... Ps>
struct PLdsMax {
    static constexpr size_t value = 0;
};
template <int LPK, int P0, int... Ps>
struct PLdsMax<LPK, P0, Ps...> {
    static constexpr size_t a = PLdsBytes<P0, LPK>::value, b = PLdsMax<LPK, Ps...>::value;
    static constexpr size_t value = a > b ? a : b;
};

template <int P>
__device__ __forceinline__ R3Args p_r3_args(const Seed& seed, const PJob& J) {
    R3Args a;
    a.seed = seed;
    a.first_index = J.first_index;
    a.n = J.n;
    a.max_rounds = 1;
    a.spec = 1;
    a.list_in = nullptr;
    a.count_in = nullptr;
    a.list_out = J.list;
    a.count_out = J.list_count;
    a.attempts = J.attempts;
    a.gbits = (uint32_t*)J.g.gbits;
    a.ibits = (uint32_t*)J.g.ibits;
    a.err = J.g.err;
    a.g_in = nullptr;
    a.kfinal = J.kfinal;
    a.G = J.G;
    return a;
}

template <int P, int LPK>
__device__ __forceinline__ void p_item(const Seed& seed, const PJob& J, int stage, int local, uint8_t* lds) {
    const int G = J.G;
    switch (stage) {
        case PS_SAMPLE: {
            const int k0 = local * kPKeysPerS, k1 = min(J.n, k0 + kPKeysPerS);
            for (int key = k0; key < k1; key++)
                sample_short_key<P>(seed, J.first_index + (uint64_t)key, (int8_t*)J.g.f_rows + (size_t)key * P);
            p_signal(&J.sdone[local], 1);
            break;
        }
        case PS_R3: {
            const R3Args a = p_r3_args<P>(seed, J);
            r3_wave<P, LPK>(a, local, *(R3Lds<P, LPK>*)lds);
            p_signal(J.rcount, 1);
            break;
        }
        case PS_CHAIN: {
            const int kw0 = local * G, gsz = min(G, J.n - kw0);
            for (int s = kw0 / kPKeysPerS; s <= (kw0 + gsz - 1) / kPKeysPerS; s++)
                if (!p_wait(&J.sdone[s], 1, J.g.err)) return;
            KgPrefixWave<P>& L = *(KgPrefixWave<P>*)lds;
            kg_prefix_chain<P>(J.g, kw0, gsz, L);
            wave_sync();
            for (int j = lane_id(); j < P; j += 64) J.tinv[(size_t)local * P + j] = L.Bb[j];
            p_signal(&J.cdone[local], 1);
            break;
        }
        case PS_RECIP: {
            const int g0 = local * J.W, wn = min(J.W, J.ngroups - g0);
            for (int w = 0; w < wn; w++)
                if (!p_wait(&J.cdone[g0 + w], 1, J.g.err)) return;
            kg_shared_recip_rows<P>(J.g, g0, wn, J.tinv, J.qrow, *(KgPrefixWave<P>*)lds);
            p_signal(&J.qdone[local], 1);
            break;
        }
        case PS_RETRY: {
            if (!p_wait(J.rcount, J.nr, J.g.err)) return;
            R3Args a = p_r3_args<P>(seed, J);
            a.list_in = J.list;
            a.count_in = J.list_count;
            a.list_out = nullptr;
            a.count_out = nullptr;
            a.spec = J.retry_spec;
            a.max_rounds = ceil_div(kMaxAttempts, J.retry_spec);
            const int per_wave = (64 / kPRetryLanes) / J.retry_spec;
            const int waves = ceil_div(*(volatile int*)J.list_count, per_wave);
            for (int ws = local; ws < waves; ws += J.nt) r3_wave<P, kPRetryLanes>(a, ws, *(R3Lds<P, kPRetryLanes>*)lds);
            break;
        }
        case PS_BACK: {
            const int kw0 = local * G, gsz = min(G, J.n - kw0);
            if (!p_wait(&J.qdone[local / J.W], 1, J.g.err)) return;
            if (!p_wait(&J.kfinal[local], gsz, J.g.err)) return;
            kg_back_group<P>(J.g, local, J.tinv + (size_t)local * P, *(KgWave<P>*)lds);
            break;
        }
    }
}

template <int LPK, int... Ps>
__device__ __forceinline__ void p_dispatch(const Seed& seed, const PJob& J, int stage, int local, uint8_t* lds) {
    ((J.p == Ps ? p_item<Ps, LPK>(seed, J, stage, local, lds) : (void)0), ...);
}

// The persistent kernel: wave-sized blocks take items until the list is empty.
template <int LPK, int... Ps>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void keygen_persistent_kernel(PLaunch pl) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[PLdsMax<LPK, Ps...>::value];
    for (;;) {
        int item = 0;
        if (lane_id() == 0) item = atomicAdd(pl.next, 1);
        item = __shfl(item, 0);
        if (item >= pl.total) break;
        int lo = 0, hi = pl.nsegs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pl.segs[mid].first <= item) lo = mid;
            else hi = mid - 1;
        }
        const PSeg sg = pl.segs[lo];
        const int local = sg.local0 + (item - sg.first);
        p_dispatch<LPK, Ps...>(pl.seed, pl.jobs[sg.jobstage >> 3], sg.jobstage & 7, local, lds);
        __syncthreads();   // the next item reuses the LDS (one wave: a wave barrier)
    }
}

}  // namespace ntrup
