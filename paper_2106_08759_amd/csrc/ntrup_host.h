// Host-side internals of the library shared by its translation units: the
// context, the workspace layout, job descriptions, error plumbing and the
// per-parameter-set entry points that ntrup_pipeline.hip (compiled once per
// p) and ntrup_persist.hip (once per lanes-per-key / single-or-mixed form)
// define.  Splitting the kernels over several objects lets them compile in
// parallel; no device symbol is shared between objects.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/ntrupkg.h"
#include "ntrup_chacha.h"
#include "ntrup_params.h"

namespace ntrup {

constexpr int kParams[4] = {653, 761, 857, 1277};
constexpr int kCounterInts = 64;  // [0, 16): list counts; [32]: error bits
constexpr int kJobStreams = 4;    // concurrent branches of a mixed call
// sample_short, r3 main pass, r3 retry/final passes, group prefix + reciprocal,
// group back-substitution + encoding
constexpr int kStages = 5;
// tree form: node rows past the last key of a ragged last group (G <= 256)
constexpr int kTreeRows = 256;

inline int param_slot(int p) {
    for (int i = 0; i < 4; i++)
        if (kParams[i] == p) return i;
    return -1;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of one pipeline of n keys of degree p.
struct Ws {
    int8_t* f_rows;
    uint32_t* gbits;
    uint32_t* ibits;
    int16_t* bscr;
    int16_t* tinv;     // reciprocal of each Montgomery group's product
    uint8_t* attempts;
    int* lists[2];
    int* counters;
    int16_t* qrow;     // persistent form: partial products of the shared reciprocals
                       // (batched R/3: the group products, int8)
    int* flags;        // persistent form: dependency counters
    int8_t* r3rows;    // batched R/3: prefix products [n][p]
    int16_t* trow;     // tree form: the nodes' t values [n + kTreeRows][p] (bscr holds their b)
    uint32_t* pgbits;  // batched R/3: group products' bitsliced words [WN][2][groups]
    uint32_t* pinv;    // batched R/3: their reciprocals [WN][2][groups]
};

// Dependency counters of a persistent job of n keys (every G >= 1).
inline size_t flag_ints(size_t n) { return 4 * n + 64; }

inline size_t ws_bytes(int p, size_t n) {
    const size_t wn = (size_t)ceil_div(p, 32);
    return align256(n * p) + 2 * align256(wn * 2 * n * 4) + align256((n + kTreeRows) * p * 2) +
           align256(n * p * 2) + align256(n) + 2 * align256(n * 4) + align256(kCounterInts * 4) +
           align256(n * p * 2) + align256(flag_ints(n) * 4) + align256(n * p) + 2 * align256(wn * 2 * n * 4) +
           align256((n + kTreeRows) * p * 2);
}

inline Ws carve(void* base, int p, size_t n) {
    const size_t wn = (size_t)ceil_div(p, 32);
    char* c = (char*)base;
    Ws w;
    w.f_rows = (int8_t*)c;       c += align256(n * p);
    w.gbits = (uint32_t*)c;      c += align256(wn * 2 * n * 4);
    w.ibits = (uint32_t*)c;      c += align256(wn * 2 * n * 4);
    w.bscr = (int16_t*)c;        c += align256((n + kTreeRows) * p * 2);
    w.tinv = (int16_t*)c;        c += align256(n * p * 2);   // at most n groups
    w.attempts = (uint8_t*)c;    c += align256(n);
    w.lists[0] = (int*)c;        c += align256(n * 4);
    w.lists[1] = (int*)c;        c += align256(n * 4);
    w.counters = (int*)c;        c += align256(kCounterInts * 4);
    w.qrow = (int16_t*)c;        c += align256(n * p * 2);
    w.flags = (int*)c;           c += align256(flag_ints(n) * 4);
    w.r3rows = (int8_t*)c;       c += align256(n * p);
    w.pgbits = (uint32_t*)c;     c += align256(wn * 2 * n * 4);
    w.pinv = (uint32_t*)c;       c += align256(wn * 2 * n * 4);
    w.trow = (int16_t*)c;
    return w;
}

// Optional raw centered outputs of a job (device pointers, [n][p]; NULL = skip).
struct RawOut {
    int16_t* h;
    int8_t* f;
    int8_t* ginv;
    bool operator==(const RawOut& o) const { return h == o.h && f == o.f && ginv == o.ginv; }
};

// One keygen job as enqueued: parameter set, key range, outputs, the config
// in force and the job's offset in the context workspace.
struct JobDesc {
    int p;
    uint64_t first_index;
    size_t n;
    uint8_t* pk;
    uint8_t* sk;
    RawOut raw;
    ntrup_config cfg;
    size_t ws_off;
    bool operator==(const JobDesc& o) const {
        return p == o.p && first_index == o.first_index && n == o.n && pk == o.pk && sk == o.sk && raw == o.raw &&
               memcmp(&cfg, &o.cfg, sizeof cfg) == 0 && ws_off == o.ws_off;
    }
};

// What a captured graph was built from; a call replays it when all match.
struct GraphKey {
    uint32_t seed[8];
    void* ws;
    std::vector<JobDesc> jobs;
    bool operator==(const GraphKey& o) const {
        return memcmp(seed, o.seed, sizeof seed) == 0 && ws == o.ws && jobs == o.jobs;
    }
};

}  // namespace ntrup

struct ntrup_ctx {
    int device = 0;
    int last_hip_error = 0;
    void* ws = nullptr;
    size_t ws_cap = 0;
    size_t ws_budget = 0;           // 0: unbounded; else the most workspace the context may hold
    ntrup_config cfg[4];
    std::vector<int*> last_err;     // error words of the last keygen call
    std::vector<ntrup::JobDesc> one_job;   // the job list of ntrup_batch_keygen_noalloc
    hipStream_t cap_stream = nullptr;
    hipStream_t job_streams[ntrup::kJobStreams] = {};
    // side stream of single-job calls: the prefix half of the group stage
    // (and the batched R/3 stage) runs there beside the R/3 stage
    hipStream_t side_stream = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    hipEvent_t graph_done = nullptr;   // after the last graph launch
    hipEvent_t fork_event = nullptr;
    std::vector<hipEvent_t> join_events;
    // end of the last call that used the workspace, and the stream it ran on:
    // a call on another stream waits for it first (calls on one context
    // share the workspace)
    hipEvent_t call_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    bool have_graph = false;
    ntrup::GraphKey gkey;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // stage timing: kStages+1 events per recorded pipeline
    std::vector<hipEvent_t> tev;
    std::vector<char> t_side;       // pipeline ran its side stream
    int t_max = 0, t_used = 0;
};

namespace ntrup {

inline int hip_fail(ntrup_ctx* ctx, hipError_t e) {
    ctx->last_hip_error = (int)e;
    return NTRUP_EIO;
}

#define NTRUP_HIP(ctx, expr)                             \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_);  \
    } while (0)

inline unsigned grid_for(size_t items, size_t per_block) { return (unsigned)((items + per_block - 1) / per_block); }

// Event slot of stage boundary b of the current timed pipeline, or null.
inline hipEvent_t stage_event(ntrup_ctx* ctx, int b) {
    if (ctx->t_used >= ctx->t_max) return nullptr;
    return ctx->tev[(size_t)ctx->t_used * (kStages + 1) + b];
}

// Grow the context workspace to `bytes` (never beyond its budget).
int ensure_ws(ntrup_ctx* ctx, size_t bytes);

// ---- defined per parameter set in ntrup_pipeline.hip ----------------------

// Enqueue the whole KeyGen pipeline of one job on `st` (see ntrup_pipeline.hip).
template <int P>
int enqueue_keygen(ntrup_ctx* ctx, const ntrup_config& cfg, const Seed& seed, uint64_t first_index, size_t n,
                   uint8_t* pk, uint8_t* sk, const RawOut& raw, const Ws& w, hipStream_t st, bool side_ok,
                   bool zero_err);

template <int P>
int op_decode_raw(ntrup_ctx* ctx, size_t n, const uint8_t* pk, const uint8_t* sk, const RawOut& raw,
                  hipStream_t st);
template <int P>
int op_mul_rq(ntrup_ctx* ctx, bool mfma, const int16_t* a, const int16_t* b, int16_t* c, size_t n, bool small_a,
              hipStream_t st);
template <int P>
int op_mul_r3(ntrup_ctx* ctx, const int8_t* a, const int8_t* b, int8_t* c, size_t n, hipStream_t st);
template <int P>
int op_recip_rq(ntrup_ctx* ctx, bool jump, const int16_t* a, int16_t* out, int32_t* ok, size_t n, hipStream_t st);
template <int P>
int op_recip_r3(ntrup_ctx* ctx, int lpk, const int8_t* a, int8_t* out, int32_t* ok, size_t n, hipStream_t st);
template <int P>
int op_batch_inv_rq(ntrup_ctx* ctx, bool mfma, const int16_t* a, int16_t* out, size_t n, size_t group_size,
                    hipStream_t st);
template <int P>
int op_sample(ntrup_ctx* ctx, const Seed& sd, uint64_t first_index, size_t n, int attempt, int8_t* f, int8_t* g,
              hipStream_t st);

// Encapsulation / decapsulation core (ntrup_kem.h): r sampled on the
// encapsulation stream, c = Round(h r); r' = decrypt(c) with the weight
// check, and with h the re-encryption check.
template <int P>
int op_encap(ntrup_ctx* ctx, const Seed& sd, uint64_t first_index, size_t n, const int16_t* h, int16_t* c, int8_t* r,
             hipStream_t st);
template <int P>
int op_decap(ntrup_ctx* ctx, size_t n, const int16_t* c, const int8_t* f, const int8_t* ginv, const int16_t* h,
             int8_t* r, uint8_t* ok, hipStream_t st);

// Clear `count` ints (a fill kernel, not a memset node, so that captured
// graphs replay it reliably).
void launch_zero_ints(int* p, int count, hipStream_t st);

// ---- the persistent form: ntrup_persist.hip ------------------------------
struct PLaunch;
template <int LPK>
int launch_persistent_single(ntrup_ctx* ctx, int p, const PLaunch& pl, hipStream_t st);
template <int LPK>
int launch_persistent_mixed(ntrup_ctx* ctx, const PLaunch& pl, hipStream_t st);

}  // namespace ntrup
