// C ABI of the batched KeyGen library: argument checking, workspace, launch
// sequencing and hipGraph replay.  See include/ntrupkg.h for the contract.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/ntrupkg.h"
#include "ntrup_kernels.h"
#include "ntrup_keygen.h"
#include "ntrup_persist.h"
#include "ntrup_r3batch.h"

using namespace ntrup;

namespace {

constexpr int kParams[4] = {653, 761, 857, 1277};
constexpr int kCounterInts = 64;  // [0, 16): list counts; [32]: error bits

int param_slot(int p) {
    for (int i = 0; i < 4; i++)
        if (kParams[i] == p) return i;
    return -1;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

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
    uint32_t* pgbits;  // batched R/3: group products' bitsliced words [WN][2][groups]
    uint32_t* pinv;    // batched R/3: their reciprocals [WN][2][groups]
};

// Dependency counters of a persistent job of n keys (every G >= 1).
size_t flag_ints(size_t n) { return 4 * n + 64; }

size_t ws_bytes(int p, size_t n) {
    const size_t wn = (size_t)ceil_div(p, 32);
    return align256(n * p) + 2 * align256(wn * 2 * n * 4) + 2 * align256(n * p * 2) + align256(n) +
           2 * align256(n * 4) + align256(kCounterInts * 4) + align256(n * p * 2) + align256(flag_ints(n) * 4) +
           align256(n * p) + 2 * align256(wn * 2 * n * 4);
}

Ws carve(void* base, int p, size_t n) {
    const size_t wn = (size_t)ceil_div(p, 32);
    char* c = (char*)base;
    Ws w;
    w.f_rows = (int8_t*)c;       c += align256(n * p);
    w.gbits = (uint32_t*)c;      c += align256(wn * 2 * n * 4);
    w.ibits = (uint32_t*)c;      c += align256(wn * 2 * n * 4);
    w.bscr = (int16_t*)c;        c += align256(n * p * 2);
    w.tinv = (int16_t*)c;        c += align256(n * p * 2);   // at most n groups
    w.attempts = (uint8_t*)c;    c += align256(n);
    w.lists[0] = (int*)c;        c += align256(n * 4);
    w.lists[1] = (int*)c;        c += align256(n * 4);
    w.counters = (int*)c;        c += align256(kCounterInts * 4);
    w.qrow = (int16_t*)c;        c += align256(n * p * 2);
    w.flags = (int*)c;           c += align256(flag_ints(n) * 4);
    w.r3rows = (int8_t*)c;       c += align256(n * p);
    w.pgbits = (uint32_t*)c;     c += align256(wn * 2 * n * 4);
    w.pinv = (uint32_t*)c;
    return w;
}

// One keygen job as enqueued: parameter set, key range, outputs, the config
// in force and the job's offset in the context workspace.
struct JobDesc {
    int p;
    uint64_t first_index;
    size_t n;
    uint8_t* pk;
    uint8_t* sk;
    ntrup_config cfg;
    size_t ws_off;
    bool operator==(const JobDesc& o) const {
        return p == o.p && first_index == o.first_index && n == o.n && pk == o.pk && sk == o.sk &&
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

constexpr int kJobStreams = 4;  // concurrent branches of a mixed call

}  // namespace

struct ntrup_ctx {
    int device = 0;
    int last_hip_error = 0;
    void* ws = nullptr;
    size_t ws_cap = 0;
    ntrup_config cfg[4];
    std::vector<int*> last_err;     // error words of the last keygen call
    hipStream_t cap_stream = nullptr;
    hipStream_t job_streams[kJobStreams] = {};
    // side stream of single-job calls: Short sampling and the prefix half of
    // the group stage run there beside the R/3 stage (they need only f)
    hipStream_t side_stream = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    hipEvent_t graph_done = nullptr;   // after the last graph launch
    hipEvent_t fork_event = nullptr;
    std::vector<hipEvent_t> join_events;
    bool have_graph = false;
    GraphKey gkey;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // stage timing: kStages+1 events per recorded pipeline
    std::vector<hipEvent_t> tev;
    std::vector<char> t_side;       // pipeline ran its side stream
    int t_max = 0, t_used = 0;
};

namespace {
// sample_short, r3 main pass, r3 retry/final passes, group prefix + reciprocal,
// group back-substitution + encoding
constexpr int kStages = 5;
}

namespace {

int hip_fail(ntrup_ctx* ctx, hipError_t e) {
    ctx->last_hip_error = (int)e;
    return NTRUP_EIO;
}

#define NTRUP_HIP(ctx, expr)                             \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_);  \
    } while (0)

int set_device(ntrup_ctx* ctx) {
    NTRUP_HIP(ctx, hipSetDevice(ctx->device));
    return 0;
}

int ensure_ws(ntrup_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->ws_cap) return 0;
    if (ctx->ws) {
        NTRUP_HIP(ctx, hipDeviceSynchronize());
        NTRUP_HIP(ctx, hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_cap = 0;
        ctx->have_graph = false;  // captured pointers are stale
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        ctx->last_hip_error = (int)e;
        return NTRUP_ENOMEM;
    }
    ctx->ws = p;
    ctx->ws_cap = bytes;
    return 0;
}

Seed make_seed(const uint8_t* s) {
    Seed k;
    for (int i = 0; i < 8; i++)
        k.k[i] = (uint32_t)s[4 * i] | ((uint32_t)s[4 * i + 1] << 8) | ((uint32_t)s[4 * i + 2] << 16) |
                 ((uint32_t)s[4 * i + 3] << 24);
    return k;
}

unsigned grid_for(size_t items, size_t per_block) { return (unsigned)((items + per_block - 1) / per_block); }

// R/3 pass over up to n keys with lpk lanes per key and a.spec attempts per
// key side by side: 64 / (lpk * spec) keys per one-wave block.
template <int P>
void launch_r3(int lpk, size_t n, const R3Args& a, hipStream_t st) {
    const size_t kpb = (size_t)(64 / lpk / a.spec);
    const dim3 grid(grid_for(n, kpb)), blk(64);
    switch (lpk) {
        case 1: hipLaunchKernelGGL((r3_kernel<P, 1>), grid, blk, 0, st, a); break;
        case 2: hipLaunchKernelGGL((r3_kernel<P, 2>), grid, blk, 0, st, a); break;
        case 4: hipLaunchKernelGGL((r3_kernel<P, 4>), grid, blk, 0, st, a); break;
        default: hipLaunchKernelGGL((r3_kernel<P, 8>), grid, blk, 0, st, a); break;
    }
}

// Event slot of stage boundary b of the current timed pipeline, or null.
hipEvent_t stage_event(ntrup_ctx* ctx, int b) {
    if (ctx->t_used >= ctx->t_max) return nullptr;
    return ctx->tev[(size_t)ctx->t_used * (kStages + 1) + b];
}

// Enqueue the whole KeyGen pipeline of one job on `st`.  side_ok: with the
// matrix-core engine, the prefix half of the group stage (which needs only
// f) runs on ctx->side_stream beside the R/3 stage, forked from st after
// Short sampling and joined before the back-substitution.  Otherwise -- graph
// capture, the jobs of a mixed call (already concurrent branches), the plain
// form -- every stage runs on st.  zero_err: also clear the error word (once
// per API call).
//
// Stage events: 0 start; 1 end of sampling; 2 end of the prefix kernel
// (the product engine 0 records it right after 1); 3 end of the R/3 main
// pass; 4 end of the R/3 retry passes; 5 end.
template <int P>
int enqueue_keygen(ntrup_ctx* ctx, const ntrup_config& cfg, const Seed& seed, uint64_t first_index,
                   size_t n, uint8_t* pk, uint8_t* sk, const Ws& w, hipStream_t st, bool side_ok, bool zero_err) {
    const bool mfma = cfg.product_engine == 1;
    const bool side = side_ok && mfma;
    hipStream_t ss = side ? ctx->side_stream : st;
    auto mark = [&](int b, hipStream_t on) {
        if (hipEvent_t ev = stage_event(ctx, b)) (void)hipEventRecord(ev, on);
    };
    GroupArgs g;
    g.n = (int)n;
    g.G = cfg.group_size;
    g.f_rows = w.f_rows;
    g.gbits = w.gbits;
    g.ibits = w.ibits;
    g.bscr = w.bscr;
    g.pk = pk;
    g.sk = sk;
    g.err = w.counters + 32;
    g.a_in = nullptr;
    g.c_out = nullptr;
    const int W = cfg.inverse_share;

    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, w.counters, zero_err ? kCounterInts : 16);
    mark(0, st);
    // batched R/3 needs no f: its whole stage runs on the side stream from
    // the start, beside sampling and the prefix kernel (which stay on st)
    const bool r3_first = side && cfg.r3_batch;
    hipStream_t sp = r3_first ? st : ss;   // prefix kernel
    hipStream_t sr = r3_first ? ss : st;   // R/3 stage
    if (r3_first) {
        NTRUP_HIP(ctx, hipEventRecord(ctx->side_fork, st));
        NTRUP_HIP(ctx, hipStreamWaitEvent(ss, ctx->side_fork, 0));
    }
    hipLaunchKernelGGL(sample_short_kernel<P>, dim3(grid_for(n, 4)), dim3(256), 0, st, seed, first_index, (int)n,
                       w.f_rows);
    mark(1, st);
    if (side && !r3_first) {
        NTRUP_HIP(ctx, hipEventRecord(ctx->side_fork, st));
        NTRUP_HIP(ctx, hipStreamWaitEvent(ss, ctx->side_fork, 0));
    }
    if (mfma) {
        const dim3 grid(grid_for(n, (size_t)cfg.group_size * W)), blk(64 * W);
        switch (W) {
            case 1: hipLaunchKernelGGL((keygen_prefix_kernel<P, 1>), grid, blk, 0, sp, g, w.tinv); break;
            case 2: hipLaunchKernelGGL((keygen_prefix_kernel<P, 2>), grid, blk, 0, sp, g, w.tinv); break;
            case 4: hipLaunchKernelGGL((keygen_prefix_kernel<P, 4>), grid, blk, 0, sp, g, w.tinv); break;
            default:
                if constexpr (P != 1277) hipLaunchKernelGGL((keygen_prefix_kernel<P, 8>), grid, blk, 0, sp, g, w.tinv);
                break;
        }
        // with a side stream, the back-substitution (which needs only f) runs
        // there too, and only h = g c and the encoding follow the R/3 stage
        if (side)
            hipLaunchKernelGGL((keygen_cinv_kernel<P>), dim3(grid_for(n, cfg.group_size)), dim3(64), 0, sp, g,
                               (const int16_t*)w.tinv);
    }
    mark(2, sp);
    if (side && !r3_first) NTRUP_HIP(ctx, hipEventRecord(ctx->side_join, ss));
    R3Args a;
    memset(&a, 0, sizeof a);
    a.seed = seed;
    a.first_index = first_index;
    a.n = (int)n;
    a.attempts = w.attempts;
    a.gbits = w.gbits;
    a.ibits = w.ibits;
    a.err = w.counters + 32;
    a.g_in = nullptr;
    const int R = cfg.retry_passes;
    if (cfg.r3_batch) {
        // batched R/3 reciprocals: screen, prefix products, group reciprocals,
        // back-substitution; groups whose product is not a unit go to the
        // per-key divstep pass
        R3bArgs<P> b;
        b.seed = seed;
        b.first_index = first_index;
        b.n = (int)n;
        b.G = cfg.group_size;
        b.gbits = w.gbits;
        b.ibits = w.ibits;
        b.attempts = w.attempts;
        b.rows = w.r3rows;
        b.pj = (int8_t*)w.qrow;
        b.pinv = w.pinv;
        b.pok = (const uint8_t*)w.lists[1];
        b.fb_list = w.lists[0];
        b.fb_count = w.counters;
        b.err = w.counters + 32;
        b.screen = cfg.r3_batch == 1;
        // retry list: lists[0] and counters[1] (the fallback reuses lists[0]
        // afterwards, with counters[0]); retry draws in the group-reciprocal
        // buffers (pgbits, pinv: 2 [WN][2][n] words), which are written later
        b.rt_list = w.lists[0];
        b.rt_count = w.counters + 1;
        b.rt_scratch = w.pgbits;
        b.rt_cap = (int)(2 * n / kR3bRetryDraws);
        const unsigned ngroups = grid_for(n, cfg.group_size);
        hipLaunchKernelGGL((r3b_sample_kernel<P>), dim3(grid_for(n * (size_t)ceil_div(P, 32), 256)), dim3(256), 0, sr,
                           b);
        hipLaunchKernelGGL((r3b_screen_kernel<P>), dim3(grid_for(n, 256)), dim3(256), 0, sr, b);
        if (b.screen) {
            hipLaunchKernelGGL((r3b_retry_sample_kernel<P>), dim3(256), dim3(256), 0, sr, b);
            hipLaunchKernelGGL((r3b_retry_screen_kernel<P>), dim3(64), dim3(256), 0, sr, b);
        }
        hipLaunchKernelGGL((r3b_prefix_kernel<P>), dim3(ngroups), dim3(64), 0, sr, b);
        R3Args gi;
        memset(&gi, 0, sizeof gi);
        gi.n = (int)ngroups;
        gi.max_rounds = 1;
        gi.spec = 1;
        gi.attempts = (uint8_t*)w.lists[1];
        gi.gbits = w.pgbits;
        gi.ibits = w.pinv;
        gi.err = w.counters + 32;
        gi.g_in = (const int8_t*)w.qrow;
        launch_r3<P>(8, ngroups, gi, sr);   // latency-bound: few products, most lanes per product
        hipLaunchKernelGGL((r3b_back_kernel<P>), dim3(ngroups), dim3(64), 0, sr, b);
        mark(3, sr);
        a.list_in = w.lists[0];
        a.count_in = w.counters;
        a.list_out = nullptr;
        a.count_out = nullptr;
        a.spec = cfg.retry_parallel_attempts;
        a.max_rounds = ceil_div(kMaxAttempts, a.spec);
        launch_r3<P>(cfg.retry_lanes_per_key, n, a, sr);
    }
    for (int pass = 0; pass <= R + 1 && !cfg.r3_batch; pass++) {
        const bool last = pass == R + 1;
        a.list_in = pass == 0 ? nullptr : w.lists[(pass - 1) & 1];
        a.count_in = pass == 0 ? nullptr : w.counters + (pass - 1);
        a.list_out = last ? nullptr : w.lists[pass & 1];
        a.count_out = last ? nullptr : w.counters + pass;
        a.spec = pass == 0 ? 1 : cfg.retry_parallel_attempts;
        a.max_rounds = last ? ceil_div(kMaxAttempts, a.spec) : 1;
        launch_r3<P>(pass == 0 ? cfg.lanes_per_key : cfg.retry_lanes_per_key, n, a, sr);
        if (pass == 0) mark(3, sr);
    }
    mark(4, sr);
    if (r3_first) NTRUP_HIP(ctx, hipEventRecord(ctx->side_join, ss));
    if (side) NTRUP_HIP(ctx, hipStreamWaitEvent(st, ctx->side_join, 0));
    if (mfma && side) {
        const unsigned per = grid_for(n, 8);
        hipLaunchKernelGGL((keygen_h_kernel<P>), dim3(8 * per), dim3(64), 0, st, g, (int)per);
    } else if (mfma) {
        hipLaunchKernelGGL((keygen_back_kernel<P>), dim3(grid_for(n, cfg.group_size)), dim3(64), 0, st, g,
                           (const int16_t*)w.tinv);
    } else {
        hipLaunchKernelGGL((group_kernel<P, true>), dim3(grid_for(n, cfg.group_size)), dim3(64), 0, st, g);
    }
    mark(5, st);
    if (ctx->t_used < ctx->t_max) ctx->t_side[ctx->t_used++] = r3_first ? 3 : side ? 1 : 0;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e);
    return 0;
}

int enqueue_dispatch(ntrup_ctx* ctx, int p, const ntrup_config& cfg, const Seed& seed, uint64_t first_index,
                     size_t n, uint8_t* pk, uint8_t* sk, const Ws& w, hipStream_t st, bool side_ok, bool zero_err) {
    switch (p) {
        case 653: return enqueue_keygen<653>(ctx, cfg, seed, first_index, n, pk, sk, w, st, side_ok, zero_err);
        case 761: return enqueue_keygen<761>(ctx, cfg, seed, first_index, n, pk, sk, w, st, side_ok, zero_err);
        case 857: return enqueue_keygen<857>(ctx, cfg, seed, first_index, n, pk, sk, w, st, side_ok, zero_err);
        case 1277: return enqueue_keygen<1277>(ctx, cfg, seed, first_index, n, pk, sk, w, st, side_ok, zero_err);
    }
    return NTRUP_EINVAL;
}

// ---------------------------------------------------------------------------
// Persistent form: every stage of every job as items of one work list, run by
// one launch of keygen_persistent_kernel (see ntrup_persist.h).
// ---------------------------------------------------------------------------
template <int LPK, int... Ps>
int launch_persistent(ntrup_ctx* ctx, const PLaunch& pl, hipStream_t st) {
    auto kernel = keygen_persistent_kernel<LPK, Ps...>;
    int per_cu = 0, cus = 0;
    NTRUP_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0));
    NTRUP_HIP(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int grid = std::max(1, std::min(pl.total, std::max(1, per_cu) * cus));
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, st, pl);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template <int LPK>
int launch_persistent_p(ntrup_ctx* ctx, int p, bool mixed, const PLaunch& pl, hipStream_t st) {
    if (mixed) return launch_persistent<LPK, 653, 761, 857, 1277>(ctx, pl, st);
    switch (p) {
        case 653: return launch_persistent<LPK, 653>(ctx, pl, st);
        case 761: return launch_persistent<LPK, 761>(ctx, pl, st);
        case 857: return launch_persistent<LPK, 857>(ctx, pl, st);
        case 1277: return launch_persistent<LPK, 1277>(ctx, pl, st);
    }
    return NTRUP_EINVAL;
}

// The work list of `jobs` (each with cfg.persistent set; the R/3 lanes per
// key of the first job apply to all): stage counts, dependency counters in
// each job's workspace (zeroed here), segments in the order S | R and C
// interleaved in 8 chunks | Q | T | B, job by job within each stage.
int enqueue_persistent(ntrup_ctx* ctx, const Seed& sd, const std::vector<JobDesc>& jobs, hipStream_t st) {
    if (jobs.empty() || jobs.size() > (size_t)kPMaxJobs) return NTRUP_EINVAL;
    PLaunch pl;
    memset(&pl, 0, sizeof pl);
    pl.seed = sd;
    pl.njobs = (int)jobs.size();
    const int lpk = jobs[0].cfg.lanes_per_key;
    bool mixed = false;
    for (size_t j = 0; j < jobs.size(); j++) {
        const JobDesc& jd = jobs[j];
        mixed = mixed || jd.p != jobs[0].p;
        const Ws w = carve((char*)ctx->ws + jd.ws_off, jd.p, jd.n);
        PJob& J = pl.jobs[j];
        const int n = (int)jd.n;
        J.p = jd.p;
        J.n = n;
        J.G = jd.cfg.group_size;
        J.W = jd.cfg.inverse_share;
        J.ns = (int)grid_for(n, kPKeysPerS);
        J.nr = (int)grid_for(n, 64 / lpk);
        J.ngroups = (int)grid_for(n, J.G);
        J.nq = (int)grid_for(J.ngroups, J.W);
        J.nt = std::min(64, std::max(1, (int)grid_for(n, 512)));
        J.retry_spec = jd.cfg.retry_parallel_attempts;
        J.first_index = jd.first_index;
        J.g.n = n;
        J.g.G = J.G;
        J.g.f_rows = w.f_rows;
        J.g.gbits = w.gbits;
        J.g.ibits = w.ibits;
        J.g.bscr = w.bscr;
        J.g.pk = jd.pk;
        J.g.sk = jd.sk;
        J.g.err = w.counters + 32;
        J.g.a_in = nullptr;
        J.g.c_out = nullptr;
        J.tinv = w.tinv;
        J.qrow = w.qrow;
        J.attempts = w.attempts;
        J.list = w.lists[0];
        J.list_count = w.counters;
        J.sdone = w.flags;
        J.cdone = J.sdone + J.ns;
        J.qdone = J.cdone + J.ngroups;
        J.kfinal = J.qdone + J.nq;
        J.rcount = J.kfinal + J.ngroups;
        const int used = J.ns + 2 * J.ngroups + J.nq + 2;   // rcount, then the list's next index (job 0)
        hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, w.counters, kCounterInts);
        hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for(used, 256)), dim3(256), 0, st, w.flags, used);
        if (j == 0) pl.next = J.rcount + 1;
    }
    auto add = [&](int job, int stage, int local0, int count) {
        if (count <= 0) return;
        PSeg& g = pl.segs[pl.nsegs++];
        g.first = pl.total;
        g.local0 = local0;
        g.count = count;
        g.jobstage = job * 8 + stage;
        pl.total += count;
    };
    constexpr int kChunks = 8;
    static_assert(kPMaxJobs * (4 + 2 * kChunks) <= kPMaxSegs, "segment table");
    for (int j = 0; j < pl.njobs; j++) add(j, PS_SAMPLE, 0, pl.jobs[j].ns);
    for (int c = 0; c < kChunks; c++)
        for (int j = 0; j < pl.njobs; j++) {
            const PJob& J = pl.jobs[j];
            add(j, PS_R3, J.nr * c / kChunks, J.nr * (c + 1) / kChunks - J.nr * c / kChunks);
            add(j, PS_CHAIN, J.ngroups * c / kChunks, J.ngroups * (c + 1) / kChunks - J.ngroups * c / kChunks);
        }
    for (int j = 0; j < pl.njobs; j++) add(j, PS_RECIP, 0, pl.jobs[j].nq);
    for (int j = 0; j < pl.njobs; j++) add(j, PS_RETRY, 0, pl.jobs[j].nt);
    for (int j = 0; j < pl.njobs; j++) add(j, PS_BACK, 0, pl.jobs[j].ngroups);
    NTRUP_HIP(ctx, hipGetLastError());
    return lpk == 2 ? launch_persistent_p<2>(ctx, jobs[0].p, mixed, pl, st)
                    : launch_persistent_p<4>(ctx, jobs[0].p, mixed, pl, st);
}

bool valid_config(const ntrup_config& c) {
    auto lpk_ok = [](int l) { return l == 1 || l == 2 || l == 4 || l == 8; };
    return c.group_size >= 1 && c.group_size <= 1024 && lpk_ok(c.lanes_per_key) &&
           lpk_ok(c.retry_lanes_per_key) && lpk_ok(c.retry_parallel_attempts) &&
           c.retry_lanes_per_key * c.retry_parallel_attempts <= 64 && c.retry_passes >= 0 &&
           c.retry_passes <= 8 && (c.use_graph == 0 || c.use_graph == 1) &&
           (c.product_engine == 0 || c.product_engine == 1) &&
           (c.inverse_share == 1 || c.inverse_share == 2 || c.inverse_share == 4 || c.inverse_share == 8) &&
           (c.persistent == 0 ||
            (c.persistent == 1 && c.product_engine == 1 && (c.lanes_per_key == 2 || c.lanes_per_key == 4))) &&
           (c.r3_batch == 0 || ((c.r3_batch == 1 || c.r3_batch == 2) && c.product_engine == 1 && c.persistent == 0));
}

int check_job(int p, size_t n, const void* pk, const void* sk) {
    if (param_slot(p) < 0 || n == 0 || n > 0x7FFFFFFF || !pk || !sk) return NTRUP_EINVAL;
    return 0;
}

template <int P>
int op_recip_r3(ntrup_ctx* ctx, int lpk, const int8_t* a, int8_t* out, int32_t* ok, size_t n, hipStream_t st) {
    if (int r = ensure_ws(ctx, ws_bytes(P, n))) return r;
    const Ws w = carve(ctx->ws, P, n);
    R3Args ar;
    memset(&ar, 0, sizeof ar);
    ar.n = (int)n;
    ar.max_rounds = 1;
    ar.spec = 1;
    ar.attempts = w.attempts;
    ar.gbits = w.gbits;
    ar.ibits = w.ibits;
    ar.err = w.counters + 32;
    ar.g_in = a;
    launch_r3<P>(lpk, n, ar, st);
    hipLaunchKernelGGL(unpack_bits_kernel<P>, dim3(grid_for(n, 256)), dim3(256), 0, st, (int)n, w.ibits, out);
    hipLaunchKernelGGL(copy_flags_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, (int)n, w.attempts, ok);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

}  // namespace

extern "C" {

int ntrup_params(int p, int* q, int* w, size_t* pkb, size_t* skb) {
    int qq, ww;
    switch (p) {
        case 653: qq = Param<653>::q; ww = Param<653>::w; break;
        case 761: qq = Param<761>::q; ww = Param<761>::w; break;
        case 857: qq = Param<857>::q; ww = Param<857>::w; break;
        case 1277: qq = Param<1277>::q; ww = Param<1277>::w; break;
        default: return NTRUP_EINVAL;
    }
    if (q) *q = qq;
    if (w) *w = ww;
    if (pkb) *pkb = (size_t)pk_bytes(p);
    if (skb) *skb = (size_t)sk_bytes(p);
    return 0;
}

const char* ntrup_strerror(int code) {
    switch (code) {
        case NTRUP_OK: return "ok";
        case NTRUP_EIO: return "HIP call failed";
        case NTRUP_EAGAIN: return "no invertible g within the attempt cap";
        case NTRUP_ENOMEM: return "device allocation failed";
        case NTRUP_EINVAL: return "invalid argument";
        case NTRUP_EFAULT: return "group product not a unit";
        case NTRUP_ETIME: return "a persistent-kernel item waited too long for its inputs";
    }
    return "unknown error";
}

int ntrup_ctx_create(ntrup_ctx** out, int device) {
    if (!out) return NTRUP_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return NTRUP_EINVAL;
    ntrup_ctx* ctx = new (std::nothrow) ntrup_ctx();
    if (!ctx) return NTRUP_ENOMEM;
    ctx->device = device;
    for (int i = 0; i < 4; i++) ctx->cfg[i] = ntrup_config{32, 2, 8, 4, 1, 1, 1, 4, 0, 0};
    bool ok = set_device(ctx) == 0 && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < kJobStreams; i++)
        ok = hipStreamCreateWithFlags(&ctx->job_streams[i], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->side_join, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->graph_done, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        ntrup_ctx_destroy(ctx);
        return NTRUP_EIO;
    }
    *out = ctx;
    return 0;
}

int ntrup_ctx_destroy(ntrup_ctx* ctx) {
    if (!ctx) return NTRUP_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (hipStream_t js : ctx->job_streams)
        if (js) (void)hipStreamDestroy(js);
    if (ctx->side_stream) (void)hipStreamDestroy(ctx->side_stream);
    if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
    if (ctx->side_join) (void)hipEventDestroy(ctx->side_join);
    if (ctx->graph_done) (void)hipEventDestroy(ctx->graph_done);
    if (ctx->fork_event) (void)hipEventDestroy(ctx->fork_event);
    for (hipEvent_t e : ctx->join_events) (void)hipEventDestroy(e);
    if (ctx->ws) (void)hipFree(ctx->ws);
    for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
    delete ctx;
    return 0;
}

int ntrup_ctx_reserve(ntrup_ctx* ctx, int p, size_t n) {
    if (!ctx || param_slot(p) < 0 || n == 0) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    return ensure_ws(ctx, ws_bytes(p, n));
}

size_t ntrup_ctx_workspace_bytes(const ntrup_ctx* ctx) { return ctx ? ctx->ws_cap : 0; }

int ntrup_last_hip_error(const ntrup_ctx* ctx) { return ctx ? ctx->last_hip_error : 0; }

int ntrup_get_config(const ntrup_ctx* ctx, int p, ntrup_config* cfg) {
    const int s = param_slot(p);
    if (!ctx || s < 0 || !cfg) return NTRUP_EINVAL;
    *cfg = ctx->cfg[s];
    return 0;
}

int ntrup_set_config(ntrup_ctx* ctx, int p, const ntrup_config* cfg) {
    const int s = param_slot(p);
    if (!ctx || s < 0 || !cfg || !valid_config(*cfg)) return NTRUP_EINVAL;
    if (p == 1277 && cfg->inverse_share > 4) return NTRUP_EINVAL;  // 8 waves of p = 1277 exceed LDS/VGPRs
    ctx->cfg[s] = *cfg;
    return 0;
}

int ntrup_batch_keygen(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n, uint8_t* pk,
                       uint8_t* sk, void* stream) {
    ntrup_job job;
    job.p = p;
    job.first_index = first_index;
    job.n = n;
    job.pk = pk;
    job.sk = sk;
    return ntrup_batch_keygen_mixed(ctx, seed, &job, 1, stream);
}

int ntrup_keygen_plain(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n, uint8_t* pk,
                       uint8_t* sk, void* stream) {
    if (!ctx || !seed) return NTRUP_EINVAL;
    if (int r = check_job(p, n, pk, sk)) return r;
    if (int r = set_device(ctx)) return r;
    if (int r = ensure_ws(ctx, ws_bytes(p, 1))) return r;
    ntrup_config cfg = ctx->cfg[param_slot(p)];
    cfg.group_size = 1;
    const Seed sd = make_seed(seed);
    const Ws w = carve(ctx->ws, p, 1);
    ctx->last_err.assign(1, w.counters + 32);
    size_t pkb, skb;
    ntrup_params(p, nullptr, nullptr, &pkb, &skb);
    for (size_t i = 0; i < n; i++) {
        int r = enqueue_dispatch(ctx, p, cfg, sd, first_index + i, 1, pk + i * pkb, sk + i * skb, w,
                                 (hipStream_t)stream, false, i == 0);
        if (r) return r;
    }
    return 0;
}

namespace {

// Enqueue every job on `st`: one job directly; several jobs on the context's
// job streams between a fork and a join on `st`, so that they run
// concurrently (and form parallel branches when captured).
// side_ok: a single job may fork its side stream (eager launches only: a
// captured graph stays one linear stream per job).
int enqueue_jobs(ntrup_ctx* ctx, const Seed& sd, const std::vector<JobDesc>& jobs, hipStream_t st, bool side_ok) {
    bool persistent = jobs.size() <= (size_t)kPMaxJobs;
    for (const JobDesc& j : jobs) persistent = persistent && j.cfg.persistent;
    if (persistent) {
        // one launch for every job; stage events: all of the call in "fused"
        for (int b = 0; b < kStages; b++)
            if (hipEvent_t ev = stage_event(ctx, b)) (void)hipEventRecord(ev, st);
        int r = enqueue_persistent(ctx, sd, jobs, st);
        if (hipEvent_t ev = stage_event(ctx, kStages)) (void)hipEventRecord(ev, st);
        if (ctx->t_used < ctx->t_max) ctx->t_side[ctx->t_used++] = 2;
        return r;
    }
    if (jobs.size() == 1) {
        const JobDesc& j = jobs[0];
        return enqueue_dispatch(ctx, j.p, j.cfg, sd, j.first_index, j.n, j.pk, j.sk,
                                carve((char*)ctx->ws + j.ws_off, j.p, j.n), st, side_ok, true);
    }
    if (!ctx->fork_event) NTRUP_HIP(ctx, hipEventCreateWithFlags(&ctx->fork_event, hipEventDisableTiming));
    while (ctx->join_events.size() < jobs.size()) {
        hipEvent_t e;
        NTRUP_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->join_events.push_back(e);
    }
    NTRUP_HIP(ctx, hipEventRecord(ctx->fork_event, st));
    for (size_t i = 0; i < jobs.size(); i++) {
        const JobDesc& j = jobs[i];
        hipStream_t js = ctx->job_streams[i % kJobStreams];
        NTRUP_HIP(ctx, hipStreamWaitEvent(js, ctx->fork_event, 0));
        // the jobs already run as concurrent branches: each stays on its own
        // stream (no second-level fork inside a forked branch)
        int r = enqueue_dispatch(ctx, j.p, j.cfg, sd, j.first_index, j.n, j.pk, j.sk,
                                 carve((char*)ctx->ws + j.ws_off, j.p, j.n), js, false, true);
        if (r) return r;
        NTRUP_HIP(ctx, hipEventRecord(ctx->join_events[i], js));
    }
    for (size_t i = 0; i < jobs.size(); i++) NTRUP_HIP(ctx, hipStreamWaitEvent(st, ctx->join_events[i], 0));
    return 0;
}

}  // namespace

int ntrup_batch_keygen_mixed(ntrup_ctx* ctx, const uint8_t* seed, const ntrup_job* jobs, size_t njobs,
                             void* stream) {
    if (!ctx || !seed || !jobs || njobs == 0 || njobs > 4096) return NTRUP_EINVAL;
    std::vector<JobDesc> jd(njobs);
    size_t total = 0;
    bool graph = ctx->t_max == 0;
    for (size_t j = 0; j < njobs; j++) {
        if (int r = check_job(jobs[j].p, jobs[j].n, jobs[j].pk, jobs[j].sk)) return r;
        jd[j] = JobDesc{jobs[j].p, jobs[j].first_index, jobs[j].n, jobs[j].pk, jobs[j].sk,
                        ctx->cfg[param_slot(jobs[j].p)], total};
        graph = graph && jd[j].cfg.use_graph;
        total += ws_bytes(jobs[j].p, jobs[j].n);
    }
    if (int r = set_device(ctx)) return r;
    if (int r = ensure_ws(ctx, total)) return r;
    const Seed sd = make_seed(seed);
    ctx->last_err.clear();
    for (const JobDesc& j : jd) ctx->last_err.push_back(carve((char*)ctx->ws + j.ws_off, j.p, j.n).counters + 32);
    hipStream_t st = (hipStream_t)stream;
    if (!graph) return enqueue_jobs(ctx, sd, jd, st, true);

    GraphKey key;
    memcpy(key.seed, sd.k, sizeof key.seed);
    key.ws = ctx->ws;
    key.jobs = jd;
    if (!ctx->have_graph || !(ctx->gkey == key)) {
        // the previous graph may still run: wait for its last launch first
        if (ctx->exec && ctx->graph_done) NTRUP_HIP(ctx, hipEventSynchronize(ctx->graph_done));
        if (ctx->exec) { (void)hipGraphExecDestroy(ctx->exec); ctx->exec = nullptr; }
        if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
        ctx->have_graph = false;
        NTRUP_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        int r = enqueue_jobs(ctx, sd, jd, ctx->cap_stream, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
        if (r) { if (g) (void)hipGraphDestroy(g); return r; }
        if (e != hipSuccess) return hip_fail(ctx, e);
        ctx->graph = g;
        NTRUP_HIP(ctx, hipGraphInstantiate(&ctx->exec, g, nullptr, nullptr, 0));
        ctx->gkey = key;
        ctx->have_graph = true;
    }
    NTRUP_HIP(ctx, hipGraphLaunch(ctx->exec, st));
    NTRUP_HIP(ctx, hipEventRecord(ctx->graph_done, st));
    return 0;
}

int ntrup_ctx_timing_begin(ntrup_ctx* ctx, int max_pipelines) {
    if (!ctx || max_pipelines < 0 || max_pipelines > 100000) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const size_t need = (size_t)max_pipelines * (kStages + 1);
    while (ctx->tev.size() < need) {
        hipEvent_t e;
        NTRUP_HIP(ctx, hipEventCreate(&e));
        ctx->tev.push_back(e);
    }
    ctx->t_side.assign((size_t)max_pipelines, 0);
    ctx->t_max = max_pipelines;
    ctx->t_used = 0;
    return 0;
}

int ntrup_ctx_timing_end(ntrup_ctx* ctx, double* ms, int nstages, int* npipelines) {
    if (!ctx || !ms || nstages < kStages + 1) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    for (int s = 0; s < nstages; s++) ms[s] = 0.0;
    for (int c = 0; c < ctx->t_used; c++) {
        // events: 0 start, 1 sampled, 2 prefix kernel done, 3 R/3 main pass
        // done, 4 R/3 retries done, 5 end (see enqueue_keygen)
        hipEvent_t* ev = &ctx->tev[(size_t)c * (kStages + 1)];
        NTRUP_HIP(ctx, hipEventSynchronize(ev[kStages]));
        float t[kStages + 1][kStages + 1] = {};
        for (int i = 0; i <= kStages; i++)
            for (int j = i + 1; j <= kStages; j++) NTRUP_HIP(ctx, hipEventElapsedTime(&t[i][j], ev[i], ev[j]));
        if (ctx->t_side[c] == 2) {
            ms[kStages] += t[0][kStages];                     // the persistent fused kernel
            continue;
        }
        ms[0] += t[0][1];                                     // sample_short
        ms[3] += t[1][2];                                     // group prefix + reciprocal
        ms[2] += t[3][4];                                     // R/3 retries
        if (ctx->t_side[c] == 3) {
            ms[1] += t[0][3];                                 // batched R/3 from the start, beside sampling
            ms[4] += t[2][4] >= 0.f ? t[4][5] : t[2][5];      // back-substitution, from its later input
        } else if (ctx->t_side[c]) {
            ms[1] += t[1][3];                                 // R/3 main pass, beside the prefix kernel
            ms[4] += t[2][4] >= 0.f ? t[4][5] : t[2][5];      // back-substitution, from its later input
        } else {
            ms[1] += t[2][3];
            ms[4] += t[4][5];
        }
    }
    if (npipelines) *npipelines = ctx->t_used;
    ctx->t_max = 0;
    ctx->t_used = 0;
    return 0;
}

int ntrup_ctx_status(ntrup_ctx* ctx, void* stream) {
    if (!ctx) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    NTRUP_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    int bits = 0;
    for (int* e : ctx->last_err) {
        int v = 0;
        NTRUP_HIP(ctx, hipMemcpy(&v, e, sizeof v, hipMemcpyDeviceToHost));
        bits |= v;
    }
    if (bits & 4) return NTRUP_ETIME;
    if (bits & 2) return NTRUP_EFAULT;
    if (bits & 1) return NTRUP_EAGAIN;
    return 0;
}

// ---------------------------------------------------------------- single ops

int ntrup_op_mul_rq(ntrup_ctx* ctx, int p, const int16_t* a, const int16_t* b, int16_t* c, size_t n, int small_a,
                    void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !b || !c || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)n), blk(64);
    const bool mfma = ctx->cfg[param_slot(p)].product_engine == 1;
#define NTRUP_MUL(PP)                                                                              \
    case PP:                                                                                       \
        if (mfma && small_a) hipLaunchKernelGGL((mulm_kernel<PP, false>), grid, blk, 0, st, (int)n, a, b, c); \
        else if (mfma) hipLaunchKernelGGL((mulm_kernel<PP, true>), grid, blk, 0, st, (int)n, a, b, c);    \
        else if (small_a) hipLaunchKernelGGL((mul_kernel<PP, false>), grid, blk, 0, st, (int)n, a, b, c); \
        else hipLaunchKernelGGL((mul_kernel<PP, true>), grid, blk, 0, st, (int)n, a, b, c);               \
        break;
    switch (p) { NTRUP_MUL(653) NTRUP_MUL(761) NTRUP_MUL(857) NTRUP_MUL(1277) }
#undef NTRUP_MUL
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

int ntrup_op_mul_r3(ntrup_ctx* ctx, int p, const int8_t* a, const int8_t* b, int8_t* c, size_t n, void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !b || !c || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)n), blk(64);
    switch (p) {
        case 653: hipLaunchKernelGGL(mul3_kernel<653>, grid, blk, 0, st, (int)n, a, b, c); break;
        case 761: hipLaunchKernelGGL(mul3_kernel<761>, grid, blk, 0, st, (int)n, a, b, c); break;
        case 857: hipLaunchKernelGGL(mul3_kernel<857>, grid, blk, 0, st, (int)n, a, b, c); break;
        case 1277: hipLaunchKernelGGL(mul3_kernel<1277>, grid, blk, 0, st, (int)n, a, b, c); break;
    }
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

int ntrup_op_recip_rq(ntrup_ctx* ctx, int p, const int16_t* a, int16_t* out, int32_t* ok, size_t n, void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !out || !ok || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)n), blk(64);
    switch (p) {
        case 653: hipLaunchKernelGGL(recip_q_kernel<653>, grid, blk, 0, st, (int)n, a, out, ok); break;
        case 761: hipLaunchKernelGGL(recip_q_kernel<761>, grid, blk, 0, st, (int)n, a, out, ok); break;
        case 857: hipLaunchKernelGGL(recip_q_kernel<857>, grid, blk, 0, st, (int)n, a, out, ok); break;
        case 1277: hipLaunchKernelGGL(recip_q_kernel<1277>, grid, blk, 0, st, (int)n, a, out, ok); break;
    }
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}


int ntrup_op_recip_r3(ntrup_ctx* ctx, int p, const int8_t* a, int8_t* out, int32_t* ok, size_t n, void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !out || !ok || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const int lpk = ctx->cfg[param_slot(p)].lanes_per_key;
    hipStream_t st = (hipStream_t)stream;
    switch (p) {
        case 653: return op_recip_r3<653>(ctx, lpk, a, out, ok, n, st);
        case 761: return op_recip_r3<761>(ctx, lpk, a, out, ok, n, st);
        case 857: return op_recip_r3<857>(ctx, lpk, a, out, ok, n, st);
        case 1277: return op_recip_r3<1277>(ctx, lpk, a, out, ok, n, st);
    }
    return NTRUP_EINVAL;
}

int ntrup_op_batch_inv_rq(ntrup_ctx* ctx, int p, const int16_t* a, int16_t* out, size_t n, size_t group_size,
                          void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !out || n == 0 || n > 0x7FFFFFFF || group_size == 0 ||
        group_size > 1024)
        return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    if (int r = ensure_ws(ctx, ws_bytes(p, n))) return r;
    const Ws w = carve(ctx->ws, p, n);
    hipStream_t st = (hipStream_t)stream;
    GroupArgs g;
    memset(&g, 0, sizeof g);
    g.n = (int)n;
    g.G = (int)group_size;
    g.bscr = w.bscr;
    g.err = w.counters + 32;
    g.a_in = a;
    g.c_out = out;
    ctx->last_err.assign(1, w.counters + 32);
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, w.counters, kCounterInts);
    const dim3 grid(grid_for(n, group_size)), blk(64);
    const bool mfma = ctx->cfg[param_slot(p)].product_engine == 1;
#define NTRUP_INV(PP)                                                                      \
    case PP:                                                                               \
        if (mfma) hipLaunchKernelGGL((group_mfma_kernel<PP>), grid, blk, 0, st, g); \
        else hipLaunchKernelGGL((group_kernel<PP, false>), grid, blk, 0, st, g);           \
        break;
    switch (p) { NTRUP_INV(653) NTRUP_INV(761) NTRUP_INV(857) NTRUP_INV(1277) }
#undef NTRUP_INV
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

int ntrup_op_sample(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n, int attempt,
                    int8_t* f, int8_t* g, void* stream) {
    if (!ctx || param_slot(p) < 0 || !seed || n == 0 || n > 0x7FFFFF || attempt < 0 ||
        attempt >= NTRUP_MAX_ATTEMPTS)
        return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const Seed sd = make_seed(seed);
    hipStream_t st = (hipStream_t)stream;
    const unsigned gw = grid_for(n * (size_t)ceil_div(p, 32), 256);
#define NTRUP_SAMPLE(PP)                                                                                      \
    case PP:                                                                                                  \
        if (f) hipLaunchKernelGGL(sample_short_kernel<PP>, dim3(grid_for(n, 4)), dim3(256), 0, st, sd,        \
                                  first_index, (int)n, f);                                                    \
        if (g) hipLaunchKernelGGL(sample_small_kernel<PP>, dim3(gw), dim3(256), 0, st, sd, first_index, (int)n, \
                                  attempt, g);                                                                \
        break;
    switch (p) { NTRUP_SAMPLE(653) NTRUP_SAMPLE(761) NTRUP_SAMPLE(857) NTRUP_SAMPLE(1277) }
#undef NTRUP_SAMPLE
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

}  // extern "C"
