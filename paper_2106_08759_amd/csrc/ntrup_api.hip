// C ABI of the batched KeyGen library: argument checking, workspace, launch
// sequencing, stream ordering and hipGraph replay.  See include/ntrupkg.h for
// the contract.  The kernels live in the per-parameter-set objects
// (ntrup_pipeline.hip) and the persistent-kernel objects (ntrup_persist.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ntrupkg.h"
#include "ntrup_host.h"
#include "ntrup_persist.h"

using namespace ntrup;

namespace ntrup {

int ensure_ws(ntrup_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->ws_cap) return 0;
    if (ctx->ws_budget && bytes > ctx->ws_budget) return NTRUP_ENOMEM;   // nothing allocated or freed
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

void launch_zero_ints(int* p, int count, hipStream_t st) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for((size_t)count, 256)), dim3(256), 0, st, p, count);
}

}  // namespace ntrup

namespace {

// Device scratch of ntrup_batch_keygen_noalloc: the workspace of its calls,
// linked into the library (each GPU the library runs on holds one copy until
// the process ends).  Host code never passes `scratch` itself to a kernel or
// a copy: it is a host-side stand-in; scratch_ptr[d] is device d's address of
// it, taken with hipGetSymbolAddress once per device.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// Device `ctx->device`'s address of the scratch array (that device current).
int scratch_for(ntrup_ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return NTRUP_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[ctx->device]) {
        void* ptr = nullptr;
        NTRUP_HIP(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return NTRUP_EIO;
        scratch_ptr[ctx->device] = ptr;
    }
    *out = scratch_ptr[ctx->device];
    return 0;
}

int set_device(ntrup_ctx* ctx) {
    NTRUP_HIP(ctx, hipSetDevice(ctx->device));
    return 0;
}

Seed make_seed(const uint8_t* s) {
    Seed k;
    for (int i = 0; i < 8; i++)
        k.k[i] = (uint32_t)s[4 * i] | ((uint32_t)s[4 * i + 1] << 8) | ((uint32_t)s[4 * i + 2] << 16) |
                 ((uint32_t)s[4 * i + 3] << 24);
    return k;
}

// Calls on one context share its workspace.  A call enqueued on a stream
// other than the previous call's first waits for the previous call's end.
int order_after_last(ntrup_ctx* ctx, hipStream_t st) {
    if (ctx->have_last && ctx->last_stream != st) NTRUP_HIP(ctx, hipStreamWaitEvent(st, ctx->call_done, 0));
    return 0;
}

int mark_call_end(ntrup_ctx* ctx, hipStream_t st) {
    NTRUP_HIP(ctx, hipEventRecord(ctx->call_done, st));
    ctx->last_stream = st;
    ctx->have_last = true;
    return 0;
}

int enqueue_dispatch(ntrup_ctx* ctx, int p, const ntrup_config& cfg, const Seed& seed, uint64_t first_index,
                     size_t n, uint8_t* pk, uint8_t* sk, const RawOut& raw, const Ws& w, hipStream_t st,
                     bool side_ok, bool zero_err) {
    switch (p) {
        case 653: return enqueue_keygen<653>(ctx, cfg, seed, first_index, n, pk, sk, raw, w, st, side_ok, zero_err);
        case 761: return enqueue_keygen<761>(ctx, cfg, seed, first_index, n, pk, sk, raw, w, st, side_ok, zero_err);
        case 857: return enqueue_keygen<857>(ctx, cfg, seed, first_index, n, pk, sk, raw, w, st, side_ok, zero_err);
        case 1277:
            return enqueue_keygen<1277>(ctx, cfg, seed, first_index, n, pk, sk, raw, w, st, side_ok, zero_err);
    }
    return NTRUP_EINVAL;
}

// The raw arrays of a finished job (decoded from pk / sk by its p's object).
int enqueue_raw(ntrup_ctx* ctx, int p, size_t n, const uint8_t* pk, const uint8_t* sk, const RawOut& raw,
                hipStream_t st) {
    switch (p) {
        case 653: return op_decode_raw<653>(ctx, n, pk, sk, raw, st);
        case 761: return op_decode_raw<761>(ctx, n, pk, sk, raw, st);
        case 857: return op_decode_raw<857>(ctx, n, pk, sk, raw, st);
        case 1277: return op_decode_raw<1277>(ctx, n, pk, sk, raw, st);
    }
    return NTRUP_EINVAL;
}

// ---------------------------------------------------------------------------
// Persistent form: every stage of every job as items of one work list, run by
// one launch of keygen_persistent_kernel (see ntrup_persist.h).
// ---------------------------------------------------------------------------
// The work list of `jobs` (each with cfg.persistent set; the R/3 lanes per
// key of the first job apply to all): stage counts, dependency counters in
// each job's workspace (zeroed here), segments in the order S | R and C
// interleaved in 8 chunks | Q | T | B, job by job within each stage.
int enqueue_persistent(ntrup_ctx* ctx, void* base, const Seed& sd, const std::vector<JobDesc>& jobs,
                       hipStream_t st) {
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
        const Ws w = carve((char*)base + jd.ws_off, jd.p, jd.n);
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
        launch_zero_ints(w.counters, kCounterInts, st);
        launch_zero_ints(w.flags, used, st);
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
    int r;
    if (mixed) r = lpk == 2 ? launch_persistent_mixed<2>(ctx, pl, st) : launch_persistent_mixed<4>(ctx, pl, st);
    else r = lpk == 2 ? launch_persistent_single<2>(ctx, jobs[0].p, pl, st)
                      : launch_persistent_single<4>(ctx, jobs[0].p, pl, st);
    if (r) return r;
    for (const JobDesc& jd : jobs)
        if (int e = enqueue_raw(ctx, jd.p, jd.n, jd.pk, jd.sk, jd.raw, st)) return e;
    return 0;
}

bool valid_config(const ntrup_config& c) {
    auto pow2_ok = [](int l, int hi) { return l >= 1 && l <= hi && (l & (l - 1)) == 0; };
    return c.group_size >= 1 && c.group_size <= 1024 && pow2_ok(c.lanes_per_key, 64) &&
           pow2_ok(c.retry_lanes_per_key, 64) && pow2_ok(c.retry_parallel_attempts, 8) &&
           c.retry_lanes_per_key * c.retry_parallel_attempts <= 64 && c.retry_passes >= 0 &&
           c.retry_passes <= 8 && (c.use_graph == 0 || c.use_graph == 1) &&
           (c.product_engine == 0 || c.product_engine == 1) &&
           (c.inverse_share == 1 || c.inverse_share == 2 || c.inverse_share == 4 || c.inverse_share == 8) &&
           (c.persistent == 0 ||
            (c.persistent == 1 && c.product_engine == 1 && (c.lanes_per_key == 2 || c.lanes_per_key == 4))) &&
           (c.r3_batch == 0 || ((c.r3_batch == 1 || c.r3_batch == 2) && c.product_engine == 1 && c.persistent == 0)) &&
           (c.recip_jump >= 0 && c.recip_jump <= 3) &&
           (c.group_form == 0 || (c.group_form == 1 && c.product_engine == 1 && c.persistent == 0 &&
                                  c.group_size >= 2 && c.group_size <= kTreeRows &&
                                  (c.group_size & (c.group_size - 1)) == 0));
}

int check_job(int p, size_t n, const void* pk, const void* sk) {
    if (param_slot(p) < 0 || n == 0 || n > 0x7FFFFFFF || !pk || !sk) return NTRUP_EINVAL;
    return 0;
}


// Enqueue every job on `st`, its workspace at base + job.ws_off: one job
// directly; several jobs on the context's job streams between a fork and a
// join on `st`, so that they run concurrently (and form parallel branches
// when captured).  side_ok: a single job may fork its side stream (eager
// launches only: a captured graph stays one linear stream per job).
int enqueue_jobs(ntrup_ctx* ctx, void* base, const Seed& sd, const std::vector<JobDesc>& jobs, hipStream_t st,
                 bool side_ok) {
    bool persistent = jobs.size() <= (size_t)kPMaxJobs;
    for (const JobDesc& j : jobs) persistent = persistent && j.cfg.persistent;
    if (persistent) {
        // one launch for every job; stage events: all of the call in "fused"
        for (int b = 0; b < kStages; b++)
            if (hipEvent_t ev = stage_event(ctx, b)) (void)hipEventRecord(ev, st);
        int r = enqueue_persistent(ctx, base, sd, jobs, st);
        if (hipEvent_t ev = stage_event(ctx, kStages)) (void)hipEventRecord(ev, st);
        if (ctx->t_used < ctx->t_max) ctx->t_side[ctx->t_used++] = 2;
        return r;
    }
    if (jobs.size() == 1) {
        const JobDesc& j = jobs[0];
        return enqueue_dispatch(ctx, j.p, j.cfg, sd, j.first_index, j.n, j.pk, j.sk, j.raw,
                                carve((char*)base + j.ws_off, j.p, j.n), st, side_ok, true);
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
        int r = enqueue_dispatch(ctx, j.p, j.cfg, sd, j.first_index, j.n, j.pk, j.sk, j.raw,
                                 carve((char*)base + j.ws_off, j.p, j.n), js, false, true);
        if (r) return r;
        NTRUP_HIP(ctx, hipEventRecord(ctx->join_events[i], js));
    }
    for (size_t i = 0; i < jobs.size(); i++) NTRUP_HIP(ctx, hipStreamWaitEvent(st, ctx->join_events[i], 0));
    return 0;
}

// A single operation that uses the context workspace, ordered after the
// previous call on another stream and marked as the last call.
template <class F>
int ws_call(ntrup_ctx* ctx, hipStream_t st, F&& f) {
    if (int r = order_after_last(ctx, st)) return r;
    if (int r = f()) return r;
    return mark_call_end(ctx, st);
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
        case NTRUP_ENOMEM: return "device workspace over budget or allocation failed";
        case NTRUP_EINVAL: return "invalid argument";
        case NTRUP_EFAULT: return "group product not a unit";
        case NTRUP_ETIME: return "a persistent-kernel item waited too long for its inputs";
        case NTRUP_ERANGE: return "n too large for the static scratch of the allocation-free entry point";
    }
    return "unknown error";
}

int ntrup_ctx_create(ntrup_ctx** out, int device, size_t workspace_budget_bytes) {
    if (!out) return NTRUP_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return NTRUP_EINVAL;
    ntrup_ctx* ctx = new (std::nothrow) ntrup_ctx();
    if (!ctx) return NTRUP_ENOMEM;
    ctx->device = device;
    ctx->ws_budget = workspace_budget_bytes;
    ctx->one_job.reserve(1);
    ctx->last_err.reserve(kJobStreams * 4);
    for (int i = 0; i < 4; i++) ctx->cfg[i] = ntrup_config{32, 2, 8, 4, 1, 1, 1, 4, 0, 0, 1, 0};
    bool ok = set_device(ctx) == 0 && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < kJobStreams; i++)
        ok = hipStreamCreateWithFlags(&ctx->job_streams[i], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->side_join, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->graph_done, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->call_done, hipEventDisableTiming) == hipSuccess;
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
    if (ctx->call_done) (void)hipEventDestroy(ctx->call_done);
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

size_t ntrup_workspace_bytes(int p, size_t n) { return param_slot(p) < 0 ? 0 : ws_bytes(p, n); }

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
                       uint8_t* sk, int16_t* h, int8_t* f, int8_t* ginv, void* stream) {
    ntrup_job job;
    job.p = p;
    job.first_index = first_index;
    job.n = n;
    job.pk = pk;
    job.sk = sk;
    job.h = h;
    job.f = f;
    job.ginv = ginv;
    return ntrup_batch_keygen_mixed(ctx, seed, &job, 1, stream);
}

int ntrup_keygen_plain(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n, uint8_t* pk,
                       uint8_t* sk, void* stream) {
    if (!ctx || !seed) return NTRUP_EINVAL;
    if (int r = check_job(p, n, pk, sk)) return r;
    if (int r = set_device(ctx)) return r;
    if (int r = ensure_ws(ctx, ws_bytes(p, 1))) return r;
    hipStream_t st = (hipStream_t)stream;
    if (int r = order_after_last(ctx, st)) return r;
    ntrup_config cfg = ctx->cfg[param_slot(p)];
    cfg.group_size = 1;
    const Seed sd = make_seed(seed);
    const Ws w = carve(ctx->ws, p, 1);
    ctx->last_err.assign(1, w.counters + 32);
    size_t pkb, skb;
    ntrup_params(p, nullptr, nullptr, &pkb, &skb);
    const RawOut none{nullptr, nullptr, nullptr};
    for (size_t i = 0; i < n; i++) {
        int r = enqueue_dispatch(ctx, p, cfg, sd, first_index + i, 1, pk + i * pkb, sk + i * skb, none, w, st, false,
                                 i == 0);
        if (r) return r;
    }
    return mark_call_end(ctx, st);
}

int ntrup_batch_keygen_mixed(ntrup_ctx* ctx, const uint8_t* seed, const ntrup_job* jobs, size_t njobs,
                             void* stream) {
    if (!ctx || !seed || !jobs || njobs == 0 || njobs > 4096) return NTRUP_EINVAL;
    std::vector<JobDesc> jd(njobs);
    size_t total = 0;
    bool graph = ctx->t_max == 0;
    for (size_t j = 0; j < njobs; j++) {
        if (int r = check_job(jobs[j].p, jobs[j].n, jobs[j].pk, jobs[j].sk)) return r;
        jd[j] = JobDesc{jobs[j].p, jobs[j].first_index, jobs[j].n, jobs[j].pk, jobs[j].sk,
                        RawOut{jobs[j].h, jobs[j].f, jobs[j].ginv}, ctx->cfg[param_slot(jobs[j].p)], total};
        graph = graph && jd[j].cfg.use_graph;
        total += ws_bytes(jobs[j].p, jobs[j].n);
    }
    if (int r = set_device(ctx)) return r;
    if (int r = ensure_ws(ctx, total)) return r;
    const Seed sd = make_seed(seed);
    ctx->last_err.clear();
    for (const JobDesc& j : jd) ctx->last_err.push_back(carve((char*)ctx->ws + j.ws_off, j.p, j.n).counters + 32);
    hipStream_t st = (hipStream_t)stream;
    if (int r = order_after_last(ctx, st)) return r;
    if (!graph) {
        if (int r = enqueue_jobs(ctx, ctx->ws, sd, jd, st, true)) return r;
        return mark_call_end(ctx, st);
    }

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
        int r = enqueue_jobs(ctx, ctx->ws, sd, jd, ctx->cap_stream, false);
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
    return mark_call_end(ctx, st);
}

int ntrup_batch_keygen_noalloc(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n,
                               uint8_t* pk, uint8_t* sk, int16_t* h, int8_t* f, int8_t* ginv, void* stream) {
    if (!ctx || !seed) return NTRUP_EINVAL;
    if (int r = check_job(p, n, pk, sk)) return r;
    if (ws_bytes(p, n) > kScratchBytes) return NTRUP_ERANGE;
    if (int r = set_device(ctx)) return r;
    void* base = nullptr;
    if (int r = scratch_for(ctx, &base)) return r;
    // eager launches on the caller's stream only: no graph of our own (its
    // instantiation allocates) and no side stream, so that a caller may
    // capture the call into a graph of its own
    // (host vectors reserved at context creation: no host allocation either)
    std::vector<JobDesc>& jd = ctx->one_job;
    jd.assign(1, JobDesc{p, first_index, n, pk, sk, RawOut{h, f, ginv}, ctx->cfg[param_slot(p)], 0});
    jd[0].cfg.use_graph = 0;
    ctx->last_err.assign(1, carve(base, p, n).counters + 32);
    return enqueue_jobs(ctx, base, make_seed(seed), jd, (hipStream_t)stream, false);
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

#define NTRUP_BY_P(p, call)                              \
    switch (p) {                                         \
        case 653: { constexpr int P = 653; return call; }   \
        case 761: { constexpr int P = 761; return call; }   \
        case 857: { constexpr int P = 857; return call; }   \
        case 1277: { constexpr int P = 1277; return call; } \
    }                                                    \
    return NTRUP_EINVAL

int ntrup_op_mul_rq(ntrup_ctx* ctx, int p, const int16_t* a, const int16_t* b, int16_t* c, size_t n, int small_a,
                    void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !b || !c || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const bool mfma = ctx->cfg[param_slot(p)].product_engine == 1;
    NTRUP_BY_P(p, op_mul_rq<P>(ctx, mfma, a, b, c, n, small_a != 0, (hipStream_t)stream));
}

int ntrup_op_mul_r3(ntrup_ctx* ctx, int p, const int8_t* a, const int8_t* b, int8_t* c, size_t n, void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !b || !c || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    NTRUP_BY_P(p, op_mul_r3<P>(ctx, a, b, c, n, (hipStream_t)stream));
}

int ntrup_op_recip_rq(ntrup_ctx* ctx, int p, const int16_t* a, int16_t* out, int32_t* ok, size_t n, void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !out || !ok || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const bool jump = (ctx->cfg[param_slot(p)].recip_jump & 1) != 0;
    NTRUP_BY_P(p, op_recip_rq<P>(ctx, jump, a, out, ok, n, (hipStream_t)stream));
}

int ntrup_op_recip_r3(ntrup_ctx* ctx, int p, const int8_t* a, int8_t* out, int32_t* ok, size_t n, void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !out || !ok || n == 0 || n > 0x7FFFFFFF) return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const int lpk = ctx->cfg[param_slot(p)].lanes_per_key;
    hipStream_t st = (hipStream_t)stream;
    return ws_call(ctx, st, [&]() -> int { NTRUP_BY_P(p, op_recip_r3<P>(ctx, lpk, a, out, ok, n, st)); });
}

int ntrup_op_batch_inv_rq(ntrup_ctx* ctx, int p, const int16_t* a, int16_t* out, size_t n, size_t group_size,
                          void* stream) {
    if (!ctx || param_slot(p) < 0 || !a || !out || n == 0 || n > 0x7FFFFFFF || group_size == 0 ||
        group_size > 1024)
        return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const bool mfma = ctx->cfg[param_slot(p)].product_engine == 1;
    hipStream_t st = (hipStream_t)stream;
    return ws_call(ctx, st,
                   [&]() -> int { NTRUP_BY_P(p, op_batch_inv_rq<P>(ctx, mfma, a, out, n, group_size, st)); });
}

int ntrup_batch_encap(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n, const int16_t* h,
                      int16_t* c, int8_t* r, void* stream) {
    if (!ctx || param_slot(p) < 0 || !seed || n > 0x7FFFFF) return NTRUP_EINVAL;
    if (n == 0) return 0;
    if (!h || !c || !r) return NTRUP_EINVAL;
    if (int e = set_device(ctx)) return e;
    const Seed sd = make_seed(seed);
    NTRUP_BY_P(p, op_encap<P>(ctx, sd, first_index, n, h, c, r, (hipStream_t)stream));
}

int ntrup_batch_decap(ntrup_ctx* ctx, int p, size_t n, const int16_t* c, const int8_t* f, const int8_t* ginv,
                      const int16_t* h, int8_t* r, uint8_t* ok, void* stream) {
    if (!ctx || param_slot(p) < 0 || n > 0x7FFFFF) return NTRUP_EINVAL;
    if (n == 0) return 0;
    if (!c || !f || !ginv || !r) return NTRUP_EINVAL;
    if (int e = set_device(ctx)) return e;
    NTRUP_BY_P(p, op_decap<P>(ctx, n, c, f, ginv, h, r, ok, (hipStream_t)stream));
}

int ntrup_op_sample(ntrup_ctx* ctx, int p, const uint8_t* seed, uint64_t first_index, size_t n, int attempt,
                    int8_t* f, int8_t* g, void* stream) {
    if (!ctx || param_slot(p) < 0 || !seed || n == 0 || n > 0x7FFFFF || attempt < 0 ||
        attempt >= NTRUP_MAX_ATTEMPTS)
        return NTRUP_EINVAL;
    if (int r = set_device(ctx)) return r;
    const Seed sd = make_seed(seed);
    NTRUP_BY_P(p, op_sample<P>(ctx, sd, first_index, n, attempt, f, g, (hipStream_t)stream));
}

#undef NTRUP_BY_P

}  // extern "C"
