// The KeyGen stage pipeline and the single operations of one parameter set.
// Compiled once per p with -DNTRUP_P=<p> (653, 761, 857, 1277); each object
// holds the kernels of its p and the host functions that launch them.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "ntrup_host.h"
#include "ntrup_kernels.h"
#include "ntrup_kem.h"
#include "ntrup_keygen.h"
#include "ntrup_r3batch.h"
#include "ntrup_tree.h"

#ifndef NTRUP_P
#error "compile with -DNTRUP_P=653, 761, 857 or 1277"
#endif

namespace ntrup {

static_assert(kTreeRows >= kTreeMaxG, "node rows of a ragged last tree group fit the workspace");

namespace {

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
        case 16: hipLaunchKernelGGL((r3_kernel<P, 16>), grid, blk, 0, st, a); break;
        case 32: hipLaunchKernelGGL((r3_kernel<P, 32>), grid, blk, 0, st, a); break;
        case 64: hipLaunchKernelGGL((r3_kernel<P, 64>), grid, blk, 0, st, a); break;
        default: hipLaunchKernelGGL((r3_kernel<P, 8>), grid, blk, 0, st, a); break;
    }
}

// lanes per group product in the divstep reciprocals of the batched R/3
// stage (few products, so each is spread over as many lanes as pays: one
// word pair per lane, 32 lanes up to p = 1023 and a whole wave above)
template <int P>
constexpr int r3_group_lanes() { return R3Shape<P, 32>::W2 > 1 ? 64 : 32; }

// The prefix kernel with W waves per workgroup; jump: its shared reciprocal
// by jump divsteps.
template <int P, bool J>
void launch_prefix_j(int W, dim3 grid, hipStream_t st, const GroupArgs& g, int16_t* tinv) {
    const dim3 blk(64 * W);
    switch (W) {
        case 1: hipLaunchKernelGGL((keygen_prefix_kernel<P, 1, J>), grid, blk, 0, st, g, tinv); break;
        case 2: hipLaunchKernelGGL((keygen_prefix_kernel<P, 2, J>), grid, blk, 0, st, g, tinv); break;
        case 4: hipLaunchKernelGGL((keygen_prefix_kernel<P, 4, J>), grid, blk, 0, st, g, tinv); break;
        default:
            if constexpr (P != 1277) hipLaunchKernelGGL((keygen_prefix_kernel<P, 8, J>), grid, blk, 0, st, g, tinv);
            break;
    }
}

template <int P>
void launch_prefix(int W, bool jump, dim3 grid, hipStream_t st, const GroupArgs& g, int16_t* tinv) {
    if (jump) launch_prefix_j<P, true>(W, grid, st, g, tinv);
    else launch_prefix_j<P, false>(W, grid, st, g, tinv);
}

}  // namespace

// The optional raw arrays of a job, decoded from its encoded keys.
template <int P>
int op_decode_raw(ntrup_ctx* ctx, size_t n, const uint8_t* pk, const uint8_t* sk, const RawOut& raw,
                  hipStream_t st) {
    if (!raw.h && !raw.f && !raw.ginv) return 0;
    hipLaunchKernelGGL(decode_raw_kernel<P>, dim3(grid_for(n * P, 256)), dim3(256), 0, st, (int)n, pk, sk, raw.h,
                       raw.f, raw.ginv);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

// Enqueue the whole KeyGen pipeline of one job on `st`.  side_ok: with the
// matrix-core engine, the prefix half of the group stage (which needs only
// f) runs on ctx->side_stream beside the R/3 stage, forked from st after
// Short sampling and joined before h = g c.  Otherwise -- graph capture, the
// jobs of a mixed call (already concurrent branches), the plain form --
// every stage runs on st.  zero_err: also clear the error word (once per API
// call).
//
// Stage events: 0 start; 1 end of sampling; 2 end of the prefix kernel
// (the product engine 0 records it right after 1); 3 end of the R/3 main
// pass; 4 end of the R/3 retry passes; 5 end.
template <int P>
int enqueue_keygen(ntrup_ctx* ctx, const ntrup_config& cfg, const Seed& seed, uint64_t first_index, size_t n,
                   uint8_t* pk, uint8_t* sk, const RawOut& raw, const Ws& w, hipStream_t st, bool side_ok,
                   bool zero_err) {
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
    hipLaunchKernelGGL(sample_short_kernel<P>, dim3(grid_for(n, 4)), dim3(256), 0, st, seed, first_index, (int)n, 0,
                       w.f_rows);
    mark(1, st);
    if (side && !r3_first) {
        NTRUP_HIP(ctx, hipEventRecord(ctx->side_fork, st));
        NTRUP_HIP(ctx, hipStreamWaitEvent(ss, ctx->side_fork, 0));
    }
    const bool tree = mfma && cfg.group_form == 1;
    if (tree) {
        // one workgroup per group: b and t of the tree's nodes in bscr and
        // trow, c_i = 1/(3 f_i) to the key rows of tinv
        const dim3 groups(grid_for(n, cfg.group_size));
        hipLaunchKernelGGL((keygen_tree_up_kernel<P>), groups, dim3(64 * kTreeWaves), 0, sp, g, w.trow);
        if (cfg.recip_jump & 1)
            hipLaunchKernelGGL((keygen_tree_root_kernel<P, true>), groups,
                               dim3(groups.x <= 512 ? 64 * kTreeRootWaves : 64), 0, sp, g, w.trow);
        else
            hipLaunchKernelGGL((keygen_tree_root_kernel<P, false>), groups, dim3(64), 0, sp, g, w.trow);
        hipLaunchKernelGGL((keygen_tree_down_kernel<P>), groups, dim3(64 * kTreeWaves), 0, sp, g, w.trow, w.tinv);
    } else if (mfma) {
        launch_prefix<P>(W, (cfg.recip_jump & 1) != 0, dim3(grid_for(n, (size_t)cfg.group_size * W)), sp, g, w.tinv);
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
        // the group products' reciprocals: latency-bound (few products), by
        // jump divsteps on the matrix cores, one reciprocal shared by
        // kR3Share groups, or the bitsliced divsteps at the most lanes per
        // product
        if (cfg.recip_jump & 2)
            hipLaunchKernelGGL((r3_share_recip_kernel<P>), dim3(grid_for(ngroups, kR3Share)), dim3(64 * kR3Share), 0,
                               sr, (int)ngroups, (const int8_t*)w.qrow, w.pinv, (uint8_t*)w.lists[1]);
        else
            launch_r3<P>(r3_group_lanes<P>(), ngroups, gi, sr);
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
    if (tree) {
        // h = g c with c from the tree's key rows
        GroupArgs gh = g;
        gh.bscr = w.tinv;
        const unsigned per = grid_for(n, 8);
        hipLaunchKernelGGL((keygen_h_kernel<P>), dim3(8 * per), dim3(64), 0, st, gh, (int)per);
    } else if (mfma && side) {
        const unsigned per = grid_for(n, 8);
        hipLaunchKernelGGL((keygen_h_kernel<P>), dim3(8 * per), dim3(64), 0, st, g, (int)per);
    } else if (mfma) {
        hipLaunchKernelGGL((keygen_back_kernel<P>), dim3(grid_for(n, cfg.group_size)), dim3(64), 0, st, g,
                           (const int16_t*)w.tinv);
    } else {
        hipLaunchKernelGGL((group_kernel<P, true>), dim3(grid_for(n, cfg.group_size)), dim3(64), 0, st, g);
    }
    mark(5, st);
    if (int r = op_decode_raw<P>(ctx, n, pk, sk, raw, st)) return r;
    if (ctx->t_used < ctx->t_max) ctx->t_side[ctx->t_used++] = r3_first ? 3 : side ? 1 : 0;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e);
    return 0;
}

template <int P>
int op_mul_rq(ntrup_ctx* ctx, bool mfma, const int16_t* a, const int16_t* b, int16_t* c, size_t n, bool small_a,
              hipStream_t st) {
    const dim3 grid((unsigned)n), blk(64);
    if (mfma && small_a) hipLaunchKernelGGL((mulm_kernel<P, false>), grid, blk, 0, st, (int)n, a, b, c);
    else if (mfma) hipLaunchKernelGGL((mulm_kernel<P, true>), grid, blk, 0, st, (int)n, a, b, c);
    else if (small_a) hipLaunchKernelGGL((mul_kernel<P, false>), grid, blk, 0, st, (int)n, a, b, c);
    else hipLaunchKernelGGL((mul_kernel<P, true>), grid, blk, 0, st, (int)n, a, b, c);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template <int P>
int op_mul_r3(ntrup_ctx* ctx, const int8_t* a, const int8_t* b, int8_t* c, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(mul3_kernel<P>, dim3((unsigned)n), dim3(64), 0, st, (int)n, a, b, c);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template <int P>
int op_recip_rq(ntrup_ctx* ctx, bool jump, const int16_t* a, int16_t* out, int32_t* ok, size_t n, hipStream_t st) {
    if (jump)
        hipLaunchKernelGGL((recip_q_kernel<P, true>), dim3((unsigned)n), dim3(n <= 512 ? 64 * kRecipJumpWaves : 64), 0,
                           st, (int)n, a, out, ok);
    else hipLaunchKernelGGL((recip_q_kernel<P, false>), dim3((unsigned)n), dim3(64), 0, st, (int)n, a, out, ok);
    NTRUP_HIP(ctx, hipGetLastError());
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

template <int P>
int op_batch_inv_rq(ntrup_ctx* ctx, bool mfma, const int16_t* a, int16_t* out, size_t n, size_t group_size,
                    hipStream_t st) {
    if (int r = ensure_ws(ctx, ws_bytes(P, n))) return r;
    const Ws w = carve(ctx->ws, P, n);
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
    if (mfma) hipLaunchKernelGGL((group_mfma_kernel<P>), grid, blk, 0, st, g);
    else hipLaunchKernelGGL((group_kernel<P, false>), grid, blk, 0, st, g);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template <int P>
int op_sample(ntrup_ctx* ctx, const Seed& sd, uint64_t first_index, size_t n, int attempt, int8_t* f, int8_t* g,
              hipStream_t st) {
    const unsigned gw = grid_for(n * (size_t)ceil_div(P, 32), 256);
    if (f)
        hipLaunchKernelGGL(sample_short_kernel<P>, dim3(grid_for(n, 4)), dim3(256), 0, st, sd, first_index, (int)n, 0,
                           f);
    if (g) hipLaunchKernelGGL(sample_small_kernel<P>, dim3(gw), dim3(256), 0, st, sd, first_index, (int)n, attempt, g);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template <int P>
int op_encap(ntrup_ctx* ctx, const Seed& sd, uint64_t first_index, size_t n, const int16_t* h, int16_t* c, int8_t* r,
             hipStream_t st) {
    const int per = (int)((n + 7) / 8);
    hipLaunchKernelGGL(sample_short_kernel<P>, dim3(grid_for(n, 4)), dim3(256), 0, st, sd, first_index, (int)n,
                       kEncapStream, r);
    KemArgs a;
    memset(&a, 0, sizeof a);
    a.n = (int)n;
    a.per = per;
    a.h = h;
    a.c_out = c;
    a.r = r;
    hipLaunchKernelGGL(kem_encap_kernel<P>, dim3(8u * (unsigned)per), dim3(64), 0, st, a);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template <int P>
int op_decap(ntrup_ctx* ctx, size_t n, const int16_t* c, const int8_t* f, const int8_t* ginv, const int16_t* h,
             int8_t* r, uint8_t* ok, hipStream_t st) {
    const int per = (int)((n + 7) / 8);
    KemArgs a;
    memset(&a, 0, sizeof a);
    a.n = (int)n;
    a.per = per;
    a.h = h;
    a.f = f;
    a.ginv = ginv;
    a.c_in = c;
    a.r = r;
    a.ok = ok;
    hipLaunchKernelGGL(kem_decap_kernel<P>, dim3(8u * (unsigned)per), dim3(64), 0, st, a);
    NTRUP_HIP(ctx, hipGetLastError());
    return 0;
}

template int enqueue_keygen<NTRUP_P>(ntrup_ctx*, const ntrup_config&, const Seed&, uint64_t, size_t, uint8_t*,
                                     uint8_t*, const RawOut&, const Ws&, hipStream_t, bool, bool);
template int op_decode_raw<NTRUP_P>(ntrup_ctx*, size_t, const uint8_t*, const uint8_t*, const RawOut&,
                                    hipStream_t);
template int op_mul_rq<NTRUP_P>(ntrup_ctx*, bool, const int16_t*, const int16_t*, int16_t*, size_t, bool,
                                hipStream_t);
template int op_mul_r3<NTRUP_P>(ntrup_ctx*, const int8_t*, const int8_t*, int8_t*, size_t, hipStream_t);
template int op_recip_rq<NTRUP_P>(ntrup_ctx*, bool, const int16_t*, int16_t*, int32_t*, size_t, hipStream_t);
template int op_recip_r3<NTRUP_P>(ntrup_ctx*, int, const int8_t*, int8_t*, int32_t*, size_t, hipStream_t);
template int op_batch_inv_rq<NTRUP_P>(ntrup_ctx*, bool, const int16_t*, int16_t*, size_t, size_t, hipStream_t);
template int op_encap<NTRUP_P>(ntrup_ctx*, const Seed&, uint64_t, size_t, const int16_t*, int16_t*, int8_t*,
                               hipStream_t);
template int op_decap<NTRUP_P>(ntrup_ctx*, size_t, const int16_t*, const int8_t*, const int8_t*, const int16_t*,
                               int8_t*, uint8_t*, hipStream_t);
template int op_sample<NTRUP_P>(ntrup_ctx*, const Seed&, uint64_t, size_t, int, int8_t*, int8_t*, hipStream_t);

}  // namespace ntrup
