/*
 * ntrupkg.h -- batched Streamlined NTRU Prime key generation on AMD MI355X
 * (gfx950).  C ABI; no C++ or torch types.
 *
 * What it computes (OpenSSLNTRU paper, arXiv 2106.08759):
 *   KeyGen, Section 3.1: g small and invertible in R/3, 1/g in R/3, f in
 *   Short, h = g/(3f) in R/q, key pair (h, (f, 1/g)); batched as in
 *   Algorithm 1 (BatchKeyGen), the R/q reciprocals of a group of G keys shared
 *   by Montgomery's trick (Section 2.2: prefix products, one reciprocal,
 *   back-substitution; 3G-3 products + 1 reciprocal for G keys), and W such
 *   groups sharing one reciprocal through a second level of the same trick
 *   (ntrup_config.inverse_share).  R/q products run on the int8 matrix cores
 *   (exact: two 7-bit limbs per residue) or on the vector units.  The R/3
 *   reciprocal is computed per key by constant-time divsteps (the extended-gcd
 *   algorithm of Bernstein and Yang that Section 3.1 cites), which also
 *   decides invertibility.  R = Z[x]/(x^p - x - 1), parameter sets of
 *   Section 2.1 plus sntrup1277 (q = 7879, w = 492).  Also the encryption
 *   core of encapsulation and decapsulation (ntrup_batch_encap/decap).
 *
 * Determinism.  Key i of a call is a pure function of (seed, p, first_index+i):
 *   randomness is ChaCha20 (RFC 8439 block function) keyed by the 32-byte
 *   seed with nonce (key index u64 LE || p u16 LE || stream u16 LE); stream 0
 *   gives f, stream 1+k the k-th attempt at g.  So a key does not depend on n,
 *   on the group size, on the launch form or on other jobs in the same call.
 *
 * Encodings (the paper defines none; these are this library's):
 *   pk: h_i + (q-1)/2 packed as 13-bit little-endian fields, ceil(13p/8) B;
 *   sk: f then 1/g, each coefficient c as c+1 in 2 bits, four per byte,
 *       least significant first, ceil(p/4) B each.
 *
 * Memory.  Key buffers are DEVICE pointers owned by the caller; the library
 * never frees them.  The context owns a device workspace that it grows on
 * demand (hipMalloc outside of any capture), never beyond the budget given
 * to ntrup_ctx_create: a call that would need more returns NTRUP_ENOMEM and
 * allocates nothing.  ntrup_ctx_reserve sizes it in advance so that later
 * calls allocate nothing.
 *
 * Streams.  hipStream_t is passed as void*; NULL = the default stream.  All
 * keygen entry points are asynchronous: they return after enqueueing.
 * Calls on one context share its workspace, so the context orders them: a
 * call enqueued on a stream other than the previous call's waits (on the
 * device, hipStreamWaitEvent) for the previous call to finish.  Calls on
 * different contexts are independent.  ntrup_ctx_status synchronises a
 * stream and reports key-level failures.
 *
 * Errors.  0 on success, negative codes below; nothing aborts or prints.
 * A context is used by one host thread at a time.
 */
#ifndef NTRUPKG_H
#define NTRUPKG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NTRUP_OK 0
#define NTRUP_EIO (-5)      /* a HIP call failed; see ntrup_last_hip_error */
#define NTRUP_EAGAIN (-11)  /* some key found no invertible g within 64 draws */
#define NTRUP_ENOMEM (-12)  /* workspace over the context's budget, or device allocation failed */
#define NTRUP_EINVAL (-22)  /* bad parameter set, size, pointer or config */
#define NTRUP_EFAULT (-14)  /* a group product was not a unit (cannot happen in a field) */
#define NTRUP_ETIME (-62)   /* persistent form: an item's input was not ready within
                               its bounded wait (about 0.1 s); outputs are invalid */
#define NTRUP_ERANGE (-34)  /* ntrup_batch_keygen_noalloc: n exceeds its static scratch */

#define NTRUP_MAX_ATTEMPTS 64

typedef struct ntrup_ctx ntrup_ctx;

/* Sizes of parameter set p in {653, 761, 857, 1277} (Section 2.1).  Any
   output pointer may be NULL.  Returns NTRUP_EINVAL for other p. */
int ntrup_params(int p, int *q, int *w, size_t *pk_bytes, size_t *sk_bytes);

/* Create a context on HIP device `device`.  *out receives the handle.
 * workspace_budget_bytes: the most device workspace the context may ever
 * hold (0 = no limit); see ntrup_workspace_bytes for what a call needs. */
int ntrup_ctx_create(ntrup_ctx **out, int device, size_t workspace_budget_bytes);
int ntrup_ctx_destroy(ntrup_ctx *ctx);

/* Pre-size the workspace for calls of up to n keys of ring degree p. */
int ntrup_ctx_reserve(ntrup_ctx *ctx, int p, size_t n);

/* Bytes of device workspace currently held. */
size_t ntrup_ctx_workspace_bytes(const ntrup_ctx *ctx);

/* Bytes of workspace a call of n keys of parameter set p needs (a mixed call
   needs the sum over its jobs); 0 for an unknown p. */
size_t ntrup_workspace_bytes(int p, size_t n);

/* Last hipError_t seen by the context (0 if none). */
int ntrup_last_hip_error(const ntrup_ctx *ctx);
const char *ntrup_strerror(int code);

/* Tuning knobs per parameter set (chosen by the autotuner or the caller).
 *   group_size           Montgomery group size G, 1..1024 (Section 2.2's n)
 *   lanes_per_key        1, 2, 4, 8, 16, 32 or 64 lanes per key for the main R/3 pass
 *                        (more lanes: fewer registers and lower latency per
 *                        key, more cross-lane overhead; one lane per key
 *                        also skips the words of f, g, v, r that no later
 *                        divstep reads, about a fifth of the work)
 *   retry_lanes_per_key  1, 2, 4, 8, 16, 32 or 64 lanes per key for the retry passes,
 *                        which are latency-bound (few keys, a full divstep
 *                        run each)
 *   retry_parallel_attempts  1, 2, 4 or 8 consecutive g draws tried side by
 *                        side per key in the retry passes (the lowest unit
 *                        wins, so outputs do not change); retry lanes per
 *                        key times this is at most 64
 *   retry_passes         0..8 compacted passes over keys whose g was not a
 *                        unit, before a final pass that loops up to 64 draws
 *   use_graph            replay the pipeline from a captured hipGraph when
 *                        the call's arguments repeat; a captured pipeline
 *                        runs its stages on one stream, while eager launches
 *                        of a single job run the prefix products, the shared
 *                        reciprocals and the back-substitution (which need
 *                        only f) on a second stream beside the R/3 stage, and
 *                        only h = g/(3f) and the encoding after it
 *   product_engine       R/q products on the vector units (0: v_dot2 Toeplitz
 *                        dot products) or on the int8 matrix cores (1: block
 *                        Toeplitz MFMA with two 7-bit limbs); both exact
 *   inverse_share        1, 2, 4 or 8 Montgomery groups (one wave each) that
 *                        share one R/q reciprocal (product_engine 1 only;
 *                        at most 4 for p = 1277)
 *   persistent           0: the stage pipeline above (one kernel per stage);
 *                        1: one persistent fused kernel per call: sampling,
 *                        R/3, prefix chains, shared reciprocals, retries and
 *                        back-substitution of every job are items of one work
 *                        list that resident waves drain in dependency order
 *                        (requires product_engine 1 and lanes_per_key 2 or 4;
 *                        retries use 8 lanes per key; a mixed call of up to 4
 *                        jobs, all persistent, is one launch and takes the
 *                        first job's lanes_per_key)
 *   r3_batch             0: one divstep reciprocal in R/3 per key; 1: the
 *                        reciprocals of each Montgomery group of g's batched
 *                        over R/3 as in Algorithm 1 (screen of each g against
 *                        the small irreducible factors of x^p - x - 1 mod 3,
 *                        prefix products on the matrix cores, one divstep
 *                        reciprocal per group (32 lanes per group product,
 *                        64 at p = 1277),
 *                        back-substitution; a group
 *                        whose product is not a unit falls back to per-key
 *                        divsteps).  Same keys either way.  Requires
 *                        product_engine 1 and persistent 0.  2: the same
 *                        without the screen, so that every group holding a
 *                        non-unit g takes the fallback (for its tests).
 *   recip_jump           bit 0: the shared R/q reciprocal of the prefix
 *                        kernel (and ntrup_op_recip_rq); bit 1: with r3_batch,
 *                        the R/3 reciprocals of the group products -- by jump
 *                        divsteps (bit set: 48 steps at a time on the low 64
 *                        coefficients, building their 2x2 transition matrix,
 *                        which is then applied to the full polynomials on
 *                        the int8 matrix cores) or by the plain loop of
 *                        2p - 1 constant-time divsteps over the full
 *                        polynomials (bit clear; bitsliced in R/3).  Same
 *                        result.
 *   group_form           0: each Montgomery group a chain (prefix products,
 *                        the shared reciprocal, back-substitution: about 3G
 *                        dependent products on one wave); 1: a product tree
 *                        over the group's G = 2^k keys (2 <= G <= 256), the
 *                        same 3G - 3 products in 2k dependent levels shared by
 *                        the 8 waves of a workgroup, one reciprocal per
 *                        group (inverse_share unused).  Requires
 *                        product_engine 1 and persistent 0.  Same keys.    */
typedef struct {
    int group_size;
    int lanes_per_key;
    int retry_lanes_per_key;
    int retry_parallel_attempts;
    int retry_passes;
    int use_graph;
    int product_engine;
    int inverse_share;
    int persistent;
    int r3_batch;
    int recip_jump;
    int group_form;
} ntrup_config;

int ntrup_get_config(const ntrup_ctx *ctx, int p, ntrup_config *cfg);
int ntrup_set_config(ntrup_ctx *ctx, int p, const ntrup_config *cfg);

/* Batched KeyGen (Algorithm 1): keys first_index .. first_index+n-1.
 *   seed  HOST pointer, 32 bytes (copied into the launch; may be freed after)
 *   pk    device, n * pk_bytes(p) bytes, row-major by key
 *   sk    device, n * sk_bytes(p) bytes, row-major by key
 *   h     optional (NULL = skip), device int16 [n][p]: h = g/(3f) in R/q,
 *         centered in [-(q-1)/2, (q-1)/2]
 *   f     optional, device int8 [n][p]: f in Short, coefficients in {-1,0,1}
 *   ginv  optional, device int8 [n][p]: 1/g in R/3, coefficients in {-1,0,1}
 * The raw arrays are the key pair's unique values (the parity contract);
 * pk and sk are this library's encodings of them.  n >= 1 and
 * n <= 2^31 - 1.  Asynchronous on `stream`.  Key-level failures (no
 * invertible g in 64 draws: below 2^-277 per key at the worst rejection
 * rate, 4.95 % for p = 1277; below 2^-304 for p = 653) are reported by
 * ntrup_ctx_status. */
int ntrup_batch_keygen(ntrup_ctx *ctx, int p, const uint8_t *seed, uint64_t first_index, size_t n,
                       uint8_t *pk, uint8_t *sk, int16_t *h, int8_t *f, int8_t *ginv, void *stream);

/* The plain form, KeyGen of Section 3.1 one key per launch sequence (group
 * size 1, no batching): same outputs as ntrup_batch_keygen. */
int ntrup_keygen_plain(ntrup_ctx *ctx, int p, const uint8_t *seed, uint64_t first_index, size_t n,
                       uint8_t *pk, uint8_t *sk, void *stream);

/* Several parameter sets in one call (same seed); outputs identical to one
 * ntrup_batch_keygen per job. */
typedef struct {
    int p;
    uint64_t first_index;
    size_t n;
    uint8_t *pk;   /* device */
    uint8_t *sk;   /* device */
    int16_t *h;    /* optional raw outputs as in ntrup_batch_keygen; NULL = skip */
    int8_t *f;
    int8_t *ginv;
} ntrup_job;

int ntrup_batch_keygen_mixed(ntrup_ctx *ctx, const uint8_t *seed, const ntrup_job *jobs, size_t njobs,
                             void *stream);

/* The same keys as ntrup_batch_keygen, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): this call allocates nothing -- no
 * hipMalloc, hipFree or allocating library routine.  Its workspace is a
 * static device array of 32 MiB linked into the library (one copy per GPU
 * the library runs on, held until the process ends), so n is limited to
 * ntrup_workspace_bytes(p, n) <= 32 MiB (3,900 sntrup761 keys, 2,290
 * sntrup1277 keys); a larger n returns NTRUP_ERANGE and enqueues nothing.
 * The context supplies the tuning config (graph replay is not used: launches
 * are enqueued on `stream` alone, so the call may itself be captured) and
 * ntrup_ctx_status reports its key-level failures.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race and must be ordered by the caller.
 * Arguments, outputs and errors as for ntrup_batch_keygen. */
int ntrup_batch_keygen_noalloc(ntrup_ctx *ctx, int p, const uint8_t *seed, uint64_t first_index, size_t n,
                               uint8_t *pk, uint8_t *sk, int16_t *h, int8_t *f, int8_t *ginv, void *stream);

/* ---- encapsulation and decapsulation core ---------------------------------
 * The KEM's other two algorithms (Section 1: encapsulation with a public key
 * gives a ciphertext and a session key; decapsulation with the secret key
 * gives the same session key back).  The paper prints only KeyGen; these
 * compute Streamlined NTRU Prime's published encryption core on the batch:
 *   ntrup_batch_encap:  r_i in Short from stream 0x8000 of key index
 *     first_index+i (the seed and nonce layout above), c_i = Round(h_i r_i) in
 *     R/q, Round = nearest multiple of 3 of each centered coefficient;
 *   ntrup_batch_decap:  r'_i = ((3 f_i c_i in R/q) mod 3) (1/g)_i in R/3,
 *     replaced by (1, .., 1, 0, .., 0) (w ones) unless it has weight w; with
 *     h, ok_i = 1 iff Round(h_i r'_i) = c_i (the re-encryption check of the
 *     KEM), without h, ok_i = 1 iff r'_i had weight w.
 * For a key pair (h, (f, 1/g)) from ntrup_batch_keygen's raw outputs,
 * decap(encap) returns r with ok = 1.  The hashes that derive a session key
 * from r (and c), and a byte format for c, are not in the paper and are left
 * to the caller.  All arrays are device pointers, row-major [n][p], centered
 * (h, c int16; f, 1/g, r int8); ok is uint8 [n] (NULL = not written).  No
 * workspace is used and nothing is allocated; calls are asynchronous on
 * `stream` and are not ordered with other calls on the context.  n = 0 is a
 * no-op; n above 2^23, an unknown p or a missing array give NTRUP_EINVAL.
 * Decapsulation's instruction stream does not depend on the secret: the
 * weight check and the fallback are selects. */
int ntrup_batch_encap(ntrup_ctx *ctx, int p, const uint8_t *seed, uint64_t first_index, size_t n,
                      const int16_t *h, int16_t *c, int8_t *r, void *stream);
int ntrup_batch_decap(ntrup_ctx *ctx, int p, size_t n, const int16_t *c, const int8_t *f, const int8_t *ginv,
                      const int16_t *h, int8_t *r, uint8_t *ok, void *stream);

/* Synchronise `stream` and report the last keygen call on this context:
 * 0, NTRUP_EAGAIN, NTRUP_EFAULT or NTRUP_EIO. */
int ntrup_ctx_status(ntrup_ctx *ctx, void *stream);

/* Stage timing with HIP events recorded on the launch streams.  After
 * ntrup_ctx_timing_begin(ctx, m) the next m pipelines (one per job of a keygen
 * call; graph replay is bypassed meanwhile) record 6 events each, bounding
 * the stages: [0] Short sampler, [1] R/3 main pass, [2] R/3 retry and final
 * passes, [3] prefix products and group reciprocals, [4] back-substitution,
 * h = g/(3f) and encoding; [5] the persistent fused kernel (a persistent
 * call, counted once per call, puts all of its time there and none in
 * [0..4]).  With the matrix-core engine in an eager single-job call, [3]
 * runs on a side stream beside [1] and [4] is timed from the later of its
 * inputs.
 * ntrup_ctx_timing_end waits for them, writes the summed milliseconds per
 * stage to ms[0..5] (nstages >= 6), the number of pipelines timed to
 * *npipelines, and switches timing off. */
int ntrup_ctx_timing_begin(ntrup_ctx *ctx, int max_pipelines);
int ntrup_ctx_timing_end(ntrup_ctx *ctx, double *ms, int nstages, int *npipelines);

/* ---- single operations (kernel-level access, used by the tests) ----------
 * All arrays are device pointers, row-major [n][p], centered coefficients.
 * Each runs the same device code as the keygen pipeline.                   */

/* c = a * b in R/q (Section 2.1).  |a|,|b| <= (q-1)/2.  small_a != 0 selects
 * the small-operand path, which requires |a_j| <= 3.  The product engine is
 * the context's product_engine for p. */
int ntrup_op_mul_rq(ntrup_ctx *ctx, int p, const int16_t *a, const int16_t *b, int16_t *c, size_t n,
                    int small_a, void *stream);

/* c = a * b in R/3 (Section 2.1), n rows of p int8 coefficients in {-1, 0, 1}
   (device pointers), on the int8 matrix cores with the reduction mod 3: the
   product of the batched R/3 reciprocals. */
int ntrup_op_mul_r3(ntrup_ctx *ctx, int p, const int8_t *a, const int8_t *b, int8_t *c, size_t n, void *stream);

/* out = 1/a in R/q by divsteps; ok[i] = 1 iff a_i is a unit. */
int ntrup_op_recip_rq(ntrup_ctx *ctx, int p, const int16_t *a, int16_t *out, int32_t *ok, size_t n,
                      void *stream);

/* out = 1/a in R/3 by bitsliced divsteps (coefficients in {-1,0,1});
 * ok[i] = 1 iff a_i is a unit (out_i undefined otherwise). */
int ntrup_op_recip_r3(ntrup_ctx *ctx, int p, const int8_t *a, int8_t *out, int32_t *ok, size_t n,
                      void *stream);

/* Montgomery batch inversion (Section 2.2) in R/q over consecutive groups of
 * group_size rows: out_i = 1/a_i.  Every a_i must be nonzero. */
int ntrup_op_batch_inv_rq(ntrup_ctx *ctx, int p, const int16_t *a, int16_t *out, size_t n,
                          size_t group_size, void *stream);

/* The samplers: f (Short) and the attempt-th g (small) of keys
 * first_index .. first_index+n-1, as int8 rows. */
int ntrup_op_sample(ntrup_ctx *ctx, int p, const uint8_t *seed, uint64_t first_index, size_t n, int attempt,
                    int8_t *f, int8_t *g, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NTRUPKG_H */
