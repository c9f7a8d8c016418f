/*
 * ntrup_oracle.c -- plain, slow, obviously-correct CPU model of Streamlined
 * NTRU Prime key generation, used ONLY as test infrastructure.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library.  The GPU library never links or
 * calls it, and the two share no code: no headers, tables, helpers or
 * constant generators.
 *
 * What is computed (OpenSSLNTRU paper, Section 3.1, the KeyGen list):
 *   1. sample a uniform small g, repeat until g is invertible in R/3;
 *   2. 1/g in R/3;
 *   3. sample f in Short;
 *   4. h = g / (3f) in R/q;
 *   5. output (h, (f, 1/g)).
 * with R = Z[x]/(x^p - x - 1), R/3 and R/q its reductions and Short the
 * weight-w small elements (Section 2.1).
 *
 * The arithmetic is the plain definition, one key at a time:
 *   - products: schoolbook convolution of length 2p-1, then the reduction
 *     x^p = x + 1 (Section 2.1), then reduction of coefficients;
 *   - reciprocals: textbook extended Euclid over the prime field F_m
 *     (long division, Bezout coefficient), for m = 3 and m = q.
 * There is no batching (Montgomery's trick, Section 2.2, is a faster way to
 * reach exactly the same reciprocals; inverses are unique), no divsteps and
 * no blocking.
 *
 * Randomness.  The paper only says "uniform random" (Section 3.1 and
 * Algorithm 1).  The convention fixed for this library is:
 *   - ChaCha20 block function (20 rounds, 32-bit block counter, 96-bit nonce,
 *     as in RFC 8439), key = 32-byte master seed;
 *   - nonce = key index (u64 little-endian) || p (u16 LE) || stream id (u16 LE);
 *   - stream id 0 feeds f, stream id 1+k feeds the k-th attempt at g;
 *   - word i of a stream = little-endian u32 at keystream byte offset 4i.
 * Samplers (definitions of Short and small in Section 2.1):
 *   - g_i = floor(3 r_i / 2^32) - 1, i < p;
 *   - f: L_i = (r_i & ~3) | v_i with v_i = 2(r_i & 1) for i < w and v_i = 1
 *     otherwise; sort L ascending as unsigned 32-bit; f_i = (L_i & 3) - 1.
 *
 * Encodings (the paper never defines a byte format; these are the library's):
 *   - pk: each h_i + (q-1)/2 (13 bits) packed little-endian, ceil(13p/8) bytes;
 *   - sk: f then 1/g, each coefficient c as c+1 in 2 bits, 4 per byte, LSB
 *     first, ceil(p/4) bytes each.
 *
 * Encapsulation and decapsulation (the KEM's other two algorithms, Section 1)
 * are computed as their arithmetic core only; see the section at the end.
 *
 * Every function works for any odd prime modulus m and any p >= 2, so the
 * same code is checked by brute force on toy rings.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_ATTEMPTS 64
#define ORACLE_EAGAIN (-11)
#define ORACLE_EINVAL (-22)
#define ORACLE_ENOMEM (-12)

/* ------------------------------------------------------------------------ */
/* ChaCha20 block function (RFC 8439 description)                            */
/* ------------------------------------------------------------------------ */

static uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

static uint32_t load_le32(const uint8_t *b)
{
    return (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) |
           ((uint32_t)b[3] << 24);
}

static void store_le32(uint8_t *b, uint32_t v)
{
    b[0] = (uint8_t)v;
    b[1] = (uint8_t)(v >> 8);
    b[2] = (uint8_t)(v >> 16);
    b[3] = (uint8_t)(v >> 24);
}

static void quarter_round(uint32_t *x, int a, int b, int c, int d)
{
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);
}

/* 64 bytes of keystream for (key, block counter, nonce). */
void oracle_chacha20_block(const uint8_t key[32], uint32_t counter,
                           const uint8_t nonce[12], uint8_t out[64])
{
    uint32_t init[16], x[16];
    int i;
    init[0] = 0x61707865u; /* "expa" */
    init[1] = 0x3320646eu; /* "nd 3" */
    init[2] = 0x79622d32u; /* "2-by" */
    init[3] = 0x6b206574u; /* "te k" */
    for (i = 0; i < 8; i++) init[4 + i] = load_le32(key + 4 * i);
    init[12] = counter;
    for (i = 0; i < 3; i++) init[13 + i] = load_le32(nonce + 4 * i);
    memcpy(x, init, sizeof x);
    for (i = 0; i < 10; i++) {
        /* column round */
        quarter_round(x, 0, 4, 8, 12);
        quarter_round(x, 1, 5, 9, 13);
        quarter_round(x, 2, 6, 10, 14);
        quarter_round(x, 3, 7, 11, 15);
        /* diagonal round */
        quarter_round(x, 0, 5, 10, 15);
        quarter_round(x, 1, 6, 11, 12);
        quarter_round(x, 2, 7, 8, 13);
        quarter_round(x, 3, 4, 9, 14);
    }
    for (i = 0; i < 16; i++) store_le32(out + 4 * i, x[i] + init[i]);
}

/* Words 0..nwords-1 of stream `stream` of key `index` for ring degree p. */
void oracle_stream_words(const uint8_t seed[32], uint64_t index, int p,
                         int stream, uint32_t *out, int nwords)
{
    uint8_t nonce[12], block[64];
    int i, blk;
    for (i = 0; i < 8; i++) nonce[i] = (uint8_t)(index >> (8 * i));
    nonce[8] = (uint8_t)p;
    nonce[9] = (uint8_t)(p >> 8);
    nonce[10] = (uint8_t)stream;
    nonce[11] = (uint8_t)(stream >> 8);
    for (blk = 0; 16 * blk < nwords; blk++) {
        oracle_chacha20_block(seed, (uint32_t)blk, nonce, block);
        for (i = 0; i < 16 && 16 * blk + i < nwords; i++)
            out[16 * blk + i] = load_le32(block + 4 * i);
    }
}

/* ------------------------------------------------------------------------ */
/* Samplers (Section 2.1: small and Short)                                   */
/* ------------------------------------------------------------------------ */

/* Attempt k at a uniform small g: coefficients in {-1,0,1}. */
int oracle_sample_small(const uint8_t seed[32], uint64_t index, int p,
                        int attempt, int8_t *g)
{
    uint32_t *r = malloc(sizeof(uint32_t) * (size_t)p);
    int i;
    if (!r) return ORACLE_ENOMEM;
    oracle_stream_words(seed, index, p, 1 + attempt, r, p);
    for (i = 0; i < p; i++)
        g[i] = (int8_t)((int)(((uint64_t)r[i] * 3u) >> 32) - 1);
    free(r);
    return 0;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* An element of Short from stream `stream`: exactly w coefficients in
   {-1,1}, the rest 0. */
int oracle_sample_short_stream(const uint8_t seed[32], uint64_t index, int p,
                               int w, int stream, int8_t *f)
{
    uint32_t *L = malloc(sizeof(uint32_t) * (size_t)p);
    int i;
    if (!L) return ORACLE_ENOMEM;
    oracle_stream_words(seed, index, p, stream, L, p);
    for (i = 0; i < p; i++) {
        uint32_t v = (i < w) ? 2u * (L[i] & 1u) : 1u;
        L[i] = (L[i] & ~3u) | v;
    }
    qsort(L, (size_t)p, sizeof(uint32_t), cmp_u32);
    for (i = 0; i < p; i++) f[i] = (int8_t)((int)(L[i] & 3u) - 1);
    free(L);
    return 0;
}

/* f in Short for KeyGen: stream 0. */
int oracle_sample_short(const uint8_t seed[32], uint64_t index, int p, int w,
                        int8_t *f)
{
    return oracle_sample_short_stream(seed, index, p, w, 0, f);
}

/* ------------------------------------------------------------------------ */
/* Arithmetic in F_m[x] and F_m[x]/(x^p - x - 1), m an odd prime            */
/* ------------------------------------------------------------------------ */

static int64_t mod_m(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/* a^(m-2) mod m: the inverse of a nonzero a in the prime field F_m. */
static int64_t inv_mod(int64_t a, int64_t m)
{
    int64_t result = 1, base = mod_m(a, m), e = m - 2;
    while (e > 0) {
        if (e & 1) result = result * base % m;
        base = base * base % m;
        e >>= 1;
    }
    return result;
}

/* degree of a[0..n-1], -1 for the zero polynomial */
static int poly_deg(const int64_t *a, int n)
{
    int d = n - 1;
    while (d >= 0 && a[d] == 0) d--;
    return d;
}

/*
 * Product in R/m = F_m[x]/(x^p - x - 1): schoolbook convolution c = a*b of
 * length 2p-1, then for k = 2p-2 down to p replace c_k x^k by
 * c_k x^(k-p) (x + 1), i.e. add c_k into c_(k-p) and c_(k-p+1).  Both targets
 * are below p, so one pass suffices.  Inputs may be any representatives;
 * the output is in [0, m).
 */
void oracle_mul_mod(const int64_t *a, const int64_t *b, int p, int64_t m,
                    int64_t *out)
{
    int64_t *c = calloc((size_t)(2 * p - 1), sizeof(int64_t));
    int i, j, k;
    if (!c) return;
    for (i = 0; i < p; i++)
        for (j = 0; j < p; j++)
            c[i + j] = mod_m(c[i + j] + mod_m(a[i], m) * mod_m(b[j], m), m);
    for (k = 2 * p - 2; k >= p; k--) {
        c[k - p] = mod_m(c[k - p] + c[k], m);
        c[k - p + 1] = mod_m(c[k - p + 1] + c[k], m);
        c[k] = 0;
    }
    for (i = 0; i < p; i++) out[i] = c[i];
    free(c);
}

/*
 * Reciprocal in R/m by the textbook extended Euclidean algorithm on
 * (x^p - x - 1, a) over F_m.  Keeps r_prev = s_prev * a (mod x^p - x - 1)
 * and r_cur = s_cur * a, divides with remainder until the remainder is 0.
 * The last nonzero remainder is the gcd; a is a unit iff it is a nonzero
 * constant, and then 1/a = s_prev / gcd.
 * Returns 1 and writes out[0..p-1] in [0, m) if a is invertible; returns 0
 * (out zeroed) otherwise, including a = 0.  -12 if memory runs out.
 */
int oracle_inv_mod(const int64_t *a, int p, int64_t m, int64_t *out)
{
    int n = 2 * p + 2, i, ret = ORACLE_ENOMEM;
    int64_t *r_prev = calloc((size_t)n, sizeof(int64_t));
    int64_t *r_cur = calloc((size_t)n, sizeof(int64_t));
    int64_t *s_prev = calloc((size_t)n, sizeof(int64_t));
    int64_t *s_cur = calloc((size_t)n, sizeof(int64_t));
    int64_t *quo = calloc((size_t)n, sizeof(int64_t));
    int64_t *tmp = calloc((size_t)(2 * n), sizeof(int64_t));
    if (!r_prev || !r_cur || !s_prev || !s_cur || !quo || !tmp) goto done;

    /* r_prev = x^p - x - 1, s_prev = 0; r_cur = a, s_cur = 1 */
    r_prev[p] = 1;
    r_prev[1] = m - 1;
    r_prev[0] = m - 1;
    for (i = 0; i < p; i++) r_cur[i] = mod_m(a[i], m);
    s_cur[0] = 1;

    while (poly_deg(r_cur, n) >= 0) {
        int dc = poly_deg(r_cur, n), dr;
        int64_t lead_inv = inv_mod(r_cur[dc], m);
        /* long division: r_prev = quo * r_cur + rem, rem left in r_prev */
        memset(quo, 0, sizeof(int64_t) * (size_t)n);
        while ((dr = poly_deg(r_prev, n)) >= dc) {
            int shift = dr - dc;
            int64_t coef = r_prev[dr] * lead_inv % m;
            quo[shift] = coef;
            for (i = 0; i <= dc; i++)
                r_prev[i + shift] = mod_m(r_prev[i + shift] - coef * r_cur[i], m);
        }
        /* (r_prev, r_cur) <- (r_cur, rem) */
        for (i = 0; i < n; i++) {
            int64_t t = r_prev[i];
            r_prev[i] = r_cur[i];
            r_cur[i] = t;
        }
        /* (s_prev, s_cur) <- (s_cur, s_prev - quo * s_cur) */
        memset(tmp, 0, sizeof(int64_t) * (size_t)(2 * n));
        {
            int dq = poly_deg(quo, n), ds = poly_deg(s_cur, n), j;
            for (i = 0; i <= dq; i++)
                for (j = 0; j <= ds; j++)
                    tmp[i + j] = mod_m(tmp[i + j] + quo[i] * s_cur[j], m);
        }
        for (i = 0; i < n; i++) {
            int64_t next = mod_m(s_prev[i] - tmp[i], m);
            s_prev[i] = s_cur[i];
            s_cur[i] = next;
        }
    }

    if (poly_deg(r_prev, n) == 0) {
        /* gcd is the constant r_prev[0]; s_prev * a = r_prev[0] mod (x^p-x-1).
           Bezout coefficients stay below degree p, so no reduction is needed;
           check it rather than assume it. */
        int64_t ginv = inv_mod(r_prev[0], m);
        if (poly_deg(s_prev, n) >= p) { ret = ORACLE_EINVAL; goto done; }
        for (i = 0; i < p; i++) out[i] = s_prev[i] * ginv % m;
        ret = 1;
    } else {
        for (i = 0; i < p; i++) out[i] = 0;
        ret = 0;
    }
done:
    free(r_prev); free(r_cur); free(s_prev); free(s_cur); free(quo); free(tmp);
    return ret;
}

/* centered representative in [-(m-1)/2, (m-1)/2] of x in [0, m) */
static int64_t center(int64_t x, int64_t m) { return x > (m - 1) / 2 ? x - m : x; }

/* ------------------------------------------------------------------------ */
/* KeyGen (Section 3.1)                                                      */
/* ------------------------------------------------------------------------ */

/*
 * One key pair for (seed, p, q, w, index).  Outputs (all length p, centered):
 * f (Short), g (the accepted small element), ginv = 1/g in R/3,
 * h = g/(3f) in R/q.  *attempts = number of g samples drawn (>= 1).
 * Returns 0, or -11 if no invertible g appeared within 64 attempts, or -22
 * on bad parameters.
 */
int oracle_keygen(const uint8_t seed[32], int p, int q, int w, uint64_t index,
                  int8_t *f, int8_t *g, int8_t *ginv, int16_t *h, int *attempts)
{
    int64_t *a = NULL, *b = NULL, *c = NULL;
    int i, k, ok = 0, ret = 0;
    if (p < 2 || q < 5 || (q % 2) == 0 || w < 0 || w > p) return ORACLE_EINVAL;
    a = calloc((size_t)p, sizeof(int64_t));
    b = calloc((size_t)p, sizeof(int64_t));
    c = calloc((size_t)p, sizeof(int64_t));
    if (!a || !b || !c) { ret = ORACLE_ENOMEM; goto done; }

    /* 1-2: small g, resampled until invertible in R/3; its reciprocal */
    for (k = 0; k < ORACLE_MAX_ATTEMPTS && !ok; k++) {
        if ((ret = oracle_sample_small(seed, index, p, k, g)) != 0) goto done;
        for (i = 0; i < p; i++) a[i] = g[i];
        ok = oracle_inv_mod(a, p, 3, b);
        if (ok < 0) { ret = ok; goto done; }
    }
    *attempts = k;
    if (!ok) { ret = ORACLE_EAGAIN; goto done; }
    for (i = 0; i < p; i++) ginv[i] = (int8_t)center(b[i], 3);

    /* 3: f in Short */
    if ((ret = oracle_sample_short(seed, index, p, w, f)) != 0) goto done;

    /* 4: h = g * (3f)^-1 in R/q */
    for (i = 0; i < p; i++) a[i] = 3 * (int64_t)f[i];
    ok = oracle_inv_mod(a, p, q, b);
    if (ok != 1) { ret = ok < 0 ? ok : ORACLE_EINVAL; goto done; }
    for (i = 0; i < p; i++) a[i] = g[i];
    oracle_mul_mod(a, b, p, q, c);
    for (i = 0; i < p; i++) h[i] = (int16_t)center(c[i], q);
    ret = 0;
done:
    free(a); free(b); free(c);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* Encodings                                                                 */
/* ------------------------------------------------------------------------ */

/* pk: h_i + (q-1)/2 as 13-bit little-endian fields; ceil(13p/8) bytes. */
void oracle_encode_pk(const int16_t *h, int p, int q, uint8_t *pk)
{
    int nbytes = (13 * p + 7) / 8, i, bit;
    memset(pk, 0, (size_t)nbytes);
    for (i = 0; i < p; i++) {
        uint32_t v = (uint32_t)(h[i] + (q - 1) / 2);
        for (bit = 0; bit < 13; bit++) {
            int pos = 13 * i + bit;
            if ((v >> bit) & 1u) pk[pos / 8] |= (uint8_t)(1u << (pos % 8));
        }
    }
}

/* sk: f then ginv, each coefficient c stored as c+1 in 2 bits, LSB first. */
void oracle_encode_sk(const int8_t *f, const int8_t *ginv, int p, uint8_t *sk)
{
    int half = (p + 3) / 4, i;
    memset(sk, 0, (size_t)(2 * half));
    for (i = 0; i < p; i++) {
        sk[i / 4] |= (uint8_t)((f[i] + 1) << (2 * (i % 4)));
        sk[half + i / 4] |= (uint8_t)((ginv[i] + 1) << (2 * (i % 4)));
    }
}

/* CPU-baseline driver: keys index0 .. index0+n-1, outputs discarded except
   a checksum so that nothing is optimised away.  Returns the number of keys
   that completed, or a negative error. */
long oracle_keygen_range(const uint8_t seed[32], int p, int q, int w,
                         uint64_t index0, long n, uint64_t *checksum)
{
    int8_t *f = malloc((size_t)p), *g = malloc((size_t)p), *gi = malloc((size_t)p);
    int16_t *h = malloc(sizeof(int16_t) * (size_t)p);
    long done = 0, j;
    uint64_t sum = 0;
    int att, i;
    if (!f || !g || !gi || !h) { done = ORACLE_ENOMEM; goto out; }
    for (j = 0; j < n; j++) {
        int ret = oracle_keygen(seed, p, q, w, index0 + (uint64_t)j, f, g, gi, h, &att);
        if (ret != 0) { done = ret; goto out; }
        for (i = 0; i < p; i++) sum = sum * 31u + (uint64_t)(uint16_t)h[i];
        done++;
    }
out:
    *checksum = sum;
    free(f); free(g); free(gi); free(h);
    return done;
}

/* ------------------------------------------------------------------------ */
/* Encapsulation and decapsulation core                                      */
/* ------------------------------------------------------------------------ */
/*
 * The paper uses sntrup as a KEM (Section 1: key generation, encapsulation
 * with a public key, decapsulation with the secret key) and prints only the
 * KeyGen steps.  What follows is the published Streamlined NTRU Prime core,
 * restated:
 *   encrypt(r, h), r in Short:  c = Round(h r) in R/q, where Round replaces
 *     each centered coefficient by the nearest multiple of 3;
 *   decrypt(c, f, v = 1/g):  e = 3 f c in R/q, centered; e reduced mod 3;
 *     r' = e v in R/3, centered; if r' does not have weight w it is replaced
 *     by the fixed weight-w element (1, ..., 1, 0, ..., 0) (w ones first);
 *   decapsulation with the public key also encrypts r' again and reports
 *     whether that gives c back.
 * For a key pair and r in Short, decrypt(encrypt(r)) = r: the centered 3 f c
 * equals g r + 3 f (c - h r) over Z when q > 16 w + 1 (every coefficient is
 * below 8 w in size), so reducing mod 3 leaves g r.  The hashes that turn r
 * and c into a session key, and a byte format for c, are not in the paper
 * and are not computed here.
 * Encapsulation draws r with the Short sampler from stream 0x8000 of the
 * key's index (KeyGen uses streams 0 .. 64).
 */
#define ORACLE_ENCAP_STREAM 0x8000

/* nearest multiple of 3 to x: 3 floor((x + 1) / 3) */
static int64_t round3(int64_t x)
{
    int64_t y = x + 1;
    int64_t fl = y >= 0 ? y / 3 : -((-y + 2) / 3);
    return 3 * fl;
}

/* c = Round(h r) in R/q (h and r centered; c centered, a multiple of 3). */
int oracle_encrypt(const int16_t *h, const int8_t *r, int p, int q, int16_t *c)
{
    int64_t *a = calloc((size_t)p, sizeof(int64_t));
    int64_t *b = calloc((size_t)p, sizeof(int64_t));
    int64_t *t = calloc((size_t)p, sizeof(int64_t));
    int i, ret = ORACLE_ENOMEM;
    if (!a || !b || !t) goto done;
    for (i = 0; i < p; i++) { a[i] = h[i]; b[i] = r[i]; }
    oracle_mul_mod(a, b, p, q, t);
    for (i = 0; i < p; i++) c[i] = (int16_t)round3(center(t[i], q));
    ret = 0;
done:
    free(a); free(b); free(t);
    return ret;
}

/* r' = decrypt(c) as above; returns 1 if r' had weight w, 0 if it was
   replaced by the fixed element, or a negative error. */
int oracle_decrypt(const int16_t *c, const int8_t *f, const int8_t *ginv,
                   int p, int q, int w, int8_t *r)
{
    int64_t *a = calloc((size_t)p, sizeof(int64_t));
    int64_t *b = calloc((size_t)p, sizeof(int64_t));
    int64_t *t = calloc((size_t)p, sizeof(int64_t));
    int i, weight = 0, ret = ORACLE_ENOMEM;
    if (!a || !b || !t) goto done;
    /* e = 3 f c in R/q, centered, then mod 3 */
    for (i = 0; i < p; i++) { a[i] = 3 * (int64_t)f[i]; b[i] = c[i]; }
    oracle_mul_mod(a, b, p, q, t);
    for (i = 0; i < p; i++) a[i] = mod_m(center(t[i], q), 3);
    /* r' = e v in R/3 */
    for (i = 0; i < p; i++) b[i] = ginv[i];
    oracle_mul_mod(a, b, p, 3, t);
    for (i = 0; i < p; i++) {
        r[i] = (int8_t)center(t[i], 3);
        weight += r[i] != 0;
    }
    if (weight != w)
        for (i = 0; i < p; i++) r[i] = (int8_t)(i < w ? 1 : 0);
    ret = weight == w;
done:
    free(a); free(b); free(t);
    return ret;
}

/* Encapsulation core for key `index`: r in Short from the encapsulation
   stream, c = encrypt(r, h). */
int oracle_encap(const uint8_t seed[32], int p, int q, int w, uint64_t index,
                 const int16_t *h, int16_t *c, int8_t *r)
{
    int ret = oracle_sample_short_stream(seed, index, p, w, ORACLE_ENCAP_STREAM, r);
    if (ret != 0) return ret;
    return oracle_encrypt(h, r, p, q, c);
}

/* Decapsulation core: r' = decrypt(c).  With h (not NULL) returns 1 iff
   encrypt(r', h) = c; without h, 1 iff r' had weight w.  0 otherwise, or a
   negative error. */
int oracle_decap(const int16_t *c, const int8_t *f, const int8_t *ginv,
                 const int16_t *h, int p, int q, int w, int8_t *r)
{
    int16_t *c2;
    int i, ok = oracle_decrypt(c, f, ginv, p, q, w, r);
    if (ok < 0 || !h) return ok;
    c2 = malloc(sizeof(int16_t) * (size_t)p);
    if (!c2) return ORACLE_ENOMEM;
    ok = oracle_encrypt(h, r, p, q, c2);
    if (ok == 0) {
        ok = 1;
        for (i = 0; i < p; i++) ok &= c2[i] == c[i];
    }
    free(c2);
    return ok;
}
