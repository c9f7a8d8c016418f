/* Driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host only): every exported oracle function on
 * the four parameter sets and on edge inputs, so that an out-of-bounds
 * access, a leak or undefined arithmetic anywhere in it aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_chacha20_block(const uint8_t key[32], uint32_t counter, const uint8_t nonce[12], uint8_t out[64]);
void oracle_stream_words(const uint8_t seed[32], uint64_t index, int p, int stream, uint32_t *out, int nwords);
int oracle_sample_small(const uint8_t seed[32], uint64_t index, int p, int attempt, int8_t *g);
int oracle_sample_short_stream(const uint8_t seed[32], uint64_t index, int p, int w, int stream, int8_t *f);
void oracle_mul_mod(const int64_t *a, const int64_t *b, int p, int64_t m, int64_t *out);
int oracle_inv_mod(const int64_t *a, int p, int64_t m, int64_t *out);
int oracle_keygen(const uint8_t seed[32], int p, int q, int w, uint64_t index, int8_t *f, int8_t *g, int8_t *ginv,
                  int16_t *h, int *attempts);
void oracle_encode_pk(const int16_t *h, int p, int q, uint8_t *pk);
void oracle_encode_sk(const int8_t *f, const int8_t *ginv, int p, uint8_t *sk);
long oracle_keygen_range(const uint8_t seed[32], int p, int q, int w, uint64_t index0, long n, uint64_t *checksum);
int oracle_encap(const uint8_t seed[32], int p, int q, int w, uint64_t index, const int16_t *h, int16_t *c,
                 int8_t *r);
int oracle_decap(const int16_t *c, const int8_t *f, const int8_t *ginv, const int16_t *h, int p, int q, int w,
                 int8_t *r);

static int fail(const char *what, int p) {
    printf("FAIL %s p=%d\n", what, p);
    return 1;
}

int main(void) {
    static const int P[4][3] = {{653, 4621, 288}, {761, 4591, 286}, {857, 5167, 322}, {1277, 7879, 492}};
    uint8_t seed[32], nonce[12] = {0}, block[64];
    uint32_t words[100];
    int k, i;
    for (i = 0; i < 32; i++) seed[i] = (uint8_t)i;
    oracle_chacha20_block(seed, 0xFFFFFFFFu, nonce, block);
    oracle_stream_words(seed, ~0ull, 1277, 0xFFFF, words, 100);
    for (k = 0; k < 4; k++) {
        const int p = P[k][0], q = P[k][1], w = P[k][2];
        int8_t *f = malloc((size_t)p), *g = malloc((size_t)p), *gi = malloc((size_t)p), *r = malloc((size_t)p),
               *r2 = malloc((size_t)p);
        int16_t *h = malloc(2 * (size_t)p), *c = malloc(2 * (size_t)p);
        int64_t *a = calloc((size_t)p, 8), *b = calloc((size_t)p, 8), *o = calloc((size_t)p, 8);
        uint8_t *pk = malloc((size_t)(13 * p + 7) / 8), *sk = malloc(2 * (size_t)((p + 3) / 4));
        uint64_t cs = 0;
        int att = 0, idx;
        for (idx = 0; idx < 3; idx++) {
            if (oracle_keygen(seed, p, q, w, (uint64_t)idx, f, g, gi, h, &att) != 0) return fail("keygen", p);
            oracle_encode_pk(h, p, q, pk);
            oracle_encode_sk(f, gi, p, sk);
            if (oracle_encap(seed, p, q, w, (uint64_t)idx, h, c, r) != 0) return fail("encap", p);
            if (oracle_decap(c, f, gi, h, p, q, w, r2) != 1 || memcmp(r, r2, (size_t)p)) return fail("decap", p);
            memset(c, 0, 2 * (size_t)p);
            if (oracle_decap(c, f, gi, h, p, q, w, r2) != 0) return fail("decap of zero", p);
            for (i = 0; i < p; i++) c[i] = (int16_t)((i % 2 ? 1 : -1) * 3 * ((q - 1) / 6));
            if (oracle_decap(c, f, gi, NULL, p, q, w, r2) < 0) return fail("decap of extremes", p);
        }
        if (oracle_sample_small(seed, 7, p, 63, g) != 0) return fail("small", p);
        if (oracle_sample_short_stream(seed, 7, p, p, 0x8000, f) != 0) return fail("short w = p", p);
        for (i = 0; i < p; i++) { a[i] = (q - 1) / 2; b[i] = -(q - 1) / 2; }
        oracle_mul_mod(a, b, p, q, o);
        memset(a, 0, 8 * (size_t)p);
        if (oracle_inv_mod(a, p, 3, o) != 0 || oracle_inv_mod(a, p, q, o) != 0) return fail("inverse of 0", p);
        a[0] = 1;
        if (oracle_inv_mod(a, p, q, o) != 1) return fail("inverse of 1", p);
        if (oracle_keygen_range(seed, p, q, w, 1000, 2, &cs) != 2) return fail("range", p);
        free(f); free(g); free(gi); free(r); free(r2); free(h); free(c); free(a); free(b); free(o); free(pk); free(sk);
    }
    printf("ok\n");
    return 0;
}
