/* oracle_driver.c -- runs every entry point of the oracle (oracle/nn_oracle.c)
 * on edge and random inputs, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py.  Besides the
 * sanitizers' own checks it asserts consistencies that hold by definition
 * (skip vs repeated steps, serial vs threaded generation, Eq. 2 vs the
 * truncated digit sum, the Modified Barrett step vs the plain step) and
 * exits non-zero on the first failure.  Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nn_oracle.h"

static int fails = 0;
#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                              \
        }                                                         \
    } while (0)

static uint64_t rng = 0x9E3779B97F4A7C15ULL;
static uint64_t next64(void) { /* xorshift64* */
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return rng * 0x2545F4914F6CDD1DULL;
}

int main(void) {
    const uint64_t m = ORC_MOD;
    uint64_t z = 0;
    /* seeding: both ends of the range, and outside it */
    CHECK(orc_seed(ORC_INDEX_MIN, &z) == 0 && z > 0 && z < m);
    CHECK(orc_seed(ORC_INDEX_MAX, &z) == 0 && z > 0 && z < m);
    CHECK(orc_seed(ORC_INDEX_MIN - 1, &z) != 0);
    CHECK(orc_seed(ORC_INDEX_MAX + 1, &z) != 0);
    CHECK(orc_seed(0, &z) != 0);
    /* arithmetic at the edges of the 64-bit and modulus ranges */
    CHECK(orc_mulmod(m - 1, m - 1, m) == 1);
    CHECK(orc_mulmod(UINT64_MAX, UINT64_MAX, UINT64_MAX) == 0);
    CHECK(orc_powmod(2, 0, m) == 1);
    CHECK(orc_powmod(2, UINT64_MAX, 3) == 2);
    /* step vs skip, and the index identity z_k = index_state(a + 53 k) */
    uint64_t a = ORC_INDEX_MIN + 12345;
    CHECK(orc_seed(a, &z) == 0);
    uint64_t w = z;
    for (int k = 1; k <= 1000; ++k) {
        w = orc_step(w);
        if (k % 97 == 0) {
            CHECK(orc_skip(z, (uint64_t)k) == w);
            CHECK(orc_index_state(a + 53ULL * (uint64_t)k) == w);
        }
    }
    CHECK(orc_skip(z, 0) == z);
    CHECK(orc_skip(z, UINT64_MAX) < m);
    CHECK(orc_index_state(m - 1) == 0);
    /* digit sum = index state (Eq. 2 against the truncated definition) */
    for (int i = 0; i < 200; ++i) {
        const uint64_t n = ORC_INDEX_MIN + next64() % (ORC_INDEX_MAX - ORC_INDEX_MIN);
        CHECK(orc_digit_sum(n) == orc_index_state(n));
    }
    /* generation: empty, odd sizes, serial vs threaded, u64 vs f64 */
    enum { N = 100003 };
    uint64_t *u = malloc(N * sizeof *u), *u2 = malloc(N * sizeof *u2);
    double *f = malloc(N * sizeof *f), *f2 = malloc(N * sizeof *f2);
    if (!u || !u2 || !f || !f2) return 2;
    CHECK(orc_gen_u64(z, 0, u) == z);
    const uint64_t zn = orc_gen_u64(z, N, u);
    CHECK(orc_gen_f64(z, N, f) == zn);
    CHECK(zn == orc_skip(z, N));
    CHECK(orc_gen_par(z, N, u2, 0, 0) == zn && memcmp(u, u2, N * sizeof *u) == 0);
    CHECK(orc_gen_par(z, N, f2, 1, 3) == zn && memcmp(f, f2, N * sizeof *f) == 0);
    CHECK(orc_gen_par(z, 7, u2, 0, 64) == orc_skip(z, 7));
    for (int i = 0; i < N; i += 101) {
        CHECK(u[i] > 0 && u[i] < m);
        CHECK(f[i] > 0.0 && f[i] < 1.0 && f[i] == orc_to_f64(u[i]));
    }
    CHECK(orc_max_threads() >= 1);
    /* the paper's Modified Barrett step against the plain step */
    for (int i = 0; i < 100000; ++i) {
        uint64_t s = 1 + next64() % (m - 1);
        if (s % 3 == 0) continue;
        CHECK(orc_modbarrett_step(s) == orc_step(s));
    }
    CHECK(orc_gen_f64_modbarrett(z, N, f2) == zn && memcmp(f, f2, N * sizeof *f) == 0);
    /* the generic modulus 3^e, e = 1..40 */
    for (int e = 1; e <= 40; ++e) {
        const uint64_t me = orc_g_modulus(e);
        CHECK(me > 0);
        const uint64_t n = me + 100;
        CHECK(orc_g_digit_sum(n, e) == orc_g_index_state(n, e));
        CHECK(orc_g_step(1, e, 53) < me);
    }
    /* the 3^40 generator */
    uint64_t z40 = 0;
    CHECK(orc_e40_seed(ORC_E40_INDEX_MIN, &z40) == 0 && z40 > 0 && z40 < ORC_E40_MOD);
    CHECK(orc_e40_seed(ORC_E40_INDEX_MAX, &z40) == 0 && z40 < ORC_E40_MOD);
    CHECK(orc_e40_seed(ORC_E40_INDEX_MIN - 1, &z40) != 0);
    CHECK(orc_e40_seed(ORC_E40_INDEX_MIN + 777, &z40) == 0);
    const uint64_t z40n = orc_e40_gen_u64(z40, N, u);
    CHECK(orc_e40_gen_f64(z40, N, f) == z40n && z40n == orc_e40_skip(z40, N));
    uint64_t w40 = z40;
    for (int k = 0; k < 1000; ++k) w40 = orc_e40_step(w40);
    CHECK(orc_e40_skip(z40, 1000) == w40 && u[999] == w40);
    for (int i = 0; i < N; i += 101) {
        CHECK(u[i] > 0 && u[i] < ORC_E40_MOD);
        CHECK(f[i] > 0.0 && f[i] < 1.0 && f[i] == orc_e40_to_f64(u[i]));
    }
    CHECK(orc_e40_to_f64(ORC_E40_MOD - 1) < 1.0);
    free(u);
    free(u2);
    free(f);
    free(f2);
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
