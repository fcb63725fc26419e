/*
 * nn_oracle.h -- plain, slow, obviously correct CPU oracle for the
 * alpha_{2,3} normal-number LCG of Beliakov, Johnstone, Creighton and Wilkin,
 * "Parallel random variates generator for GPUs based on normal numbers"
 * (Algorithm BB and Eqs. 1-3 of Section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this code: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Every modular product is computed as (unsigned __int128)a*b % m and every
 * power by square-and-multiply over the full 64-bit exponent; nothing is
 * blocked, fused or reordered beyond the definitions cited per function.
 *
 * Conventions (readings of the paper where it leaves a choice open):
 *  - step-then-emit: a call that emits n values from state z emits
 *    z_1..z_n (Eq. 3 applied before each output) and returns z_n;
 *  - f64 output is the IEEE round-to-nearest product double(z) * R with
 *    R = RN(1/3^33), the reciprocal the paper's listings multiply by.
 */
#ifndef NN_ORACLE_H
#define NN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 3^33, the modulus of Eqs. 2-3 (Section 2, Algorithm BB). */
#define ORC_MOD 5559060566555523ULL
/* Seed (starting index) range of Algorithm BB step 1, both ends inclusive. */
#define ORC_INDEX_MIN (ORC_MOD + 100ULL)
#define ORC_INDEX_MAX 9007199254740992ULL /* 2^53 */

/* Modular product a*b mod m for m < 2^64, via a 128-bit product. */
uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t m);
/* b^e mod m by square-and-multiply over all 64 bits of e. */
uint64_t orc_powmod(uint64_t b, uint64_t e, uint64_t m);

/* Eq. 2: z0 = 2^(a - 3^33) * floor(3^33 / 2) mod 3^33.
 * Returns 0 and writes *z0 for a in [ORC_INDEX_MIN, ORC_INDEX_MAX],
 * returns -1 (and writes nothing) otherwise. */
int orc_seed(uint64_t a, uint64_t *z0);

/* Eq. 3: one step z -> 2^53 * z mod 3^33. */
uint64_t orc_step(uint64_t z);

/* Skip-ahead (Section 2, last paragraph): the state k steps after z,
 * z * (2^53)^k mod 3^33, with k used as given (no reduction by the period). */
uint64_t orc_skip(uint64_t z, uint64_t k);

/* Eq. 2 evaluated at an arbitrary position n >= 3^33:
 * 2^(n - 3^33) * floor(3^33/2) mod 3^33.  Returns 0 for n < 3^33. */
uint64_t orc_index_state(uint64_t n);

/* The definition of alpha_{2,3} (Section 2) truncated after k = 33 and
 * scaled by 3^33: sum_{k=1}^{33} 3^(33-k) * (2^(n - 3^k) mod 3^k) mod 3^33,
 * i.e. 3^33 times the fractional part of sum_{k<=33} 2^(n-3^k)/3^k.
 * Requires n >= 3^33 (returns 0 otherwise). */
uint64_t orc_digit_sum(uint64_t n);

/* The paper's conversion to a variate in (0,1): RN(double(z) * RN(1/3^33)). */
double orc_to_f64(uint64_t z);

/* Serial generation (Algorithm BB step 3): emits z_1..z_n after z into out
 * (raw states or variates) and returns z_n (z itself when n == 0). */
uint64_t orc_gen_u64(uint64_t z, uint64_t n, uint64_t *out);
uint64_t orc_gen_f64(uint64_t z, uint64_t n, double *out);

/* The same output computed by nthreads OpenMP threads, each starting its
 * contiguous chunk from orc_skip (the skip-ahead partition of the
 * Introduction).  kind 0 = u64, 1 = f64.  nthreads <= 0 uses all threads.
 * Returns z_n. */
uint64_t orc_gen_par(uint64_t z, uint64_t n, void *out, int kind, int nthreads);
/* Number of threads orc_gen_par would use for nthreads <= 0. */
int orc_max_threads(void);

/* Generic analogue (Section 2, the LCG behind Eq. 1 at modulus 3^e):
 * modulus 3^e, multiplier 2^b mod 3^e, for 1 <= e <= 40. */
uint64_t orc_g_modulus(int e);
uint64_t orc_g_step(uint64_t z, int e, int b);
/* 2^(n - 3^e) * floor(3^e / 2) mod 3^e (Eq. 1 numerator); n >= 3^e. */
uint64_t orc_g_index_state(uint64_t n, int e);
/* sum_{k=1}^{e} 3^(e-k) * (2^(n-3^k) mod 3^k) mod 3^e: the definition of
 * alpha_{2,3} truncated after k = e, scaled by 3^e; n >= 3^e. */
uint64_t orc_g_digit_sum(uint64_t n, int e);

/* The larger modulus 3^40 that Section 2 names for a longer period: the same
 * generator with m = 3^40 (period 2*3^39), multiplier 2^53 (53 bits per
 * step, as Eq. 3), seeded by Eq. 2 with 3^40 in place of 3^33.  Readings:
 * starting indices a in [3^40 + 100, 2^64 - 1] (Algorithm BB's lower bound
 * carried over, the upper bound is the 64-bit index type); variates
 * RN(RN(z) * RN(1/3^40)), where RN(z) rounds the 64-bit state to binary64. */
#define ORC_E40_MOD 12157665459056928801ULL /* 3^40 */
#define ORC_E40_INDEX_MIN (ORC_E40_MOD + 100ULL)
#define ORC_E40_INDEX_MAX 18446744073709551615ULL /* 2^64 - 1 */
/* Eq. 2 at modulus 3^40; 0 and *z0 written for a in range, -1 otherwise. */
int orc_e40_seed(uint64_t a, uint64_t *z0);
/* One step z -> 2^53 z mod 3^40. */
uint64_t orc_e40_step(uint64_t z);
/* z * (2^53)^k mod 3^40, k used as given. */
uint64_t orc_e40_skip(uint64_t z, uint64_t k);
/* RN(RN(z) * RN(1/3^40)). */
double orc_e40_to_f64(uint64_t z);
/* Serial generation at modulus 3^40, step-then-emit; returns z_n. */
uint64_t orc_e40_gen_u64(uint64_t z, uint64_t n, uint64_t *out);
uint64_t orc_e40_gen_f64(uint64_t z, uint64_t n, double *out);

/* Modified Barrett step of Section 3.1 (the paper's fastest serial method),
 * valid for 0 < z < 3^33: 2^53 * z mod 3^33 without a division.  Kept only
 * as the paper-comparable CPU rate; the plain definition above is the oracle. */
uint64_t orc_modbarrett_step(uint64_t z);
uint64_t orc_gen_f64_modbarrett(uint64_t z, uint64_t n, double *out);

#ifdef __cplusplus
}
#endif

#endif /* NN_ORACLE_H */
