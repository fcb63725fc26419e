/*
 * nn_oracle.c -- the CPU oracle (test infrastructure; see nn_oracle.h).
 *
 * Each function restates a definition of Section 2 of Beliakov et al.
 * (Algorithm BB, Eqs. 1-3, the definition of alpha_{2,3}) with 128-bit
 * integer products; the paper's reduction methods of Section 3 are not used
 * here except orc_modbarrett_step, which is kept only as a timing comparator.
 */
#include "nn_oracle.h"

#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* RN(1/3^33): the reciprocal the paper's listings multiply a state by. */
static const double ORC_RECIP = 1.0 / 5559060566555523.0;

uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)(((u128)a * (u128)b) % (u128)m);
}

uint64_t orc_powmod(uint64_t b, uint64_t e, uint64_t m)
{
    uint64_t result = 1 % m;
    uint64_t base = b % m;
    while (e != 0) {
        if (e & 1u)
            result = orc_mulmod(result, base, m);
        base = orc_mulmod(base, base, m);
        e >>= 1;
    }
    return result;
}

uint64_t orc_g_modulus(int e)
{
    uint64_t m = 1;
    for (int i = 0; i < e; i++)
        m *= 3;
    return m;
}

/* Eq. 1 numerator / Eq. 2 at modulus 3^e and position n >= 3^e. */
uint64_t orc_g_index_state(uint64_t n, int e)
{
    uint64_t m = orc_g_modulus(e);
    if (n < m)
        return 0;
    return orc_mulmod(orc_powmod(2, n - m, m), m / 2, m);
}

uint64_t orc_g_step(uint64_t z, int e, int b)
{
    uint64_t m = orc_g_modulus(e);
    return orc_mulmod(orc_powmod(2, (uint64_t)b, m), z, m);
}

int orc_seed(uint64_t a, uint64_t *z0)
{
    if (a < ORC_INDEX_MIN || a > ORC_INDEX_MAX)
        return -1;
    *z0 = orc_index_state(a);
    return 0;
}

uint64_t orc_index_state(uint64_t n)
{
    return orc_g_index_state(n, 33);
}

/* The multiplier of Eq. 3, 2^53 reduced mod 3^33. */
static uint64_t orc_multiplier(void)
{
    return orc_powmod(2, 53, ORC_MOD);
}

uint64_t orc_step(uint64_t z)
{
    /* 2^53 * z mod 3^33 straight from Eq. 3. */
    return orc_mulmod(orc_multiplier(), z, ORC_MOD);
}

uint64_t orc_skip(uint64_t z, uint64_t k)
{
    return orc_mulmod(z, orc_powmod(orc_multiplier(), k, ORC_MOD), ORC_MOD);
}

uint64_t orc_g_digit_sum(uint64_t n, int e)
{
    const uint64_t m = orc_g_modulus(e);
    if (n < m)
        return 0;
    uint64_t acc = 0;
    uint64_t three_k = 1;
    for (int k = 1; k <= e; k++) {
        three_k *= 3; /* 3^k */
        uint64_t term = orc_powmod(2, n - three_k, three_k); /* 2^(n-3^k) mod 3^k */
        uint64_t scale = m / three_k;                        /* 3^(e-k) */
        /* the sum of two residues can pass 2^64 once m > 2^63 (e = 40) */
        acc = (uint64_t)(((u128)acc + orc_mulmod(term, scale, m)) % m);
    }
    return acc;
}

uint64_t orc_digit_sum(uint64_t n)
{
    return orc_g_digit_sum(n, 33);
}

double orc_to_f64(uint64_t z)
{
    return (double)z * ORC_RECIP;
}

uint64_t orc_gen_u64(uint64_t z, uint64_t n, uint64_t *out)
{
    const uint64_t a = orc_multiplier();
    for (uint64_t k = 0; k < n; k++) {
        z = orc_mulmod(a, z, ORC_MOD);
        out[k] = z;
    }
    return z;
}

uint64_t orc_gen_f64(uint64_t z, uint64_t n, double *out)
{
    const uint64_t a = orc_multiplier();
    for (uint64_t k = 0; k < n; k++) {
        z = orc_mulmod(a, z, ORC_MOD);
        out[k] = orc_to_f64(z);
    }
    return z;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

uint64_t orc_gen_par(uint64_t z, uint64_t n, void *out, int kind, int nthreads)
{
    int nt = nthreads > 0 ? nthreads : orc_max_threads();
    if ((uint64_t)nt > n)
        nt = n > 0 ? (int)n : 1;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static, 1)
#endif
    for (int j = 0; j < nt; j++) {
        uint64_t lo = (uint64_t)(((u128)n * (u128)j) / (u128)nt);
        uint64_t hi = (uint64_t)(((u128)n * (u128)(j + 1)) / (u128)nt);
        uint64_t start = orc_skip(z, lo);
        if (kind == 0)
            orc_gen_u64(start, hi - lo, (uint64_t *)out + lo);
        else
            orc_gen_f64(start, hi - lo, (double *)out + lo);
    }
    return orc_skip(z, n);
}

/* ------------------------------------------------------ modulus 3^40 -- */

static const double ORC_E40_RECIP = 1.0 / 12157665459056928801.0; /* RN(1/3^40) */

int orc_e40_seed(uint64_t a, uint64_t *z0)
{
    if (a < ORC_E40_INDEX_MIN)
        return -1;
    *z0 = orc_g_index_state(a, 40);
    return 0;
}

uint64_t orc_e40_step(uint64_t z)
{
    return orc_mulmod(1ULL << 53, z, ORC_E40_MOD); /* 2^53 < 3^40 */
}

uint64_t orc_e40_skip(uint64_t z, uint64_t k)
{
    return orc_mulmod(z, orc_powmod(1ULL << 53, k, ORC_E40_MOD), ORC_E40_MOD);
}

double orc_e40_to_f64(uint64_t z)
{
    return (double)z * ORC_E40_RECIP;
}

uint64_t orc_e40_gen_u64(uint64_t z, uint64_t n, uint64_t *out)
{
    for (uint64_t k = 0; k < n; k++) {
        z = orc_e40_step(z);
        out[k] = z;
    }
    return z;
}

uint64_t orc_e40_gen_f64(uint64_t z, uint64_t n, double *out)
{
    for (uint64_t k = 0; k < n; k++) {
        z = orc_e40_step(z);
        out[k] = orc_e40_to_f64(z);
    }
    return z;
}

/* Modified Barrett (Section 3.1): with mu = floor(2^106 / m) and k = 53,
 * q3 = floor(mu * z / 2^53), r = 2^53 - (q3 * m mod 2^53), then at most one
 * subtraction of m.  Correct for 0 < z < m. */
uint64_t orc_modbarrett_step(uint64_t z)
{
    const uint64_t mu = (uint64_t)(((u128)1 << 106) / (u128)ORC_MOD);
    const uint64_t two53 = 1ULL << 53;
    uint64_t q3 = (uint64_t)(((u128)mu * (u128)z) >> 53);
    uint64_t r2 = (q3 * ORC_MOD) & (two53 - 1);
    uint64_t r = two53 - r2;
    if (r >= ORC_MOD)
        r -= ORC_MOD;
    return r;
}

uint64_t orc_gen_f64_modbarrett(uint64_t z, uint64_t n, double *out)
{
    for (uint64_t k = 0; k < n; k++) {
        z = orc_modbarrett_step(z);
        out[k] = orc_to_f64(z);
    }
    return z;
}
