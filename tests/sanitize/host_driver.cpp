// host_driver.cpp -- the library's host-side arithmetic (csrc/nn_host.hpp,
// csrc/nn_arith.hpp, csrc/nn_e40.hpp and the device header's
// nn_dev_mulmod, all of which also compile for the host) under
// AddressSanitizer and UndefinedBehaviorSanitizer, checked against the
// oracle on edge and random inputs.  Built by tests/test_oracle_sanitized.py
// with a host compiler only; test infrastructure.
#include <stdint.h>
#include <math.h>
#include <stdio.h>

#include "nn_e40.hpp"
#include "nn_host.hpp"

extern "C" {
#include "nn_oracle.h"
}

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            if (fails < 20) fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

static uint64_t rng = 0xD1B54A32D192ED03ULL;
static uint64_t next64() {  // xorshift64*
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return rng * 0x2545F4914F6CDD1DULL;
}

static uint64_t unit(uint64_t m) {  // a random unit modulo a power of 3
    for (;;) {
        const uint64_t z = 1 + next64() % (m - 1);
        if (z % 3) return z;
    }
}

static void check_mult(uint64_t v, uint64_t z) {
    const nn::Mult f = nn::make_mult(v);
    const uint64_t want = orc_mulmod(z, v, ORC_MOD);
    CHECK((uint64_t)nn::mm_fp64((double)z, f.v, f.qh, f.ql) == want);
    CHECK((uint64_t)nn_dev_mulmod((double)z, nn_dev_mult{f.v, f.qh, f.ql}) == want);
    CHECK(nn::mm_barrett(z, v) == want);
    CHECK(nn::mm_shoup(z, v, f.shoup) == want);
    CHECK(nn::mm_montgomery(z, f.mont) == want);
}

int main() {
    const uint64_t m = ORC_MOD;
    CHECK(nn::kMod == m && nn::e40::kMod == ORC_E40_MOD);
    // the four reductions at the ends of the unit range and at random
    const uint64_t edge[] = {1, 2, 4, m - 1, m - 2, m - 4, nn::kMult, nn::kHalf, nn::kHalf + 1};
    for (uint64_t v : edge)
        for (uint64_t z : edge) check_mult(v, z);
    for (int i = 0; i < 200000; ++i) check_mult(unit(m), unit(m));
    // the step multiplier and its powers, as the kernels take them
    for (int i = 0; i < 2000; ++i) {
        const uint64_t k = next64() >> (next64() % 64);
        check_mult(nn::MultPowers::get().pow(k), unit(m));
        const uint64_t s = unit(m);
        CHECK(nn::h_skip(s, k) == orc_skip(s, k));
        CHECK(nn::mm_modbarrett_step(s) == orc_step(s));
    }
    CHECK(nn::h_skip(1, 0) == 1);
    CHECK(nn::h_skip(1, nn::kPeriod) == 1);
    CHECK(nn::h_skip(7, UINT64_MAX) == orc_skip(7, UINT64_MAX));
    // seeding (Eq. 2) at the ends of the index range and at random
    uint64_t z = 0;
    const uint64_t idx[] = {ORC_INDEX_MIN, ORC_INDEX_MIN + 1, ORC_INDEX_MAX - 1, ORC_INDEX_MAX};
    for (uint64_t a : idx) CHECK(orc_seed(a, &z) == 0 && nn::h_seed(a) == z);
    for (int i = 0; i < 2000; ++i) {
        const uint64_t a = ORC_INDEX_MIN + next64() % (ORC_INDEX_MAX - ORC_INDEX_MIN);
        CHECK(orc_seed(a, &z) == 0 && nn::h_seed(a) == z && nn::valid_state(z));
    }
    CHECK(!nn::valid_state(0) && !nn::valid_state(m) && !nn::valid_state(3));
    // variates: RN(z RN(3^-33)) on both sides
    for (int i = 0; i < 10000; ++i) {
        const uint64_t s = unit(m);
        CHECK(nn::VarFP64::to_f64((double)s) == orc_to_f64(s));
        CHECK(nn::VarBarrett::to_f64(s) == orc_to_f64(s));
    }
    // 3^40: Montgomery step against the oracle's
    const uint64_t m40 = ORC_E40_MOD;
    const uint64_t mont = (uint64_t)(((nn::u128)nn::e40::kMult << 64) % m40);
    const uint64_t e40_edge[] = {1, 2, m40 - 1, m40 - 2, nn::e40::kHalf, 1ULL << 63};
    for (uint64_t s : e40_edge) CHECK(nn::e40::mm40(s, mont) == orc_e40_step(s));
    for (int i = 0; i < 200000; ++i) {
        const uint64_t s = unit(m40);
        CHECK(nn::e40::mm40(s, mont) == orc_e40_step(s));
        CHECK(nn::e40::to_f64(s) == orc_e40_to_f64(s));
    }
    // 3^40, the FP64 limb step: single products from canonical limbs, and
    // long chains through the redundant form (the bounds the step relies
    // on), against the oracle's exact products
    const uint64_t l_edge[] = {1,           2,           nn::e40::kLimb - 1, nn::e40::kLimb + 1,
                               m40 - 1,     m40 - 2,     nn::e40::kHalf,     nn::e40::kMult,
                               m40 - nn::e40::kLimb + 1, (nn::e40::kLimb - 1) * nn::e40::kLimb + 1};
    auto l_edge_of = [&](int i) { return l_edge[i]; };
    // a state converted straight from its limbs (a launch's first outputs),
    // and the limbs' bound, which the conversions rely on
    for (int c = 0; c < 20000; ++c) {
        const uint64_t s = c < 10 ? l_edge_of(c) : unit(m40);
        const nn::e40::L2 z = nn::e40::limbs(s);
        CHECK(fabs(z.lo) <= 0.5 * nn::e40::kB && z.hi >= 0.0 && z.hi <= nn::e40::kB);
        CHECK(nn::e40::to_u64(z) == s && nn::e40::to_f64(z) == orc_e40_to_f64(s));
    }
    for (uint64_t v : l_edge)
        for (uint64_t s : l_edge) {
            const nn::e40::L2 r = nn::e40::mul40l(nn::e40::limbs(s), nn::e40::make_mult40l(v));
            const uint64_t want = (uint64_t)(((nn::u128)s * v) % m40);
            CHECK(nn::e40::to_u64(r) == want);
            CHECK(nn::e40::to_f64(r) == orc_e40_to_f64(want));
        }
    for (int c = 0; c < 200; ++c) {
        const uint64_t v = c < 100 ? unit(m40) : (c < 150 ? m40 - 1 - (uint64_t)c : orc_e40_skip(1, next64()));
        const nn::e40::Mult40L mv = nn::e40::make_mult40l(v);
        uint64_t want = unit(m40);
        nn::e40::L2 s = nn::e40::limbs(want);
        for (int k = 0; k < 5000; ++k) {
            s = nn::e40::mul40l(s, mv);
            want = (uint64_t)(((nn::u128)want * v) % m40);
            CHECK(nn::e40::to_u64(s) == want);
            CHECK(nn::e40::to_f64(s) == orc_e40_to_f64(want));
            CHECK(fabs(s.hi) < 2.01 * nn::e40::kB && fabs(s.lo) <= 0.5001 * nn::e40::kB);
        }
    }
    // the generator's own multiplier, stepped, against the oracle's steps
    {
        uint64_t z = 0;
        CHECK(orc_e40_seed(ORC_E40_INDEX_MIN + 4242, &z) == 0);
        nn::e40::L2 s = nn::e40::limbs(z);
        const nn::e40::Mult40L m1 = nn::e40::make_mult40l(nn::e40::kMult);
        for (int k = 0; k < 100000; ++k) {
            s = nn::e40::mul40l(s, m1);
            z = orc_e40_step(z);
            CHECK(nn::e40::to_u64(s) == z && nn::e40::to_f64(s) == orc_e40_to_f64(z));
        }
    }
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("host driver ok\n");
    return 0;
}
