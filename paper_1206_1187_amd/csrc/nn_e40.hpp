// nn_e40.hpp -- the generator at the larger modulus 3^40 that Section 2
// names for a longer period (2*3^39): Eq. 3 with m = 3^40 and the same
// multiplier 2^53 (still 53 bits of alpha_{2,3} per step), Eq. 2 with 3^40
// in place of 3^33.  m > 2^63, so states need all 64 bits and the product
// of two of them 128: the FP64 reduction of the 3^33 path does not apply.
// The step uses Montgomery's reduction with R = 2^64 and multipliers kept in
// Montgomery form (v R mod m), so states stay in standard form.
#pragma once

#include <stdint.h>

#include "nn_arith.hpp"

namespace nn {
namespace e40 {

constexpr uint64_t kMod = 12157665459056928801ULL;  // 3^40
constexpr uint64_t kPeriod = 2ULL * (kMod / 3ULL);   // 2*3^39
constexpr uint64_t kMult = 1ULL << 53;               // 2^53 < 3^40
constexpr uint64_t kHalf = kMod / 2ULL;              // floor(3^40/2) (Eq. 2)
constexpr uint64_t kIndexMin = kMod + 100ULL;
constexpr double kRecip = 1.0 / 12157665459056928801.0;  // RN(1/3^40)

constexpr uint64_t neg_inv() {
    uint64_t x = kMod;
    for (int i = 0; i < 6; ++i) x *= 2ULL - kMod * x;
    return 0ULL - x;
}
constexpr uint64_t kNInv = neg_inv();  // -m^{-1} mod 2^64
static_assert(kMod * (0ULL - kNInv) == 1ULL, "Montgomery inverse");
static_assert(kMod > (1ULL << 63), "3^40 needs the full 64 bits");

// A fixed multiplier v and its Montgomery form v 2^64 mod m.
struct Mult40 {
    uint64_t v;
    uint64_t mont;
};

// REDC(z * vmont) = v z mod m for z < m.  With T = z vmont < m^2 and
// u = (T mod 2^64) (-1/m) mod 2^64, T + u m is a multiple of 2^64 and
// S = (T + u m) / 2^64 < 2m; 2m > 2^64, so S is formed in 128 bits: the
// low words of T and u m sum to 0 or 2^64, a carry of (T mod 2^64 != 0).
NN_HD uint64_t mm40(uint64_t z, uint64_t vmont) {
    const u128 t = (u128)z * vmont;
    const uint64_t tl = (uint64_t)t;
    const uint64_t u = tl * kNInv;
    const u128 um = (u128)u * kMod;
    const u128 s = (t >> 64) + (um >> 64) + (tl != 0);
    return (uint64_t)(s >= kMod ? s - kMod : s);
}

NN_HD double to_f64(uint64_t z) { return (double)z * kRecip; }

}  // namespace e40
}  // namespace nn
