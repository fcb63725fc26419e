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

// The FP64 step: base-B limbs, B = 3^20 < 2^32, m = B^2.  For a state
// z = x1 B + x0 and a multiplier v = j1 B + j0 the term x1 j1 B^2 is a
// multiple of m, so
//     v z = (x1 j0 + x0 j1 + c) B + r   (mod m),   x0 j0 = c B + r,
// three products of integers below 2^33, each reduced modulo B exactly in
// FP64: the product as ph + pl (two-product, exact), a quotient rounded
// from ph/B (off by at most one from the nearest), the remainder formed by
// one FMA and one add, both exact because it is an integer below 2^34.
// States stay redundant (limbs() starts them so): x0 = r in about
// [-B/2, B/2] and x1 the unreduced sum, below 2.01 B in magnitude; the
// output takes z from them directly (top() below).  Multipliers are
// canonical: 0 <= j0, j1 < B.
constexpr uint64_t kLimb = 3486784401ULL;  // 3^20
constexpr double kB = 3486784401.0;
constexpr double kRB = 1.0 / 3486784401.0;      // RN(1/B)
constexpr double kHalfRB = 0.5 / 3486784401.0;  // RN(1/(2B)) = RN(1/B)/2
static_assert(kLimb * kLimb == kMod, "3^40 = (3^20)^2");

struct L2 {
    double lo;  // x0
    double hi;  // x1
};

struct Mult40L {
    double j0;  // v mod B
    double j1;  // v div B
};

// x j - q B for q the rounded quotient: x j mod B up to one B either way.
NN_HD double rem_b(double x, double j, double* q_out) {
    const double ph = x * j;
    const double pl = __builtin_fma(x, j, -ph);
    const double q = __builtin_rint(ph * kRB);
    *q_out = q;
    return __builtin_fma(-q, kB, ph) + pl;
}

NN_HD L2 mul40l(L2 z, Mult40L v) {
    double c, qa, qb;
    const double r = rem_b(z.lo, v.j0, &c);
    const double ta = rem_b(z.hi, v.j0, &qa);
    const double tb = rem_b(z.lo, v.j1, &qb);
    return L2{r, ta + tb + c};
}

// A state's limbs in the form the step keeps: z = x1 B + x0 with
// |x0| <= B/2 (x0 = z mod B, less B above B/2) and 0 <= x1 <= B.
NN_HD L2 limbs(uint64_t z) {
    const uint64_t q = z / kLimb, r = z % kLimb;
    return r > kLimb / 2 ? L2{(double)r - kB, (double)(q + 1)} : L2{(double)r, (double)q};
}

// The output needs z = x1 B + x0 mod m in [0, m), not canonical limbs:
// z = (x1 - f B) B + x0 for f = floor((x1 + x0/B) / B).  x0 is a nonzero
// integer in (-B, B) (a state is a unit, so x0 is not a multiple of B), so
// x1 + x0/B lies strictly between x1 and x1 + 1 for x0 > 0 and between
// x1 - 1 and x1 for x0 < 0, and neither open interval holds a multiple of
// B: f = floor((x1 + 1/2) / B) or floor((x1 - 1/2) / B), the half taking
// x0's sign.  That quotient is at least 1/(2B) away from an integer, far
// beyond the rounding of the one FMA that forms it, so its floor is exact.
// top() returns x1 - f B, in [0, B) for x0 > 0 and [1, B] for x0 < 0, and
// z = top B + x0 lies in (0, m).
NN_HD double top(L2 z) {
    const double f = __builtin_floor(__builtin_fma(z.hi, kRB, __builtin_copysign(kHalfRB, z.lo)));
    return __builtin_fma(-f, kB, z.hi);
}

// top < 2^32 and |x0| < 2^31: z formed modulo 2^64, where it is exact.
NN_HD uint64_t to_u64(L2 z) {
    return (uint64_t)(uint32_t)top(z) * kLimb + (uint64_t)(int64_t)(int32_t)z.lo;
}

// RN(z) is one FMA: top B + x0 formed exactly and rounded once.
NN_HD double to_f64(L2 z) { return __builtin_fma(top(z), kB, z.lo) * kRecip; }

inline Mult40L make_mult40l(uint64_t v) { return Mult40L{(double)(v % kLimb), (double)(v / kLimb)}; }

}  // namespace e40
}  // namespace nn
