// nn_arith.hpp -- exact arithmetic modulo 3^33 shared by the gfx950 kernels
// and their host build (the same source, compiled for both sides).
//
// The generator (Section 2, Eq. 3) multiplies a 53-bit state by a 53-bit
// multiplier modulo m = 3^33 ~ 2^52.3, a 106-bit product.  CDNA has no
// 64x64-bit integer multiplier, so the step loop offers four exact
// reductions (chosen by measurement):
//
//  * mm_fp64   -- FP64 FMA: the product as an exact double-double
//                 (two-product), a quotient estimate from a double-double
//                 v/m, and an exactly computed remainder;
//  * mm_barrett -- Barrett's reduction with k = 53, mu = floor(2^106/m)
//                 (Section 3.1, Algorithm Barrett), two final corrections;
//  * mm_shoup   -- Shoup's fixed-multiplier quotient floor(v 2^64 / m);
//  * mm_montgomery -- Montgomery reduction with R = 2^64, the multiplier
//                 pre-scaled by R so states stay in standard form.
//
// Every function takes a state z (a unit, 1 <= z < m) and a fixed
// multiplier described by `Mult` and returns v*z mod m in [1, m).
#pragma once

#include <stdint.h>

#include "nn_device.h"

#if defined(__HIPCC__)
#define NN_HD __host__ __device__ __forceinline__
#else
#define NN_HD inline
#endif

namespace nn {

typedef unsigned __int128 u128;

constexpr uint64_t kMod = 5559060566555523ULL;               // 3^33
constexpr uint64_t kPeriod = 2ULL * (kMod / 3ULL);            // 2*3^32
constexpr uint64_t kMult = (uint64_t)(((u128)1 << 53) % kMod); // 2^53 mod 3^33 (Eq. 3)
constexpr uint64_t kHalf = kMod / 2ULL;                       // floor(3^33/2) (Eq. 2)
constexpr double kModD = 5559060566555523.0;
constexpr double kRecip = 1.0 / 5559060566555523.0;           // RN(1/3^33)
constexpr uint64_t kBarrettMu = (uint64_t)(((u128)1 << 106) / kMod);

// -m^{-1} mod 2^64 by Newton iteration (m odd).
constexpr uint64_t mont_neg_inv() {
    uint64_t x = kMod;  // correct to 3 bits for odd m
    for (int i = 0; i < 6; ++i) x *= 2ULL - kMod * x;
    return 0ULL - x;
}
constexpr uint64_t kMontNInv = mont_neg_inv();
static_assert(kMod * (0ULL - kMontNInv) == 1ULL, "Montgomery inverse");
static_assert(kMod < (1ULL << 53) && (1ULL << 53) < 2 * kMod, "m is a 53-bit number");

// A fixed multiplier v (a unit mod m) with the data each reduction needs.
struct Mult {
    double v;        // v, exact as a double (v < 2^53)
    double qh, ql;   // v/m as an unevaluated double-double sum qh + ql
    uint64_t vi;     // v
    uint64_t shoup;  // floor(v * 2^64 / m)
    uint64_t mont;   // v * 2^64 mod m
};

// ---------------------------------------------------------------- FP64 --
// v z mod m, exact, for z, v in [1, m): the reduction of the public device
// header (nn_dev_mulmod, whose comment carries the bounds) with q m formed
// as a two-product sh + sl and r summed as (ph - sh) + (pl - sl): ph - sh is
// exact (Sterbenz, or an integer difference below 2^53), pl - sl an integer
// below 2^53, r an integer below m.  Three more instructions than
// nn_dev_mulmod's single fused q m; the kernels that store every output use
// this form because their stores, spaced by the longer instruction stream,
// write faster on MI355X (same GPU, same shapes: plain u64 6.8-6.9 against
// 5.8 TB/s, interleaved batch 6.1 against 5.8 TB/s).  The fused consumer,
// bound by its arithmetic, uses nn_dev_mulmod (VarFP64Fused).  Translation
// units are built with FP contraction off so no product is fused into a
// neighbouring add.
NN_HD double mm_fp64(double z, double v, double qh, double ql) {
    const double mod = (double)kMod;
    const double ph = v * z;
    const double pl = __builtin_fma(v, z, -ph);
    const double q = __builtin_rint(__builtin_fma(z, qh, z * ql));
    const double sh = q * mod;
    const double sl = __builtin_fma(q, mod, -sh);
    const double r = (ph - sh) + (pl - sl);
    return r < 0.0 ? r + mod : r;
}

// ------------------------------------------------------------- Barrett --
// Algorithm Barrett (Section 3.1) with k = 53: q1 = x >> 52,
// q3 = (q1 mu) >> 54 underestimates floor(x/m) by at most 2.
NN_HD uint64_t mm_barrett(uint64_t a, uint64_t b) {
    const u128 x = (u128)a * b;
    const uint64_t q1 = (uint64_t)(x >> 52);
    const uint64_t q3 = (uint64_t)(((u128)q1 * kBarrettMu) >> 54);
    uint64_t r = (uint64_t)x - q3 * kMod;  // < 3m, exact modulo 2^64
    if (r >= kMod) r -= kMod;
    if (r >= kMod) r -= kMod;
    return r;
}

// --------------------------------------------------------------- Shoup --
// q = floor(z * floor(v 2^64/m) / 2^64) is floor(v z/m) or one less.
NN_HD uint64_t mm_shoup(uint64_t z, uint64_t v, uint64_t vshoup) {
    const uint64_t q = (uint64_t)(((u128)z * vshoup) >> 64);
    const uint64_t r = v * z - q * kMod;  // in [0, 2m), exact modulo 2^64
    return r >= kMod ? r - kMod : r;
}

// ---------------------------------------------------------- Montgomery --
// REDC(z * vmont) = z * v * 2^64 * 2^-64 = v z (mod m).  T < m^2 and
// U m < 2^117, so T + U m fits 128 bits and the result is below 2m.
NN_HD uint64_t mm_montgomery(uint64_t z, uint64_t vmont) {
    const u128 t = (u128)z * vmont;
    const uint64_t u = (uint64_t)t * kMontNInv;
    const u128 s = t + (u128)u * kMod;
    const uint64_t r = (uint64_t)(s >> 64);
    return r >= kMod ? r - kMod : r;
}

// ---------------------------------------------------- Modified Barrett --
// Section 3.1's Modified Barrett reduction, which only computes the step of
// Eq. 3 itself, 2^53 z mod m: with x = 2^53 z, Barrett's first quotient
// digit floor(x / 2^53) is z and x mod 2^53 is 0, so the quotient estimate
// is q = floor(mu z / 2^53) (mu = floor(2^106/m) as above) and the
// remainder is 2^53 - (q m mod 2^53), brought below m by one subtraction.
// Exact for z < m: q is floor(x/m) or one less and the true remainder stays
// below 2^53 in both cases.
NN_HD uint64_t mm_modbarrett_step(uint64_t z) {
    const uint64_t q = (uint64_t)(((u128)kBarrettMu * z) >> 53);
    const uint64_t low53 = (q * kMod) & ((1ULL << 53) - 1);
    const uint64_t r = (1ULL << 53) - low53;
    return r >= kMod ? r - kMod : r;
}

// ----------------------------------------------------- variant policies --
// State type, conversion and one multiplication per reduction.
struct VarFP64 {
    typedef double S;
    static NN_HD S load(uint64_t x) { return (double)x; }
    static NN_HD S mul(S z, const Mult& f) { return mm_fp64(z, f.v, f.qh, f.ql); }
    static NN_HD uint64_t to_u64(S z) { return (uint64_t)z; }
    static NN_HD double to_f64(S z) { return z * kRecip; }
};
// The FP64 state with nn_dev_mulmod's shorter reduction (fused consumer).
struct VarFP64Fused {
    typedef double S;
    static NN_HD S load(uint64_t x) { return (double)x; }
    static NN_HD S mul(S z, const Mult& f) { return nn_dev_mulmod(z, nn_dev_mult{f.v, f.qh, f.ql}); }
    static NN_HD uint64_t to_u64(S z) { return (uint64_t)z; }
    static NN_HD double to_f64(S z) { return z * kRecip; }
};
struct VarBarrett {
    typedef uint64_t S;
    static NN_HD S load(uint64_t x) { return x; }
    static NN_HD S mul(S z, const Mult& f) { return mm_barrett(z, f.vi); }
    static NN_HD uint64_t to_u64(S z) { return z; }
    static NN_HD double to_f64(S z) { return (double)z * kRecip; }
};
struct VarShoup {
    typedef uint64_t S;
    static NN_HD S load(uint64_t x) { return x; }
    static NN_HD S mul(S z, const Mult& f) { return mm_shoup(z, f.vi, f.shoup); }
    static NN_HD uint64_t to_u64(S z) { return z; }
    static NN_HD double to_f64(S z) { return (double)z * kRecip; }
};
struct VarMontgomery {
    typedef uint64_t S;
    static NN_HD S load(uint64_t x) { return x; }
    static NN_HD S mul(S z, const Mult& f) { return mm_montgomery(z, f.mont); }
    static NN_HD uint64_t to_u64(S z) { return z; }
    static NN_HD double to_f64(S z) { return (double)z * kRecip; }
};

}  // namespace nn
