// nn_host.hpp -- host-side modular arithmetic of the library: seeding by
// starting index (Eq. 2), skip-ahead (Section 2, last paragraph) and the
// per-launch multipliers the kernels consume.
#pragma once

#include <stdint.h>

#include <cmath>
#include <mutex>

#include "nn_arith.hpp"

namespace nn {

// Exact v*z mod m on the host (Barrett, the same exact routine as the
// device's integer path).
inline uint64_t h_mulmod(uint64_t a, uint64_t b) { return mm_barrett(a, b); }

inline bool valid_state(uint64_t s) { return s != 0 && s < kMod && s % 3 != 0; }

// base^e mod m by square-and-multiply.
inline uint64_t h_powmod(uint64_t base, uint64_t e) {
    uint64_t r = 1, b = base % kMod;
    while (e) {
        if (e & 1) r = h_mulmod(r, b);
        b = h_mulmod(b, b);
        e >>= 1;
    }
    return r;
}

// (2^53)^k mod m through byte tables: kMult^(j * 256^i) for i < 7, j < 256
// (256^7 = 2^56 exceeds the period, the largest exponent after reduction).
class MultPowers {
  public:
    static const MultPowers& get() {
        static MultPowers p;
        return p;
    }
    uint64_t pow(uint64_t k) const {
        k %= kPeriod;  // 2^53 has order exactly 2*3^32 modulo 3^33
        uint64_t r = 1;
        for (int i = 0; k != 0; ++i, k >>= 8) {
            const uint32_t j = (uint32_t)(k & 0xff);
            if (j) r = h_mulmod(r, tab_[i][j]);
        }
        return r;
    }

  private:
    MultPowers() {
        uint64_t step = kMult;  // kMult^(256^i)
        for (int i = 0; i < 7; ++i) {
            tab_[i][0] = 1;
            for (int j = 1; j < 256; ++j) tab_[i][j] = h_mulmod(tab_[i][j - 1], step);
            step = h_mulmod(tab_[i][255], step);
        }
    }
    uint64_t tab_[7][256];
};

inline uint64_t h_skip(uint64_t s, uint64_t k) { return h_mulmod(s, MultPowers::get().pow(k)); }

// Eq. 2: z0 = 2^(a - 3^33) * floor(3^33/2) mod 3^33.
inline uint64_t h_seed(uint64_t a) { return h_mulmod(h_powmod(2, a - kMod), kHalf); }

// The reduction data of a fixed multiplier v (a unit).
inline Mult make_mult(uint64_t v) {
    Mult f;
    f.v = (double)v;  // exact, v < 2^53
    f.vi = v;
    // F = floor(v * 2^128 / m) as two 64-bit quotient digits.
    const u128 n1 = (u128)v << 64;
    const uint64_t q1 = (uint64_t)(n1 / kMod);  // < 2^64 since v < m
    const uint64_t r1 = (uint64_t)(n1 % kMod);
    const uint64_t q2 = (uint64_t)(((u128)r1 << 64) / kMod);
    f.shoup = q1;
    f.mont = r1;  // v * 2^64 mod m
    // Normalise F and split its top 106 bits into qh + ql (v/m >= 2^-53,
    // so at least 75 significant bits are present).
    const u128 F = ((u128)q1 << 64) | q2;
    int lz = 0;
    if (q1 == 0)
        lz = 64 + __builtin_clzll(q2);
    else
        lz = __builtin_clzll(q1);
    const u128 G = F << lz;
    const uint64_t hi53 = (uint64_t)(G >> 75);
    const uint64_t lo53 = (uint64_t)(G >> 22) & ((1ULL << 53) - 1);
    f.qh = std::ldexp((double)hi53, -53 - lz);
    f.ql = std::ldexp((double)lo53, -106 - lz);
    return f;
}

}  // namespace nn
