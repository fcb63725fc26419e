// nn_kernels.hpp -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"

namespace nn {

// Skip-ahead tables on the device: t_lo[l] = 2^(53 l) for l < 1024 and
// t_hi[j] = 2^(53 * 1024 j) for j < 16384 (mod 3^33), so the multiplier of
// any offset t < 2^24 is t_hi[t >> 10] * t_lo[t & 1023].
constexpr uint32_t kLoBits = 10;
constexpr uint32_t kLoSize = 1u << kLoBits;
constexpr uint32_t kHiSize = 1u << 14;
constexpr uint64_t kMaxThreads = (uint64_t)kLoSize * kHiSize;  // 2^24

// Plain generation: thread t of T = grid*block emits elements t + i*T for
// i < e_full, plus element t + e_full*T when t < rem (count = e_full*T+rem).
// `base` is state * 2^53 (the first output of the call), J = (2^53)^T.
struct GenArgs {
    uint64_t* out;
    uint64_t T;
    uint64_t e_full;
    uint32_t rem;
    uint64_t base;
    Mult J;
    const Mult* t_lo;
    const Mult* t_hi;
};

hipError_t launch_generate(int mulmod, int kind, int unroll, bool nontemporal, uint32_t grid,
                           uint32_t block, hipStream_t stream, const GenArgs& a);

hipError_t launch_fill(int unroll, bool nontemporal, uint32_t grid, uint32_t block,
                       hipStream_t stream, uint64_t* out, uint64_t T, uint64_t e_full,
                       uint32_t rem, uint64_t value);

}  // namespace nn
