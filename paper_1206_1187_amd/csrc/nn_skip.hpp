// nn_skip.hpp -- device skip-ahead by any offset (Section 2: any iterate is
// reachable directly) through the four 13-bit-per-level tables t_sk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"
#include "nn_batch.hpp"

namespace nn {

// src * (2^53)^k for any k < 2^52 through the four 13-bit skip tables.
template <class V>
__device__ __forceinline__ typename V::S skip_any(uint64_t src, uint64_t k,
                                                  const Mult* __restrict__ t_sk) {
    typename V::S z = V::load(src);
#pragma unroll
    for (uint32_t lvl = 0; lvl < kSkipLevels; ++lvl)
        z = V::mul(z, t_sk[lvl * kSkipSize + ((k >> (kSkipBits * lvl)) & (kSkipSize - 1))]);
    return z;
}

}  // namespace nn
