// nn_device.hpp -- device helpers shared by the plain and batched kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"
#include "nn_kernels.hpp"

namespace nn {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// base * (2^53)^k for k < 2^25 through the two skip tables.
template <class V>
__device__ __forceinline__ typename V::S thread_start(uint64_t base, uint64_t k,
                                                      const Mult* __restrict__ t_lo,
                                                      const Mult* __restrict__ t_hi) {
    typename V::S z = V::load(base);
    z = V::mul(z, t_hi[k >> kLoBits]);
    z = V::mul(z, t_lo[k & (kLoSize - 1)]);
    return z;
}

// The 64-bit pattern stored for a state: the state itself or its variate.
template <class V, int KIND>
__device__ __forceinline__ uint64_t out_bits(typename V::S z) {
    if constexpr (KIND == 0)
        return V::to_u64(z);
    else
        return (uint64_t)__double_as_longlong(V::to_f64(z));
}

template <bool NT, class P, class X>
__device__ __forceinline__ void put(P* p, X x) {
    if constexpr (NT)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

}  // namespace nn
