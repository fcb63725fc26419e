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

// Address-space views.  Stores through a global pointer count only against
// the vector-memory counter; through a generic (flat) pointer they also
// count against the scalar one, so every wait for a scalar load would wait
// for them too.  Data read through a constant pointer must not change while
// the kernel runs (it is written before the launch); uniform loads through
// it go to the scalar unit, and the loop that consumes them never waits on
// its own outstanding stores.
template <class T>
using global_ptr = __attribute__((address_space(1))) T*;
template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ global_ptr<T> as_global(T* p) {
    return (global_ptr<T>)p;
}
template <class T>
__device__ __forceinline__ const_ptr<T> as_const(const T* p) {
    return (const_ptr<T>)p;
}

template <bool NT, class P, class X>
__device__ __forceinline__ void put(P* p, X x) {
    if constexpr (NT)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

}  // namespace nn
