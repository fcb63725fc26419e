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

// Flat layout start: the states of lane l's pair (outputs 2l and 2l + 1)
// of the chunk that begins u = b*R rows of kFlatPerBlock outputs after the
// output whose state is `base`: two multiplications by uniform table
// entries (scalar loads that hit L2), one by the lane's offset, one by M1.
// tabs is the device table allocation (t_lo at 0, t_flo and t_fhi at their
// offsets); b*R < kFlatMaxRowsPerLaunch.
template <class V>
__device__ __forceinline__ void flat_start(uint64_t b, uint32_t l, int R, uint64_t base,
                                           const Mult* __restrict__ tabs, const Mult& M1,
                                           typename V::S& za, typename V::S& zb) {
    const uint64_t u = b * (uint64_t)R;
    const Mult hi = tabs[kFlatHiOffset + u / kFlatLoSize];
    const Mult lo = tabs[kFlatLoOffset + u % kFlatLoSize];
    const Mult lane = tabs[2u * l];  // t_lo: (2^53)^(2l)
    za = V::mul(V::mul(V::mul(V::load(base), hi), lo), lane);
    zb = V::mul(za, M1);
}

// XCD runs (see kFlatXcdRun): the chunk (or record) that workgroup w takes
// when runs of kFlatXcds*kFlatXcdRun workgroups give XCD x = w mod kFlatXcds
// the kFlatXcdRun consecutive ones [x kFlatXcdRun, (x + 1) kFlatXcdRun) of
// its run.  A permutation of every whole run.
__device__ __forceinline__ uint64_t xcd_run_index(uint64_t w) {
    constexpr uint64_t run = (uint64_t)kFlatXcds * kFlatXcdRun;
    const uint64_t r = w % run;
    return w - r + (r % kFlatXcds) * kFlatXcdRun + r / kFlatXcds;
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
