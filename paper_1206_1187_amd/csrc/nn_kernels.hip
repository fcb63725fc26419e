// nn_kernels.hip -- gfx950 kernels of the alpha_{2,3} generator.
//
// Layout (serial order in memory, coalesced stores): with T = grid*block
// threads, thread t starts at element t by skip-ahead and then strides by
// T using the jump multiplier J = (2^53)^T, so a wavefront's 64 lanes always
// store 64 consecutive elements (512 contiguous bytes).  Eq. 3 applied T
// times is one multiplication by J (Section 2: any iterate is reachable
// directly), which keeps memory order equal to sequence order, unlike the
// paper's strided layout of Section 3.2.
#include <hip/hip_runtime.h>

#include "nn_kernels.hpp"

namespace nn {

template <class V>
__device__ __forceinline__ typename V::S thread_start(uint64_t base, uint64_t t,
                                                      const Mult* __restrict__ t_lo,
                                                      const Mult* __restrict__ t_hi) {
    typename V::S z = V::load(base);
    z = V::mul(z, t_hi[t >> kLoBits]);
    z = V::mul(z, t_lo[t & (kLoSize - 1)]);
    return z;
}

template <class V, int KIND>
__device__ __forceinline__ uint64_t out_bits(typename V::S z) {
    if constexpr (KIND == 0)
        return V::to_u64(z);
    else
        return (uint64_t)__double_as_longlong(V::to_f64(z));
}

template <bool NT>
__device__ __forceinline__ void put(uint64_t* p, uint64_t x) {
    if constexpr (NT)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

template <class V, int KIND, int UNROLL, bool NT>
__global__ __launch_bounds__(1024) void k_generate(uint64_t* __restrict__ out, uint64_t T,
                                                   uint64_t e_full, uint32_t rem, uint64_t base,
                                                   Mult J, const Mult* __restrict__ t_lo,
                                                   const Mult* __restrict__ t_hi) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool extra = t < rem;
    if (e_full == 0 && !extra) return;
    typename V::S z = thread_start<V>(base, t, t_lo, t_hi);
    uint64_t* row = out;  // uniform: row i starts at element i*T
#pragma unroll UNROLL
    for (uint64_t i = 0; i < e_full; ++i) {
        put<NT>(row + t, out_bits<V, KIND>(z));
        row += T;
        z = V::mul(z, J);
    }
    if (extra) put<NT>(row + t, out_bits<V, KIND>(z));
}

// The paper's "Constant" kernel (Section 4.2): the same stores, a fixed value.
template <int UNROLL, bool NT>
__global__ __launch_bounds__(1024) void k_fill(uint64_t* __restrict__ out, uint64_t T,
                                               uint64_t e_full, uint32_t rem, uint64_t value) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t* row = out;
#pragma unroll UNROLL
    for (uint64_t i = 0; i < e_full; ++i) {
        put<NT>(row + t, value);
        row += T;
    }
    if (t < rem) put<NT>(row + t, value);
}

template <class V, int KIND, int U, bool NT>
static hipError_t gen_one(uint32_t grid, uint32_t block, hipStream_t s, const GenArgs& a) {
    hipLaunchKernelGGL((k_generate<V, KIND, U, NT>), dim3(grid), dim3(block), 0, s, a.out, a.T,
                       a.e_full, a.rem, a.base, a.J, a.t_lo, a.t_hi);
    return hipGetLastError();
}

template <class V, int KIND, bool NT>
static hipError_t gen_u(int unroll, uint32_t grid, uint32_t block, hipStream_t s,
                        const GenArgs& a) {
    switch (unroll) {
        case 1: return gen_one<V, KIND, 1, NT>(grid, block, s, a);
        case 2: return gen_one<V, KIND, 2, NT>(grid, block, s, a);
        case 4: return gen_one<V, KIND, 4, NT>(grid, block, s, a);
        case 8: return gen_one<V, KIND, 8, NT>(grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <class V>
static hipError_t gen_v(int kind, int unroll, bool nt, uint32_t grid, uint32_t block,
                        hipStream_t s, const GenArgs& a) {
    if (kind == 0)
        return nt ? gen_u<V, 0, true>(unroll, grid, block, s, a)
                  : gen_u<V, 0, false>(unroll, grid, block, s, a);
    return nt ? gen_u<V, 1, true>(unroll, grid, block, s, a)
              : gen_u<V, 1, false>(unroll, grid, block, s, a);
}

hipError_t launch_generate(int mulmod, int kind, int unroll, bool nt, uint32_t grid,
                           uint32_t block, hipStream_t s, const GenArgs& a) {
    switch (mulmod) {
        case 1: return gen_v<VarFP64>(kind, unroll, nt, grid, block, s, a);
        case 2: return gen_v<VarBarrett>(kind, unroll, nt, grid, block, s, a);
        case 3: return gen_v<VarShoup>(kind, unroll, nt, grid, block, s, a);
        case 4: return gen_v<VarMontgomery>(kind, unroll, nt, grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <int U, bool NT>
static hipError_t fill_one(uint32_t grid, uint32_t block, hipStream_t s, uint64_t* out,
                           uint64_t T, uint64_t e_full, uint32_t rem, uint64_t value) {
    hipLaunchKernelGGL((k_fill<U, NT>), dim3(grid), dim3(block), 0, s, out, T, e_full, rem,
                       value);
    return hipGetLastError();
}

hipError_t launch_fill(int unroll, bool nt, uint32_t grid, uint32_t block, hipStream_t s,
                       uint64_t* out, uint64_t T, uint64_t e_full, uint32_t rem,
                       uint64_t value) {
#define NN_FILL_CASE(U)                                                          \
    case U:                                                                      \
        return nt ? fill_one<U, true>(grid, block, s, out, T, e_full, rem, value) \
                  : fill_one<U, false>(grid, block, s, out, T, e_full, rem, value);
    switch (unroll) {
        NN_FILL_CASE(1)
        NN_FILL_CASE(2)
        NN_FILL_CASE(4)
        NN_FILL_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef NN_FILL_CASE
}

}  // namespace nn
