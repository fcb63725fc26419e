// nn_strided.hip -- the paper's own output layout (Section 3.2), kept as an
// option for comparison: T = count / E threads, thread t makes the E
// consecutive elements t*E .. t*E + E-1 with the Modified Barrett step of
// Section 3.1 and stores its i-th one at out[t + i*T], so for each i the
// lanes of a wavefront store contiguously (coalesced) and the array holds the
// sequence transposed: out[t + i*T] = z_(t*E + i + 1).  Readers that know the
// layout read it back the same way, as the paper notes.
#include <hip/hip_runtime.h>

#include "nn_device.hpp"
#include "nn_skip.hpp"

namespace nn {

template <int KIND, bool NT>
__global__ __launch_bounds__(1024) void k_generate_strided(uint64_t* out, uint64_t T, uint32_t E,
                                                           uint64_t base, const Mult* t_sk) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    uint64_t z = skip_any<VarShoup>(base, t * E, t_sk);  // element t*E
    const global_ptr<uint64_t> o = as_global(out) + t;
#pragma unroll 8
    for (uint32_t i = 0; i < E; ++i) {
        const uint64_t bits = KIND == 0 ? z : (uint64_t)__double_as_longlong((double)z * kRecip);
        put<NT>(o + i * T, bits);
        z = mm_modbarrett_step(z);
    }
}

hipError_t launch_generate_strided(int kind, bool nt, uint32_t grid, uint32_t block,
                                   hipStream_t s, uint64_t* out, uint64_t T, uint32_t E,
                                   uint64_t base, const Mult* t_sk) {
    if (kind == 0) {
        if (nt)
            k_generate_strided<0, true><<<grid, block, 0, s>>>(out, T, E, base, t_sk);
        else
            k_generate_strided<0, false><<<grid, block, 0, s>>>(out, T, E, base, t_sk);
    } else {
        if (nt)
            k_generate_strided<1, true><<<grid, block, 0, s>>>(out, T, E, base, t_sk);
        else
            k_generate_strided<1, false><<<grid, block, 0, s>>>(out, T, E, base, t_sk);
    }
    return hipGetLastError();
}

}  // namespace nn
