// example.hip -- a consumer kernel written against the public device header
// (include/nn_device.h) the way a simulation would use it; built by
// build.py next to this file and called by tests/test_gpu_devapi.py.
//
// Mode 0: thread t of T takes elements t, t+T, t+2T, ... (one skip, then a
//         jump multiplier of (2^53)^T per step).
// Mode 1: thread t takes the consecutive elements t*E .. t*E+E-1 with
//         nn_dev_next and the multiplier 2^53.
// Either way element x (0-based) of the output is the (x+1)-th state after
// `state` as a variate, so the array equals nn_generate's.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_device.h"

__global__ void k_strided_consumer(double state, uint64_t count, uint64_t T,
                                   const nn_dev_mult* table, nn_dev_mult jump, double* out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double z = nn_dev_skip(state, t + 1, table);
    for (uint64_t x = t; x < count; x += T) {
        out[x] = nn_dev_variate(z);
        z = nn_dev_mulmod(z, jump);
    }
}

__global__ void k_consecutive_consumer(double state, uint64_t count, uint64_t E,
                                       const nn_dev_mult* table, nn_dev_mult one, double* out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t x0 = t * E;
    if (x0 >= count) return;
    double z = nn_dev_skip(state, x0, table);  // the state before element x0
    for (uint64_t x = x0; x < x0 + E && x < count; ++x) out[x] = nn_dev_next(&z, one);
}

extern "C" int example_generate(int mode, uint64_t state, uint64_t count, uint64_t threads_or_e,
                                const nn_dev_mult* table, nn_dev_mult mult, double* out,
                                void* stream) {
    if (!table || !out || !threads_or_e) return 1;
    const uint32_t block = 256;
    if (mode == 0) {
        const uint64_t T = threads_or_e;
        const uint32_t grid = (uint32_t)((T + block - 1) / block);
        k_strided_consumer<<<grid, block, 0, (hipStream_t)stream>>>((double)state, count, T,
                                                                     table, mult, out);
    } else {
        const uint64_t E = threads_or_e;
        const uint64_t T = (count + E - 1) / E;
        const uint32_t grid = (uint32_t)((T + block - 1) / block);
        k_consecutive_consumer<<<grid, block, 0, (hipStream_t)stream>>>((double)state, count, E,
                                                                         table, mult, out);
    }
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
