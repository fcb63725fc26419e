// nn_batch.hip -- persistent kernel of the batched form.
//
// Each stream is cut into tiles of rows*2*block outputs.  Workgroup w
// processes tiles w, w + grid, w + 2*grid, ... of the batch (so the tiles
// written at any moment are neighbours, as in the plain row layout).  Inside
// a tile, lane l owns the aligned output pair (x_a, x_b) of each row and
// steps both states by (2^53)^(2*block) per row.  Pairs are aligned to the
// global output index, so the 16-byte stores stay aligned for any stream
// offset: a stream at an odd offset starts and may end with a half pair.
// Element x of a window is src * (2^53)^(pos + x + 1).
#include <hip/hip_runtime.h>

#include "nn_batch.hpp"
#include "nn_device.hpp"

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

template <class V, int KIND, bool NT, bool INDEXED>
__global__ __launch_bounds__(1024) void k_batch(BatchArgs a) {
    const BatchHeader* hdr = a.ws;
    const uint32_t n_desc = hdr->n_desc;
    const uint32_t n_tiles = hdr->n_tiles;
    uint64_t* const out = hdr->out;
    const BatchDesc* __restrict__ desc = reinterpret_cast<const BatchDesc*>(hdr + 1);
    const uint64_t* __restrict__ tiles = reinterpret_cast<const uint64_t*>(desc + n_desc);
    const uint32_t B = blockDim.x;
    const uint32_t l = threadIdx.x;
    const uint64_t S = 2ull * B * a.rows;  // tile size in the padded index

    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint64_t w = tiles[t];
        const BatchDesc D = desc[w >> 32];
        const uint64_t j = (uint32_t)w;
        // Padded index p = x + s, s = 1 for streams at odd output offsets.
        const uint32_t s = (uint32_t)(D.out_off & 1u);
        const uint64_t P0 = j * S;
        const uint64_t Lp = D.len + s;
        const uint64_t P1 = P0 + S < Lp ? P0 + S : Lp;
        const uint32_t rows = (uint32_t)((P1 - P0 + 2ull * B - 1) / (2ull * B));
        // Row r, lane l: x_b = P0 + 2(rB + l) + 1 - s, x_a = x_b - 1.
        const uint64_t xb0 = P0 + 2ull * l + 1 - s;
        uint64_t* const pair0 = out + (D.out_off - s) + P0 + 2ull * l;  // global index of x_a, even
        typename V::S zb;
        if constexpr (INDEXED)
            zb = skip_any<V>(hdr->states[D.src], D.pos + xb0 + 1, a.t_sk);
        else
            zb = thread_start<V>(D.src, xb0 + 1, a.t_lo, a.t_hi);
        typename V::S za = V::mul(zb, a.Minv);
        for (uint32_t r = 0; r < rows; ++r) {
            const uint64_t xb = xb0 + 2ull * r * B;
            const bool vb = xb < D.len;
            const bool va = xb >= 1 && xb - 1 < D.len;
            uint64_t* const p = pair0 + 2ull * r * B;
            if (va && vb) {
                u64x2 v;
                v.x = out_bits<V, KIND>(za);
                v.y = out_bits<V, KIND>(zb);
                put<NT>(reinterpret_cast<u64x2*>(p), v);
            } else if (vb) {
                put<NT>(p + 1, out_bits<V, KIND>(zb));
            } else if (va) {
                put<NT>(p, out_bits<V, KIND>(za));
            }
            za = V::mul(za, a.JB);
            zb = V::mul(zb, a.JB);
        }
    }
}

template <class V, int KIND, bool NT>
static const void* kernel_kvn(bool indexed) {
    return indexed ? reinterpret_cast<const void*>(&k_batch<V, KIND, NT, true>)
                   : reinterpret_cast<const void*>(&k_batch<V, KIND, NT, false>);
}

template <class V, int KIND>
static const void* kernel_kv(bool nt, bool indexed) {
    return nt ? kernel_kvn<V, KIND, true>(indexed) : kernel_kvn<V, KIND, false>(indexed);
}

template <class V>
static const void* kernel_v(int kind, bool nt, bool indexed) {
    return kind == 0 ? kernel_kv<V, 0>(nt, indexed) : kernel_kv<V, 1>(nt, indexed);
}

const void* batch_kernel(int mulmod, int kind, bool nt, bool indexed) {
    switch (mulmod) {
        case 1: return kernel_v<VarFP64>(kind, nt, indexed);
        case 2: return kernel_v<VarBarrett>(kind, nt, indexed);
        case 3: return kernel_v<VarShoup>(kind, nt, indexed);
        case 4: return kernel_v<VarMontgomery>(kind, nt, indexed);
        default: return nullptr;
    }
}

hipError_t launch_batch(int mulmod, int kind, bool nt, bool indexed, uint32_t grid,
                        uint32_t block, hipStream_t s, const BatchArgs& a) {
    const void* k = batch_kernel(mulmod, kind, nt, indexed);
    if (!k) return hipErrorInvalidValue;
    BatchArgs copy = a;
    void* params[] = {&copy};
    return hipLaunchKernel(k, dim3(grid), dim3(block), params, 0, s);
}

}  // namespace nn
