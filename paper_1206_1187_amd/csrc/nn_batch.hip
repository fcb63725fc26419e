// nn_batch.hip -- persistent kernel of the batched form.
//
// The batch is a sequence of rows of 2*block outputs (each window cut into
// ceil((len + s)/(2*block)) rows, s = 1 for windows at odd output offsets).
// Workgroup w processes the contiguous row range
// [n_rows*w/grid, n_rows*(w+1)/grid): inside a window it keeps stepping its
// lanes' states by (2^53)^(2*block) per row, exactly as the plain row
// kernel, and it skips ahead afresh only when it enters a new window.  Lane
// l owns the aligned output pair (x_a, x_b) of each row; pairs are aligned
// to the global output index, so the 16-byte stores stay aligned for any
// window offset (a window at an odd offset starts, and may end, with a half
// pair).  Element x of a window is src * (2^53)^(pos + x + 1).
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

// Stores row r's pair of lane l: x_b = 2(jr*B + l) + 1 - s, x_a = x_b - 1.
// `full` (uniform) says every pair of the row lies inside the window.
template <class V, int KIND, bool NT>
__device__ __forceinline__ void store_pair(uint64_t* out, const BatchDesc& D, uint64_t xb,
                                           typename V::S za, typename V::S zb, bool full) {
    uint64_t* const q = out + (D.out_off + xb - 1);  // global index of x_a, even
    if (full) {
        u64x2 v;
        v.x = out_bits<V, KIND>(za);
        v.y = out_bits<V, KIND>(zb);
        put<NT>(reinterpret_cast<u64x2*>(q), v);
        return;
    }
    const bool vb = xb < D.len;
    const bool va = xb >= 1 && xb - 1 < D.len;
    uint64_t* const p = out + (D.out_off + xb - 1);  // global index of x_a, even
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
}

// Workgroups form clusters of `cluster` consecutive workgroups; cluster c
// takes the contiguous row range [n_rows*c/C, n_rows*(c+1)/C) of the C =
// grid/cluster clusters, and member i of the cluster takes its rows
// r0 + i, r0 + i + cluster, ...  Two rows in flight: (za, zb) hold row r
// and (zc, zd) row r + cluster of the current window; all four advance by
// JB2 = (2^53)^(4*block*cluster) per step.
template <class V, int KIND, bool NT, bool INDEXED>
__global__ __launch_bounds__(1024) void k_batch(BatchArgs a) {
    const BatchHeader* hdr = a.ws;
    const uint32_t n_desc = hdr->n_desc;
    const uint64_t n_rows = hdr->n_rows;
    uint64_t* const out = hdr->out;
    const BatchDesc* __restrict__ desc = reinterpret_cast<const BatchDesc*>(hdr + 1);
    const uint32_t B = blockDim.x;
    const uint32_t l = threadIdx.x;
    const uint32_t K = a.cluster;
    const uint32_t n_clusters = gridDim.x / K;
    const uint32_t c = blockIdx.x / K;
    const uint32_t i = blockIdx.x % K;
    const uint64_t r1 = n_rows * (c + 1) / n_clusters;
    const uint64_t r_first = n_rows * c / n_clusters + i;
    if (r_first >= r1 || n_desc == 0) return;
    // The last window whose first row is at or before r_first (binary search).
    uint32_t lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (desc[mid].row_start <= r_first)
            lo = mid;
        else
            hi = mid - 1;
    }
    uint32_t d = lo;
    BatchDesc D = desc[d];
    uint64_t next_start = d + 1 < n_desc ? desc[d + 1].row_start : n_rows;
    bool fresh = true;
    typename V::S za = V::load(1), zb = V::load(1), zc = V::load(1), zd = V::load(1);
    for (uint64_t r = r_first; r < r1;) {
        if (r >= next_start) {  // enter a later window (empty ones have no rows)
            do {
                ++d;
                next_start = d + 1 < n_desc ? desc[d + 1].row_start : n_rows;
            } while (r >= next_start);
            D = desc[d];
            fresh = true;
        }
        const uint32_t s = (uint32_t)(D.out_off & 1u);
        const uint64_t xb = 2ull * ((r - D.row_start) * B + l) + 1 - s;
        if (fresh) {
            // src * (2^53)^(pos + x_b + 1): the window's element x_b.
            if constexpr (INDEXED)
                zb = skip_any<V>(hdr->states[D.src], D.pos + xb + 1, a.t_sk);
            else
                zb = skip_any<V>(D.src, D.pos + xb + 1, a.t_sk);
            za = V::mul(zb, a.Minv);
            zc = V::mul(za, a.JB);
            zd = V::mul(zb, a.JB);
            fresh = false;
        }
        const uint64_t seg_end = next_start < r1 ? next_start : r1;
        // Row jr covers window elements [2 jr B - s, 2 (jr + 1) B - s).
        const uint64_t jr = r - D.row_start;
        const bool full0 = (jr > 0 || s == 0) && 2ull * (jr + 1) * B - s <= D.len;
        const bool full1 = 2ull * (jr + K + 1) * B - s <= D.len;
        store_pair<V, KIND, NT>(out, D, xb, za, zb, full0);
        if (r + K < seg_end) {
            store_pair<V, KIND, NT>(out, D, xb + 2ull * B * K, zc, zd, full1);
            za = V::mul(za, a.JB2);
            zb = V::mul(zb, a.JB2);
            zc = V::mul(zc, a.JB2);
            zd = V::mul(zd, a.JB2);
            r += 2ull * K;
        } else {
            // The window or the range ends within the next K rows: one row.
            za = V::mul(za, a.JB);
            zb = V::mul(zb, a.JB);
            zc = V::mul(zc, a.JB);
            zd = V::mul(zd, a.JB);
            r += K;
        }
    }
}

// Pre-pass of the interleaved kernel: the window of every batch row.
__global__ __launch_bounds__(256) void k_batch_map(BatchArgs a) {
    const BatchHeader* hdr = a.ws;
    const uint32_t n_desc = hdr->n_desc;
    const uint64_t n_rows = hdr->n_rows;
    const BatchDesc* __restrict__ desc = reinterpret_cast<const BatchDesc*>(hdr + 1);
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n_desc - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (desc[mid].row_start <= r)
                lo = mid;
            else
                hi = mid - 1;
        }
        a.row_desc[r] = lo;
    }
}

// src * (2^53)^k, k < 2^56, through the LDS copy of the 8-bit skip tables.
__device__ __forceinline__ double skip8(uint64_t src, uint64_t k, const double* t8) {
    double z = (double)src;
#pragma unroll
    for (uint32_t lvl = 0; lvl < kSkip8Levels; ++lvl) {
        const double* e = t8 + 3 * (lvl * kSkip8Size + ((k >> (8 * lvl)) & 0xff));
        z = mm_fp64(z, e[0], e[1], e[2]);
    }
    return z;
}

// Interleaved batch kernel: workgroup w takes batch rows w, w + G, ...;
// while a lane's window continues its state moves G rows with JG,
// otherwise it skips ahead afresh through the LDS tables.
template <int KIND, bool NT, bool INDEXED>
__global__ __launch_bounds__(256) void k_batch_il(BatchArgs a) {
    __shared__ double t8[kSkip8Levels * kSkip8Size * 3];
    for (uint32_t i = threadIdx.x; i < kSkip8Levels * kSkip8Size * 3; i += blockDim.x)
        t8[i] = a.t8[i];
    __syncthreads();
    const BatchHeader* hdr = a.ws;
    const uint64_t n_rows = hdr->n_rows;
    uint64_t* const out = hdr->out;
    const BatchDesc* __restrict__ desc = reinterpret_cast<const BatchDesc*>(hdr + 1);
    const uint32_t B = blockDim.x;
    const uint32_t l = threadIdx.x;
    const uint64_t G = gridDim.x;
    uint32_t d_prev = 0xffffffffu;
    BatchDesc D;
    double za = 1.0, zb = 1.0;
    for (uint64_t r = blockIdx.x; r < n_rows; r += G) {
        const uint32_t d = a.row_desc[r];
        const bool same = d == d_prev;
        if (!same) D = desc[d];
        const uint32_t s = (uint32_t)(D.out_off & 1u);
        const uint64_t xb = 2ull * ((r - D.row_start) * B + l) + 1 - s;
        if (same) {
            za = mm_fp64(za, a.JG.v, a.JG.qh, a.JG.ql);
            zb = mm_fp64(zb, a.JG.v, a.JG.qh, a.JG.ql);
        } else {
            uint64_t src;
            if constexpr (INDEXED)
                src = hdr->states[D.src];
            else
                src = D.src;
            zb = skip8(src, D.pos + xb + 1, t8);
            za = mm_fp64(zb, a.Minv.v, a.Minv.qh, a.Minv.ql);
            d_prev = d;
        }
        const uint64_t jr = r - D.row_start;
        const bool full = (jr > 0 || s == 0) && 2ull * (jr + 1) * B - s <= D.len;
        store_pair<VarFP64, KIND, NT>(out, D, xb, za, zb, full);
    }
}

const void* batch_map_kernel() { return reinterpret_cast<const void*>(&k_batch_map); }

template <int KIND, bool NT>
static const void* il_kn(bool indexed) {
    return indexed ? reinterpret_cast<const void*>(&k_batch_il<KIND, NT, true>)
                   : reinterpret_cast<const void*>(&k_batch_il<KIND, NT, false>);
}

const void* batch_il_kernel(int kind, bool nt, bool indexed) {
    if (kind == 0) return nt ? il_kn<0, true>(indexed) : il_kn<0, false>(indexed);
    return nt ? il_kn<1, true>(indexed) : il_kn<1, false>(indexed);
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
