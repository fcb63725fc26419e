// nn_kernels.hip -- gfx950 kernels of the alpha_{2,3} generator.
//
// Layout (serial order in memory, coalesced stores): with T = grid*block
// threads, each owning W consecutive elements per row, row i covers
// elements [i*W*T, (i+1)*W*T) and thread t writes elements
// i*W*T + W*t .. + W-1.  A thread starts at element W*t by skip-ahead and
// then moves one row per step with the jump multiplier J = (2^53)^(W*T):
// Eq. 3 applied W*T times is one multiplication by J (Section 2: any iterate
// is reachable directly).  A wavefront's 64 lanes therefore store 64*W
// consecutive elements (512 or 1024 contiguous bytes) per row, and memory
// order equals sequence order, unlike the paper's strided layout of
// Section 3.2.
#include <hip/hip_runtime.h>

#include "nn_device.hpp"

namespace nn {

// W = 1: one element per thread and row.
template <class V, int KIND, int UNROLL, bool NT>
__global__ __launch_bounds__(1024) void k_generate1(uint64_t* __restrict__ out, uint64_t T,
                                                    uint64_t e_full, uint32_t rem, uint64_t base,
                                                    Mult J, Mult M1,
                                                    const Mult* __restrict__ t_lo,
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

// W = 2: two consecutive elements per thread and row, one 16-byte store.
// Requires a 16-byte aligned output.
template <class V, int KIND, int UNROLL, bool NT>
__global__ __launch_bounds__(1024) void k_generate2(uint64_t* __restrict__ out, uint64_t T,
                                                    uint64_t e_full, uint32_t rem, uint64_t base,
                                                    Mult J, Mult M1,
                                                    const Mult* __restrict__ t_lo,
                                                    const Mult* __restrict__ t_hi) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t rem_pairs = rem >> 1;
    const bool extra_pair = t < rem_pairs;
    const bool extra_one = (rem & 1u) && t == rem_pairs;
    if (e_full == 0 && !extra_pair && !extra_one) return;
    typename V::S za = thread_start<V>(base, 2ull * t, t_lo, t_hi);
    typename V::S zb = V::mul(za, M1);
    u64x2* row = reinterpret_cast<u64x2*>(out);
#pragma unroll UNROLL
    for (uint64_t i = 0; i < e_full; ++i) {
        u64x2 v;
        v.x = out_bits<V, KIND>(za);
        v.y = out_bits<V, KIND>(zb);
        put<NT>(row + t, v);
        row += T;
        za = V::mul(za, J);
        zb = V::mul(zb, J);
    }
    if (extra_pair) {
        u64x2 v;
        v.x = out_bits<V, KIND>(za);
        v.y = out_bits<V, KIND>(zb);
        put<NT>(row + t, v);
    } else if (extra_one) {
        put<NT>(reinterpret_cast<uint64_t*>(row + t), out_bits<V, KIND>(za));
    }
}

// W = 2 with IL rows in flight per thread: 2*IL independent multiplication
// chains per lane, each advanced by JI = J^IL per trip.
template <class V, int KIND, int UNROLL, bool NT, int IL>
__global__ __launch_bounds__(1024) void k_generate2_ilp(uint64_t* __restrict__ out, uint64_t T,
                                                        uint64_t e_full, uint32_t rem,
                                                        uint64_t base, Mult J, Mult M1, Mult JI,
                                                        const Mult* __restrict__ t_lo,
                                                        const Mult* __restrict__ t_hi) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t rem_pairs = rem >> 1;
    const bool extra_pair = t < rem_pairs;
    const bool extra_one = (rem & 1u) && t == rem_pairs;
    if (e_full == 0 && !extra_pair && !extra_one) return;
    typename V::S za[IL], zb[IL];
    za[0] = thread_start<V>(base, 2ull * t, t_lo, t_hi);
    zb[0] = V::mul(za[0], M1);
#pragma unroll
    for (int r = 1; r < IL; ++r) {
        za[r] = V::mul(za[r - 1], J);
        zb[r] = V::mul(zb[r - 1], J);
    }
    u64x2* row = reinterpret_cast<u64x2*>(out);
    uint64_t i = 0;
#pragma unroll UNROLL
    for (; i + IL <= e_full; i += IL) {
#pragma unroll
        for (int r = 0; r < IL; ++r) {
            u64x2 v;
            v.x = out_bits<V, KIND>(za[r]);
            v.y = out_bits<V, KIND>(zb[r]);
            put<NT>(row + r * T + t, v);
            za[r] = V::mul(za[r], JI);
            zb[r] = V::mul(zb[r], JI);
            // Each row's store stays next to its own two multiplications:
            // left to itself the scheduler bunches the stores of a trip
            // together, which writes about 8 % slower on MI355X.
            __builtin_amdgcn_sched_barrier(0);
        }
        row += IL * T;
    }
    // Fewer than IL full rows remain, then the partial row; za[r], zb[r]
    // hold rows i + r.
    const uint32_t left = (uint32_t)(e_full - i);
    typename V::S pa = za[0], pb = zb[0];
#pragma unroll
    for (int r = 0; r < IL; ++r) {
        if ((uint32_t)r < left) {
            u64x2 v;
            v.x = out_bits<V, KIND>(za[r]);
            v.y = out_bits<V, KIND>(zb[r]);
            put<NT>(row + r * T + t, v);
        }
        if ((uint32_t)r == left) {
            pa = za[r];
            pb = zb[r];
        }
    }
    row += left * T;
    if (extra_pair) {
        u64x2 v;
        v.x = out_bits<V, KIND>(pa);
        v.y = out_bits<V, KIND>(pb);
        put<NT>(row + t, v);
    } else if (extra_one) {
        put<NT>(reinterpret_cast<uint64_t*>(row + t), out_bits<V, KIND>(pa));
    }
}

// Fused consumer (the paper's point that variates usually feed a simulation
// directly, Section 3.2; its Table 2 removes the memory traffic): the same
// generation as k_generate2_ilp with IL = 2, the outputs summed in
// registers.  Kind 0 sums raw states modulo 2^64 (exact in any order).
template <class V, int KIND>
__global__ __launch_bounds__(1024) void k_consume(uint64_t T, uint64_t e_full, uint32_t rem,
                                                  uint64_t base, Mult J, Mult M1, Mult JI,
                                                  const Mult* __restrict__ t_lo,
                                                  const Mult* __restrict__ t_hi, void* result) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    typename V::S za0 = thread_start<V>(base, 2ull * t, t_lo, t_hi);
    typename V::S zb0 = V::mul(za0, M1);
    typename V::S za1 = V::mul(za0, J);
    typename V::S zb1 = V::mul(zb0, J);
    uint64_t su = 0;
    double sf = 0.0;
    auto take = [&](typename V::S z) {
        if constexpr (KIND == 0)
            su += V::to_u64(z);
        else
            sf += V::to_f64(z);
    };
    uint64_t i = 0;
    for (; i + 2 <= e_full; i += 2) {
        take(za0);
        take(zb0);
        take(za1);
        take(zb1);
        za0 = V::mul(za0, JI);
        zb0 = V::mul(zb0, JI);
        za1 = V::mul(za1, JI);
        zb1 = V::mul(zb1, JI);
    }
    typename V::S pa = za0, pb = zb0;
    if (i < e_full) {  // one full row left
        take(za0);
        take(zb0);
        pa = za1;
        pb = zb1;
    }
    const uint32_t rem_pairs = rem >> 1;
    if (t < rem_pairs) {
        take(pa);
        take(pb);
    } else if ((rem & 1u) && t == rem_pairs) {
        take(pa);
    }
    // Reduce across the wavefront, then one atomic per wavefront.
    for (int off = 32; off > 0; off >>= 1) {
        if constexpr (KIND == 0)
            su += (uint64_t)__shfl_xor((unsigned long long)su, off, 64);
        else
            sf += __shfl_xor(sf, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if constexpr (KIND == 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(result), (unsigned long long)su);
        else
            atomicAdd(reinterpret_cast<double*>(result), sf);
    }
}

template <class V>
static hipError_t consume_v(int kind, uint32_t grid, uint32_t block, hipStream_t s,
                            const GenArgs& a, void* result) {
    if (kind == 0)
        hipLaunchKernelGGL((k_consume<V, 0>), dim3(grid), dim3(block), 0, s, a.T, a.e_full,
                           a.rem, a.base, a.J, a.M1, a.JI, a.t_lo, a.t_hi, result);
    else
        hipLaunchKernelGGL((k_consume<V, 1>), dim3(grid), dim3(block), 0, s, a.T, a.e_full,
                           a.rem, a.base, a.J, a.M1, a.JI, a.t_lo, a.t_hi, result);
    return hipGetLastError();
}

hipError_t launch_consume(int mulmod, int kind, uint32_t grid, uint32_t block, hipStream_t s,
                          const GenArgs& a, void* result) {
    switch (mulmod) {
        case 1: return consume_v<VarFP64Fused>(kind, grid, block, s, a, result);
        case 2: return consume_v<VarBarrett>(kind, grid, block, s, a, result);
        case 3: return consume_v<VarShoup>(kind, grid, block, s, a, result);
        case 4: return consume_v<VarMontgomery>(kind, grid, block, s, a, result);
        default: return hipErrorInvalidValue;
    }
}

// The paper's "Constant" kernel (Section 4.2): the same stores, a fixed value.
template <int W, int UNROLL, bool NT>
__global__ __launch_bounds__(1024) void k_fill(uint64_t* __restrict__ out, uint64_t T,
                                               uint64_t e_full, uint32_t rem, uint64_t value) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (W == 1) {
        uint64_t* row = out;
#pragma unroll UNROLL
        for (uint64_t i = 0; i < e_full; ++i) {
            put<NT>(row + t, value);
            row += T;
        }
        if (t < rem) put<NT>(row + t, value);
    } else {
        u64x2 v;
        v.x = value;
        v.y = value;
        u64x2* row = reinterpret_cast<u64x2*>(out);
#pragma unroll UNROLL
        for (uint64_t i = 0; i < e_full; ++i) {
            put<NT>(row + t, v);
            row += T;
        }
        if (t < (rem >> 1))
            put<NT>(row + t, v);
        else if ((rem & 1u) && t == (rem >> 1))
            put<NT>(reinterpret_cast<uint64_t*>(row + t), value);
    }
}

// The flat kernels' multipliers in a static device array of this module:
// the lane offsets (2^53)^(2l) for l < kFlatBlock, then t_flo and t_fhi.
// Its address is a link-time constant of the code, so a workgroup issues
// its table loads at once instead of after the load of a table pointer
// from its arguments.  Filled per device at set-up (upload_flat_symbol).
__device__ Mult flat_sym[kFlatSymEntries];

// flat_start over flat_sym: the states of lane l's pair (outputs 2l and
// 2l + 1) of the chunk that begins u = b*R rows after the output whose state
// is `base`.  b*R < kFlatMaxRowsPerLaunch.
template <class V>
__device__ __forceinline__ void flat_start_sym(uint64_t b, uint32_t l, int R, uint64_t base,
                                               const Mult& M1, typename V::S& za,
                                               typename V::S& zb) {
    const uint64_t u = b * (uint64_t)R;
    const Mult hi = flat_sym[kFlatSymHi + u / kFlatLoSize];
    const Mult lo = flat_sym[kFlatSymLo + u % kFlatLoSize];
    const Mult lane = flat_sym[kFlatSymLane + l];
    za = V::mul(V::mul(V::mul(V::load(base), hi), lo), lane);
    zb = V::mul(za, M1);
}

hipError_t upload_flat_symbol(const Mult* entries) {
    return hipMemcpyToSymbol(HIP_SYMBOL(flat_sym), entries, sizeof(Mult) * kFlatSymEntries, 0,
                             hipMemcpyHostToDevice);
}

// The chunk that workgroup w writes: w itself (G = 0), or its XCD-run
// chunk (G = kFlatXcdRun, in launches of whole runs).
template <int G>
__device__ __forceinline__ uint64_t flat_chunk(uint64_t w) {
    static_assert(G == 0 || G == (int)kFlatXcdRun, "XCD runs of kFlatXcdRun chunks");
    if constexpr (G == 0)
        return w;
    else
        return xcd_run_index(w);
}

// Flat layout (see launch_generate_flat).  Workgroup w writes the R rows of
// kFlatPerBlock outputs of chunk b = flat_chunk<G>(w), from element
// kFlatPerBlock*R*b on, lane l the pair 2l of each row, and exits.  Its start is two multiplications by uniform
// table entries (scalar loads that hit L2), then one by the lane's offset;
// after that one multiplication per output.  Each row: its store, then the
// two multiplications to the next.
//
// A workgroup lives a few microseconds, so its start must not wait on more
// round trips of scalar-load latency than needed: the tables sit at a fixed
// address (flat_sym), so their loads go out with the load of the base, the
// whole-chunk kernel takes no count and tests nothing, and the table
// indices are in range for every lane.  A ragged last chunk goes to
// k_generate_flat_tail.
template <class V, int KIND, bool NT, int R, int G>
__global__ __launch_bounds__(kFlatBlock) void k_generate_flat(uint64_t base,
                                                              uint64_t* __restrict__ out,
                                                              Mult M1, Mult J) {
    extern __shared__ char occupancy_cap[];  // dynamic LDS only limits residency
    (void)occupancy_cap;
    const uint64_t b = flat_chunk<G>(blockIdx.x);
    const uint32_t l = threadIdx.x;
    typename V::S za, zb;
    flat_start_sym<V>(b, l, R, base, M1, za, zb);
    u64x2* p = reinterpret_cast<u64x2*>(out + (uint64_t)kFlatPerBlock * R * b + 2u * l);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        u64x2 v;
        v.x = out_bits<V, KIND>(za);
        v.y = out_bits<V, KIND>(zb);
        put<NT>(p + r * kFlatBlock, v);
        if (r + 1 < R) {
            za = V::mul(za, J);
            zb = V::mul(zb, J);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The last, partial chunk: `count` < kFlatPerBlock*R outputs from `out`,
// one workgroup (b = 0 relative to `base`).
template <class V, int KIND, bool NT, int R>
__global__ __launch_bounds__(kFlatBlock) void k_generate_flat_tail(uint64_t base,
                                                                   uint64_t* __restrict__ out,
                                                                   Mult M1, Mult J,
                                                                   uint64_t count) {
    const uint32_t l = threadIdx.x;
    typename V::S za, zb;
    flat_start_sym<V>(0, l, R, base, M1, za, zb);
    uint64_t k = 2u * l;
    for (int r = 0; r < R && k < count; ++r, k += kFlatPerBlock) {
        if (k + 1 < count) {
            u64x2 v;
            v.x = out_bits<V, KIND>(za);
            v.y = out_bits<V, KIND>(zb);
            put<NT>(reinterpret_cast<u64x2*>(out + k), v);
        } else {
            put<NT>(out + k, out_bits<V, KIND>(za));
        }
        za = V::mul(za, J);
        zb = V::mul(zb, J);
    }
}

// The paper's "Constant" kernel (Section 4.2) for the flat layout: exactly
// k_generate_flat's stores with the arithmetic taken out -- whole chunks of
// R rows of kFlatPerBlock outputs, no count test, each row's store followed
// by the same scheduling barrier, and a ragged last chunk in a separate
// one-workgroup kernel (k_fill_flat_tail).
//
// START: also the generator's start -- its three table loads (the chunk's
// two row multipliers and the lane's offset) -- with only a comparison in
// place of its multiplications, so the stores wait for the same loads:
// the generator minus its arithmetic.  (The entries are positive, so the
// comparison always keeps `value`.)
template <bool NT, int R, bool START, int G>
__global__ __launch_bounds__(kFlatBlock) void k_fill_flat(uint64_t* __restrict__ out,
                                                          uint64_t value) {
    extern __shared__ char occupancy_cap[];
    (void)occupancy_cap;
    const uint64_t b = flat_chunk<G>(blockIdx.x);
    u64x2 v;
    v.x = value;
    if constexpr (START) {
        const uint64_t u = b * R;
        const double hi = flat_sym[kFlatSymHi + u / kFlatLoSize].v;
        const double lo = flat_sym[kFlatSymLo + u % kFlatLoSize].v;
        const double lane = flat_sym[kFlatSymLane + threadIdx.x].v;
        v.x = hi + lo + lane > 0.0 ? value : 0;
    }
    v.y = v.x;
    u64x2* p = reinterpret_cast<u64x2*>(out + (uint64_t)kFlatPerBlock * R * b + 2u * threadIdx.x);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        put<NT>(p + r * kFlatBlock, v);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The last, partial chunk of a fill: `count` < kFlatPerBlock*R outputs.
template <bool NT, int R>
__global__ __launch_bounds__(kFlatBlock) void k_fill_flat_tail(uint64_t* __restrict__ out,
                                                               uint64_t count, uint64_t value) {
    u64x2 v;
    v.x = value;
    v.y = value;
    uint64_t k = 2u * threadIdx.x;
    for (int r = 0; r < R && k < count; ++r, k += kFlatPerBlock) {
        if (k + 1 < count)
            put<NT>(reinterpret_cast<u64x2*>(out + k), v);
        else
            put<NT>(out + k, value);
    }
}

template <class V, int KIND, bool NT, int R>
static hipError_t flat_one(uint32_t lds, hipStream_t s, const FlatArgs& a) {
    const uint64_t per = (uint64_t)kFlatPerBlock * R;
    const uint64_t full = a.count / per;  // whole chunks
    const uint64_t tail = a.count - full * per;
    const uint64_t runs = flat_run_chunks(R, a.xcd_runs, full);  // whole chunks in XCD runs
    if constexpr (R == 4) {
        if (runs) {
            hipLaunchKernelGGL((k_generate_flat<V, KIND, NT, R, kFlatXcdRun>),
                               dim3((uint32_t)runs), dim3(kFlatBlock), lds, s, a.base, a.out,
                               a.M1, a.J);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    if (full > runs) {
        // the whole chunks after the last run, in workgroup order from their own base
        hipLaunchKernelGGL((k_generate_flat<V, KIND, NT, R, 0>), dim3((uint32_t)(full - runs)),
                           dim3(kFlatBlock), lds, s, runs ? a.mid_base : a.base,
                           a.out + runs * per, a.M1, a.J);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tail) {
        // the tail chunk starts full*R rows in: its own base, one workgroup
        hipLaunchKernelGGL((k_generate_flat_tail<V, KIND, NT, R>), dim3(1), dim3(kFlatBlock), 0,
                           s, a.tail_base, a.out + full * per, a.M1, a.J, tail);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <class V, int KIND, bool NT>
static hipError_t flat_r(int rows, uint32_t lds, hipStream_t s, const FlatArgs& a) {
    switch (rows) {
        case 1: return flat_one<V, KIND, NT, 1>(lds, s, a);
        case 2: return flat_one<V, KIND, NT, 2>(lds, s, a);
        case 4: return flat_one<V, KIND, NT, 4>(lds, s, a);
        case 8: return flat_one<V, KIND, NT, 8>(lds, s, a);
        case 16: return flat_one<V, KIND, NT, 16>(lds, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <class V>
static hipError_t flat_v(int kind, bool nt, int rows, uint32_t lds, hipStream_t s,
                         const FlatArgs& a) {
    if (kind == 0)
        return nt ? flat_r<V, 0, true>(rows, lds, s, a) : flat_r<V, 0, false>(rows, lds, s, a);
    return nt ? flat_r<V, 1, true>(rows, lds, s, a) : flat_r<V, 1, false>(rows, lds, s, a);
}

hipError_t launch_generate_flat(int mulmod, int kind, bool nt, int rows, uint32_t lds,
                                hipStream_t s, const FlatArgs& a) {
    switch (mulmod) {
        case 1: return flat_v<VarFP64>(kind, nt, rows, lds, s, a);
        case 2: return flat_v<VarBarrett>(kind, nt, rows, lds, s, a);
        case 3: return flat_v<VarShoup>(kind, nt, rows, lds, s, a);
        case 4: return flat_v<VarMontgomery>(kind, nt, rows, lds, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <bool NT, int R, int G>
static hipError_t fill_flat_launch(uint32_t grid, uint32_t lds, hipStream_t s, bool start,
                                   uint64_t* out, uint64_t value) {
    if (start)
        hipLaunchKernelGGL((k_fill_flat<NT, R, true, G>), dim3(grid), dim3(kFlatBlock), lds, s,
                           out, value);
    else
        hipLaunchKernelGGL((k_fill_flat<NT, R, false, G>), dim3(grid), dim3(kFlatBlock), lds, s,
                           out, value);
    return hipGetLastError();
}

// Whole chunks in the generator's order (XCD runs, then workgroup order),
// then the tail.
template <bool NT, int R>
static hipError_t fill_flat_one(uint32_t lds, hipStream_t s, bool start, bool xcd_runs,
                                uint64_t* out, uint64_t count, uint64_t value) {
    const uint64_t per = (uint64_t)kFlatPerBlock * R;
    const uint64_t full = count / per;
    const uint64_t tail = count - full * per;
    const uint64_t runs = flat_run_chunks(R, xcd_runs, full);
    if constexpr (R == 4) {
        if (runs) {
            const hipError_t e =
                fill_flat_launch<NT, R, kFlatXcdRun>((uint32_t)runs, lds, s, start, out, value);
            if (e != hipSuccess) return e;
        }
    }
    if (full > runs) {
        // START: the table indices restart at the first chunk after the runs
        const hipError_t e = fill_flat_launch<NT, R, 0>((uint32_t)(full - runs), lds, s, start,
                                                        out + runs * per, value);
        if (e != hipSuccess) return e;
    }
    if (tail) {
        hipLaunchKernelGGL((k_fill_flat_tail<NT, R>), dim3(1), dim3(kFlatBlock), 0, s,
                           out + full * per, tail, value);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <bool NT>
static hipError_t fill_flat_r(int rows, uint32_t lds, hipStream_t s, bool start, bool xcd_runs,
                              uint64_t* out, uint64_t count, uint64_t value) {
    switch (rows) {
        case 1: return fill_flat_one<NT, 1>(lds, s, start, xcd_runs, out, count, value);
        case 2: return fill_flat_one<NT, 2>(lds, s, start, xcd_runs, out, count, value);
        case 4: return fill_flat_one<NT, 4>(lds, s, start, xcd_runs, out, count, value);
        case 8: return fill_flat_one<NT, 8>(lds, s, start, xcd_runs, out, count, value);
        case 16: return fill_flat_one<NT, 16>(lds, s, start, xcd_runs, out, count, value);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill_flat(bool nt, int rows, uint32_t lds, hipStream_t s, bool start,
                            bool xcd_runs, uint64_t* out, uint64_t count, uint64_t value) {
    return nt ? fill_flat_r<true>(rows, lds, s, start, xcd_runs, out, count, value)
              : fill_flat_r<false>(rows, lds, s, start, xcd_runs, out, count, value);
}

// Kernel selector: W = 1, W = 2, or W = 2 with IL = 2 or 4 rows in flight.
// ------------------------------------------------------- consecutive --
// The paper's per-thread loop (Section 3.2) with its Modified Barrett step
// (Section 3.1), kept in serial memory order by an LDS transpose.  Element
// j = t*E + e of a tile sits at LDS word j + j/E (one pad word per thread,
// so the E-strided writes of a wavefront spread over the banks).
template <int KIND, int E, int W, bool NT>
__global__ __launch_bounds__(1024) void k_generate_consec(ConsecArgs a) {
    extern __shared__ uint64_t tile[];
    const uint32_t B = blockDim.x;
    const uint32_t t = threadIdx.x;
    const uint64_t per_tile = (uint64_t)B * E;
    const uint64_t n_tiles = (a.count + per_tile - 1) / per_tile;
    uint64_t ti = blockIdx.x;
    if (ti >= n_tiles) return;
    // The state of this thread's first element in tile ti.
    uint64_t z0 = thread_start<VarShoup>(a.base, ti * per_tile + (uint64_t)t * E, a.t_lo, a.t_hi);
    const global_ptr<uint64_t> out = as_global(a.out);
    for (; ti < n_tiles; ti += gridDim.x) {
        uint64_t z = z0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint64_t bits = KIND == 0 ? z : (uint64_t)__double_as_longlong((double)z * kRecip);
            tile[t * (E + 1) + e] = bits;
            z = mm_modbarrett_step(z);
        }
        z0 = VarShoup::mul(z0, a.J);
        __syncthreads();
        const uint64_t first = ti * per_tile;
        const uint64_t here = a.count - first < per_tile ? a.count - first : per_tile;
        if (W == 2 && here == per_tile) {
#pragma unroll
            for (int i = 0; i < E / 2; ++i) {
                const uint32_t j = 2 * (i * B + t);  // even, so j and j+1 share a thread
                const uint32_t w = j + j / E;
                u64x2 v;
                v.x = tile[w];
                v.y = tile[w + 1];
                put<NT>(reinterpret_cast<global_ptr<u64x2>>(out + first + j), v);
            }
        } else {
            for (uint32_t j = t; j < here; j += B) put<NT>(out + first + j, tile[j + j / E]);
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

template <int KIND, int E, int W>
static hipError_t consec_one(bool nt, uint32_t grid, uint32_t block, hipStream_t s,
                             const ConsecArgs& a) {
    const uint32_t lds = consec_lds_bytes(block, E);
    if (nt) {
        k_generate_consec<KIND, E, W, true><<<grid, block, lds, s>>>(a);
    } else {
        k_generate_consec<KIND, E, W, false><<<grid, block, lds, s>>>(a);
    }
    return hipGetLastError();
}

template <int KIND, int W>
static hipError_t consec_e(int E, bool nt, uint32_t grid, uint32_t block, hipStream_t s,
                           const ConsecArgs& a) {
    switch (E) {
        case 2: return consec_one<KIND, 2, W>(nt, grid, block, s, a);
        case 4: return consec_one<KIND, 4, W>(nt, grid, block, s, a);
        case 8: return consec_one<KIND, 8, W>(nt, grid, block, s, a);
        case 16: return consec_one<KIND, 16, W>(nt, grid, block, s, a);
        case 32: return consec_one<KIND, 32, W>(nt, grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_generate_consec(int kind, int E, int width, bool nt, uint32_t grid,
                                  uint32_t block, hipStream_t s, const ConsecArgs& a) {
    if (kind == 0)
        return width == 2 ? consec_e<0, 2>(E, nt, grid, block, s, a)
                          : consec_e<0, 1>(E, nt, grid, block, s, a);
    return width == 2 ? consec_e<1, 2>(E, nt, grid, block, s, a)
                      : consec_e<1, 1>(E, nt, grid, block, s, a);
}

template <class V, int KIND, int W, int IL, int U, bool NT>
static hipError_t gen_one(uint32_t grid, uint32_t block, hipStream_t s, const GenArgs& a) {
    if constexpr (W == 1)
        hipLaunchKernelGGL((k_generate1<V, KIND, U, NT>), dim3(grid), dim3(block), 0, s, a.out,
                           a.T, a.e_full, a.rem, a.base, a.J, a.M1, a.t_lo, a.t_hi);
    else if constexpr (IL == 1)
        hipLaunchKernelGGL((k_generate2<V, KIND, U, NT>), dim3(grid), dim3(block), 0, s, a.out,
                           a.T, a.e_full, a.rem, a.base, a.J, a.M1, a.t_lo, a.t_hi);
    else
        hipLaunchKernelGGL((k_generate2_ilp<V, KIND, U, NT, IL>), dim3(grid), dim3(block), 0, s,
                           a.out, a.T, a.e_full, a.rem, a.base, a.J, a.M1, a.JI, a.t_lo,
                           a.t_hi);
    return hipGetLastError();
}

template <class V, int KIND, int W, int IL, bool NT>
static hipError_t gen_u(int unroll, uint32_t grid, uint32_t block, hipStream_t s,
                        const GenArgs& a) {
    switch (unroll) {
        case 1: return gen_one<V, KIND, W, IL, 1, NT>(grid, block, s, a);
        case 2: return gen_one<V, KIND, W, IL, 2, NT>(grid, block, s, a);
        case 4: return gen_one<V, KIND, W, IL, 4, NT>(grid, block, s, a);
        case 8: return gen_one<V, KIND, W, IL, 8, NT>(grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <class V, int KIND, int W, int IL>
static hipError_t gen_n(int unroll, bool nt, uint32_t grid, uint32_t block, hipStream_t s,
                        const GenArgs& a) {
    return nt ? gen_u<V, KIND, W, IL, true>(unroll, grid, block, s, a)
              : gen_u<V, KIND, W, IL, false>(unroll, grid, block, s, a);
}

template <class V, int KIND>
static hipError_t gen_k(int width, int unroll, int ilp, bool nt, uint32_t grid, uint32_t block,
                        hipStream_t s, const GenArgs& a) {
    if (width == 1 && ilp == 1) return gen_n<V, KIND, 1, 1>(unroll, nt, grid, block, s, a);
    if (width == 2 && ilp == 1) return gen_n<V, KIND, 2, 1>(unroll, nt, grid, block, s, a);
    if (width == 2 && ilp == 2) return gen_n<V, KIND, 2, 2>(unroll, nt, grid, block, s, a);
    if (width == 2 && ilp == 4) return gen_n<V, KIND, 2, 4>(unroll, nt, grid, block, s, a);
    return hipErrorInvalidValue;
}

template <class V>
static hipError_t gen_v(int kind, int width, int unroll, int ilp, bool nt, uint32_t grid,
                        uint32_t block, hipStream_t s, const GenArgs& a) {
    return kind == 0 ? gen_k<V, 0>(width, unroll, ilp, nt, grid, block, s, a)
                     : gen_k<V, 1>(width, unroll, ilp, nt, grid, block, s, a);
}

hipError_t launch_generate(int mulmod, int kind, int width, int unroll, int ilp, bool nt,
                           uint32_t grid, uint32_t block, hipStream_t s, const GenArgs& a) {
    switch (mulmod) {
        case 1: return gen_v<VarFP64>(kind, width, unroll, ilp, nt, grid, block, s, a);
        case 2: return gen_v<VarBarrett>(kind, width, unroll, ilp, nt, grid, block, s, a);
        case 3: return gen_v<VarShoup>(kind, width, unroll, ilp, nt, grid, block, s, a);
        case 4: return gen_v<VarMontgomery>(kind, width, unroll, ilp, nt, grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <int W, int U, bool NT>
static hipError_t fill_one(uint32_t grid, uint32_t block, hipStream_t s, uint64_t* out,
                           uint64_t T, uint64_t e_full, uint32_t rem, uint64_t value) {
    hipLaunchKernelGGL((k_fill<W, U, NT>), dim3(grid), dim3(block), 0, s, out, T, e_full, rem,
                       value);
    return hipGetLastError();
}

template <int W>
static hipError_t fill_w(int unroll, bool nt, uint32_t grid, uint32_t block, hipStream_t s,
                         uint64_t* out, uint64_t T, uint64_t e_full, uint32_t rem,
                         uint64_t value) {
#define NN_FILL_CASE(U)                                                              \
    case U:                                                                          \
        return nt ? fill_one<W, U, true>(grid, block, s, out, T, e_full, rem, value) \
                  : fill_one<W, U, false>(grid, block, s, out, T, e_full, rem, value);
    switch (unroll) {
        NN_FILL_CASE(1)
        NN_FILL_CASE(2)
        NN_FILL_CASE(4)
        NN_FILL_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef NN_FILL_CASE
}

hipError_t launch_fill(int width, int unroll, bool nt, uint32_t grid, uint32_t block,
                       hipStream_t s, uint64_t* out, uint64_t T, uint64_t e_full, uint32_t rem,
                       uint64_t value) {
    if (width == 1) return fill_w<1>(unroll, nt, grid, block, s, out, T, e_full, rem, value);
    if (width == 2) return fill_w<2>(unroll, nt, grid, block, s, out, T, e_full, rem, value);
    return hipErrorInvalidValue;
}

}  // namespace nn
