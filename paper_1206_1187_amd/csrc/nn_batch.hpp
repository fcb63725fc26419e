// nn_batch.hpp -- the batched form: many streams (windows of the sequence)
// written by one persistent kernel whose arguments never change, so the
// launch can live in a hipGraph and be replayed for every batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"

namespace nn {

// One stream after host preparation: `base` = state * 2^53 (its first
// output), `len` outputs written from element `out_off` of the output.
// Streams longer than kBatchMaxLen are split by the host.
struct BatchDesc {
    uint64_t base;
    uint64_t len;
    uint64_t out_off;
};

constexpr uint64_t kBatchMaxLen = 1ull << 24;

// Device workspace image, uploaded per batch as one contiguous block:
// header, then n_desc descriptors, then n_tiles tile words
// (desc index << 32 | tile index within the descriptor).
struct BatchHeader {
    uint64_t* out;
    uint32_t n_desc;
    uint32_t n_tiles;
    uint64_t pad[6];
};
static_assert(sizeof(BatchHeader) == 64, "header is one 64-byte line");

// Kernel arguments (fixed for the life of a plan).
struct BatchArgs {
    const BatchHeader* ws;  // device workspace
    uint32_t rows;          // rows of 2*block outputs per tile
    Mult JB;                // (2^53)^(2*block): one row
    Mult Minv;              // (2^53)^-1
    const Mult* t_lo;
    const Mult* t_hi;
};

// The kernel entry for (mulmod, kind, nontemporal); its single parameter is
// a BatchArgs passed by value.
const void* batch_kernel(int mulmod, int kind, bool nontemporal);

hipError_t launch_batch(int mulmod, int kind, bool nontemporal, uint32_t grid, uint32_t block,
                        hipStream_t stream, const BatchArgs& a);

}  // namespace nn
