// nn_batch.hpp -- the batched form: many streams (windows of the sequence)
// written by one persistent kernel whose arguments never change, so the
// launch can live in a hipGraph and be replayed for every batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"

namespace nn {

// One stream window after host preparation: `len` outputs written from
// element `out_off` of the output; output x is src * (2^53)^(pos + x + 1).
//  * direct batches: src = the state, pos = the piece's offset in the
//    stream (streams longer than kBatchMaxLen are split by the host);
//  * indexed batches (the served form): src = a row of the device-resident
//    stream-state table, pos = the window's position in that stream
//    (reduced modulo the period).
// The batch is cut into rows of 2*block outputs aligned to global output
// pairs; row_start is the index of the window's first row in the batch
// (a prefix sum of ceil((len + (out_off & 1)) / (2*block))).
struct BatchDesc {
    uint64_t src;
    uint64_t pos;
    uint64_t len;
    uint64_t out_off;
    uint64_t row_start;
};

constexpr uint64_t kBatchMaxLen = 1ull << 24;

// Device workspace image, uploaded per batch as one contiguous block:
// the header, then n_desc descriptors.
struct BatchHeader {
    uint64_t* out;
    uint32_t n_desc;
    uint32_t pad0;
    uint64_t n_rows;
    const uint64_t* states;  // indexed batches: the stream-state table
    uint64_t pad[4];
};
static_assert(sizeof(BatchHeader) == 64, "header is one 64-byte line");

// Skip tables of the indexed form: t_sk[lvl][j] = (2^53)^(j * 2^(13 lvl)),
// lvl < 4, j < 8192, so any exponent below 2^52 costs four multiplications.
constexpr uint32_t kSkipBits = 13;
constexpr uint32_t kSkipSize = 1u << kSkipBits;
constexpr uint32_t kSkipLevels = 4;

// Kernel arguments (fixed for the life of a plan).
struct BatchArgs {
    const BatchHeader* ws;  // device workspace
    Mult JB;                // (2^53)^(2*block): one row
    Mult JB2;               // (2^53)^(4*block): two rows
    Mult Minv;              // (2^53)^-1
    const Mult* t_lo;
    const Mult* t_hi;
    const Mult* t_sk;       // kSkipLevels * kSkipSize entries (indexed batches)
};

// The kernel entry for (mulmod, kind, nontemporal, indexed); its single
// parameter is a BatchArgs passed by value.
const void* batch_kernel(int mulmod, int kind, bool nontemporal, bool indexed);

hipError_t launch_batch(int mulmod, int kind, bool nontemporal, bool indexed, uint32_t grid,
                        uint32_t block, hipStream_t stream, const BatchArgs& a);

}  // namespace nn
