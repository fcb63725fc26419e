// nn_kernels.hpp -- launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"

namespace nn {

// Skip-ahead tables on the device: t_lo[l] = 2^(53 l) for l < 1024 and
// t_hi[j] = 2^(53 * 1024 j) for j < 32768 (mod 3^33), so the multiplier of
// any offset k < 2^25 is t_hi[k >> 10] * t_lo[k & 1023].
constexpr uint32_t kLoBits = 10;
constexpr uint32_t kLoSize = 1u << kLoBits;
constexpr uint32_t kHiSize = 1u << 15;
constexpr uint64_t kMaxOffset = (uint64_t)kLoSize * kHiSize;  // 2^25
constexpr uint64_t kMaxThreads = kMaxOffset / 2;             // 2^24

// Plain generation.  Each of the T = grid*block threads owns W consecutive
// elements per row (W = 1: 8-byte stores, W = 2: 16-byte stores); row i
// covers elements [i*W*T, (i+1)*W*T).  count = e_full*W*T + rem with
// rem < W*T: the last, partial row holds `rem` elements.  `base` is
// state * 2^53 (the first output of the call), J = (2^53)^(W*T) and
// M1 = 2^53 with its reduction data.
struct GenArgs {
    uint64_t* out;
    uint64_t T;
    uint64_t e_full;
    uint32_t rem;
    uint64_t base;
    Mult J;
    Mult M1;
    Mult JI;  // J^ilp: the step of a thread that advances ilp rows at once
    const Mult* t_lo;
    const Mult* t_hi;
};

// ilp (width 2 only): rows a thread keeps in flight, 1, 2 or 4.
hipError_t launch_generate(int mulmod, int kind, int width, int unroll, int ilp,
                           bool nontemporal, uint32_t grid, uint32_t block, hipStream_t stream,
                           const GenArgs& a);

// Fused consumer: the row layout's states (W = 2, IL rows in flight) are
// consumed in registers instead of stored: each thread adds its outputs
// (raw states modulo 2^64 for kind 0, variates in binary64 for kind 1) and
// one atomic per thread folds the partial sums into *result.
hipError_t launch_consume(int mulmod, int kind, uint32_t grid, uint32_t block, hipStream_t s,
                          const GenArgs& a, void* result);

// Flat layout: workgroup b of 256 threads writes R rows of 512 elements,
// [512 R b, 512 R (b + 1)) of the launch, two consecutive ones per lane in
// one 16-byte store per row, and exits.  Its chunk starts u = R b rows of
// 512 in, from base * t_fhi[u >> 10] * t_flo[u & 1023] with
// t_flo[j] = (2^53)^(512 j) and t_fhi[i] = (2^53)^(512 * 1024 i): two small
// tables that stay in L2 (a workgroup lives a few microseconds, so its start
// must not wait on DRAM).
constexpr uint32_t kFlatBlock = 256;
constexpr uint32_t kFlatPerBlock = 2 * kFlatBlock;
constexpr uint32_t kFlatLoSize = 1024;
constexpr uint32_t kFlatHiSize = 2048;
constexpr uint64_t kFlatMaxRowsPerLaunch = (uint64_t)kFlatLoSize * kFlatHiSize;  // 2^21
// The device tables are one allocation of Mult entries: t_lo (kLoSize),
// t_hi (kHiSize), the four 8192-entry skip levels, then t_flo and t_fhi.
// The flat kernels take the allocation's start and these fixed offsets, so
// one kernel-argument load gives them every table.
constexpr uint64_t kFlatLoOffset = (uint64_t)kLoSize + kHiSize + 4ull * 8192ull;
constexpr uint64_t kFlatHiOffset = kFlatLoOffset + kFlatLoSize;
constexpr uint64_t kFlatMaxCount = kFlatMaxRowsPerLaunch * kFlatPerBlock;  // 2^30 per launch

// Rows per workgroup of the flat layout: 1, 2, 4, 8 or 16.  Defaults from
// sweeps on MI355X (2^30 f64 outputs): four rows (16 KiB per workgroup) and
// temporal stores, with the residency cap of occupancy 4 (33 280 bytes of
// dynamic LDS per workgroup).  The rate has a cliff in the LDS per
// workgroup: 6.2-6.35 TB/s at 31 744 bytes or less, 7.4-7.5 TB/s from
// 32 256 to 40 960 bytes; non-temporal stores stay at 6.2-6.4 throughout.
constexpr uint32_t kFlatMaxRows = 16;
// Outputs from which an output that is only 8-byte aligned takes the flat
// layout by default (its first element in a launch of its own).
constexpr uint64_t kFlatUnalignedMin = 1ull << 22;
constexpr uint32_t kFlatDefaultRows = 4;
constexpr uint32_t kFlatDefaultOccupancy = 4;

// The flat kernels' own copy of their multipliers (a static device array):
// kFlatBlock lane offsets (2^53)^(2l), then t_flo and t_fhi.
constexpr uint32_t kFlatSymLane = 0;
constexpr uint32_t kFlatSymLo = kFlatBlock;
constexpr uint32_t kFlatSymHi = kFlatSymLo + kFlatLoSize;
constexpr uint32_t kFlatSymEntries = kFlatSymHi + kFlatHiSize;
// Copies kFlatSymEntries entries into the current device's array.
hipError_t upload_flat_symbol(const Mult* entries);

// XCD runs: the 8 XCDs take consecutive workgroups in turn, so with chunks in
// workgroup order each XCD writes every eighth 16 KiB chunk.  With four rows
// per workgroup the whole chunks are taken in runs of 8*kFlatXcdRun
// workgroups instead, in which XCD x writes the kFlatXcdRun consecutive
// chunks [x kFlatXcdRun, (x + 1) kFlatXcdRun) of the run (4 MiB).  Whole
// chunks beyond the last full run keep workgroup order (a launch of their
// own from mid_base).
constexpr uint32_t kFlatXcds = 8;
constexpr uint32_t kFlatXcdRun = 256;
// Whole chunks of a flat launch that go to the XCD-run kernel (runs: the
// launch takes XCD runs at all).
inline uint64_t flat_run_chunks(int rows, bool runs, uint64_t whole_chunks) {
    const uint64_t run = (uint64_t)kFlatXcds * kFlatXcdRun;
    return rows == 4 && runs ? whole_chunks / run * run : 0;
}

struct FlatArgs {
    uint64_t* out;   // 16-byte aligned
    uint64_t count;  // <= kFlatMaxCount
    uint64_t base;   // state of out[0]
    uint64_t mid_base;   // state of the first output after the XCD runs (flat_run_chunks)
    uint64_t tail_base;  // state of the first output of the partial last chunk, if any
    Mult M1;         // 2^53
    Mult J;          // (2^53)^kFlatPerBlock: the next row of a lane
    bool xcd_runs;   // 4 rows: whole chunks in XCD runs (else address order)
};

// rows: rows per workgroup (1, 2, 4, 8, 16); lds_bytes > 0 caps the
// resident workgroups per compute unit.
hipError_t launch_generate_flat(int mulmod, int kind, bool nontemporal, int rows,
                                uint32_t lds_bytes, hipStream_t stream, const FlatArgs& a);
// start: the fill that keeps the generator's table loads (NN_FILL_WITH_START).
hipError_t launch_fill_flat(bool nontemporal, int rows, uint32_t lds_bytes, hipStream_t stream,
                            bool start, bool xcd_runs, uint64_t* out, uint64_t count,
                            uint64_t value);

// Consecutive layout: the output is cut into tiles of block*E elements;
// workgroup w makes tiles w, w + grid, ...  In a tile, thread t makes
// elements t*E .. t*E + E-1 one after another with the Modified Barrett
// step by 2^53, parks them in LDS, and the workgroup then stores the tile
// in serial order, lane-contiguous (16 bytes per lane when width 2).
// `base` is state * 2^53 (element 0), J = (2^53)^(grid*block*E) moves a
// thread to its next tile, and grid*block*E <= kMaxOffset.
constexpr uint32_t kConsecMaxE = 32;

struct ConsecArgs {
    uint64_t* out;
    uint64_t count;
    uint64_t base;
    Mult J;
    const Mult* t_lo;
    const Mult* t_hi;
};

// E in {2, 4, 8, 16, 32}, width 1 or 2; lds_bytes = block*(E+1)*8.
hipError_t launch_generate_consec(int kind, int E, int width, bool nontemporal, uint32_t grid,
                                  uint32_t block, hipStream_t stream, const ConsecArgs& a);

inline uint32_t consec_lds_bytes(uint32_t block, uint32_t E) { return block * (E + 1) * 8; }

hipError_t launch_fill(int width, int unroll, bool nontemporal, uint32_t grid, uint32_t block,
                       hipStream_t stream, uint64_t* out, uint64_t T, uint64_t e_full,
                       uint32_t rem, uint64_t value);

}  // namespace nn
