// nn_batch.hpp -- the batched form: many streams (windows of the sequence)
// written by one persistent kernel whose arguments never change, so the
// launch can live in a hipGraph and be replayed for every batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_arith.hpp"
#include "nn_kernels.hpp"

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
    uint32_t mode;  // chunked kernel: kChunkPerRecord or kChunkOwned
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

// The device-side API's skip tables (nn_dev_skip_table): 8 bits per level,
// t8[lvl][j] = (2^53)^(j * 2^(8 lvl)), lvl < 7 (2^56 > the period), three
// doubles (v, qh, ql) per entry.
constexpr uint32_t kSkip8Levels = NN_DEV_SKIP_LEVELS;
constexpr uint32_t kSkip8Size = NN_DEV_SKIP_SIZE;
static_assert(kSkip8Levels == 7 && kSkip8Size == 256, "8-bit levels covering 2^56");
static_assert(sizeof(nn_dev_mult) == 3 * sizeof(double), "t8 entries are nn_dev_mult");

// Interleaved kernel: rows of 2*kIlPairs*block outputs, lane l owning the
// pairs 2 (e block + l), 2 (e block + l) + 1, e < kIlPairs (each store of
// a wavefront is 1 KiB contiguous), kIlRows rows in flight per lane.
constexpr uint32_t kIlPairs = 1;
constexpr uint32_t kIlRows = 4;
// One record per batch row, written by a pre-pass.
// Element k of a row (k < W = 2*kIlPairs*block) has
// the state z * (2^53)^k and goes to output index g + k, and it belongs to
// the row's window iff lo <= k < hi.  Rows are aligned to the output (g is
// a multiple of W), so lo < W fits below g.
struct RowRec {
    double z;       // state of the row's element 0
    uint64_t info;  // g | lo | hi << 52 (see kRecMulti for the chunked kernel's other form)
};
static_assert(sizeof(RowRec) == 16, "one 16-byte record per row");
constexpr uint64_t kRecIndexMask = (1ull << 51) - 1;  // g | lo (output indices < 2^51)
constexpr uint32_t kRecHiShift = 52;
// Chunked kernel, one workgroup per chunk: a chunk that more windows share
// has its first window's record with bit kRecMulti set and, in place of g,
// (d + 1) << 11 | lo, d that window's index: the chunk's other windows are
// the next windows, d + 1, d + 2, ..., whose records for it are the ext
// records (the record of each window's first chunk).
constexpr uint32_t kRecMulti = 51;
// An ext record of an empty window.
constexpr uint64_t kRecEmpty = ~0ull;
// Records are stored workgroup-major: each workgroup of the row kernel reads
// the records of its rows as one contiguous run (per = ceil(ceil(n_rows / C)
// / K) of them, C = grid / K clusters of K workgroups), kRecChunk at a time
// through LDS.
constexpr uint32_t kRecChunk = 4096;

// Kernel arguments (fixed for the life of a plan but for n_rec and out).
struct BatchArgs {
    // Chunked kernel: its record array and, set for each batch (the plan
    // updates its graph node's arguments with the grid), the record count and
    // the output; record and count lead, so one scalar load fetches both.
    RowRec* rec;            // row records (device workspace; interleaved kernels too)
    uint64_t n_rec;
    uint64_t* out;
    RowRec* ext;            // chunked, owned mode: each window's first-chunk record
    const BatchHeader* ws;  // device workspace
    uint32_t cluster;       // workgroups sharing a row range (both batch kernels)
    Mult JB;                // (2^53)^(2*block*cluster): the next row of a lane
    Mult JB2;               // (2^53)^(4*block*cluster): two such rows
    Mult Minv;              // (2^53)^-1
    const Mult* t_lo;
    const Mult* t_hi;
    const Mult* t_sk;       // kSkipLevels * kSkipSize entries
    Mult JR;                // (2^53)^(row_outs*256): a pre-pass thread's next row
    uint32_t grid;          // workgroups of the row kernel
    uint32_t block;         // threads per workgroup of the row kernel
    uint32_t row_outs;      // outputs per row (2*kIlPairs*block, a power of two)
};

// Interleaved kernels (FP64 reduction, block 64, 128 or 256): the pre-pass
// writes every row's record, then the row kernel's clusters of `cluster`
// workgroups each take a contiguous range of rows and interleave them
// (cluster = grid: workgroup w takes rows w, w + grid, ..., one write front
// as in the plain row layout).
const void* batch_rec_kernel(bool indexed);
const void* batch_rows_kernel(int kind, bool nontemporal);

// Chunked kernel (FP64 reduction, 256 threads): the pre-pass writes one
// record per chunk of kChunkOuts outputs and window that meet (rows of
// kChunkOuts outputs in k_batch_rec's terms, one cluster of one workgroup,
// so the records lie in window order); by default the chunk kernel has one
// workgroup per record, dispatched in record order like the plain flat
// layout's chunks (a fixed grid takes the records round-robin instead).
constexpr uint32_t kChunkRows = 4;
constexpr uint32_t kChunkOuts = kChunkRows * 512;
// The chunked kernel's multipliers in a static device array of its module:
// (2^53)^(2l) for l < kFlatBlock, then (2^53)^(2l+1) (a lane's pair, each
// half contiguous so a wave's loads of either are), then (2^53)^kFlatPerBlock
// (one row).  Filled per device at set-up.
constexpr uint32_t kChunkSymEntries = 2 * kFlatBlock + 1;
hipError_t upload_chunk_symbol(const Mult* entries);
// Records of the chunked kernel lie in record order (record j at j; the
// pre-pass writes them as one cluster of one workgroup).  The kernel takes
// them in the plain flat layout's XCD runs (xcd_run_index): in each run of
// kFlatXcds*kFlatXcdRun workgroups, XCD x takes the kFlatXcdRun consecutive
// records [x kFlatXcdRun, (x + 1) kFlatXcdRun) of the run, so one XCD's
// records share its L2's lines and it writes 4 MiB of consecutive chunks;
// records after the last full run go in workgroup order.
// Record modes of the chunked kernel (BatchHeader::mode):
//  * per record: a record per chunk and window that meet, one workgroup each
//    (windows in any order; a chunk that windows share is written by
//    several workgroups);
//  * owned: windows sorted by output offset and disjoint (the host checks),
//    a record per chunk, so every chunk is written by one workgroup, which
//    also writes the chunk's other windows from their ext records.  The
//    descriptors' row_start then holds k | first_shared << 62 |
//    last_shared << 63: k the chunk number of the window's first chunk
//    (chunks that windows meet, numbered in output order), first_shared
//    whether that chunk holds the end of an earlier window, last_shared
//    whether the window's last chunk holds the start of a later one.
constexpr uint32_t kChunkPerRecord = 0;
constexpr uint32_t kChunkOwned = 1;
constexpr uint64_t kDescFirstShared = 1ull << 62;
constexpr uint64_t kDescLastShared = 1ull << 63;
const void* batch_chunks_kernel(int kind, bool nontemporal);

// The kernel entry for (mulmod, kind, nontemporal, indexed); its single
// parameter is a BatchArgs passed by value.
const void* batch_kernel(int mulmod, int kind, bool nontemporal, bool indexed);

hipError_t launch_batch(int mulmod, int kind, bool nontemporal, bool indexed, uint32_t grid,
                        uint32_t block, hipStream_t stream, const BatchArgs& a);

// A batch of at most kInlineDescs windows passed by value in the kernel
// arguments (the header, then the descriptors, laid out as in the
// workspace), launched without an upload.
constexpr uint32_t kInlineDescs = 16;
struct BatchInline {
    BatchHeader hdr;
    BatchDesc desc[kInlineDescs];
};
static_assert(sizeof(BatchInline) == sizeof(BatchHeader) + kInlineDescs * sizeof(BatchDesc),
              "descriptors follow the header as in the workspace");

hipError_t launch_batch_inline(int mulmod, int kind, bool nontemporal, bool indexed,
                               uint32_t grid, uint32_t block, hipStream_t stream,
                               const BatchArgs& a, const BatchInline& in);

// A small batch of the FP64 reduction in the kernel arguments, each window
// written as the plain generator's flat layout writes an output: chunks of
// kChunkRows rows of 512 outputs, one workgroup each, dispatched in order
// (a window's chunks after the previous window's).  The host gives each
// window's start state, so a workgroup's start is the plain flat kernel's.
// Window element x has the state base * (2^53)^(x + s), s = out_off mod 2
// (chunks are aligned to output pairs, so the 16-byte stores stay aligned).
struct FlatWin {
    uint64_t base;     // state of window element -s
    uint64_t len;      // outputs, > 0
    uint64_t out_off;  // output index of window element 0
    uint32_t s;        // out_off & 1
    uint32_t chunk0;   // the window's first chunk (workgroup index)
};
struct BatchFlatInline {
    uint64_t* out;
    uint32_t n;
    uint32_t pad;
    FlatWin w[kInlineDescs];
};

// grid = the windows' chunks in total; lds caps residency as for the
// plain flat layout.
hipError_t launch_batch_flat_inline(int kind, bool nontemporal, uint32_t grid, uint32_t lds,
                                    hipStream_t stream, const Mult* tabs, const Mult& M1,
                                    const Mult& J, const BatchFlatInline& in);

// ------------------------------------------- batches without allocation --
// nn_generate_batch_static runs the chunked kernel with its workspace in one
// static device array per device instead of a plan's allocations.  Layout
// of that array (offsets in bytes):
//   0                 BatchHeader, written by k_static_descs
//   kStaticDescOff    BatchDesc[kStaticMaxStreams], prepared by k_static_descs
//   kStaticRawOff     the caller's nn_stream_desc[n], copied in by the host
//   kStaticRecOff     chunk records (RowRec), written by k_batch_rec
// A window of length L at output offset o has ceil((L + o mod kChunkOuts) /
// kChunkOuts) < L / kChunkOuts + 2 records, so kStaticMaxStreams windows of
// kStaticMaxOutputs outputs in all never need more than kStaticMaxRecords.
constexpr uint32_t kStaticMaxStreams = 1u << 16;
constexpr uint64_t kStaticMaxOutputs = 1ull << 31;
constexpr uint64_t kStaticMaxRecords = kStaticMaxOutputs / kChunkOuts + 2ull * kStaticMaxStreams;
constexpr uint64_t static_align(uint64_t x) { return (x + 255) & ~(uint64_t)255; }
constexpr uint64_t kStaticDescOff = sizeof(BatchHeader);
constexpr uint64_t kStaticRawOff =
    static_align(kStaticDescOff + (uint64_t)kStaticMaxStreams * sizeof(BatchDesc));
constexpr uint64_t kStaticRecOff =
    static_align(kStaticRawOff + (uint64_t)kStaticMaxStreams * 3 * sizeof(uint64_t));
constexpr uint64_t kStaticScratchBytes = kStaticRecOff + kStaticMaxRecords * sizeof(RowRec);

// Prepares a static batch on the device (one workgroup of 1024 threads):
// the n copied descriptors {state, length, out_offset} become BatchDescs
// (src = state, pos = 0, row_start = the prefix sum of the windows' chunk
// records), and the header gets out, n and the record count.  Windows of
// length 0 get no record.
hipError_t launch_static_descs(hipStream_t stream, void* scratch, uint32_t n, uint64_t* out);

// --------------------------------------------------- device request queue --
// The served form's low-latency path: a persistent kernel serves requests
// that the host publishes in a ring in fine-grained (coherent) host memory,
// so a request costs no launch.  Every live workgroup walks the ring in
// order; the rows of an entry (2*block outputs each) are claimed a few at a
// time by whichever workgroups reach it, so any workgroup may leave between
// entries and the rest finish the work.  A workgroup leaves when the host
// sets `stop`, after `idle_ticks` without a new entry, or after `max_ticks`
// of life; an entry is then either complete or untouched, and the host
// relaunches from the first incomplete one.
// The host computes each entry's start state (it holds every stream's
// state), so a claim starts from three independent table loads and no
// skip-ahead on the device.
struct QueueEntry {
    uint64_t base;   // state of the window's element -1: output x is base * (2^53)^(x + 1)
    uint64_t count;  // outputs, in (0, kQueueMaxCount]
    uint64_t out;    // device address of output 0, 16-byte aligned
    uint64_t pad;
};

struct QueueShared {  // host memory, fine-grained
    uint64_t head;    // host: entries [0, head) are published
    uint64_t stop;    // host: leave once no published entry is left
    uint64_t pad[6];
};

constexpr uint32_t kQueueRowsPerClaim = 4;
constexpr uint32_t kQueueMaxRowsPerClaim = 64;
// Rows are the flat layout's rows (kFlatPerBlock outputs, 256 threads), so
// a row's start is base * t_fhi[u >> 10] * t_flo[u & 1023] for row u < 2^21.
constexpr uint64_t kQueueMaxCount = kFlatMaxCount;

struct QueueArgs {
    QueueShared* sh;
    const QueueEntry* entries;  // host memory, cap entries (ring)
    uint64_t* done;             // host memory, cap entries: seq + 1 once entry seq is complete
    uint64_t* claim;            // device, cap entries: (round << 32) | rows claimed
    uint64_t* fin;              // device, cap entries: rows finished
    uint32_t cap;               // ring capacity, a power of two
    uint32_t cap_log2;
    uint64_t start;             // first entry of this launch
    const Mult* tabs;           // the device table allocation (t_lo, t_flo, t_fhi)
    Mult JB;                    // (2^53)^kFlatPerBlock: a lane's next row
    uint64_t idle_ticks;        // wall-clock ticks
    uint64_t max_ticks;
};

hipError_t launch_queue(int kind, uint32_t grid, uint32_t block, hipStream_t stream,
                        const QueueArgs& a);

// The paper's strided layout (nn_strided.hip): T threads, E consecutive
// elements each, out[t + i*T] = element t*E + i; base is element 0's state.
hipError_t launch_generate_strided(int kind, bool nontemporal, uint32_t grid, uint32_t block,
                                   hipStream_t stream, uint64_t* out, uint64_t T, uint32_t E,
                                   uint64_t base, const Mult* t_sk);

}  // namespace nn
