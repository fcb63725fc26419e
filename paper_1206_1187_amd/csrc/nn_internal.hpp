// nn_internal.hpp -- state shared by the C-ABI translation units: status
// reporting, per-device tables and batch plans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "nn.h"
#include "nn_arith.hpp"
#include "nn_batch.hpp"

namespace nn {

// Records a detail string for nn_last_error() and returns `status`.
int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int ok();

struct DeviceTables {
    bool ready = false;
    Mult* t_lo = nullptr;       // kLoSize entries
    Mult* t_hi = nullptr;       // kHiSize entries
    Mult* t_sk = nullptr;       // kSkipLevels * kSkipSize entries
    double* t8 = nullptr;       // kSkip8Levels * kSkip8Size * 3 doubles
    Mult* t_flo = nullptr;      // kFlatLoSize entries (flat layout)
    Mult* t_fhi = nullptr;      // kFlatHiSize entries (flat layout)
    void* scratch = nullptr;    // this device's copy of the static batch workspace
    int cus = 0;
    uint32_t lds_per_cu = 0;
    uint32_t lds_per_block = 0;
};

// Tables of the current device (set up on first use).
int current_device(DeviceTables** out);

// Per-kind launch defaults.
struct KindDefaults {
    uint32_t mulmod, grid_num, grid_den, unroll, ilp;
};
const KindDefaults& kind_defaults(int kind);
constexpr uint32_t kDefaultBlock = 256;

}  // namespace nn

// A batch plan: two slots, each a device workspace, a pinned staging copy
// of it and a graph of the batch kernel (with the interleaved kernel's
// row-record pre-pass before it).  Batches alternate between the slots, so the
// host prepares batch i+1 while batch i runs; a slot is reused only after
// the batch that last used it has finished.
struct nn_batch_slot {
    size_t ws_bytes = 0;
    void* ws_dev = nullptr;
    void* ws_host = nullptr;      // pinned staging, same layout as ws_dev
    nn::RowRec* rec = nullptr;    // device, cap_rows + 2 grid records (interleaved, chunked)
    nn::RowRec* ext = nullptr;    // device, cap_desc first-chunk records (chunked)
    hipEvent_t done = nullptr;
    bool pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t main_node = nullptr;  // the batch kernel's node
    uint32_t main_grid = 0;              // its grid as last set (chunked kernel, set per batch)
    hipGraphNode_t rec_node = nullptr;   // the record pre-pass's node (interleaved, indexed chunked)
    hipEvent_t ready = nullptr;          // overlapped plans: this slot's upload and pre-pass done
    uint32_t rec_grid = 0;               // its grid as last set (one workgroup per window)
    nn::BatchArgs args;
};

struct nn_batch_plan {
    std::mutex mu;  // one batch call at a time per plan
    int device = 0;
    int kind = 0;
    bool indexed = false;
    uint32_t mulmod = 0, block = 0, grid = 0, cluster = 1;
    bool nontemporal = true, use_graph = true, interleaved = false, chunks = false;
    // Chunked plans of nn_generate_batch: each batch's descriptor upload and
    // record pre-pass run on `side`, so they overlap the previous batch's
    // chunk kernel; the caller's stream waits for them (event `ready` of the
    // slot) and runs the chunk kernel.  They touch only the slot's own
    // workspace, which the host has seen free (plan_wait) before reuse.
    bool overlap = false;
    hipStream_t side = nullptr;
    uint64_t cap_rows = 0;
    uint32_t map_grid = 0;
    uint32_t max_streams = 0;
    uint64_t max_outputs = 0;
    uint32_t cap_desc = 0;
    // small batches of the FP64 reduction (the flat inline kernel)
    const uint64_t* host_states = nullptr;  // indexed plans: host copy of the state table
    const nn::Mult* tabs = nullptr;         // the device tables
    nn::Mult M1, J512;                      // 2^53 and (2^53)^512
    uint32_t occupancy = 0;                 // chunk kernel: resident workgroups per CU
    uint32_t flat_lds = 0;                  // its residency cap as dynamic LDS
    nn_batch_slot slot[2];
    int next = 0;  // the slot of the next batch
};

namespace nn {

// Creates a plan on the current device.  Indexed plans read window states
// from `states` (a device table; `host_states` is its host copy, read for
// batches small enough to travel in the kernel arguments) and take
// descriptors with src = row.
int plan_create(int kind, uint32_t max_streams, uint64_t max_outputs, const nn_batch_cfg* cfg,
                bool indexed, const uint64_t* states, const uint64_t* host_states,
                nn_batch_plan** out);
void plan_release(nn_batch_plan* p);

// Waits until the next batch's slot is free (the batch before the previous
// one has finished).
int plan_wait(nn_batch_plan* p);
// True when every batch of the plan has finished on the device.
bool plan_idle(nn_batch_plan* p);
// Staged descriptors of the next batch (capacity p->cap_desc); valid after
// plan_wait().
inline BatchDesc* plan_staged_descs(nn_batch_plan* p) {
    return reinterpret_cast<BatchDesc*>(reinterpret_cast<BatchHeader*>(p->slot[p->next].ws_host) +
                                        1);
}
// Fills in the row prefix of the `nd` staged descriptors (their src, pos,
// len and out_off set by the caller), uploads them and launches on
// `stream`, and records the plan's completion event.  The caller checked
// nd <= p->cap_desc and holds p->mu.
int plan_launch_staged(nn_batch_plan* p, uint32_t nd, void* out, hipStream_t stream);

// Device request queue (host side in nn_queue.hip, kernel in nn_batch.hip).
struct DeviceQueue;
int queue_create(int kind, uint32_t workgroups, uint32_t capacity, double idle_s,
                 DeviceQueue** out);
// Waits for published entries to finish, stops the kernel, frees.
void queue_destroy(DeviceQueue* q);
// Publishes a request: `count` outputs (0 < count <= kQueueMaxCount) to a
// 16-byte aligned `out`, output x being base * (2^53)^(x + 1); NN_ERANGE when
// the ring is full.  Launches the kernel if it is not running.
int queue_submit(DeviceQueue* q, uint64_t base, uint64_t count, void* out, uint64_t* seq_out);
bool queue_done(DeviceQueue* q, uint64_t seq);
// Relaunches the kernel if it has left while published entries are incomplete.
int queue_keep_running(DeviceQueue* q);

}  // namespace nn
