// nn_queue.hip -- host side of the device request queue (the served form's
// low-latency path; the kernel is k_queue in nn_batch.hip).
//
// The ring, its head and stop words and the per-entry completion words live
// in one fine-grained (coherent) pinned host allocation; the per-slot row
// claim and row count words in device memory.  The host publishes an entry
// by writing it, then storing head with release order; it learns completion
// from the entry's completion word.  The kernel runs on its own stream at
// the default priority and leaves by itself (stop, idle time, life limit);
// the host relaunches it, from the first incomplete entry, when entries are
// waiting and it has left.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>

#include "nn_host.hpp"
#include "nn_internal.hpp"

namespace nn {

struct DeviceQueue {
    int device = 0;
    int kind = 0;
    uint32_t workgroups = 0;
    uint32_t cap = 0;
    void* host_mem = nullptr;  // QueueShared, entries[cap], done[cap]
    QueueShared* sh = nullptr;
    QueueEntry* entries = nullptr;
    volatile uint64_t* done = nullptr;
    void* dev_mem = nullptr;  // claim[cap], fin[cap]
    hipStream_t stream = nullptr;
    hipEvent_t exited = nullptr;
    bool launched = false;
    uint64_t next_seq = 0;  // next entry to publish
    uint64_t low = 0;       // every entry below is complete
    QueueArgs args;
};

namespace {

int relaunch(DeviceQueue* q) {
    // Entries below `low` are complete; the one at `low` is incomplete or
    // unpublished, and (the kernel having left) untouched.
    while (q->low < q->next_seq && q->done[q->low & (q->cap - 1)] == q->low + 1) ++q->low;
    q->args.start = q->low;
    hipError_t e = launch_queue(q->kind, q->workgroups, 256, q->stream, q->args);
    if (e == hipSuccess) e = hipEventRecord(q->exited, q->stream);
    if (e != hipSuccess) return fail(NN_EHIP, "queue launch: %s", hipGetErrorString(e));
    q->launched = true;
    return NN_OK;
}

bool kernel_running(DeviceQueue* q) {
    return q->launched && hipEventQuery(q->exited) == hipErrorNotReady;
}

}  // namespace

int queue_create(int kind, uint32_t workgroups, uint32_t capacity, double idle_s,
                 DeviceQueue** out) {
    if (capacity == 0 || (capacity & (capacity - 1)) || capacity > (1u << 20))
        return fail(NN_EINVAL, "queue capacity %u: a power of two up to 2^20", capacity);
    if (workgroups == 0 || workgroups > 1024)
        return fail(NN_EINVAL, "queue workgroups %u: 1 to 1024", workgroups);
    if (!(idle_s > 0.0) || idle_s > 10.0)
        return fail(NN_EINVAL, "queue idle time %g s: in (0, 10]", idle_s);
    DeviceTables* d = nullptr;
    int st = current_device(&d);
    if (st) return st;
    DeviceQueue* q = new (std::nothrow) DeviceQueue();
    if (!q) return fail(NN_ENOMEM, "queue allocation");
    (void)hipGetDevice(&q->device);
    q->kind = kind;
    q->workgroups = workgroups;
    q->cap = capacity;
    const size_t host_bytes = sizeof(QueueShared) + capacity * (sizeof(QueueEntry) + 8);
    hipError_t e = hipHostMalloc(&q->host_mem, host_bytes, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipMalloc(&q->dev_mem, capacity * 16ull);
    if (e == hipSuccess) e = hipMemset(q->dev_mem, 0, capacity * 16ull);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->exited, hipEventDisableTiming);
    int rate_khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, q->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();  // the claim words are zero before any launch
    if (e != hipSuccess || rate_khz <= 0) {
        queue_destroy(q);
        return fail(NN_EHIP, "queue set-up: %s", hipGetErrorString(e));
    }
    memset(q->host_mem, 0, host_bytes);
    q->sh = (QueueShared*)q->host_mem;
    q->entries = (QueueEntry*)(q->sh + 1);
    q->done = (volatile uint64_t*)(q->entries + capacity);
    QueueArgs& a = q->args;
    a.sh = q->sh;
    a.entries = q->entries;
    a.done = (uint64_t*)q->done;
    a.claim = (uint64_t*)q->dev_mem;
    a.fin = a.claim + capacity;
    a.cap = capacity;
    a.cap_log2 = (uint32_t)__builtin_ctz(capacity);
    a.start = 0;
    a.tabs = d->t_lo;  // the table allocation: t_lo at 0, t_flo and t_fhi at their offsets
    a.JB = make_mult(MultPowers::get().pow(kFlatPerBlock));
    const double ticks_per_s = rate_khz * 1e3;
    a.idle_ticks = (uint64_t)(idle_s * ticks_per_s);
    a.max_ticks = (uint64_t)(60.0 * ticks_per_s);  // a launch lives at most a minute
    *out = q;
    return NN_OK;
}

void queue_destroy(DeviceQueue* q) {
    if (!q) return;
    if (q->sh) __atomic_store_n(&q->sh->stop, 1ull, __ATOMIC_RELEASE);
    if (q->launched) (void)hipEventSynchronize(q->exited);  // serves what is published, then leaves
    if (q->exited) (void)hipEventDestroy(q->exited);
    if (q->stream) (void)hipStreamDestroy(q->stream);
    if (q->dev_mem) (void)hipFree(q->dev_mem);
    if (q->host_mem) (void)hipHostFree(q->host_mem);
    delete q;
}

int queue_submit(DeviceQueue* q, uint64_t base, uint64_t count, void* out, uint64_t* seq_out) {
    if (count == 0 || count > kQueueMaxCount || ((uintptr_t)out % 16))
        return fail(NN_EINVAL, "queue entry: 0 < count <= 2^30 and a 16-byte aligned output");
    const uint64_t seq = q->next_seq;
    const uint32_t slot = (uint32_t)(seq & (q->cap - 1));
    if (seq >= q->cap && q->done[slot] != seq - q->cap + 1)
        return fail(NN_ERANGE, "device queue full");  // the slot's previous entry is running
    QueueEntry& e = q->entries[slot];
    e.base = base;
    e.count = count;
    e.out = (uint64_t)(uintptr_t)out;
    e.pad = 0;
    __atomic_store_n(&q->sh->head, seq + 1, __ATOMIC_RELEASE);
    q->next_seq = seq + 1;
    *seq_out = seq;
    if (!kernel_running(q)) return relaunch(q);
    return NN_OK;
}

bool queue_done(DeviceQueue* q, uint64_t seq) {
    return q->done[seq & (q->cap - 1)] == seq + 1;
}

int queue_keep_running(DeviceQueue* q) {
    if (q->next_seq == 0 || kernel_running(q)) return NN_OK;
    while (q->low < q->next_seq && q->done[q->low & (q->cap - 1)] == q->low + 1) ++q->low;
    if (q->low == q->next_seq) return NN_OK;  // nothing waits
    return relaunch(q);
}

}  // namespace nn
