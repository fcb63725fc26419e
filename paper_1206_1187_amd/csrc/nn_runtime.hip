// nn_runtime.hip -- status reporting, per-device skip tables and batch plans
// (shared by the C-ABI entry points of the plain, batched and served forms).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nn_host.hpp"
#include "nn_internal.hpp"
#include "nn_kernels.hpp"

namespace nn {

namespace {
thread_local std::string g_last_error;
}

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int ok() {
    g_last_error.clear();
    return NN_OK;
}

const char* last_error() { return g_last_error.c_str(); }

// Defaults from launch-shape sweeps on MI355X (256 CUs, bulk outputs of
// 2^28..2^30): 16-byte stores per lane from 256-thread workgroups on a
// fraction of the CUs (fewer concurrent writers keep the HBM write stream
// closer to sequential).  F64 output: the FP64 reduction with four rows in
// flight, unrolled 8 times, on CUs/2 workgroups; U64 output: the FP64
// reduction with two rows in flight on 3*CUs/4 workgroups.
const KindDefaults& kind_defaults(int kind) {
    static const KindDefaults d[2] = {
        {NN_MULMOD_FP64, 3, 4, 2, 2},  // NN_OUT_U64
        {NN_MULMOD_FP64, 1, 2, 8, 4},  // NN_OUT_F64
    };
    return d[kind == NN_OUT_F64 ? 1 : 0];
}

namespace {

// The workspace of nn_generate_batch_static (layout in nn_batch.hpp): every
// device that loads the library holds its own copy until the process ends.
// Host code never names it after set-up: hipGetSymbolAddress gives each
// device's address once (DeviceTables::scratch), and that pointer is what
// kernels, copies and fills receive.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_dev_mutex;
DeviceTables g_dev[kMaxDevices];

// Host copies of the device tables (built once, shared by all devices):
// t_lo, t_hi, then the four 13-bit skip levels.
const std::vector<Mult>& host_mult_tables() {
    static std::vector<Mult> tab = [] {
        std::vector<Mult> t(kLoSize + kHiSize + kSkipLevels * kSkipSize);
        uint64_t p = 1;
        for (uint32_t l = 0; l < kLoSize; ++l) {  // (2^53)^l
            t[l] = make_mult(p);
            p = h_mulmod(p, kMult);
        }
        const uint64_t step = p;  // (2^53)^1024
        uint64_t q = 1;
        for (uint32_t j = 0; j < kHiSize; ++j) {  // (2^53)^(1024 j)
            t[kLoSize + j] = make_mult(q);
            q = h_mulmod(q, step);
        }
        Mult* sk = t.data() + kLoSize + kHiSize;
        for (uint32_t lvl = 0; lvl < kSkipLevels; ++lvl) {  // (2^53)^(j 2^(13 lvl))
            const uint64_t unit = MultPowers::get().pow(1ull << (kSkipBits * lvl));
            uint64_t r = 1;
            for (uint32_t j = 0; j < kSkipSize; ++j) {
                sk[lvl * kSkipSize + j] = make_mult(r);
                r = h_mulmod(r, unit);
            }
        }
        return t;
    }();
    return tab;
}

// Host copy of the 8-bit skip tables: (v, qh, ql) of (2^53)^(j 2^(8 lvl)).
const std::vector<double>& host_skip8_table() {
    static std::vector<double> tab = [] {
        std::vector<double> t(kSkip8Levels * kSkip8Size * 3);
        for (uint32_t lvl = 0; lvl < kSkip8Levels; ++lvl) {
            const uint64_t unit = MultPowers::get().pow(1ull << (8 * lvl));
            uint64_t r = 1;
            for (uint32_t j = 0; j < kSkip8Size; ++j) {
                const Mult m = make_mult(r);
                double* e = &t[3 * (lvl * kSkip8Size + j)];
                e[0] = m.v;
                e[1] = m.qh;
                e[2] = m.ql;
                r = h_mulmod(r, unit);
            }
        }
        return t;
    }();
    return tab;
}

// Host copy of the flat layout's chunk multipliers: (2^53)^(512 j) for
// j < kFlatLoSize, then (2^53)^(512 kFlatLoSize i) for i < kFlatHiSize.
const std::vector<Mult>& host_flat_tables() {
    static std::vector<Mult> tab = [] {
        std::vector<Mult> t(kFlatLoSize + kFlatHiSize);
        const uint64_t row = MultPowers::get().pow(kFlatPerBlock);
        uint64_t p = 1;
        for (uint32_t j = 0; j < kFlatLoSize; ++j, p = h_mulmod(p, row)) t[j] = make_mult(p);
        const uint64_t big = p;  // (2^53)^(512 kFlatLoSize)
        p = 1;
        for (uint32_t i = 0; i < kFlatHiSize; ++i, p = h_mulmod(p, big))
            t[kFlatLoSize + i] = make_mult(p);
        return t;
    }();
    return tab;
}

// Set up tables on `dev`, which must be the current device.
int ensure_device_current(int dev, DeviceTables** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(NN_ENODEV, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    DeviceTables& d = g_dev[dev];
    if (!d.ready) {
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess)
            return fail(NN_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
            return fail(NN_ENODEV, "device %d is %s, this library is built for gfx950", dev,
                        prop.gcnArchName);
        const std::vector<Mult>& h = host_mult_tables();
        const std::vector<Mult>& hb = host_flat_tables();
        const std::vector<double>& h8 = host_skip8_table();
        const size_t mult_bytes = h.size() * sizeof(Mult);
        const size_t blk_bytes = hb.size() * sizeof(Mult);
        const size_t t8_bytes = h8.size() * sizeof(double);
        void* mem = nullptr;
        e = hipMalloc(&mem, mult_bytes + blk_bytes + t8_bytes);
        if (e != hipSuccess) return fail(NN_ENOMEM, "hipMalloc tables: %s", hipGetErrorString(e));
        e = hipMemcpy(mem, h.data(), mult_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char*)mem + mult_bytes, hb.data(), blk_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char*)mem + mult_bytes + blk_bytes, h8.data(), t8_bytes,
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return fail(NN_EHIP, "table upload: %s", hipGetErrorString(e));
        }
        d.t_lo = (Mult*)mem;
        d.t_hi = d.t_lo + kLoSize;
        d.t_sk = d.t_hi + kHiSize;
        d.t_flo = (Mult*)((char*)mem + mult_bytes);
        d.t_fhi = d.t_flo + kFlatLoSize;
        static_assert(kFlatLoOffset == (uint64_t)kLoSize + kHiSize + kSkipLevels * kSkipSize,
                      "the flat tables follow the skip tables");
        d.t8 = (double*)((char*)mem + mult_bytes + blk_bytes);
        {
            // the flat kernels' static copy: even t_lo entries, t_flo, t_fhi
            std::vector<Mult> sym(kFlatSymEntries);
            for (uint32_t l = 0; l < kFlatBlock; ++l) sym[kFlatSymLane + l] = h[2u * l];
            std::copy(hb.begin(), hb.end(), sym.begin() + kFlatSymLo);
            e = upload_flat_symbol(sym.data());
            // the chunked batch kernel's: t_lo's even entries below 2*kFlatBlock,
            // then its odd ones, then one row's step
            std::vector<Mult> cs;
            for (uint32_t l = 0; l < kFlatBlock; ++l) cs.push_back(h[2u * l]);
            for (uint32_t l = 0; l < kFlatBlock; ++l) cs.push_back(h[2u * l + 1]);
            cs.push_back(make_mult(MultPowers::get().pow(kFlatPerBlock)));
            if (e == hipSuccess) e = upload_chunk_symbol(cs.data());
            if (e != hipSuccess) {
                (void)hipFree(mem);
                return fail(NN_EHIP, "static table upload: %s", hipGetErrorString(e));
            }
        }
        void* ws = nullptr;
        e = hipGetSymbolAddress(&ws, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return fail(NN_EHIP, "static batch workspace address: %s", hipGetErrorString(e));
        }
        d.scratch = ws;
        d.cus = prop.multiProcessorCount;
        d.lds_per_cu = (uint32_t)prop.maxSharedMemoryPerMultiProcessor;
        d.lds_per_block = (uint32_t)prop.sharedMemPerBlock;
        d.ready = true;
    }
    *out = &d;
    return NN_OK;
}

}  // namespace

int current_device(DeviceTables** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NN_ENODEV, "hipGetDevice: %s", hipGetErrorString(e));
    return ensure_device_current(dev, out);
}

// ---------------------------------------------------------------- plans --

void plan_release(nn_batch_plan* p) {
    if (p->side) (void)hipStreamSynchronize(p->side);
    for (nn_batch_slot& q : p->slot) {
        if (q.done) {
            (void)hipEventSynchronize(q.done);
            (void)hipEventDestroy(q.done);
        }
        if (q.ready) (void)hipEventDestroy(q.ready);
        if (q.exec) (void)hipGraphExecDestroy(q.exec);
        if (q.graph) (void)hipGraphDestroy(q.graph);
        if (q.ws_dev) (void)hipFree(q.ws_dev);
        if (q.rec) (void)hipFree(q.rec);
        if (q.ext) (void)hipFree(q.ext);
        if (q.ws_host) (void)hipHostFree(q.ws_host);
    }
    if (p->side) (void)hipStreamDestroy(p->side);
    delete p;
}

namespace {

// Device and pinned memory, event and graph of one slot.
int slot_create(nn_batch_plan* p, nn_batch_slot& q, const DeviceTables& d,
                const uint64_t* states) {
    q.ws_bytes = sizeof(BatchHeader) + (size_t)p->cap_desc * sizeof(BatchDesc);
    hipError_t e = hipMalloc(&q.ws_dev, q.ws_bytes);
    if (e == hipSuccess && (p->interleaved || p->chunks))  // grid * per <= rows + clusters + grid
        e = hipMalloc((void**)&q.rec, (p->cap_rows + 2ull * p->grid) * sizeof(RowRec));
    if (e == hipSuccess && p->chunks)
        e = hipMalloc((void**)&q.ext, (size_t)p->cap_desc * sizeof(RowRec));
    if (e != hipSuccess)
        return fail(NN_ENOMEM, "batch workspace (%zu bytes): %s", q.ws_bytes, hipGetErrorString(e));
    e = hipHostMalloc(&q.ws_host, q.ws_bytes, hipHostMallocDefault);
    if (e != hipSuccess)
        return fail(NN_ENOMEM, "pinned staging (%zu bytes): %s", q.ws_bytes, hipGetErrorString(e));
    BatchHeader* hdr = (BatchHeader*)q.ws_host;
    memset(hdr, 0, sizeof *hdr);
    hdr->states = states;
    e = hipEventCreateWithFlags(&q.done, hipEventDisableTiming);
    if (e == hipSuccess && p->overlap) e = hipEventCreateWithFlags(&q.ready, hipEventDisableTiming);
    if (e != hipSuccess) return fail(NN_EHIP, "event: %s", hipGetErrorString(e));
    const uint32_t block = p->block, cluster = p->cluster;
    q.args.ws = (const BatchHeader*)q.ws_dev;
    q.args.cluster = cluster;
    q.args.JB = make_mult(MultPowers::get().pow(2ull * block * cluster));
    q.args.JB2 = make_mult(MultPowers::get().pow(4ull * block * cluster));
    q.args.Minv = make_mult(MultPowers::get().pow(kPeriod - 1));
    q.args.t_lo = d.t_lo;
    q.args.t_hi = d.t_hi;
    q.args.t_sk = d.t_sk;
    q.args.rec = q.rec;
    q.args.ext = q.ext;
    q.args.row_outs = 2u * kIlPairs * block;
    q.args.grid = p->grid;
    q.args.block = block;
    if (p->chunks) {
        // the pre-pass writes chunk records in record order: rows of
        // kChunkOuts outputs, one cluster of one workgroup
        q.args.row_outs = kChunkOuts;
        q.args.grid = 1;
        q.args.cluster = 1;
    }
    q.args.JR = make_mult(MultPowers::get().pow((uint64_t)q.args.row_outs * 256));
    if (!p->use_graph) return NN_OK;
    // The graph holds the kernels; the descriptor upload before each replay
    // is an ordinary async copy on the same stream (a copy node from pinned
    // host memory measured slower on MI355X).
    e = hipGraphCreate(&q.graph, 0);
    hipGraphNode_t last = nullptr;
    void* params[] = {&q.args};
    if (e == hipSuccess && (p->interleaved || p->chunks) && !p->overlap) {
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof kp);
        kp.func = const_cast<void*>(batch_rec_kernel(p->indexed));
        kp.gridDim = dim3(p->map_grid);
        kp.blockDim = dim3(256);
        kp.kernelParams = params;
        e = hipGraphAddKernelNode(&last, q.graph, nullptr, 0, &kp);
        q.rec_node = last;
        q.rec_grid = p->map_grid;
    }
    if (e == hipSuccess) {
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof kp);
        kp.func = p->chunks ? const_cast<void*>(batch_chunks_kernel(p->kind, p->nontemporal))
                  : p->interleaved
                      ? const_cast<void*>(batch_rows_kernel(p->kind, p->nontemporal))
                      : const_cast<void*>(
                            batch_kernel((int)p->mulmod, p->kind, p->nontemporal, p->indexed));
        kp.gridDim = dim3(p->grid ? p->grid : 1);  // chunked, grid 0: set per batch
        kp.blockDim = dim3(block);
        kp.sharedMemBytes = p->chunks ? p->flat_lds : 0;
        kp.kernelParams = params;
        kp.extra = nullptr;
        e = hipGraphAddKernelNode(&q.main_node, q.graph, last ? &last : nullptr, last ? 1 : 0,
                                  &kp);
        q.main_grid = p->grid ? p->grid : 1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&q.exec, q.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(NN_EHIP, "batch graph: %s", hipGetErrorString(e));
    return NN_OK;
}

}  // namespace

int plan_create(int kind, uint32_t max_streams, uint64_t max_outputs, const nn_batch_cfg* cfg,
                bool indexed, const uint64_t* states, const uint64_t* host_states,
                nn_batch_plan** plan_out) {
    if (!plan_out) return fail(NN_EINVAL, "plan_out is NULL");
    if (kind != NN_OUT_U64 && kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %d unknown", kind);
    if (max_streams == 0) return fail(NN_EINVAL, "max_streams must be positive");
    nn_batch_cfg c = {0, 0, 0, 0, 0, 0};
    if (cfg) c = *cfg;
    if (c.flags &
        ~(NN_CFG_TEMPORAL_STORES | NN_BATCH_NO_GRAPH | NN_BATCH_INTERLEAVED | NN_BATCH_CHUNKS))
        return fail(NN_EINVAL, "unknown batch flags 0x%x", c.flags);
    const bool chunks = (c.flags & NN_BATCH_CHUNKS) != 0;
    if (chunks && (c.flags & NN_BATCH_INTERLEAVED))
        return fail(NN_EINVAL, "NN_BATCH_CHUNKS and NN_BATCH_INTERLEAVED are exclusive");
    if (chunks && ((c.block && c.block != 256) || c.cluster > 1 ||
                   (c.mulmod && c.mulmod != NN_MULMOD_FP64)))
        return fail(NN_EINVAL, "the chunked batch kernel has 256 threads, no clusters and the "
                               "FP64 reduction");
    if (c.occupancy && !chunks)
        return fail(NN_EINVAL, "occupancy applies to the chunked batch kernel only");
    if (c.occupancy && (c.occupancy < 2 || c.occupancy > 16))
        return fail(NN_EINVAL, "occupancy %u: must be 0 or in [2, 16]", c.occupancy);
    DeviceTables* d = nullptr;
    int st = current_device(&d);
    if (st) return st;
    const KindDefaults& kd = kind_defaults(kind);
    const uint32_t block = c.block ? c.block : kDefaultBlock;
    if (block < 64 || block > 1024 || block % 64)
        return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", block);
    const bool interleaved = (c.flags & NN_BATCH_INTERLEAVED) != 0;
    uint32_t cluster = c.cluster ? c.cluster : 1;
    if (cluster > 64 && !interleaved) return fail(NN_EINVAL, "cluster %u: at most 64", cluster);
    const uint32_t mulmod = c.mulmod ? c.mulmod : kd.mulmod;
    if (mulmod > NN_MULMOD_MONTGOMERY)
        return fail(NN_EINVAL, "mulmod %u: batches take FP64, Barrett, Shoup or Montgomery",
                    mulmod);
    uint32_t grid = c.grid;
    if (chunks) {
        // grid 0: one workgroup per record, dispatched in output order
    } else if (!grid) {
        grid = (uint32_t)((uint64_t)d->cus * kd.grid_num / kd.grid_den);
        if (!grid) grid = 1;
    }
    if (!c.grid) grid = (grid + cluster - 1) / cluster * cluster;
    if (interleaved && !c.cluster) cluster = grid;  // one range: all workgroups interleave
    if (grid > (1u << 20)) return fail(NN_EINVAL, "grid %u too large", grid);
    if (grid % cluster) return fail(NN_EINVAL, "grid %u is not a multiple of cluster %u", grid, cluster);
    // Direct batches split streams into pieces of at most kBatchMaxLen.
    const uint64_t cap_desc = (uint64_t)max_streams + (indexed ? 0 : max_outputs / kBatchMaxLen + 1);
    if (cap_desc > 0xffffffffull) return fail(NN_ERANGE, "batch capacity too large");

    nn_batch_plan* p = new (std::nothrow) nn_batch_plan();
    if (!p) return fail(NN_ENOMEM, "plan allocation");
    (void)hipGetDevice(&p->device);
    p->kind = kind;
    p->indexed = indexed;
    p->mulmod = mulmod;
    p->block = block;
    p->grid = grid;
    p->nontemporal = !(c.flags & NN_CFG_TEMPORAL_STORES);
    p->use_graph = !(c.flags & NN_BATCH_NO_GRAPH);
    p->interleaved = (c.flags & NN_BATCH_INTERLEAVED) != 0;
    p->chunks = chunks;
    p->overlap = chunks && !indexed;
    if (p->interleaved &&
        (mulmod != NN_MULMOD_FP64 || (block & (block - 1)) || block > 256)) {
        plan_release(p);
        return fail(NN_EINVAL, "the interleaved batch kernel needs the FP64 reduction and "
                    "block 64, 128 or 256");
    }
    p->cluster = cluster;
    p->cap_rows = max_outputs / (chunks ? (uint64_t)kChunkOuts : 2ull * block) + 2 * cap_desc;
    p->map_grid = (uint32_t)(d->cus > 0 ? d->cus * 4 : 64);
    p->max_streams = max_streams;
    p->max_outputs = max_outputs;
    p->cap_desc = (uint32_t)cap_desc;
    p->host_states = host_states;
    p->tabs = d->t_lo;
    p->M1 = make_mult(kMult);
    p->J512 = make_mult(MultPowers::get().pow(kFlatPerBlock));
    // the chunk kernel's residency cap: dynamic LDS that leaves room for
    // `occupancy` workgroups per compute unit, not one more
    p->occupancy = c.occupancy ? c.occupancy : kFlatDefaultOccupancy;
    p->flat_lds = (d->lds_per_cu / (p->occupancy + 1) / 512 + 1) * 512;
    if (p->flat_lds > d->lds_per_block) p->flat_lds = 0;
    if (p->overlap) {
        // default priority; non-blocking, so it does not wait for the null stream
        hipError_t e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (e != hipSuccess) {
            plan_release(p);
            return fail(NN_EHIP, "batch side stream: %s", hipGetErrorString(e));
        }
    }
    for (nn_batch_slot& q : p->slot) {
        st = slot_create(p, q, *d, states);
        if (st) {
            plan_release(p);
            return st;
        }
    }
    *plan_out = p;
    return NN_OK;
}

int plan_wait(nn_batch_plan* p) {
    nn_batch_slot& q = p->slot[p->next];
    if (!q.pending) return NN_OK;
    hipError_t e = hipEventSynchronize(q.done);
    if (e != hipSuccess)
        return fail(NN_EHIP, "waiting for an earlier batch: %s", hipGetErrorString(e));
    q.pending = false;
    return NN_OK;
}

bool plan_idle(nn_batch_plan* p) {
    bool idle = true;
    for (nn_batch_slot& q : p->slot) {
        if (!q.pending) continue;
        if (hipEventQuery(q.done) == hipSuccess)
            q.pending = false;
        else
            idle = false;
    }
    return idle;
}

int plan_launch_staged(nn_batch_plan* p, uint32_t nd, void* out, hipStream_t stream) {
    nn_batch_slot& q = p->slot[p->next];
    // A small batch travels in the kernel arguments (no upload to wait for)
    // and runs the blocked kernel whichever kernel the plan has; larger ones
    // of an interleaved plan run its pre-pass and row kernel.
    const bool in_args = nd <= kInlineDescs;
    const bool il = (p->interleaved || p->chunks) && !in_args;
    const uint64_t row = p->chunks && !in_args ? (uint64_t)kChunkOuts
                                               : (il ? 2ull * kIlPairs : 2ull) * p->block;
    BatchHeader* hdr = (BatchHeader*)q.ws_host;
    BatchDesc* dd = plan_staged_descs(p);
    uint64_t rows = 0;
    for (uint32_t k = 0; k < nd; ++k) {
        dd[k].row_start = rows;
        // rows aligned to output pairs (blocked kernel) or to whole rows
        // of the output (interleaved kernel; chunks for the chunked one)
        const uint64_t s = dd[k].out_off & (il ? row - 1 : 1u);
        rows += (dd[k].len + s + row - 1) / row;
        // row records hold output indices in 52 bits
        if (il && dd[k].out_off + dd[k].len > (1ull << 51))
            return fail(NN_ERANGE, "interleaved and chunked batches take output indices below "
                                   "2^51");
    }
    if (il && rows > p->cap_rows)
        return fail(NN_ERANGE, "batch of %llu rows, plan holds %llu", (unsigned long long)rows,
                    (unsigned long long)p->cap_rows);
    // The chunked kernel's owned mode (one record, and one workgroup, per
    // chunk) needs the non-empty windows sorted by output offset and
    // disjoint.  Windows are independent, so they are sorted here if they
    // are not (a server's batches come in admission order); overlapping
    // windows take a record per chunk and window.
    bool owned = p->chunks && !in_args;
    if (owned) {
        bool sorted = true;
        for (uint32_t k = 1; k < nd && sorted; ++k) sorted = dd[k - 1].out_off <= dd[k].out_off;
        if (!sorted)
            std::sort(dd, dd + nd,
                      [](const BatchDesc& x, const BatchDesc& y) { return x.out_off < y.out_off; });
    }
    uint64_t end = 0;
    for (uint32_t k = 0; k < nd && owned; ++k) {
        if (!dd[k].len) continue;
        if (dd[k].out_off < end) owned = false;
        end = dd[k].out_off + dd[k].len;
    }
    if (owned) {
        // chunks numbered in output order; a window whose first chunk holds
        // the previous window's end starts at that chunk's number
        uint64_t K = 0, prev_last = 0;
        int64_t prev = -1;
        for (uint32_t k = 0; k < nd; ++k) {
            BatchDesc& D = dd[k];
            if (!D.len) {
                D.row_start = 0;
                continue;
            }
            const uint64_t first = D.out_off / row, last = (D.out_off + D.len - 1) / row;
            const bool shared = prev >= 0 && prev_last == first;
            const uint64_t k0 = shared ? K - 1 : K;
            K = k0 + (last - first + 1);
            if (shared) dd[prev].row_start |= kDescLastShared;
            D.row_start = k0 | (shared ? kDescFirstShared : 0);
            prev = k;
            prev_last = last;
        }
        rows = K;
    }
    hdr->out = (uint64_t*)out;
    hdr->n_desc = nd;
    hdr->mode = owned ? kChunkOwned : kChunkPerRecord;
    hdr->n_rows = rows;
    const size_t bytes = sizeof(BatchHeader) + nd * sizeof(BatchDesc);
    hipError_t e;
    if (in_args && p->mulmod == NN_MULMOD_FP64 && (!p->indexed || p->host_states)) {
        // each window as the plain flat layout writes it, from a start state
        // computed here (so no skip-ahead on the device)
        BatchFlatInline in;
        memset(&in, 0, sizeof in);
        in.out = (uint64_t*)out;
        in.n = nd;
        uint64_t chunks = 0;
        for (uint32_t k = 0; k < nd; ++k) {
            const BatchDesc& D = dd[k];
            FlatWin& w = in.w[k];
            w.s = (uint32_t)(D.out_off & 1u);
            const uint64_t src = p->indexed ? p->host_states[D.src] : D.src;
            w.base = h_skip(src, (D.pos % kPeriod) + 1 - w.s);  // element -s
            w.len = D.len;
            w.out_off = D.out_off;
            w.chunk0 = (uint32_t)chunks;
            chunks += (D.len + w.s + kChunkOuts - 1) / kChunkOuts;
        }
        e = launch_batch_flat_inline(p->kind, p->nontemporal, (uint32_t)chunks, p->flat_lds,
                                     stream, p->tabs, p->M1, p->J512, in);
        if (e != hipSuccess) return fail(NN_EHIP, "batch launch: %s", hipGetErrorString(e));
        e = hipEventRecord(q.done, stream);
        if (e != hipSuccess) return fail(NN_EHIP, "batch event: %s", hipGetErrorString(e));
        q.pending = true;
        p->next ^= 1;
        return NN_OK;
    }
    if (in_args) {
        BatchInline in;
        memset(&in, 0, sizeof in);
        memcpy(&in, q.ws_host, bytes);
        e = launch_batch_inline((int)p->mulmod, p->kind, p->nontemporal, p->indexed, p->grid,
                                p->block, stream, q.args, in);
        if (e != hipSuccess) return fail(NN_EHIP, "batch launch: %s", hipGetErrorString(e));
        e = hipEventRecord(q.done, stream);
        if (e != hipSuccess) return fail(NN_EHIP, "batch event: %s", hipGetErrorString(e));
        q.pending = true;
        p->next ^= 1;
        return NN_OK;
    }
    // overlapped plans upload and run the pre-pass on the side stream
    const hipStream_t up = p->overlap ? p->side : stream;
    e = hipMemcpyAsync(q.ws_dev, q.ws_host, bytes, hipMemcpyHostToDevice, up);
    // the chunked kernel's workgroups: one per record unless the plan fixed a grid;
    // its arguments carry the record count and the output
    const uint32_t chunk_grid = p->grid ? p->grid : (uint32_t)rows;
    q.args.n_rec = rows;
    q.args.out = (uint64_t*)out;
    // the record pre-pass: a workgroup per window (the window's skip-ahead is
    // its one long dependent chain), at least one
    const uint32_t rec_grid = nd < 1 ? 1u : nd > 65535 ? 65535u : nd;
    if (e == hipSuccess && p->overlap) {
        BatchArgs copy = q.args;
        void* params[] = {&copy};
        e = hipLaunchKernel(batch_rec_kernel(p->indexed), dim3(rec_grid), dim3(256), params, 0,
                            p->side);
        if (e == hipSuccess) e = hipEventRecord(q.ready, p->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, q.ready, 0);
    }
    if (e == hipSuccess && p->use_graph && q.rec_node && rec_grid != q.rec_grid) {
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof kp);
        void* params[] = {&q.args};
        kp.func = const_cast<void*>(batch_rec_kernel(p->indexed));
        kp.gridDim = dim3(rec_grid);
        kp.blockDim = dim3(256);
        kp.kernelParams = params;
        e = hipGraphExecKernelNodeSetParams(q.exec, q.rec_node, &kp);
        if (e == hipSuccess) q.rec_grid = rec_grid;
    }
    if (e == hipSuccess && p->use_graph && p->chunks) {
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof kp);
        void* params[] = {&q.args};
        kp.func = const_cast<void*>(batch_chunks_kernel(p->kind, p->nontemporal));
        kp.gridDim = dim3(chunk_grid);
        kp.blockDim = dim3(p->block);
        kp.sharedMemBytes = p->flat_lds;
        kp.kernelParams = params;
        e = hipGraphExecKernelNodeSetParams(q.exec, q.main_node, &kp);
        if (e == hipSuccess) q.main_grid = chunk_grid;
    }
    if (e == hipSuccess && p->use_graph) {
        e = hipGraphLaunch(q.exec, stream);
    } else if (e == hipSuccess) {
        BatchArgs copy = q.args;
        void* params[] = {&copy};
        if (p->interleaved || p->chunks) {
            if (!p->overlap)
                e = hipLaunchKernel(batch_rec_kernel(p->indexed), dim3(rec_grid), dim3(256),
                                    params, 0, stream);
            if (e == hipSuccess && p->chunks)
                e = hipLaunchKernel(batch_chunks_kernel(p->kind, p->nontemporal),
                                    dim3(chunk_grid), dim3(kFlatBlock), params, p->flat_lds,
                                    stream);
            else if (e == hipSuccess)
                e = hipLaunchKernel(batch_rows_kernel(p->kind, p->nontemporal), dim3(p->grid),
                                    dim3(p->block), params, 0, stream);
        } else {
            e = launch_batch((int)p->mulmod, p->kind, p->nontemporal, p->indexed, p->grid,
                             p->block, stream, q.args);
        }
    }
    if (e != hipSuccess) return fail(NN_EHIP, "batch launch: %s", hipGetErrorString(e));
    e = hipEventRecord(q.done, stream);
    if (e != hipSuccess) return fail(NN_EHIP, "batch event: %s", hipGetErrorString(e));
    q.pending = true;
    p->next ^= 1;
    return NN_OK;
}

}  // namespace nn
