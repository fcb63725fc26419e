// nn_server.hip -- the served form: continuous batching of variate
// requests over device-resident stream states.
//
// A request (stream, count) gets the next `count` outputs of its stream,
// in arrival order: its window [pos, pos + count) is fixed at submission.
// The device holds each stream's state at position 0 (a table of 8-byte
// states); a window's outputs are table[stream] * (2^53)^(pos + x + 1),
// computed on the device (four-level skip tables), so a request's bytes do
// not depend on which batch it rides in or what else is in flight.
//
// Scheduling, on every poll: harvest finished batches; admit requests from
// the head of the arrival queue while the output pool has room and slots
// are free; launch the admitted requests as one batch on any idle lane (a
// batch plan with its own HIP stream).  Requests arriving while batches run
// are admitted as memory and slots free up and launched on the next idle
// lane, so work from successive arrivals overlaps on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "nn.h"
#include "nn_host.hpp"
#include "nn_internal.hpp"

using namespace nn;

namespace {

// Best-fit allocator over [0, size) with coalescing of free neighbours.
class PoolAllocator {
  public:
    explicit PoolAllocator(uint64_t size) : size_(size) {
        if (size) insert_free(0, size);
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = round(bytes);
        auto it = by_size_.lower_bound(bytes);
        if (it == by_size_.end()) return false;
        const uint64_t o = it->second, sz = it->first;
        erase_free(o, sz);
        if (sz > bytes) insert_free(o + bytes, sz - bytes);
        *off = o;
        used_ += bytes;
        if (used_ > peak_) peak_ = used_;
        return true;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = round(bytes);
        used_ -= bytes;
        uint64_t o = off, sz = bytes;
        auto next = by_off_.lower_bound(o);
        if (next != by_off_.end() && next->first == o + sz) {
            sz += next->second;
            erase_free(next->first, next->second);
        }
        auto prev = by_off_.lower_bound(o);
        if (prev != by_off_.begin()) {
            --prev;
            if (prev->first + prev->second == o) {
                o = prev->first;
                sz += prev->second;
                erase_free(prev->first, prev->second);
            }
        }
        insert_free(o, sz);
    }
    static uint64_t round(uint64_t b) { return (b + 255) & ~uint64_t(255); }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t size() const { return size_; }

  private:
    void insert_free(uint64_t o, uint64_t sz) {
        by_off_[o] = sz;
        by_size_.emplace(sz, o);
    }
    void erase_free(uint64_t o, uint64_t sz) {
        by_off_.erase(o);
        auto r = by_size_.equal_range(sz);
        for (auto it = r.first; it != r.second; ++it)
            if (it->second == o) {
                by_size_.erase(it);
                break;
            }
    }
    uint64_t size_, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> by_off_;
    std::multimap<uint64_t, uint64_t> by_size_;
};

enum ReqState { kQueued, kAdmitted, kInFlight, kDone };

struct Request {
    uint64_t ticket = 0;
    uint32_t stream = 0;
    uint64_t count = 0;
    uint64_t pos = 0;  // window start, reduced modulo the period
    uint64_t pool_off = 0;
    bool has_region = false;
    ReqState state = kQueued;
    int status = NN_OK;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

struct Lane {
    nn_batch_plan* plan = nullptr;
    hipStream_t stream = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
    double t_complete = 0;  // fake device: simulated completion time
    int status = NN_OK;     // fake device: injected launch failure
};

}  // namespace

struct nn_server {
    std::mutex mu;
    nn_server_cfg cfg;
    bool fake = false;
    int device = 0;
    uint32_t n_streams = 0;
    std::vector<uint64_t> host_states;  // state at position 0 of each stream
    std::vector<uint64_t> next_pos;     // next window start of each stream
    uint64_t* dev_states = nullptr;
    char* pool = nullptr;  // device memory, or host memory with the fake device
    bool own_pool = true;
    PoolAllocator* alloc = nullptr;
    std::vector<Lane> lanes;
    nn::DeviceQueue* dq = nullptr;                          // NN_SERVER_DEVICE_QUEUE
    std::vector<std::pair<uint64_t, uint64_t>> qflight;     // (queue entry, ticket)
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<uint64_t> queue;    // arrival order, not yet admitted
    std::vector<uint64_t> pending;  // admitted, not yet launched
    uint64_t pending_outputs = 0;
    std::deque<uint64_t> finished;  // done, not yet reported by poll
    uint32_t slots_used = 0;
    uint64_t next_ticket = 1;
    uint32_t inject_failures = 0;
    double fake_now = 0;
    std::chrono::steady_clock::time_point t0;
    nn_server_stats stats;

    double now() const {
        if (fake) return fake_now;
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

constexpr uint64_t kDefaultBatchOutputs = 1ull << 27;
constexpr uint32_t kDefaultBatchRequests = 4096;
constexpr uint32_t kDefaultSlots = 65536;
constexpr uint32_t kDefaultLanes = 2;

void server_free(nn_server* s) {
    if (s->dq) queue_destroy(s->dq);  // before the pool and the state table
    for (Lane& l : s->lanes) {
        if (l.plan) plan_release(l.plan);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
    if (s->fake) {
        if (s->own_pool) free(s->pool);
    } else {
        if (s->pool && s->own_pool) (void)hipFree(s->pool);
        if (s->dev_states) (void)hipFree(s->dev_states);
    }
    delete s->alloc;
    delete s;
}

void finish(nn_server* s, Request& r, int status, double t) {
    r.state = kDone;
    r.status = status;
    r.t_done = t;
    s->finished.push_back(r.ticket);
    if (status == NN_OK)
        ++s->stats.completed;
    else
        ++s->stats.failed;
    if (s->stats.in_flight) --s->stats.in_flight;
}

// Fake device: the outputs of one window computed on the host.
void fake_fill(nn_server* s, const Request& r) {
    uint64_t* out = (uint64_t*)(s->pool + r.pool_off);
    uint64_t z = h_skip(s->host_states[r.stream], r.pos);
    for (uint64_t x = 0; x < r.count; ++x) {
        z = h_mulmod(z, kMult);
        if (s->cfg.kind == NN_OUT_F64) {
            const double v = (double)z * kRecip;
            memcpy(&out[x], &v, 8);
        } else {
            out[x] = z;
        }
    }
}

void harvest(nn_server* s) {
    const double t = s->now();
    if (s->dq && !s->qflight.empty()) {
        for (size_t i = 0; i < s->qflight.size();) {
            if (queue_done(s->dq, s->qflight[i].first)) {
                finish(s, s->reqs[s->qflight[i].second], NN_OK, t);
                s->qflight[i] = s->qflight.back();
                s->qflight.pop_back();
            } else {
                ++i;
            }
        }
        if (!s->qflight.empty() && queue_keep_running(s->dq) != NN_OK) {
            for (auto& f : s->qflight) finish(s, s->reqs[f.second], NN_EHIP, t);
            s->qflight.clear();
        }
    }
    for (Lane& l : s->lanes) {
        if (!l.busy) continue;
        bool done;
        if (s->fake)
            done = t >= l.t_complete;
        else
            done = plan_idle(l.plan);
        if (!done) continue;
        for (uint64_t tk : l.tickets) finish(s, s->reqs[tk], l.status, t);
        l.tickets.clear();
        l.busy = false;
        l.status = NN_OK;
    }
}

// True when no batch is running or waiting for a lane.
bool batches_idle(const nn_server* s) {
    if (!s->pending.empty()) return false;
    for (const Lane& l : s->lanes)
        if (l.busy) return false;
    return true;
}

// Admits from the head of the queue; returns true if anything was admitted.
bool admit(nn_server* s) {
    bool any = false;
    const double t = s->now();
    while (!s->queue.empty()) {
        Request& r = s->reqs[s->queue.front()];
        if (s->slots_used >= s->cfg.max_slots) break;
        // Small requests take the device queue while the server is lightly
        // loaded: no batch running or waiting, and at most two entries in
        // flight per queue workgroup.  Under load the batch lanes take
        // everything (each batch spreads over the whole device), and the
        // queue kernel, left idle, exits and frees its compute units.
        const bool small = s->dq && r.count && r.count <= s->cfg.queue_max_outputs &&
                           s->qflight.size() < 2ull * s->cfg.queue_workgroups &&
                           batches_idle(s);
        if (!small) {
            if (s->pending.size() >= s->cfg.max_batch_requests) break;
            if (s->pending_outputs + r.count > s->cfg.max_batch_outputs) break;
        }
        if (r.count) {
            uint64_t off = 0;
            if (!s->alloc->alloc(r.count * 8, &off)) break;  // head of line waits for memory
            r.pool_off = off;
            r.has_region = true;
        }
        r.state = kAdmitted;
        r.t_admit = t;
        ++s->slots_used;
        s->queue.pop_front();
        if (small) {
            // Straight to the device queue, no batch launch.
            uint64_t seq = 0;
            // output x of the window is state(0) * (2^53)^(pos + x + 1)
            const uint64_t base = h_skip(s->host_states[r.stream], r.pos);
            const int st = queue_submit(s->dq, base, r.count, s->pool + r.pool_off, &seq);
            if (st == NN_OK) {
                r.state = kInFlight;
                r.t_launch = t;
                ++s->stats.in_flight;
                s->qflight.emplace_back(seq, r.ticket);
                any = true;
                continue;
            }
            if (st != NN_ERANGE) {  // the queue kernel could not be launched
                ++s->stats.in_flight;
                finish(s, r, st, t);
                any = true;
                continue;
            }
            // The ring is full: the batch path takes it.
        }
        if (r.count == 0) {
            ++s->stats.in_flight;
            finish(s, r, NN_OK, t);
        } else {
            s->pending.push_back(r.ticket);
            s->pending_outputs += r.count;
        }
        any = true;
    }
    if (s->stats.pool_peak < s->alloc->peak()) s->stats.pool_peak = s->alloc->peak();
    return any;
}

// Launches the pending batch on an idle lane; returns true if launched.
bool launch(nn_server* s) {
    if (s->pending.empty()) return false;
    Lane* lane = nullptr;
    for (Lane& l : s->lanes)
        if (!l.busy) {
            lane = &l;
            break;
        }
    if (!lane) return false;
    const double t = s->now();
    int status = NN_OK;
    if (s->fake) {
        if (s->inject_failures) {
            --s->inject_failures;
            status = NN_EHIP;
        } else {
            for (uint64_t tk : s->pending) fake_fill(s, s->reqs[tk]);
        }
        lane->t_complete =
            t + s->cfg.fake_latency_s +
            (s->cfg.fake_bytes_per_s > 0 ? 8.0 * s->pending_outputs / s->cfg.fake_bytes_per_s : 0);
    } else {
        std::lock_guard<std::mutex> lock(lane->plan->mu);
        status = plan_wait(lane->plan);
        if (status == NN_OK) {
            BatchDesc* dd = plan_staged_descs(lane->plan);
            uint32_t nd = 0;
            for (uint64_t tk : s->pending) {
                const Request& r = s->reqs[tk];
                dd[nd].src = r.stream;
                dd[nd].pos = r.pos;
                dd[nd].len = r.count;
                dd[nd].out_off = r.pool_off / 8;
                dd[nd].row_start = 0;
                ++nd;
            }
            status = plan_launch_staged(lane->plan, nd, s->pool, lane->stream);
        }
    }
    lane->tickets.swap(s->pending);
    s->pending.clear();
    s->pending_outputs = 0;
    lane->busy = true;
    lane->status = status;
    if (!s->fake && status != NN_OK) lane->t_complete = t;  // reported on the next harvest
    for (uint64_t tk : lane->tickets) {
        Request& r = s->reqs[tk];
        r.state = kInFlight;
        r.t_launch = t;
        ++s->stats.in_flight;
    }
    ++s->stats.batches;
    if (!s->fake && status != NN_OK) {
        // The plan enqueued nothing: report the batch as failed right away.
        for (uint64_t tk : lane->tickets) finish(s, s->reqs[tk], status, t);
        lane->tickets.clear();
        lane->busy = false;
        lane->status = NN_OK;
    }
    return true;
}

void progress(nn_server* s) {
    for (int guard = 0; guard < 1 << 20; ++guard) {
        harvest(s);
        const bool a = admit(s);
        const bool l = launch(s);
        if (!a && !l) break;
    }
}

}  // namespace

extern "C" {

int nn_server_create(const nn_server_cfg* cfg, const uint64_t* stream_states, uint32_t n_streams,
                     nn_server** out) {
    if (!cfg || !out) return fail(NN_EINVAL, "NULL argument");
    if (n_streams == 0 || !stream_states) return fail(NN_EINVAL, "no streams");
    for (uint32_t i = 0; i < n_streams; ++i)
        if (!valid_state(stream_states[i]))
            return fail(NN_EINVAL, "stream %u: state %llu is not a unit modulo 3^33", i,
                        (unsigned long long)stream_states[i]);
    nn_server_cfg c = *cfg;
    if (c.kind != NN_OUT_U64 && c.kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %u unknown", c.kind);
    if (c.flags & ~(NN_SERVER_FAKE_DEVICE | NN_SERVER_DEVICE_QUEUE))
        return fail(NN_EINVAL, "unknown server flags 0x%x", c.flags);
    if ((c.flags & NN_SERVER_DEVICE_QUEUE) && (c.flags & NN_SERVER_FAKE_DEVICE))
        return fail(NN_EINVAL, "the device queue needs a GPU");
    if (!c.queue_max_outputs) c.queue_max_outputs = 1ull << 18;
    if (c.queue_max_outputs > kQueueMaxCount)
        return fail(NN_EINVAL, "queue_max_outputs %llu: at most 2^30",
                    (unsigned long long)c.queue_max_outputs);
    if (!c.queue_workgroups) c.queue_workgroups = 16;
    if (!c.queue_capacity) c.queue_capacity = 1024;
    if (!(c.queue_idle_s > 0.0)) c.queue_idle_s = 0.05;
    if (!c.pool_bytes) return fail(NN_EINVAL, "pool_bytes must be positive");
    if (!c.max_batch_outputs) c.max_batch_outputs = kDefaultBatchOutputs;
    if (!c.max_batch_requests) c.max_batch_requests = kDefaultBatchRequests;
    if (!c.max_slots) c.max_slots = kDefaultSlots;
    if (!c.lanes) c.lanes = kDefaultLanes;
    if (c.lanes > 64) return fail(NN_EINVAL, "lanes %u: at most 64", c.lanes);
    if (c.max_batch_outputs > (1ull << 40)) return fail(NN_ERANGE, "max_batch_outputs too large");
    nn_server* s = new (std::nothrow) nn_server();
    if (!s) return fail(NN_ENOMEM, "server allocation");
    memset(&s->stats, 0, sizeof s->stats);
    s->cfg = c;
    s->fake = (c.flags & NN_SERVER_FAKE_DEVICE) != 0;
    s->n_streams = n_streams;
    s->host_states.assign(stream_states, stream_states + n_streams);
    s->next_pos.assign(n_streams, 0);
    s->alloc = new (std::nothrow) PoolAllocator(c.pool_bytes);
    s->t0 = std::chrono::steady_clock::now();
    s->lanes.resize(c.lanes);
    if (!s->alloc) {
        server_free(s);
        return fail(NN_ENOMEM, "pool allocator");
    }
    if (c.pool) {
        if ((uintptr_t)c.pool % 256) {
            server_free(s);
            return fail(NN_EINVAL, "pool %p is not 256-byte aligned", c.pool);
        }
        s->pool = (char*)c.pool;
        s->own_pool = false;
        // Regions are rounded up to 256 bytes: only whole units are usable.
        delete s->alloc;
        s->alloc = new (std::nothrow) PoolAllocator(c.pool_bytes & ~uint64_t(255));
        if (!s->alloc) {
            server_free(s);
            return fail(NN_ENOMEM, "pool allocator");
        }
    }
    if (s->fake) {
        if (!s->pool) s->pool = (char*)aligned_alloc(256, PoolAllocator::round(c.pool_bytes));
        if (!s->pool) {
            server_free(s);
            return fail(NN_ENOMEM, "fake pool of %llu bytes", (unsigned long long)c.pool_bytes);
        }
        *out = s;
        return ok();
    }
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess && !s->pool)
        e = hipMalloc((void**)&s->pool, PoolAllocator::round(c.pool_bytes));
    if (e != hipSuccess) {
        server_free(s);
        return fail(NN_ENOMEM, "output pool of %llu bytes: %s", (unsigned long long)c.pool_bytes,
                    hipGetErrorString(e));
    }
    e = hipMalloc((void**)&s->dev_states, n_streams * sizeof(uint64_t));
    if (e == hipSuccess)
        e = hipMemcpy(s->dev_states, stream_states, n_streams * sizeof(uint64_t),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        server_free(s);
        return fail(NN_EHIP, "stream-state table: %s", hipGetErrorString(e));
    }
    for (Lane& l : s->lanes) {
        e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            server_free(s);
            return fail(NN_EHIP, "lane stream: %s", hipGetErrorString(e));
        }
        int st = plan_create((int)c.kind, c.max_batch_requests, c.max_batch_outputs, &c.batch,
                             true, s->dev_states, s->host_states.data(), &l.plan);
        if (st) {
            server_free(s);
            return st;
        }
    }
    if (c.flags & NN_SERVER_DEVICE_QUEUE) {
        int st = queue_create((int)c.kind, c.queue_workgroups, c.queue_capacity, c.queue_idle_s,
                              &s->dq);
        if (st) {
            server_free(s);
            return st;
        }
    }
    *out = s;
    return ok();
}

int nn_server_destroy(nn_server* s) {
    if (s) server_free(s);
    return ok();
}

int nn_server_submit(nn_server* s, uint32_t stream_id, uint64_t count, uint64_t* ticket_out) {
    if (!s || !ticket_out) return fail(NN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    if (stream_id >= s->n_streams)
        return fail(NN_EINVAL, "stream %u of %u", stream_id, s->n_streams);
    if (count > s->cfg.max_batch_outputs || count > s->alloc->size() / 8)
        return fail(NN_ERANGE, "request of %llu outputs can never be admitted (pool %llu bytes, "
                    "batch %llu outputs)", (unsigned long long)count,
                    (unsigned long long)s->alloc->size(),
                    (unsigned long long)s->cfg.max_batch_outputs);
    Request r;
    r.ticket = s->next_ticket++;
    r.stream = stream_id;
    r.count = count;
    r.pos = s->next_pos[stream_id];
    s->next_pos[stream_id] = (r.pos + count) % kPeriod;
    r.t_submit = s->now();
    s->reqs.emplace(r.ticket, r);
    s->queue.push_back(r.ticket);
    ++s->stats.submitted;
    *ticket_out = r.ticket;
    return ok();
}

int nn_server_poll(nn_server* s, nn_completion* out, uint32_t max_out, uint32_t* n_out) {
    if (!s || !n_out || (max_out && !out)) return fail(NN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    progress(s);
    uint32_t n = 0;
    while (n < max_out && !s->finished.empty()) {
        const Request& r = s->reqs[s->finished.front()];
        s->finished.pop_front();
        nn_completion& c = out[n++];
        c.ticket = r.ticket;
        c.count = r.count;
        c.position = r.pos;
        c.data = r.has_region ? (void*)(s->pool + r.pool_off) : nullptr;
        c.t_submit = r.t_submit;
        c.t_admit = r.t_admit;
        c.t_launch = r.t_launch;
        c.t_done = r.t_done;
        c.stream_id = r.stream;
        c.status = r.status;
    }
    *n_out = n;
    return ok();
}

int nn_server_release(nn_server* s, uint64_t ticket) {
    if (!s) return fail(NN_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(NN_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request& r = it->second;
    if (r.state != kDone) return fail(NN_EINVAL, "ticket %llu is not finished", (unsigned long long)ticket);
    for (uint64_t tk : s->finished)
        if (tk == ticket) return fail(NN_EINVAL, "ticket %llu not yet reported by poll",
                                      (unsigned long long)ticket);
    if (r.has_region) s->alloc->release(r.pool_off, r.count * 8);
    --s->slots_used;
    ++s->stats.released;
    s->reqs.erase(it);
    return ok();
}

int nn_server_cancel(nn_server* s, uint64_t ticket) {
    if (!s) return fail(NN_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != kQueued)
        return fail(NN_EINVAL, "ticket %llu is not queued", (unsigned long long)ticket);
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
        if (*q == ticket) {
            s->queue.erase(q);
            break;
        }
    // The window stays assigned: later requests of the stream keep their
    // positions, so a cancellation never shifts anyone else's outputs.
    Request& r = it->second;
    r.state = kDone;
    r.status = NN_ECANCELED;
    r.t_done = s->now();
    ++s->slots_used;  // released like any finished request
    s->finished.push_back(ticket);
    ++s->stats.failed;
    return ok();
}

int nn_server_stats_get(nn_server* s, nn_server_stats* out) {
    if (!s || !out) return fail(NN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    out->queued = s->queue.size();
    out->pending = s->pending.size();
    out->pool_used = s->alloc->used();
    out->pool_peak = s->alloc->peak();
    out->slots_used = s->slots_used;
    out->now = s->now();
    return ok();
}

int nn_server_set_clock(nn_server* s, double now) {
    if (!s) return fail(NN_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->fake) return fail(NN_EINVAL, "the clock is settable on the fake device only");
    if (now < s->fake_now) return fail(NN_EINVAL, "the clock cannot go back");
    s->fake_now = now;
    return ok();
}

int nn_server_inject_failures(nn_server* s, uint32_t n) {
    if (!s) return fail(NN_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->fake) return fail(NN_EINVAL, "failures are injectable on the fake device only");
    s->inject_failures = n;
    return ok();
}

// --------------------------------------------------------------- replay --

// p50 and p99 of v (reordered in place); zero for an empty v.
static void percentiles(std::vector<double>& v, double* p50, double* p99) {
    *p50 = *p99 = 0.0;
    if (v.empty()) return;
    const size_t i50 = (v.size() - 1) / 2, i99 = (size_t)((v.size() - 1) * 0.99);
    std::nth_element(v.begin(), v.begin() + i50, v.end());
    *p50 = v[i50];
    std::nth_element(v.begin(), v.begin() + i99, v.end());
    *p99 = v[i99];
}

static void stage_stats(std::vector<double>& seen, std::vector<double>& launch,
                        std::vector<double>& done, nn_replay_stats* st) {
    percentiles(seen, &st->seen_p50, &st->seen_p99);
    percentiles(launch, &st->launch_p50, &st->launch_p99);
    percentiles(done, &st->done_p50, &st->done_p99);
}

static int replay_check(const double* t_arrive, const uint32_t* stream_id, const uint64_t* count,
                        uint64_t n, double time_scale, double* latency_out) {
    if (n && (!t_arrive || !stream_id || !count || !latency_out))
        return fail(NN_EINVAL, "NULL trace array");
    if (!(time_scale > 0)) return fail(NN_EINVAL, "time_scale must be positive");
    for (uint64_t i = 1; i < n; ++i)
        if (t_arrive[i] < t_arrive[i - 1]) return fail(NN_EINVAL, "arrival times must not decrease");
    return NN_OK;
}

int nn_server_replay(nn_server* s, const double* t_arrive, const uint32_t* stream_id,
                     const uint64_t* count, uint64_t n, double time_scale, double timeout_s,
                     double* latency_out, nn_replay_stats* stats_out) {
    if (!s) return fail(NN_EINVAL, "NULL server");
    int st = replay_check(t_arrive, stream_id, count, n, time_scale, latency_out);
    if (st) return st;
    if (s->fake) return fail(NN_EINVAL, "replay runs in real time: not on the fake device");
    std::vector<nn_completion> buf(1024);
    std::vector<double> st_seen(n), st_launch(n), st_done(n);
    uint64_t first_ticket = 0, i = 0, done = 0, failed = 0, variates = 0;
    const double t0 = s->now();
    while (done < n) {
        const double now = s->now() - t0;
        while (i < n && t_arrive[i] / time_scale <= now) {
            uint64_t tk = 0;
            st = nn_server_submit(s, stream_id[i], count[i], &tk);
            if (st) return st;
            if (i == 0) first_ticket = tk;
            ++i;
        }
        uint32_t got = 0;
        st = nn_server_poll(s, buf.data(), (uint32_t)buf.size(), &got);
        if (st) return st;
        for (uint32_t k = 0; k < got; ++k) {
            const nn_completion& c = buf[k];
            const uint64_t idx = c.ticket - first_ticket;
            latency_out[idx] = c.t_done - t0 - t_arrive[idx] / time_scale;
            st_seen[idx] = c.t_submit - t0 - t_arrive[idx] / time_scale;
            st_launch[idx] = c.t_launch - c.t_submit;
            st_done[idx] = c.t_done - c.t_launch;
            if (c.status != NN_OK) ++failed;
            variates += c.count;
            st = nn_server_release(s, c.ticket);
            if (st) return st;
            ++done;
        }
        if (timeout_s > 0 && s->now() - t0 > timeout_s)
            return fail(NN_ERANGE, "replay timed out with %llu of %llu requests done",
                        (unsigned long long)done, (unsigned long long)n);
    }
    if (stats_out) {
        stats_out->wall_s = s->now() - t0;
        stats_out->requests = n;
        stats_out->variates = variates;
        stats_out->failed = failed;
        stage_stats(st_seen, st_launch, st_done, stats_out);
    }
    return ok();
}

int nn_replay_per_request(const uint64_t* stream_states, uint32_t n_streams,
                          const double* t_arrive, const uint32_t* stream_id, const uint64_t* count,
                          uint64_t n, double time_scale, double timeout_s, void* pool_dev,
                          uint64_t pool_elems, int kind, void* stream, double* latency_out,
                          nn_replay_stats* stats_out) {
    int st = replay_check(t_arrive, stream_id, count, n, time_scale, latency_out);
    if (st) return st;
    if (!stream_states || !n_streams) return fail(NN_EINVAL, "no streams");
    if (!pool_dev || (uintptr_t)pool_dev % 8) return fail(NN_EINVAL, "bad pool");
    for (uint64_t k = 0; k < n; ++k) {
        if (stream_id[k] >= n_streams) return fail(NN_EINVAL, "request %llu: unknown stream",
                                                    (unsigned long long)k);
        if (count[k] > pool_elems) return fail(NN_ERANGE, "request %llu larger than the pool",
                                               (unsigned long long)k);
    }
    std::vector<uint64_t> pos(n_streams, 0);
    struct Flight {
        hipEvent_t ev;
        uint64_t idx, used;
        double t_enq;  // the launch and its event are enqueued
    };
    std::vector<double> st_seen(n), st_launch(n), st_done(n);
    std::deque<Flight> flights;
    std::vector<hipEvent_t> free_events;
    uint64_t head = 0, used = 0, i = 0, done = 0, variates = 0;
    uint64_t* pool = (uint64_t*)pool_dev;
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&] {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    st = NN_OK;
    while (done < n && st == NN_OK) {
        const double t = now();
        while (i < n && t_arrive[i] / time_scale <= t) {
            const uint64_t c = count[i];
            uint64_t start = head, waste = 0;
            if (head + c > pool_elems) {
                start = 0;
                waste = pool_elems - head;
            }
            if (used + waste + c > pool_elems) break;  // wait for the oldest to finish
            uint64_t state = h_skip(stream_states[stream_id[i]], pos[stream_id[i]]);
            pos[stream_id[i]] = (pos[stream_id[i]] + c) % kPeriod;
            if (c) {
                st = nn_generate_ex(&state, c, pool + start, kind, stream, nullptr);
                if (st) break;
            }
            hipEvent_t ev;
            if (free_events.empty()) {
                if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                    st = fail(NN_EHIP, "event creation");
                    break;
                }
            } else {
                ev = free_events.back();
                free_events.pop_back();
            }
            if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
                st = fail(NN_EHIP, "event record");
                break;
            }
            const double t_enq = now();
            st_seen[i] = t - t_arrive[i] / time_scale;
            st_launch[i] = t_enq - t;
            flights.push_back({ev, i, waste + c, t_enq});
            used += waste + c;
            head = start + c;
            ++i;
        }
        while (!flights.empty() && hipEventQuery(flights.front().ev) == hipSuccess) {
            const Flight f = flights.front();
            flights.pop_front();
            const double t_done = now();
            latency_out[f.idx] = t_done - t_arrive[f.idx] / time_scale;
            st_done[f.idx] = t_done - f.t_enq;
            variates += count[f.idx];
            used -= f.used;
            free_events.push_back(f.ev);
            ++done;
        }
        if (timeout_s > 0 && now() > timeout_s) {
            st = fail(NN_ERANGE, "replay timed out with %llu of %llu requests done",
                      (unsigned long long)done, (unsigned long long)n);
        }
    }
    (void)hipStreamSynchronize((hipStream_t)stream);
    for (const Flight& f : flights) (void)hipEventDestroy(f.ev);
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    if (st) return st;
    if (stats_out) {
        stats_out->wall_s = now();
        stats_out->requests = n;
        stats_out->variates = variates;
        stats_out->failed = 0;
        stage_stats(st_seen, st_launch, st_done, stats_out);
    }
    return ok();
}

}  // extern "C"
