// nn_capi.hip -- the extern "C" boundary declared in include/nn.h.
//
// Host work per generating call: validate, pick the launch shape, compute
// base = state*2^53 and the jump J = (2^53)^T with its reduction data,
// enqueue one kernel, and advance the caller's state by skip-ahead.  No
// allocation and no synchronisation happen on this path after the one-time
// per-device table upload.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>
#include <vector>

#include "nn.h"
#include "nn_host.hpp"
#include "nn_kernels.hpp"

using namespace nn;

namespace {

thread_local std::string g_last_error;

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

constexpr int kMaxDevices = 64;

struct DeviceTables {
    bool ready = false;
    Mult* t_lo = nullptr;  // device, kLoSize entries
    Mult* t_hi = nullptr;  // device, kHiSize entries
    int cus = 0;
};

std::mutex g_dev_mutex;
DeviceTables g_dev[kMaxDevices];

// Host copies of the skip-ahead tables (built once, shared by all devices).
const std::vector<Mult>& host_tables() {
    static std::vector<Mult> tab = [] {
        std::vector<Mult> t(kLoSize + kHiSize);
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
        const std::vector<Mult>& h = host_tables();
        void* mem = nullptr;
        e = hipMalloc(&mem, h.size() * sizeof(Mult));
        if (e != hipSuccess) return fail(NN_ENOMEM, "hipMalloc tables: %s", hipGetErrorString(e));
        e = hipMemcpy(mem, h.data(), h.size() * sizeof(Mult), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return fail(NN_EHIP, "table upload: %s", hipGetErrorString(e));
        }
        d.t_lo = (Mult*)mem;
        d.t_hi = d.t_lo + kLoSize;
        d.cus = prop.multiProcessorCount;
        d.ready = true;
    }
    *out = &d;
    return NN_OK;
}

int current_device(DeviceTables** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NN_ENODEV, "hipGetDevice: %s", hipGetErrorString(e));
    return ensure_device_current(dev, out);
}

struct Resolved {
    uint32_t block, grid, mulmod, unroll;
    bool nontemporal;
};

constexpr uint32_t kDefaultBlock = 256;
constexpr uint32_t kDefaultBlocksPerCU = 8;
constexpr uint32_t kDefaultUnroll = 4;

int resolve_cfg(const nn_launch_cfg* cfg, uint64_t count, int cus, Resolved* r) {
    nn_launch_cfg c = {0, 0, 0, 0, 0};
    if (cfg) c = *cfg;
    r->block = c.block ? c.block : kDefaultBlock;
    if (r->block < 64 || r->block > 1024 || r->block % 64)
        return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", r->block);
    if (c.grid) {
        r->grid = c.grid;
    } else {
        const uint64_t need = (count + r->block - 1) / r->block;
        const uint64_t cap = (uint64_t)(cus > 0 ? cus : 1) * kDefaultBlocksPerCU;
        r->grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
    }
    if ((uint64_t)r->grid * r->block > kMaxThreads)
        return fail(NN_EINVAL, "grid*block = %llu exceeds %llu threads",
                    (unsigned long long)r->grid * r->block, (unsigned long long)kMaxThreads);
    r->mulmod = c.mulmod ? c.mulmod : NN_MULMOD_FP64;
    if (r->mulmod > NN_MULMOD_MONTGOMERY) return fail(NN_EINVAL, "mulmod %u unknown", r->mulmod);
    r->unroll = c.unroll ? c.unroll : kDefaultUnroll;
    if (r->unroll != 1 && r->unroll != 2 && r->unroll != 4 && r->unroll != 8)
        return fail(NN_EINVAL, "unroll %u: must be 1, 2, 4 or 8", r->unroll);
    if (c.flags & ~NN_CFG_TEMPORAL_STORES) return fail(NN_EINVAL, "unknown flags 0x%x", c.flags);
    r->nontemporal = !(c.flags & NN_CFG_TEMPORAL_STORES);
    return NN_OK;
}

int check_out(uint64_t count, void* out) {
    if (count > UINT64_MAX / 8) return fail(NN_ERANGE, "count %llu: count*8 overflows",
                                            (unsigned long long)count);
    if (!out) return fail(NN_EINVAL, "output pointer is NULL");
    if ((uintptr_t)out % 8) return fail(NN_EINVAL, "output pointer %p is not 8-byte aligned", out);
    if ((uintptr_t)out > UINTPTR_MAX - count * 8)
        return fail(NN_ERANGE, "output range wraps the address space");
    return NN_OK;
}

}  // namespace

extern "C" {

int nn_seed(uint64_t index, uint64_t* state_out) {
    if (!state_out) return fail(NN_EINVAL, "state_out is NULL");
    if (index < NN_INDEX_MIN || index > NN_INDEX_MAX)
        return fail(NN_EINVAL, "index %llu outside [3^33+100, 2^53]", (unsigned long long)index);
    *state_out = h_seed(index);
    return ok();
}

int nn_skip(uint64_t state, uint64_t k, uint64_t* state_out) {
    if (!state_out) return fail(NN_EINVAL, "state_out is NULL");
    if (!valid_state(state))
        return fail(NN_EINVAL, "state %llu is not a unit modulo 3^33", (unsigned long long)state);
    *state_out = h_skip(state, k);
    return ok();
}

int nn_init(int device) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return fail(NN_ENODEV, "hipGetDevice: %s", hipGetErrorString(e));
    if (device != prev) {
        e = hipSetDevice(device);
        if (e != hipSuccess) return fail(NN_ENODEV, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
    }
    DeviceTables* d = nullptr;
    int st = ensure_device_current(device, &d);
    if (device != prev) (void)hipSetDevice(prev);
    return st == NN_OK ? ok() : st;
}

int nn_default_cfg(int kind, uint64_t count, nn_launch_cfg* cfg_out) {
    if (!cfg_out) return fail(NN_EINVAL, "cfg_out is NULL");
    if (kind != NN_OUT_U64 && kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %d unknown", kind);
    DeviceTables* d = nullptr;
    int st = current_device(&d);
    if (st) return st;
    Resolved r;
    st = resolve_cfg(nullptr, count, d->cus, &r);
    if (st) return st;
    cfg_out->block = r.block;
    cfg_out->grid = r.grid;
    cfg_out->mulmod = r.mulmod;
    cfg_out->unroll = r.unroll;
    cfg_out->flags = r.nontemporal ? 0u : NN_CFG_TEMPORAL_STORES;
    return ok();
}

int nn_generate_ex(uint64_t* state, uint64_t count, void* out_dev, int kind, void* stream,
                   const nn_launch_cfg* cfg) {
    if (!state) return fail(NN_EINVAL, "state is NULL");
    if (kind != NN_OUT_U64 && kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %d unknown", kind);
    const uint64_t s = *state;
    if (!valid_state(s))
        return fail(NN_EINVAL, "state %llu is not a unit modulo 3^33", (unsigned long long)s);
    if (count == 0) return ok();
    int st = check_out(count, out_dev);
    if (st) return st;
    DeviceTables* d = nullptr;
    st = current_device(&d);
    if (st) return st;
    Resolved r;
    st = resolve_cfg(cfg, count, d->cus, &r);
    if (st) return st;

    GenArgs a;
    a.out = (uint64_t*)out_dev;
    a.T = (uint64_t)r.grid * r.block;
    a.e_full = count / a.T;
    a.rem = (uint32_t)(count % a.T);
    a.base = h_mulmod(s, kMult);
    a.J = make_mult(MultPowers::get().pow(a.T));
    a.t_lo = d->t_lo;
    a.t_hi = d->t_hi;
    hipError_t e = launch_generate((int)r.mulmod, kind, (int)r.unroll, r.nontemporal, r.grid,
                                   r.block, (hipStream_t)stream, a);
    if (e != hipSuccess) return fail(NN_EHIP, "generate launch: %s", hipGetErrorString(e));
    *state = h_skip(s, count);
    return ok();
}

int nn_generate(uint64_t* state, uint64_t count, void* out_dev, int kind, void* stream) {
    return nn_generate_ex(state, count, out_dev, kind, stream, nullptr);
}

int nn_fill(uint64_t count, void* out_dev, uint64_t value, void* stream, const nn_launch_cfg* cfg) {
    if (count == 0) return ok();
    int st = check_out(count, out_dev);
    if (st) return st;
    DeviceTables* d = nullptr;
    st = current_device(&d);
    if (st) return st;
    Resolved r;
    st = resolve_cfg(cfg, count, d->cus, &r);
    if (st) return st;
    const uint64_t T = (uint64_t)r.grid * r.block;
    hipError_t e = launch_fill((int)r.unroll, r.nontemporal, r.grid, r.block, (hipStream_t)stream,
                               (uint64_t*)out_dev, T, count / T, (uint32_t)(count % T), value);
    if (e != hipSuccess) return fail(NN_EHIP, "fill launch: %s", hipGetErrorString(e));
    return ok();
}

const char* nn_strerror(int status) {
    switch (status) {
        case NN_OK: return "ok";
        case NN_EINVAL: return "invalid argument";
        case NN_ERANGE: return "count out of range";
        case NN_EHIP: return "HIP runtime error";
        case NN_ENOMEM: return "out of memory";
        case NN_ENODEV: return "no usable gfx950 device";
        default: return "unknown status";
    }
}

const char* nn_last_error(void) { return g_last_error.c_str(); }

const char* nn_version(void) { return "nn-alpha23 0.1.0 (gfx950)"; }

int nn_debug_mulmod(int mulmod, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t* out) {
    if (n && (!a || !b || !out)) return fail(NN_EINVAL, "NULL array");
    if (mulmod < NN_MULMOD_DEFAULT || mulmod > NN_MULMOD_MONTGOMERY)
        return fail(NN_EINVAL, "mulmod %d unknown", mulmod);
    for (uint64_t i = 0; i < n; ++i)
        if (!valid_state(a[i]) || !valid_state(b[i]))
            return fail(NN_EINVAL, "pair %llu is not a pair of units", (unsigned long long)i);
    for (uint64_t i = 0; i < n; ++i) {
        const Mult f = make_mult(b[i]);
        switch (mulmod) {
            case NN_MULMOD_DEFAULT:
            case NN_MULMOD_FP64: out[i] = VarFP64::to_u64(VarFP64::mul(VarFP64::load(a[i]), f)); break;
            case NN_MULMOD_BARRETT: out[i] = VarBarrett::mul(a[i], f); break;
            case NN_MULMOD_SHOUP: out[i] = VarShoup::mul(a[i], f); break;
            default: out[i] = VarMontgomery::mul(a[i], f); break;
        }
    }
    return ok();
}

}  // extern "C"
