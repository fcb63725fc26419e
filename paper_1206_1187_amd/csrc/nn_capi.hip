// nn_capi.hip -- the extern "C" entry points of include/nn.h for the plain
// and batched forms (the served form is in nn_server.hip).
//
// Host work per plain call: validate, pick the launch shape, compute
// base = state*2^53 and the jump multiplier with its reduction data, enqueue
// one kernel, and advance the caller's state by skip-ahead.  No allocation
// and no synchronisation happen on this path after the one-time per-device
// table upload.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "nn.h"
#include "nn_host.hpp"
#include "nn_internal.hpp"
#include "nn_kernels.hpp"

using namespace nn;

namespace nn {
const char* last_error();
}

namespace {

struct Resolved {
    uint32_t block, grid, mulmod, unroll, width, occupancy, ilp;
    bool nontemporal, flat, consec, strided;
    bool xcd_runs;  // flat, 4 rows: whole chunks in XCD runs (NN_CFG_ADDRESS_ORDER clears it)
    uint32_t lds;  // dynamic LDS bytes per workgroup that cap residency
};



// `out` may be NULL (query of the defaults): it is then taken as aligned.
// nn_fill resolves through the same function, so a fill and a generation
// with the same cfg store with the same pattern.
int resolve_cfg(const nn_launch_cfg* cfg, int kind, uint64_t count, const DeviceTables& d,
                const void* out, Resolved* r) {
    const int cus = d.cus;
    const KindDefaults& kd = kind_defaults(kind);
    nn_launch_cfg c = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cfg) c = *cfg;
    const bool aligned16 = ((uintptr_t)out % 16) == 0;
    const uint32_t known = NN_CFG_TEMPORAL_STORES | NN_CFG_ROWS | NN_CFG_FLAT | NN_CFG_CONSECUTIVE |
                           NN_CFG_PAPER_STRIDED | NN_CFG_NONTEMPORAL_STORES | NN_CFG_ADDRESS_ORDER;
    if (c.flags & ~known) return fail(NN_EINVAL, "unknown flags 0x%x", c.flags);
    r->xcd_runs = !(c.flags & NN_CFG_ADDRESS_ORDER);
    const uint32_t store_flags = c.flags & (NN_CFG_TEMPORAL_STORES | NN_CFG_NONTEMPORAL_STORES);
    if (store_flags == (NN_CFG_TEMPORAL_STORES | NN_CFG_NONTEMPORAL_STORES))
        return fail(NN_EINVAL, "NN_CFG_TEMPORAL_STORES and NN_CFG_NONTEMPORAL_STORES are exclusive");
    const uint32_t layouts =
        c.flags & (NN_CFG_ROWS | NN_CFG_FLAT | NN_CFG_CONSECUTIVE | NN_CFG_PAPER_STRIDED);
    if (layouts & (layouts - 1)) return fail(NN_EINVAL, "the layout flags are exclusive");
    r->nontemporal = !(c.flags & NN_CFG_TEMPORAL_STORES);
    r->consec = (c.flags & NN_CFG_CONSECUTIVE) != 0;
    r->strided = (c.flags & NN_CFG_PAPER_STRIDED) != 0;
    if ((c.flags & NN_CFG_ADDRESS_ORDER) && (r->consec || r->strided || (c.flags & NN_CFG_ROWS)))
        return fail(NN_EINVAL, "NN_CFG_ADDRESS_ORDER applies to the flat layout only");
    r->flat = false;
    if (r->strided) {
        // The paper's layout: E consecutive elements per thread, stored
        // transposed (out[t + i*T] = element t*E + i), 8-byte stores.
        r->mulmod = c.mulmod ? c.mulmod : (uint32_t)NN_MULMOD_MODBARRETT;
        if (r->mulmod != NN_MULMOD_MODBARRETT)
            return fail(NN_EINVAL, "the strided layout steps with NN_MULMOD_MODBARRETT only");
        if (c.occupancy || c.ilp > 1 || (c.width && c.width != 1) || c.grid)
            return fail(NN_EINVAL, "the strided layout takes block, unroll (elements per thread) "
                                   "and NN_CFG_TEMPORAL_STORES only");
        r->block = c.block ? c.block : 512u;
        if (r->block < 64 || r->block > 1024 || r->block % 64)
            return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", r->block);
        r->unroll = c.unroll ? c.unroll : 4096u;
        if (r->unroll == 0 || r->unroll > (1u << 20) || count % r->unroll)
            return fail(NN_EINVAL, "unroll %u: elements per thread must divide count (%llu)",
                        r->unroll, (unsigned long long)count);
        const uint64_t T = count / r->unroll;
        const uint64_t grid = (T + r->block - 1) / r->block;
        if (grid > 0x7fffffffull) return fail(NN_ERANGE, "too many threads");
        r->grid = (uint32_t)(grid ? grid : 1);
        r->width = 1;
        r->ilp = 1;
        r->occupancy = 0;
        r->lds = 0;
        return NN_OK;
    }
    if (r->consec) {
        // The paper's per-thread loop: Eq. 3's multiplier 2^53 with the
        // Modified Barrett step, serial order restored through LDS.
        r->mulmod = c.mulmod ? c.mulmod : (uint32_t)NN_MULMOD_MODBARRETT;
        if (r->mulmod != NN_MULMOD_MODBARRETT)
            return fail(NN_EINVAL, "the consecutive layout steps with NN_MULMOD_MODBARRETT only");
        if (c.occupancy) return fail(NN_EINVAL, "occupancy applies to the flat layout only");
        if (c.ilp > 1) return fail(NN_EINVAL, "ilp applies to the row layout only");
        r->occupancy = 0;
        r->lds = 0;
        r->ilp = 1;
        r->width = c.width ? c.width : (aligned16 ? 2u : 1u);
        if (r->width != 1 && r->width != 2)
            return fail(NN_EINVAL, "width %u: must be 1 or 2", r->width);
        if (r->width == 2 && !aligned16)
            return fail(NN_EINVAL, "width 2 needs a 16-byte aligned output (got %p)", out);
        // Defaults from a sweep on MI355X (2^30 f64 outputs): 512 threads
        // making 4 consecutive outputs each per tile, one workgroup per CU.
        r->block = c.block ? c.block : 512u;
        if (r->block < 64 || r->block > 1024 || r->block % 64)
            return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", r->block);
        r->unroll = c.unroll ? c.unroll : 4u;
        if (r->unroll < 2 || r->unroll > kConsecMaxE || (r->unroll & (r->unroll - 1)))
            return fail(NN_EINVAL, "unroll %u: the consecutive layout takes 2, 4, 8, 16 or 32",
                        r->unroll);
        if (consec_lds_bytes(r->block, r->unroll) > d.lds_per_block)
            return fail(NN_EINVAL, "block %u x unroll %u needs %u bytes of LDS (limit %u)",
                        r->block, r->unroll, consec_lds_bytes(r->block, r->unroll),
                        d.lds_per_block);
        const uint64_t per_tile = (uint64_t)r->block * r->unroll;
        const uint64_t max_grid = kMaxOffset / per_tile;
        if (c.grid) {
            if (c.grid > max_grid)
                return fail(NN_EINVAL, "grid %u: grid*block*unroll must not exceed 2^25", c.grid);
            r->grid = c.grid;
        } else {
            const uint64_t tiles = (count + per_tile - 1) / per_tile;
            uint64_t cap = (uint64_t)(cus > 0 ? cus : 1);
            if (cap > max_grid) cap = max_grid;
            r->grid = (uint32_t)(tiles < cap ? (tiles ? tiles : 1) : cap);
        }
        return NN_OK;
    }
    r->mulmod = c.mulmod ? c.mulmod : kd.mulmod;
    if (r->mulmod == NN_MULMOD_MODBARRETT)
        return fail(NN_EINVAL, "NN_MULMOD_MODBARRETT steps by 2^53 only: consecutive layout");
    if (r->mulmod > NN_MULMOD_MONTGOMERY) return fail(NN_EINVAL, "mulmod %u unknown", r->mulmod);
    // No layout flag: the flat layout unless the cfg sets a field only the
    // row layout has (block, grid, ilp, width 1; on an output that is only
    // 8-byte aligned any width, which asks for the row layout's stores); it
    // wrote faster than the row layout on every MI355X measured, for both
    // kinds (2^30 f64: 6.9 against 6.7 TB/s; 2^28 u64: 6.65 against 6.05).
    // An output that is only 8-byte aligned gets its first element from a
    // one-workgroup launch and the rest, 16-byte aligned, as usual; below
    // kFlatUnalignedMin outputs that extra launch costs more than the flat
    // layout gains, and such outputs keep the row layout (one launch).
    r->flat = (c.flags & NN_CFG_FLAT) != 0 ||
              (!(c.flags & NN_CFG_ROWS) && !c.block && !c.grid && !c.ilp &&
               (aligned16 ? c.width == 0 || c.width == 2
                          : c.width == 0 && count >= kFlatUnalignedMin));
    if ((c.flags & NN_CFG_ADDRESS_ORDER) && !r->flat)
        return fail(NN_EINVAL, "NN_CFG_ADDRESS_ORDER applies to the flat layout only");
    r->occupancy = c.occupancy ? c.occupancy : (r->flat ? kFlatDefaultOccupancy : 0u);
    r->lds = 0;
    if (r->occupancy) {
        if (r->occupancy < 2 || r->occupancy > 16)
            return fail(NN_EINVAL, "occupancy %u: must be 0 or in [2, 16]", r->occupancy);
        const uint32_t unit = 512;
        r->lds = (d.lds_per_cu / (r->occupancy + 1) / unit + 1) * unit;
        if (r->lds > d.lds_per_block || (uint64_t)r->lds * r->occupancy > d.lds_per_cu)
            return fail(NN_EINVAL, "occupancy %u not expressible on this device", r->occupancy);
    }
    if (r->flat) {
        if ((c.block && c.block != kFlatBlock) || c.grid || (c.width && c.width != 2))
            return fail(NN_EINVAL, "the flat layout has a fixed shape (block 256, width 2)");
        if (c.ilp > 1) return fail(NN_EINVAL, "ilp applies to the row layout only");
        r->block = kFlatBlock;
        r->width = 2;
        r->ilp = 1;
        // rows per workgroup; temporal stores unless asked otherwise (the
        // measured best, see kFlatDefaultRows)
        r->unroll = c.unroll ? c.unroll : kFlatDefaultRows;
        if (r->unroll == 0 || r->unroll > kFlatMaxRows || (r->unroll & (r->unroll - 1)))
            return fail(NN_EINVAL, "unroll %u: the flat layout writes 1, 2, 4, 8 or 16 rows "
                                   "per workgroup", r->unroll);
        if (!store_flags) r->nontemporal = false;
        if (r->unroll != 4) r->xcd_runs = false;
        const uint64_t chunk = count < kFlatMaxCount ? count : kFlatMaxCount;
        const uint64_t per = (uint64_t)kFlatPerBlock * r->unroll;
        r->grid = (uint32_t)((chunk + per - 1) / per);
        if (!r->grid) r->grid = 1;
        return NN_OK;
    }
    r->width = c.width ? c.width : (aligned16 ? 2u : 1u);
    if (r->width != 1 && r->width != 2)
        return fail(NN_EINVAL, "width %u: must be 1 or 2", r->width);
    if (r->width == 2 && !aligned16)
        return fail(NN_EINVAL, "width 2 needs a 16-byte aligned output (got %p)", out);
    r->block = c.block ? c.block : kDefaultBlock;
    if (r->block < 64 || r->block > 1024 || r->block % 64)
        return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", r->block);
    if (c.grid) {
        r->grid = c.grid;
    } else {
        const uint64_t per_block = (uint64_t)r->block * r->width;
        const uint64_t need = (count + per_block - 1) / per_block;
        uint64_t cap = (uint64_t)(cus > 0 ? cus : 1) * kd.grid_num / kd.grid_den;
        if (cap == 0) cap = 1;
        r->grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
    }
    if ((uint64_t)r->grid * r->block > kMaxThreads)
        return fail(NN_EINVAL, "grid*block = %llu exceeds %llu threads",
                    (unsigned long long)r->grid * r->block, (unsigned long long)kMaxThreads);
    r->unroll = c.unroll ? c.unroll : kd.unroll;
    if (r->unroll != 1 && r->unroll != 2 && r->unroll != 4 && r->unroll != 8)
        return fail(NN_EINVAL, "unroll %u: must be 1, 2, 4 or 8", r->unroll);
    r->ilp = c.ilp ? c.ilp : (r->width == 2 ? kd.ilp : 1u);
    if (r->ilp != 1 && r->ilp != 2 && r->ilp != 4)
        return fail(NN_EINVAL, "ilp %u: must be 1, 2 or 4", r->ilp);
    if (r->ilp > 1 && r->width != 2) return fail(NN_EINVAL, "ilp > 1 needs width 2");
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

int nn_dev_mult_pow(uint64_t k, nn_dev_mult* out) {
    if (!out) return fail(NN_EINVAL, "out is NULL");
    const Mult m = make_mult(h_skip(1, k));
    out->v = m.v;
    out->qh = m.qh;
    out->ql = m.ql;
    return ok();
}

int nn_dev_skip_table(const nn_dev_mult** table_out) {
    if (!table_out) return fail(NN_EINVAL, "table_out is NULL");
    DeviceTables* d = nullptr;
    const int st = current_device(&d);
    if (st != NN_OK) return st;
    *table_out = reinterpret_cast<const nn_dev_mult*>(d->t8);
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
    int st = current_device(&d);
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
    st = resolve_cfg(nullptr, kind, count, *d, nullptr, &r);
    if (st) return st;
    cfg_out->width = r.width;
    cfg_out->block = r.block;
    cfg_out->grid = r.grid;
    cfg_out->mulmod = r.mulmod;
    cfg_out->unroll = r.unroll;
    cfg_out->occupancy = r.occupancy;
    cfg_out->ilp = r.ilp;
    cfg_out->flags = (r.nontemporal ? 0u : NN_CFG_TEMPORAL_STORES) |
                     (r.flat ? NN_CFG_FLAT : NN_CFG_ROWS);
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
    st = resolve_cfg(cfg, kind, count, *d, out_dev, &r);
    if (st) return st;

    if (r.strided) {
        hipError_t e = launch_generate_strided(kind, r.nontemporal, r.grid, r.block,
                                               (hipStream_t)stream, (uint64_t*)out_dev,
                                               count / r.unroll, r.unroll, h_mulmod(s, kMult),
                                               d->t_sk);
        if (e != hipSuccess) return fail(NN_EHIP, "generate launch: %s", hipGetErrorString(e));
        *state = h_skip(s, count);
        return ok();
    }
    if (r.consec) {
        ConsecArgs ca;
        ca.out = (uint64_t*)out_dev;
        ca.count = count;
        ca.base = h_mulmod(s, kMult);
        ca.J = make_mult(MultPowers::get().pow((uint64_t)r.grid * r.block * r.unroll));
        ca.t_lo = d->t_lo;
        ca.t_hi = d->t_hi;
        hipError_t e = launch_generate_consec(kind, (int)r.unroll, (int)r.width, r.nontemporal,
                                              r.grid, r.block, (hipStream_t)stream, ca);
        if (e != hipSuccess) return fail(NN_EHIP, "generate launch: %s", hipGetErrorString(e));
        *state = h_skip(s, count);
        return ok();
    }
    if (r.flat) {
        FlatArgs f;
        f.M1 = make_mult(kMult);
        f.J = make_mult(MultPowers::get().pow(kFlatPerBlock));
        f.xcd_runs = r.xcd_runs;
        // an output that is only 8-byte aligned: its first element alone
        // (the tail kernel with one output), then the 16-byte aligned rest
        const uint64_t head = ((uintptr_t)out_dev % 16) ? 1 : 0;
        if (head) {
            f.out = (uint64_t*)out_dev;
            f.count = 1;
            f.base = f.mid_base = f.tail_base = h_skip(s, 1);
            hipError_t e = launch_generate_flat((int)r.mulmod, kind, r.nontemporal, (int)r.unroll,
                                                r.lds, (hipStream_t)stream, f);
            if (e != hipSuccess)
                return fail(NN_EHIP, "generate launch: %s", hipGetErrorString(e));
        }
        for (uint64_t off = head; off < count; off += kFlatMaxCount) {
            const uint64_t n = count - off < kFlatMaxCount ? count - off : kFlatMaxCount;
            f.out = (uint64_t*)out_dev + off;
            f.count = n;
            f.base = h_skip(s, off + 1);  // the first output of this chunk
            const uint64_t per = (uint64_t)kFlatPerBlock * r.unroll;
            f.mid_base = h_skip(f.base, flat_run_chunks((int)r.unroll, r.xcd_runs, n / per) * per);
            f.tail_base = h_skip(f.base, n / per * per);
            hipError_t e = launch_generate_flat((int)r.mulmod, kind, r.nontemporal, (int)r.unroll,
                                                r.lds, (hipStream_t)stream, f);
            if (e != hipSuccess)
                return fail(NN_EHIP, "generate launch: %s", hipGetErrorString(e));
        }
        *state = h_skip(s, count);
        return ok();
    }
    if (r.lds)
        return fail(NN_EINVAL, "occupancy applies to the flat layout only");

    GenArgs a;
    a.out = (uint64_t*)out_dev;
    a.T = (uint64_t)r.grid * r.block;
    const uint64_t row = a.T * r.width;
    a.e_full = count / row;
    a.rem = (uint32_t)(count % row);
    a.base = h_mulmod(s, kMult);
    const uint64_t jump = MultPowers::get().pow(row);
    a.J = make_mult(jump);
    a.M1 = make_mult(kMult);
    a.JI = make_mult(MultPowers::get().pow(row * r.ilp));
    a.t_lo = d->t_lo;
    a.t_hi = d->t_hi;
    hipError_t e = launch_generate((int)r.mulmod, kind, (int)r.width, (int)r.unroll, (int)r.ilp,
                                   r.nontemporal, r.grid, r.block, (hipStream_t)stream, a);
    if (e != hipSuccess) return fail(NN_EHIP, "generate launch: %s", hipGetErrorString(e));
    *state = h_skip(s, count);
    return ok();
}

int nn_generate(uint64_t* state, uint64_t count, void* out_dev, int kind, void* stream) {
    return nn_generate_ex(state, count, out_dev, kind, stream, nullptr);
}

int nn_consume(uint64_t* state, uint64_t count, int kind, void* result_dev, void* stream,
               const nn_launch_cfg* cfg) {
    if (!state) return fail(NN_EINVAL, "state is NULL");
    if (kind != NN_OUT_U64 && kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %d unknown", kind);
    const uint64_t s = *state;
    if (!valid_state(s))
        return fail(NN_EINVAL, "state %llu is not a unit modulo 3^33", (unsigned long long)s);
    if (count == 0) return ok();
    if (!result_dev || (uintptr_t)result_dev % 8)
        return fail(NN_EINVAL, "result pointer %p must be non-NULL and 8-byte aligned", result_dev);
    DeviceTables* d = nullptr;
    int st = current_device(&d);
    if (st) return st;
    nn_launch_cfg c = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cfg) c = *cfg;
    if (c.flags || c.occupancy || (c.width && c.width != 2) || (c.ilp && c.ilp != 2) || c.unroll)
        return fail(NN_EINVAL, "nn_consume takes block, grid and mulmod only");
    const KindDefaults& kd = kind_defaults(NN_OUT_F64);
    const uint32_t block = c.block ? c.block : kDefaultBlock;
    if (block < 64 || block > 1024 || block % 64)
        return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", block);
    const uint32_t mulmod = c.mulmod ? c.mulmod : kd.mulmod;
    if (mulmod > NN_MULMOD_MONTGOMERY)
        return fail(NN_EINVAL, "mulmod %u: nn_consume takes FP64, Barrett, Shoup or Montgomery",
                    mulmod);
    uint32_t grid = c.grid;
    if (!grid) {
        // No stores to keep sequential: fill the device.
        const uint64_t need = (count + 2ull * block - 1) / (2ull * block);
        const uint64_t cap = (uint64_t)(d->cus > 0 ? d->cus : 1) * 8;
        grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
    }
    if ((uint64_t)grid * block > kMaxThreads)
        return fail(NN_EINVAL, "grid*block exceeds %llu threads", (unsigned long long)kMaxThreads);
    GenArgs a;
    a.out = nullptr;
    a.T = (uint64_t)grid * block;
    const uint64_t row = 2 * a.T;
    a.e_full = count / row;
    a.rem = (uint32_t)(count % row);
    a.base = h_mulmod(s, kMult);
    const uint64_t jump = MultPowers::get().pow(row);
    a.J = make_mult(jump);
    a.M1 = make_mult(kMult);
    a.JI = make_mult(MultPowers::get().pow(2 * row));
    a.t_lo = d->t_lo;
    a.t_hi = d->t_hi;
    hipError_t e = launch_consume((int)mulmod, kind, grid, block, (hipStream_t)stream, a, result_dev);
    if (e != hipSuccess) return fail(NN_EHIP, "consume launch: %s", hipGetErrorString(e));
    *state = h_skip(s, count);
    return ok();
}

int nn_fill(uint64_t count, void* out_dev, uint64_t value, void* stream, const nn_launch_cfg* cfg) {
    if (count == 0) return ok();
    int st = check_out(count, out_dev);
    if (st) return st;
    DeviceTables* d = nullptr;
    st = current_device(&d);
    if (st) return st;
    nn_launch_cfg c;
    memset(&c, 0, sizeof c);
    if (cfg) c = *cfg;
    const bool with_start = (c.flags & NN_FILL_WITH_START) != 0;
    c.flags &= ~NN_FILL_WITH_START;
    Resolved r;
    st = resolve_cfg(&c, NN_OUT_F64, count, *d, out_dev, &r);
    if (st) return st;
    if (r.consec || r.strided) return fail(NN_EINVAL, "nn_fill has no consecutive layout");
    if (with_start && !r.flat) return fail(NN_EINVAL, "NN_FILL_WITH_START needs the flat layout");
    if (r.flat) {
        // as nn_generate: an 8-byte aligned output's first element alone
        const uint64_t head = ((uintptr_t)out_dev % 16) ? 1 : 0;
        if (head) {
            hipError_t e = launch_fill_flat(r.nontemporal, (int)r.unroll, r.lds,
                                            (hipStream_t)stream, with_start, r.xcd_runs,
                                            (uint64_t*)out_dev, 1, value);
            if (e != hipSuccess) return fail(NN_EHIP, "fill launch: %s", hipGetErrorString(e));
        }
        for (uint64_t off = head; off < count; off += kFlatMaxCount) {
            const uint64_t n = count - off < kFlatMaxCount ? count - off : kFlatMaxCount;
            hipError_t e = launch_fill_flat(r.nontemporal, (int)r.unroll, r.lds,
                                            (hipStream_t)stream, with_start, r.xcd_runs,
                                            (uint64_t*)out_dev + off, n, value);
            if (e != hipSuccess) return fail(NN_EHIP, "fill launch: %s", hipGetErrorString(e));
        }
        return ok();
    }
    if (r.lds) return fail(NN_EINVAL, "occupancy applies to the flat layout only");
    const uint64_t T = (uint64_t)r.grid * r.block;
    const uint64_t row = T * r.width;
    hipError_t e = launch_fill((int)r.width, (int)r.unroll, r.nontemporal, r.grid, r.block,
                               (hipStream_t)stream, (uint64_t*)out_dev, T, count / row,
                               (uint32_t)(count % row), value);
    if (e != hipSuccess) return fail(NN_EHIP, "fill launch: %s", hipGetErrorString(e));
    return ok();
}

int nn_batch_plan_create(int kind, uint32_t max_streams, uint64_t max_outputs,
                         const nn_batch_cfg* cfg, nn_batch_plan** plan_out) {
    int st = plan_create(kind, max_streams, max_outputs, cfg, false, nullptr, nullptr, plan_out);
    return st == NN_OK ? ok() : st;
}

int nn_batch_plan_destroy(nn_batch_plan* plan) {
    if (plan) plan_release(plan);
    return ok();
}

int nn_batch_plan_cfg(const nn_batch_plan* plan, nn_batch_cfg* cfg_out) {
    if (!plan || !cfg_out) return fail(NN_EINVAL, "NULL argument");
    cfg_out->block = plan->block;
    cfg_out->grid = plan->grid;
    cfg_out->cluster = plan->cluster;
    cfg_out->mulmod = plan->mulmod;
    cfg_out->flags = (plan->nontemporal ? 0u : NN_CFG_TEMPORAL_STORES) |
                     (plan->use_graph ? 0u : NN_BATCH_NO_GRAPH) |
                     (plan->interleaved ? NN_BATCH_INTERLEAVED : 0u) |
                     (plan->chunks ? NN_BATCH_CHUNKS : 0u);
    cfg_out->occupancy = plan->chunks ? plan->occupancy : 0u;
    return ok();
}

int nn_generate_batch(nn_batch_plan* plan, const nn_stream_desc* descs, uint32_t n, void* out_dev,
                      void* stream, uint64_t* final_states) {
    if (!plan) return fail(NN_EINVAL, "plan is NULL");
    if (plan->indexed) return fail(NN_EINVAL, "plan belongs to a server");
    if (n && !descs) return fail(NN_EINVAL, "descs is NULL");
    uint64_t total = 0, pieces = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const nn_stream_desc& q = descs[i];
        if (!valid_state(q.state))
            return fail(NN_EINVAL, "stream %u: state %llu is not a unit modulo 3^33", i,
                        (unsigned long long)q.state);
        if (q.length > UINT64_MAX / 8 || q.out_offset > UINT64_MAX / 8 - q.length)
            return fail(NN_ERANGE, "stream %u: output range overflows", i);
        total += q.length;
        if (total < q.length) return fail(NN_ERANGE, "total outputs overflow");
        pieces += (q.length + kBatchMaxLen - 1) / kBatchMaxLen;
    }
    if (total) {
        if (!out_dev) return fail(NN_EINVAL, "output pointer is NULL");
        if ((uintptr_t)out_dev % 16)
            return fail(NN_EINVAL, "batch output %p must be 16-byte aligned", out_dev);
    }
    if (n > plan->max_streams)
        return fail(NN_ERANGE, "batch of %u streams, plan holds %u", n, plan->max_streams);
    if (total > plan->max_outputs)
        return fail(NN_ERANGE, "batch of %llu outputs, plan holds %llu", (unsigned long long)total,
                    (unsigned long long)plan->max_outputs);
    if (pieces > plan->cap_desc)
        return fail(NN_ERANGE, "batch needs %llu stream pieces, plan holds %u",
                    (unsigned long long)pieces, plan->cap_desc);
    std::lock_guard<std::mutex> lock(plan->mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
        return fail(NN_EINVAL, "plan belongs to device %d, current device is %d", plan->device, dev);
    if (total == 0) {
        if (final_states)
            for (uint32_t i = 0; i < n; ++i) final_states[i] = descs[i].state;
        return ok();
    }
    int st = plan_wait(plan);
    if (st) return st;
    BatchDesc* dd = plan_staged_descs(plan);
    uint32_t nd = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const nn_stream_desc& q = descs[i];
        for (uint64_t off = 0; off < q.length; off += kBatchMaxLen) {
            const uint64_t len = q.length - off < kBatchMaxLen ? q.length - off : kBatchMaxLen;
            dd[nd].src = q.state;  // the device skips ahead by pos
            dd[nd].pos = off % kPeriod;
            dd[nd].len = len;
            dd[nd].out_off = q.out_offset + off;
            ++nd;
        }
    }
    st = plan_launch_staged(plan, nd, out_dev, (hipStream_t)stream);
    if (st) return st;
    if (final_states)
        for (uint32_t i = 0; i < n; ++i) final_states[i] = h_skip(descs[i].state, descs[i].length);
    return ok();
}

int nn_generate_batch_static(const nn_stream_desc* descs, uint32_t n, void* out_dev, int kind,
                             void* stream, uint64_t* final_states) {
    if (kind != NN_OUT_U64 && kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %d unknown", kind);
    if (n && !descs) return fail(NN_EINVAL, "descs is NULL");
    if (n > kStaticMaxStreams)
        return fail(NN_ERANGE, "batch of %u streams, the static workspace holds %u", n,
                    kStaticMaxStreams);
    uint64_t total = 0, records = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const nn_stream_desc& q = descs[i];
        if (!valid_state(q.state))
            return fail(NN_EINVAL, "stream %u: state %llu is not a unit modulo 3^33", i,
                        (unsigned long long)q.state);
        if (q.length > kStaticMaxOutputs)
            return fail(NN_ERANGE, "stream %u: %llu outputs, the static workspace holds %llu", i,
                        (unsigned long long)q.length, (unsigned long long)kStaticMaxOutputs);
        if (q.length && q.out_offset > (1ull << 51) - q.length)
            return fail(NN_ERANGE, "stream %u: output indices reach 2^51", i);
        total += q.length;
        if (total > kStaticMaxOutputs)
            return fail(NN_ERANGE, "batch of more than %llu outputs",
                        (unsigned long long)kStaticMaxOutputs);
        if (q.length)
            records += (q.length + (q.out_offset & (kChunkOuts - 1)) + kChunkOuts - 1) / kChunkOuts;
    }
    if (total) {
        if (!out_dev) return fail(NN_EINVAL, "output pointer is NULL");
        if ((uintptr_t)out_dev % 16)
            return fail(NN_EINVAL, "batch output %p must be 16-byte aligned", out_dev);
    }
    DeviceTables* d = nullptr;
    int st = current_device(&d);
    if (st) return st;
    if (total == 0) {
        if (final_states)
            for (uint32_t i = 0; i < n; ++i) final_states[i] = descs[i].state;
        return ok();
    }
    if (records > kStaticMaxRecords)  // cannot happen within the limits above
        return fail(NN_ERANGE, "batch of %llu chunk records", (unsigned long long)records);
    const hipStream_t s = (hipStream_t)stream;
    char* ws = static_cast<char*>(d->scratch);
    // the caller's descriptors, then the descriptors and header the kernels read
    hipError_t e = hipMemcpyAsync(ws + kStaticRawOff, descs, (size_t)n * sizeof(nn_stream_desc),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_static_descs(s, ws, n, static_cast<uint64_t*>(out_dev));
    // the chunked plan's arguments (nn_runtime.hip, slot_create) over the static workspace
    BatchArgs a;
    memset(&a, 0, sizeof a);
    a.ws = reinterpret_cast<const BatchHeader*>(ws);
    a.JB = make_mult(MultPowers::get().pow(kFlatPerBlock));
    a.Minv = make_mult(MultPowers::get().pow(kPeriod - 1));
    a.t_lo = d->t_lo;
    a.t_hi = d->t_hi;
    a.t_sk = d->t_sk;
    a.rec = reinterpret_cast<RowRec*>(ws + kStaticRecOff);
    a.row_outs = kChunkOuts;
    a.grid = 1;
    a.cluster = 1;
    a.block = kFlatBlock;
    a.JR = make_mult(MultPowers::get().pow((uint64_t)kChunkOuts * 256));
    a.n_rec = records;
    a.out = static_cast<uint64_t*>(out_dev);
    uint32_t lds = (d->lds_per_cu / (kFlatDefaultOccupancy + 1) / 512 + 1) * 512;
    if (lds > d->lds_per_block) lds = 0;
    void* params[] = {&a};
    // the record pre-pass: a workgroup per window
    if (e == hipSuccess)
        e = hipLaunchKernel(batch_rec_kernel(false), dim3(n > 65535 ? 65535u : n), dim3(256),
                            params, 0, s);
    if (e == hipSuccess)
        e = hipLaunchKernel(batch_chunks_kernel(kind, true), dim3((uint32_t)records),
                            dim3(kFlatBlock), params, lds, s);
    if (e != hipSuccess) return fail(NN_EHIP, "static batch launch: %s", hipGetErrorString(e));
    if (final_states)
        for (uint32_t i = 0; i < n; ++i) final_states[i] = h_skip(descs[i].state, descs[i].length);
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
        case NN_ECANCELED: return "request cancelled";
        default: return "unknown status";
    }
}

const char* nn_last_error(void) { return last_error(); }

const char* nn_version(void) { return "nn-alpha23 0.1.0 (gfx950)"; }

int nn_debug_mulmod(int mulmod, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t* out) {
    if (n && (!a || !b || !out)) return fail(NN_EINVAL, "NULL array");
    if ((mulmod < NN_MULMOD_DEFAULT || mulmod > NN_MULMOD_MODBARRETT) &&
        mulmod != NN_DEBUG_DEVICE_MULMOD)
        return fail(NN_EINVAL, "mulmod %d unknown", mulmod);
    for (uint64_t i = 0; i < n; ++i)
        if (!valid_state(a[i]) || !valid_state(b[i]))
            return fail(NN_EINVAL, "pair %llu is not a pair of units", (unsigned long long)i);
    if (mulmod == NN_MULMOD_MODBARRETT) {
        for (uint64_t i = 0; i < n; ++i)
            if (b[i] != kMult)
                return fail(NN_EINVAL, "NN_MULMOD_MODBARRETT multiplies by 2^53 only (pair %llu)",
                            (unsigned long long)i);
        for (uint64_t i = 0; i < n; ++i) out[i] = mm_modbarrett_step(a[i]);
        return ok();
    }
    for (uint64_t i = 0; i < n; ++i) {
        const Mult f = make_mult(b[i]);
        switch (mulmod) {
            case NN_MULMOD_DEFAULT:
            case NN_MULMOD_FP64: out[i] = VarFP64::to_u64(VarFP64::mul(VarFP64::load(a[i]), f)); break;
            case NN_DEBUG_DEVICE_MULMOD:
                out[i] = (uint64_t)nn_dev_mulmod((double)a[i], nn_dev_mult{f.v, f.qh, f.ql});
                break;
            case NN_MULMOD_BARRETT: out[i] = VarBarrett::mul(a[i], f); break;
            case NN_MULMOD_SHOUP: out[i] = VarShoup::mul(a[i], f); break;
            default: out[i] = VarMontgomery::mul(a[i], f); break;
        }
    }
    return ok();
}

}  // extern "C"
