// nn_batch.hip -- persistent kernel of the batched form.
//
// The batch is a sequence of rows of 2*block outputs (each window cut into
// ceil((len + s)/(2*block)) rows, s = 1 for windows at odd output offsets).
// Workgroup w processes the contiguous row range
// [n_rows*w/grid, n_rows*(w+1)/grid): inside a window it keeps stepping its
// lanes' states by (2^53)^(2*block) per row, exactly as the plain row
// kernel, and it skips ahead afresh only when it enters a new window.  Lane
// l owns the aligned output pair (x_a, x_b) of each row; pairs are aligned
// to the global output index, so the 16-byte stores stay aligned for any
// window offset (a window at an odd offset starts, and may end, with a half
// pair).  Element x of a window is src * (2^53)^(pos + x + 1).
#include <hip/hip_runtime.h>

#include "nn_batch.hpp"
#include "nn_device.hpp"
#include "nn_skip.hpp"

namespace nn {

// A descriptor read through the scalar unit, field by field.
__device__ __forceinline__ BatchDesc load_desc(const_ptr<BatchDesc> p) {
    BatchDesc D;
    D.src = p->src;
    D.pos = p->pos;
    D.len = p->len;
    D.out_off = p->out_off;
    D.row_start = p->row_start;
    return D;
}

// Stores row r's pair of lane l: x_b = 2(jr*B + l) + 1 - s, x_a = x_b - 1.
// `full` (uniform) says every pair of the row lies inside the window.
template <class V, int KIND, bool NT>
__device__ __forceinline__ void store_pair(global_ptr<uint64_t> out, const BatchDesc& D,
                                           uint64_t xb, typename V::S za, typename V::S zb,
                                           bool full) {
    const global_ptr<uint64_t> p = out + (D.out_off + xb - 1);  // global index of x_a, even
    if (full) {
        u64x2 v;
        v.x = out_bits<V, KIND>(za);
        v.y = out_bits<V, KIND>(zb);
        put<NT>(reinterpret_cast<global_ptr<u64x2>>(p), v);
        return;
    }
    const bool vb = xb < D.len;
    const bool va = xb >= 1 && xb - 1 < D.len;
    if (va && vb) {
        u64x2 v;
        v.x = out_bits<V, KIND>(za);
        v.y = out_bits<V, KIND>(zb);
        put<NT>(reinterpret_cast<global_ptr<u64x2>>(p), v);
    } else if (vb) {
        put<NT>(p + 1, out_bits<V, KIND>(zb));
    } else if (va) {
        put<NT>(p, out_bits<V, KIND>(za));
    }
}

// The window holding row r, given a window d at or before it (row_start
// of d <= r): each lane of the wavefront reads the first row of one of the
// next 64 windows, and a ballot finds the first that starts past r, so a
// member of a cluster passes windows it has no rows in 64 per load instead
// of one dependent load each.  Wave-uniform result.
__device__ __forceinline__ uint32_t window_of(const_ptr<BatchDesc> desc, uint32_t n_desc,
                                              uint32_t d, uint64_t r) {
    const uint32_t lane = threadIdx.x & 63u;
    for (;;) {
        const uint32_t cand = d + 1 + lane;
        const bool past = cand >= n_desc || desc[cand].row_start > r;
        const uint64_t mask = __ballot(past);
        if (mask) return d + (uint32_t)(__ffsll((unsigned long long)mask) - 1);
        d += 64;
    }
}

template <class V, int KIND>
__device__ __forceinline__ u64x2 pair_bits(typename V::S za, typename V::S zb) {
    u64x2 v;
    v.x = out_bits<V, KIND>(za);
    v.y = out_bits<V, KIND>(zb);
    return v;
}

// Workgroups form clusters of `cluster` consecutive workgroups; cluster c
// takes the contiguous row range [n_rows*c/C, n_rows*(c+1)/C) of the C =
// grid/cluster clusters, and member i of the cluster takes its rows
// r0 + i, r0 + i + cluster, ...  Each window met is one segment: a fresh
// skip-ahead, then the member's rows of that window in three parts -- the
// partial first row of a window at an odd output offset, a branch-free loop
// over full rows with two rows (four chains) in flight, and the window's
// partial last row.
template <class V, int KIND, bool NT, bool INDEXED>
__device__ __forceinline__ void batch_body(const BatchArgs& a, const const_ptr<BatchHeader> hdr) {
    const uint32_t n_desc = hdr->n_desc;
    const uint64_t n_rows = hdr->n_rows;
    const global_ptr<uint64_t> out = as_global(hdr->out);
    const const_ptr<BatchDesc> desc = reinterpret_cast<const_ptr<BatchDesc>>(hdr + 1);
    const uint32_t B = blockDim.x;
    const uint32_t l = threadIdx.x;
    const uint32_t K = a.cluster;
    const uint32_t n_clusters = gridDim.x / K;
    const uint32_t c = blockIdx.x / K;
    const uint32_t i = blockIdx.x % K;
    const uint64_t r1 = n_rows * (c + 1) / n_clusters;
    uint64_t r = n_rows * c / n_clusters + i;
    if (r >= r1 || n_desc == 0) return;
    // The last window whose first row is at or before r (binary search).
    uint32_t lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (desc[mid].row_start <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    uint32_t d = lo;
    const uint64_t BK = (uint64_t)B * K;  // pairs from one of the member's rows to the next
    uint64_t next_start = d + 1 < n_desc ? desc[d + 1].row_start : n_rows;
    while (r < r1) {
        if (r >= next_start) {
            d = window_of(desc, n_desc, d, r);
            next_start = d + 1 < n_desc ? desc[d + 1].row_start : n_rows;
        }
        const BatchDesc D = load_desc(desc + d);
        const uint64_t seg_end = next_start < r1 ? next_start : r1;
        const uint32_t s = (uint32_t)(D.out_off & 1u);
        // Row j of the window covers its elements [2 j B - s, 2 (j + 1) B - s);
        // lane l owns x_a = x_b - 1 and x_b = 2 (j B + l) + 1 - s.
        uint64_t j = r - D.row_start;
        const uint64_t j_end = seg_end - D.row_start;
        uint64_t xb = 2ull * (j * B + l) + 1 - s;
        // src * (2^53)^(pos + x_b + 1): the window's element x_b.
        typename V::S zb;
        if constexpr (INDEXED)
            zb = skip_any<V>(as_const(hdr->states)[D.src], D.pos + xb + 1, a.t_sk);
        else
            zb = skip_any<V>(D.src, D.pos + xb + 1, a.t_sk);
        typename V::S za = V::mul(zb, a.Minv);
        if (j < s) {  // row 0 of a window at an odd offset starts with a half pair
            store_pair<V, KIND, NT>(out, D, xb, za, zb, false);
            za = V::mul(za, a.JB);
            zb = V::mul(zb, a.JB);
            j += K;
            xb += 2 * BK;
        }
        // Rows below j_full lie wholly inside the window.
        const uint64_t j_full = (D.len + s) / (2ull * B);
        const uint64_t j_stop = j_full < j_end ? j_full : j_end;
        if (j < j_stop) {
            uint64_t m = (j_stop - j + K - 1) / K;  // the member's full rows
            global_ptr<u64x2> p = reinterpret_cast<global_ptr<u64x2>>(out + (D.out_off + xb - 1));
            typename V::S zc = V::mul(za, a.JB), zd = V::mul(zb, a.JB);
            j += m * K;
            xb += 2 * BK * m;
            for (; m >= 2; m -= 2) {
                // each row's store next to its own multiplications (as in
                // the plain row kernel: bunched stores write slower)
                put<NT>(p, pair_bits<V, KIND>(za, zb));
                za = V::mul(za, a.JB2);
                zb = V::mul(zb, a.JB2);
                __builtin_amdgcn_sched_barrier(0);
                put<NT>(p + BK, pair_bits<V, KIND>(zc, zd));
                zc = V::mul(zc, a.JB2);
                zd = V::mul(zd, a.JB2);
                __builtin_amdgcn_sched_barrier(0);
                p += 2 * BK;
            }
            if (m) {
                put<NT>(p, pair_bits<V, KIND>(za, zb));
                za = zc;
                zb = zd;
            }
        }
        // The window's last row when it ends inside a row.
        while (j < j_end) {
            store_pair<V, KIND, NT>(out, D, xb, za, zb, false);
            za = V::mul(za, a.JB);
            zb = V::mul(zb, a.JB);
            j += K;
            xb += 2 * BK;
        }
        r = D.row_start + j;
    }
}

// The batch read from the device workspace, written before the launch:
// scalar loads.
template <class V, int KIND, bool NT, bool INDEXED>
__global__ __launch_bounds__(1024) void k_batch(BatchArgs a) {
    batch_body<V, KIND, NT, INDEXED>(a, as_const(a.ws));
}

// A small batch carried in the kernel arguments: no upload before the
// launch, so its latency is that of a plain launch.
template <class V, int KIND, bool NT, bool INDEXED>
__global__ __launch_bounds__(1024) void k_batch_inline(BatchArgs a, BatchInline in) {
    batch_body<V, KIND, NT, INDEXED>(a, as_const(&in.hdr));
}

// Pre-pass of the interleaved kernel: every row's record, stored where its
// workgroup of the row kernel reads it.  Its rows are
// aligned to the output: row j of a window at output offset o covers
// outputs [W (floor(o / W) + j), W (floor(o / W) + j + 1)), W = 2*kIlPairs*block,
// which are its elements W j - s + k, k < W, with s = o mod W.  (Adjacent
// rows go to different workgroups, and rows that shared a cache line would
// leave partial lines in two L2s.)  Workgroups take windows d = blockIdx.x,
// + gridDim.x, ...; thread t of 256 takes the window's rows t, t + 256, ...:
// one skip-ahead to its first row, then a step of (2^53)^(W*256) per row.
//
// The chunked kernel's owned mode (kChunkOwned) numbers records by chunk:
// record k of the window's chunk j is k + j, k from the descriptor, and a
// record goes to the chunk array only if its chunk is the window's own
// first (its first chunk does not hold an earlier window's end), or a later
// chunk of the window; every window's first-chunk record also goes to ext,
// where the workgroup of a chunk that windows share finds them.  An empty
// window gets an empty ext record.
template <bool INDEXED>
__global__ __launch_bounds__(256) void k_batch_rec(BatchArgs a) {
    const const_ptr<BatchHeader> hdr = as_const(a.ws);
    const uint32_t n_desc = hdr->n_desc;
    const uint64_t n_rows = hdr->n_rows;
    const bool owned = hdr->mode == kChunkOwned;
    const const_ptr<BatchDesc> desc = reinterpret_cast<const_ptr<BatchDesc>>(hdr + 1);
    // row r -> cluster c = r / Rc, member (r - c Rc) mod K, its row (r - c Rc) / K
    const uint64_t K = a.cluster, C = a.grid / a.cluster;
    const uint64_t Rc = (n_rows + C - 1) / C;
    const uint64_t per = (Rc + K - 1) / K;
    const uint64_t W = a.row_outs;  // outputs per row, a power of two
    const global_ptr<u64x2> rec = reinterpret_cast<global_ptr<u64x2>>(as_global(a.rec));
    const global_ptr<u64x2> ext = reinterpret_cast<global_ptr<u64x2>>(as_global(a.ext));
    for (uint32_t d = blockIdx.x; d < n_desc; d += gridDim.x) {
        const BatchDesc D = load_desc(desc + d);
        if (owned && D.len == 0) {
            if (threadIdx.x == 0) {
                u64x2 E;
                E.x = 0;
                E.y = kRecEmpty;
                ext[d] = E;
            }
            continue;
        }
        const uint64_t s = D.out_off & (W - 1);
        const uint64_t nr = (D.len + s + W - 1) / W;
        uint64_t j = threadIdx.x;
        if (j >= nr) continue;
        const uint64_t r0 = owned ? D.row_start & ~(kDescFirstShared | kDescLastShared) : D.row_start;
        const bool first_shared = owned && (D.row_start & kDescFirstShared);
        const bool last_shared = owned && (D.row_start & kDescLastShared);
        uint64_t src;
        if constexpr (INDEXED)
            src = as_const(hdr->states)[D.src];
        else
            src = D.src;
        // element W j - s of the window: src * (2^53)^(pos + W j - s + 1),
        // the exponent taken modulo the period where it would be negative
        uint64_t e = D.pos + 1 + W * j;
        e = e >= s ? e - s : e + kPeriod - s;
        double z = skip_any<VarFP64>(src, e, a.t_sk);
        for (; j < nr; j += 256) {
            const uint64_t r = r0 + j;
            const uint64_t first = W * j;  // s + (window index of element 0)
            const uint64_t hi = D.len + s - first < W ? D.len + s - first : W;
            const uint64_t lo = j == 0 ? s : 0;
            u64x2 R;  // a RowRec
            R.x = __builtin_bit_cast(uint64_t, z);
            R.y = (D.out_off - s + first) | lo | (hi << kRecHiShift);
            if (owned && j == 0) ext[d] = R;
            if (!(owned && j == 0 && first_shared)) {
                if (owned && j + 1 == nr && last_shared)  // later windows share this chunk
                    R.y = ((uint64_t)(d + 1) << 11) | lo | (1ull << kRecMulti) | (hi << kRecHiShift);
                const uint64_t c = r / Rc, o = r - c * Rc;
                rec[(c * K + o % K) * per + o / K] = R;
            }
            z = VarFP64::mul(z, a.JR);
        }
    }
}

// Lane l's pair of outputs k and k + 1 of a row (states za, zb) at p,
// storing only those in [lo, hi).
template <int KIND, bool NT>
__device__ __forceinline__ void put_pair_in(global_ptr<uint64_t> p, double za, double zb,
                                            uint32_t k, uint32_t lo, uint32_t hi) {
    const bool va = k >= lo && k < hi;
    const bool vb = k + 1 >= lo && k + 1 < hi;
    if (va && vb)
        put<NT>(reinterpret_cast<global_ptr<u64x2>>(p), pair_bits<VarFP64, KIND>(za, zb));
    else if (va)
        put<NT>(p, out_bits<VarFP64, KIND>(za));
    else if (vb)
        put<NT>(p + 1, out_bits<VarFP64, KIND>(zb));
}

// Stores one row of the interleaved kernel: lane l's outputs 2 (e B + l)
// and 2 (e B + l) + 1, e < P (states z[2e], z[2e+1]; B = block), of the
// row whose record info is `info`.  CHECK: the row may be partial (a
// uniform test, then per-lane masks); otherwise it is known to lie wholly in
// its window.
template <int KIND, bool NT, bool CHECK, int P>
__device__ __forceinline__ void store_rec(global_ptr<uint64_t> out, uint64_t info,
                                          const double (&z)[2 * P], uint32_t l, uint32_t B) {
    const uint32_t W = 2u * P * B;
    const global_ptr<uint64_t> p = out + ((info & kRecIndexMask & ~(uint64_t)(W - 1)) + 2u * l);
    if constexpr (CHECK) {
        const uint32_t hi = (uint32_t)(info >> kRecHiShift);
        const uint32_t lo = (uint32_t)info & (W - 1);
        if (__builtin_expect(hi != W || lo != 0, 0)) {
#pragma unroll
            for (int e = 0; e < P; ++e)
                put_pair_in<KIND, NT>(p + 2u * e * B, z[2 * e], z[2 * e + 1], 2u * (e * B + l),
                                      lo, hi);
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < P; ++e)
        put<NT>(reinterpret_cast<global_ptr<u64x2>>(p + 2u * e * B),
                pair_bits<VarFP64, KIND>(z[2 * e], z[2 * e + 1]));
}

// The states of lane l's outputs of the row whose element 0 has state `z0`.
template <int P>
__device__ __forceinline__ void row_states(double (&z)[2 * P], double z0, const Mult (&m)[2 * P]) {
#pragma unroll
    for (int e = 0; e < 2 * P; ++e) z[e] = VarFP64::mul(z0, m[e]);
}

// Lane k's 64-bit value, read by every lane (k uniform).  readlane yields
// a signed int: each half goes through uint32_t so it is not sign-extended.
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, uint32_t k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), k);
    return (uint64_t)hi << 32 | lo;
}

// Lane k's record, read by every lane.
__device__ __forceinline__ u64x2 lane_rec(u64x2 v, uint32_t k) {
    u64x2 r;
    r.x = lane_u64(v.x, k);
    r.y = lane_u64(v.y, k);
    return r;
}

// 64 rows whose records lane k of `mine` holds (row k): IL rows in flight,
// each row stored IL rows after its multiplications.  CHECK: some of the
// rows may be partial.
template <int KIND, bool NT, bool CHECK, int P, int IL>
__device__ __forceinline__ void rows64(global_ptr<uint64_t> out, u64x2 mine,
                                       const Mult (&m)[2 * P], uint32_t l, uint32_t B) {
    static_assert(64 % IL == 0, "rows in flight divide 64");
    double z[IL][2 * P];
    uint64_t info[IL];
#pragma unroll
    for (int j = 0; j < IL; ++j) {
        const u64x2 R = lane_rec(mine, j);
        row_states<P>(z[j], __builtin_bit_cast(double, R.x), m);
        info[j] = R.y;
    }
    for (uint32_t k = IL; k < 64; k += IL) {
#pragma unroll
        for (int j = 0; j < IL; ++j) {
            store_rec<KIND, NT, CHECK, P>(out, info[j], z[j], l, B);
            const u64x2 R = lane_rec(mine, k + j);
            row_states<P>(z[j], __builtin_bit_cast(double, R.x), m);
            info[j] = R.y;
            // keeps the products here: with CHECK the compiler would sink
            // them to the branch of their store, IL rows on
#pragma unroll
            for (int e = 0; e < 2 * P; ++e) asm volatile("" ::"v"(z[j][e]));
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int j = 0; j < IL; ++j) store_rec<KIND, NT, CHECK, P>(out, info[j], z[j], l, B);
}

// Interleaved kernel: clusters of K = cluster consecutive workgroups take
// contiguous ranges of rows (of 2 P block outputs), and member i of a
// cluster takes rows i, i + K, ... of its range (K = grid: workgroup w takes
// rows w, w + grid, ...).  A row's states come from its record and the lane's
// fixed multipliers (2^53)^k for its outputs k, so rows depend on nothing
// before them.  The records are staged in LDS kRecChunk at a time (all
// loads of a chunk issued before one wait); the first chunk's length
// differs between workgroups so that they do not all stop for their next
// chunk at the same moment.  Lane j of each wavefront then holds the record
// of row 64 g + j of group g, which every lane reads by readlane: groups of
// 64 whole rows run branch-free.
template <int KIND, bool NT, int P, int IL>
__global__ __launch_bounds__(256) void k_batch_rows(BatchArgs a) {
    constexpr uint32_t kLoads = 16;  // record loads per thread and round
    __shared__ u64x2 s_rec[kRecChunk];
    const const_ptr<BatchHeader> hdr = as_const(a.ws);
    const uint64_t n_rows = hdr->n_rows;
    const global_ptr<uint64_t> out = as_global(hdr->out);
    const uint32_t l = threadIdx.x;
    const uint32_t B = blockDim.x;
    const uint32_t W = 2u * P * B;
    const uint64_t w = blockIdx.x;
    // member w mod K of cluster w / K: rows r0 + i, r0 + i + K, ... of the
    // cluster's range [r0, r_end)
    const uint64_t K = a.cluster, C = gridDim.x / a.cluster;
    const uint64_t Rc = (n_rows + C - 1) / C;
    const uint64_t per = (Rc + K - 1) / K;
    const uint64_t r0 = (w / K) * Rc, i = w % K;
    const uint64_t r_end = r0 + Rc < n_rows ? r0 + Rc : n_rows;
    if (r0 + i >= r_end) return;
    const uint64_t n_w = (r_end - r0 - i + K - 1) / K;  // this workgroup's rows
    const u64x2* __restrict__ rec = reinterpret_cast<const u64x2*>(a.rec) + w * per;
    Mult m[2 * P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
        m[2 * e] = a.t_lo[2u * (e * B + l)];
        m[2 * e + 1] = a.t_lo[2u * (e * B + l) + 1];
    }
    uint32_t chunk = kRecChunk - (uint32_t)((w * 1543u) % (kRecChunk / 2));
    for (uint64_t k0 = 0; k0 < n_w; k0 += chunk, chunk = kRecChunk) {
        const uint32_t n = n_w - k0 < chunk ? (uint32_t)(n_w - k0) : chunk;
        __syncthreads();  // every wave is done with the previous chunk
        for (uint32_t base = 0; base < n; base += kLoads * B) {
            u64x2 v[kLoads];
#pragma unroll
            for (uint32_t t = 0; t < kLoads; ++t) {
                const uint32_t i = base + t * B + l;
                v[t] = rec[k0 + (i < n ? i : 0)];
            }
#pragma unroll
            for (uint32_t t = 0; t < kLoads; ++t) {
                const uint32_t i = base + t * B + l;
                if (i < n) s_rec[i] = v[t];
            }
        }
        __syncthreads();
        for (uint32_t i0 = 0; i0 < n; i0 += 64) {
            const u64x2 mine = s_rec[(i0 + (l & 63u)) & (kRecChunk - 1)];
            const uint32_t g = n - i0 < 64 ? n - i0 : 64;
            if (g == 64) {
                const bool full =
                    (uint32_t)(mine.y >> kRecHiShift) == W && (mine.y & (W - 1)) == 0;
                if (__ballot(!full) == 0)
                    rows64<KIND, NT, false, P, IL>(out, mine, m, l, B);
                else
                    rows64<KIND, NT, true, P, IL>(out, mine, m, l, B);
                continue;
            }
            for (uint32_t k = 0; k < g; ++k) {
                const u64x2 R = lane_rec(mine, k);
                double z[2 * P];
                row_states<P>(z, __builtin_bit_cast(double, R.x), m);
                store_rec<KIND, NT, true, P>(out, R.y, z, l, B);
            }
        }
    }
}

// Chunked kernel: the flat layout of the plain generator over a batch.  The
// output is cut into aligned chunks of kChunkRows rows of 512 outputs
// (16 KiB); the pre-pass (k_batch_rec with one cluster of one workgroup and
// rows of kChunkOuts outputs) writes one record per chunk and window that
// meet, record j (in window order) at j: the state of the chunk's element 0
// as if the window covered it, the chunk's output index and the window's
// part of the chunk [lo, hi).  Workgroup w of the grid takes the virtual
// indices w, w + grid, ..., and index v the record xcd_run_index(v) while v
// lies in a whole XCD run, v after the last one: with one workgroup per
// record (the default) the dispatcher hands the chunks out in the plain flat
// layout's order (each XCD 4 MiB of consecutive chunks per run); a smaller,
// persistent grid loads the next record while it writes the current one.  Lane l's outputs of a chunk are its pairs
// 2l, 2l + 1 of each row: states z * (2^53)^(2l) and z * (2^53)^(2l+1), one
// multiplication each by the lane's fixed multipliers, then one step of
// (2^53)^512 per row.  A chunk that one window covers is stored without a
// test; one that a window starts or ends in stores the window's outputs only.
// In the owned mode (sorted, disjoint windows) there is one record per chunk
// instead, so no two workgroups write into one chunk: a chunk that several
// windows share is written whole by its workgroup, window by window.  (With
// write-back stores, chunks written in parts by workgroups on different
// XCDs cost the 10,000-window batch 12 % of its rate.)
__device__ Mult chunk_sym[kChunkSymEntries];

hipError_t upload_chunk_symbol(const Mult* entries) {
    return hipMemcpyToSymbol(HIP_SYMBOL(chunk_sym), entries, sizeof(Mult) * kChunkSymEntries, 0,
                             hipMemcpyHostToDevice);
}

template <int KIND, bool NT>
__global__ __launch_bounds__(kFlatBlock) void k_batch_chunks(BatchArgs a) {
    constexpr uint32_t C = kChunkOuts;
    const uint64_t n = a.n_rec;  // records (== hdr->n_rows)
    const const_ptr<u64x2> rec = reinterpret_cast<const_ptr<u64x2>>(as_const(a.rec));
    constexpr uint64_t kRun = (uint64_t)kFlatXcds * kFlatXcdRun;
    const uint64_t runs = n / kRun * kRun;  // records in whole XCD runs
    auto at = [&](uint64_t v) { return v < runs ? xcd_run_index(v) : v; };
    const uint32_t l = threadIdx.x;
    uint64_t j = blockIdx.x;
    // Loads before tests: the multipliers (at a fixed address) and the
    // workgroup's record go out before anything waits.  A workgroup past the
    // last record (a fixed grid larger than the batch) reads record 0, which
    // every record array holds, and leaves.
    const Mult ma = chunk_sym[l], mb = chunk_sym[kFlatBlock + l];
    const Mult JB = chunk_sym[2 * kFlatBlock];
    u64x2 cur;
    if constexpr (NT) {
        // With non-temporal stores the record is loaded through the vector
        // memory path (every lane the same 16 bytes; an index offset the
        // compiler cannot prove uniform keeps it from becoming a scalar
        // load), then made uniform: 3 % faster than the scalar load at the
        // tuned cap of 3.  With temporal stores the vector path was 30 %
        // slower, so those keep the scalar load.
        uint32_t vz;
        asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
        const global_ptr<u64x2> vrec = reinterpret_cast<global_ptr<u64x2>>(as_global(a.rec));
        const u64x2 v = vrec[at(j < n ? j : 0) + vz];
        cur.x = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v.x >> 32)) << 32) |
                (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v.x);
        cur.y = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v.y >> 32)) << 32) |
                (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v.y);
    } else {
        cur = rec[at(j < n ? j : 0)];
    }
    if (j >= n) return;
    const global_ptr<uint64_t> out = as_global(a.out);
    // one window's part [lo, hi) of the chunk at output g, from the state z0
    // of the chunk's element 0 as if the window covered it
    auto part = [&](uint64_t g, double z0, uint32_t lo, uint32_t hi) {
        const global_ptr<uint64_t> p = out + (g + 2u * l);
        double za = VarFP64::mul(z0, ma);
        double zb = VarFP64::mul(z0, mb);
#pragma unroll
        for (int r = 0; r < (int)kChunkRows; ++r) {
            put_pair_in<KIND, NT>(p + r * kFlatPerBlock, za, zb, r * kFlatPerBlock + 2u * l, lo,
                                  hi);
            za = VarFP64::mul(za, JB);
            zb = VarFP64::mul(zb, JB);
        }
    };
    for (;;) {
        const uint64_t jn = j + gridDim.x;
        // a fixed grid's next record, in flight meanwhile
        u64x2 nxt = cur;
        if (jn < n) nxt = rec[at(jn)];
        const double z0 = __builtin_bit_cast(double, cur.x);
        const uint64_t info = cur.y;
        const uint32_t hi = (uint32_t)(info >> kRecHiShift);
        const uint32_t lo = (uint32_t)info & (C - 1);
        if (hi == C && lo == 0) {
            double za = VarFP64::mul(z0, ma);
            double zb = VarFP64::mul(z0, mb);
            const global_ptr<uint64_t> p = out + ((info & kRecIndexMask) + 2u * l);
#pragma unroll
            for (int r = 0; r < (int)kChunkRows; ++r) {
                put<NT>(reinterpret_cast<global_ptr<u64x2>>(p + r * kFlatPerBlock),
                        pair_bits<VarFP64, KIND>(za, zb));
                za = VarFP64::mul(za, JB);
                zb = VarFP64::mul(zb, JB);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else if (!((info >> kRecMulti) & 1)) {
            part(info & kRecIndexMask & ~(uint64_t)(C - 1), z0, lo, hi);
        } else {
            // Owned mode, a chunk that windows d, d + 1, ... share: the later
            // windows' records are their ext records (empty windows skipped);
            // the first of them also gives the chunk's output index.
            const const_ptr<u64x2> ext = reinterpret_cast<const_ptr<u64x2>>(as_const(a.ext));
            const uint32_t n_desc = as_const(a.ws)->n_desc;
            uint64_t w = (info & kRecIndexMask) >> 11;  // d + 1
            u64x2 R;
            R.y = kRecEmpty;
            for (; w < n_desc; ++w) {
                R = ext[w];
                if (R.y != kRecEmpty) break;
            }
            const uint64_t g = R.y & kRecIndexMask & ~(uint64_t)(C - 1);
            part(g, z0, lo, hi);
            while (R.y != kRecEmpty && (R.y & kRecIndexMask & ~(uint64_t)(C - 1)) == g) {
                const uint32_t h = (uint32_t)(R.y >> kRecHiShift);
                part(g, __builtin_bit_cast(double, R.x), (uint32_t)R.y & (C - 1), h);
                if (h == C) break;  // that window reaches the chunk's end
                R.y = kRecEmpty;
                for (++w; w < n_desc; ++w) {
                    R = ext[w];
                    if (R.y != kRecEmpty) break;
                }
            }
        }
        j = jn;
        if (j >= n) break;
        cur = nxt;
    }
}

// Small batches in the kernel arguments (see BatchFlatInline): workgroup b
// finds its window among at most kInlineDescs (a uniform scan), then writes
// chunk c = b - chunk0 of it exactly as k_generate_flat writes a chunk,
// storing only the window's outputs.
template <int KIND, bool NT>
__global__ __launch_bounds__(kFlatBlock) void k_batch_flat_inline(const Mult* __restrict__ tabs,
                                                                  Mult M1, Mult J,
                                                                  BatchFlatInline in) {
    extern __shared__ char occupancy_cap[];
    (void)occupancy_cap;
    constexpr uint32_t C = kChunkOuts;
    const uint32_t b = blockIdx.x;
    uint32_t d = 0;
    for (uint32_t k = 1; k < in.n; ++k)
        if (in.w[k].chunk0 <= b) d = k;
    const FlatWin W = in.w[d];
    const uint64_t c = b - W.chunk0;
    const uint32_t l = threadIdx.x;
    double za, zb;
    flat_start<VarFP64>(c, l, (int)kChunkRows, W.base, tabs, M1, za, zb);
    // chunk-relative positions k of the window's elements k - s: [s, len + s)
    const uint64_t first = C * c;
    const global_ptr<uint64_t> p = as_global(in.out) + (W.out_off - W.s + first + 2u * l);
    const uint64_t hi = W.len + W.s;
    if (first >= W.s && first + C <= hi) {
#pragma unroll
        for (int r = 0; r < (int)kChunkRows; ++r) {
            put<NT>(reinterpret_cast<global_ptr<u64x2>>(p + r * kFlatPerBlock),
                    pair_bits<VarFP64, KIND>(za, zb));
            za = VarFP64::mul(za, J);
            zb = VarFP64::mul(zb, J);
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    // the window's first or last chunk: keep k in [s, len + s)
    const uint32_t lo = first == 0 ? W.s : 0;
    const uint32_t top = hi - first < C ? (uint32_t)(hi - first) : C;
#pragma unroll
    for (int r = 0; r < (int)kChunkRows; ++r) {
        put_pair_in<KIND, NT>(p + r * kFlatPerBlock, za, zb, r * kFlatPerBlock + 2u * l, lo, top);
        za = VarFP64::mul(za, J);
        zb = VarFP64::mul(zb, J);
    }
}

hipError_t launch_batch_flat_inline(int kind, bool nt, uint32_t grid, uint32_t lds,
                                    hipStream_t s, const Mult* tabs, const Mult& M1,
                                    const Mult& J, const BatchFlatInline& in) {
    if (kind == 0) {
        if (nt)
            hipLaunchKernelGGL((k_batch_flat_inline<0, true>), dim3(grid), dim3(kFlatBlock), lds,
                               s, tabs, M1, J, in);
        else
            hipLaunchKernelGGL((k_batch_flat_inline<0, false>), dim3(grid), dim3(kFlatBlock), lds,
                               s, tabs, M1, J, in);
    } else {
        if (nt)
            hipLaunchKernelGGL((k_batch_flat_inline<1, true>), dim3(grid), dim3(kFlatBlock), lds,
                               s, tabs, M1, J, in);
        else
            hipLaunchKernelGGL((k_batch_flat_inline<1, false>), dim3(grid), dim3(kFlatBlock), lds,
                               s, tabs, M1, J, in);
    }
    return hipGetLastError();
}

// The device request queue (see nn_batch.hpp).  Thread 0 of a workgroup
// waits for the next entry with acquire loads of the host's `head`, copies
// the entry to LDS, and claims rows with a compare-and-swap that also checks
// the slot's round, so a workgroup arriving after the entry is complete (its
// slot already reset for the next round) claims nothing.  Each claimed row
// is a row of the plain flat layout (kFlatPerBlock outputs, 16-byte stores)
// started from the entry's host-computed state.  The workgroup whose finished
// rows complete the entry resets the slot for the next round, then publishes
// seq + 1 to the host with a system-scope release.
template <int KIND>
__global__ __launch_bounds__(kFlatBlock) void k_queue(QueueArgs a) {
    __shared__ QueueEntry s_e;
    __shared__ uint32_t s_go;
    __shared__ uint64_t s_claim;
    const uint32_t l = threadIdx.x;
    const uint64_t t0 = (uint64_t)wall_clock64();
    uint64_t last = t0;
    for (uint64_t seq = a.start;; ++seq) {
        const uint32_t slot = (uint32_t)(seq & (a.cap - 1));
        if (l == 0) {
            uint32_t go = 0;
            for (;;) {
                const uint64_t h =
                    __hip_atomic_load(&a.sh->head, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                const uint64_t now = (uint64_t)wall_clock64();
                if (h > seq) {
                    go = 1;
                    last = now;
                    break;
                }
                if (__hip_atomic_load(&a.sh->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM))
                    break;
                if (now - last > a.idle_ticks || now - t0 > a.max_ticks) break;
                __builtin_amdgcn_s_sleep(8);
            }
            if (go) s_e = a.entries[slot];
            s_go = go;
        }
        __syncthreads();
        if (!s_go) return;
        const QueueEntry E = s_e;
        const uint64_t rows = (E.count + kFlatPerBlock - 1) / kFlatPerBlock;
        const uint64_t round = (seq >> a.cap_log2) & 0xffffffffull;
        const global_ptr<uint64_t> out = as_global(reinterpret_cast<uint64_t*>(E.out));
        // Rows are claimed ceil(rows / workgroups) at a time (at least
        // kQueueRowsPerClaim, at most kQueueMaxRowsPerClaim), so a small entry
        // costs each workgroup one claim; a claim that takes the last rows
        // also tells its workgroup that nothing is left.
        uint64_t per_claim = (rows + gridDim.x - 1) / gridDim.x;
        per_claim = per_claim < kQueueRowsPerClaim ? kQueueRowsPerClaim
                  : per_claim > kQueueMaxRowsPerClaim ? kQueueMaxRowsPerClaim : per_claim;
        uint64_t mine = 0;
        for (bool more = true; more;) {
            __syncthreads();  // s_claim and s_e are rewritten below
            if (l == 0) {
                uint64_t first = ~0ull;
                uint64_t old =
                    __hip_atomic_load(&a.claim[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                while ((old >> 32) == round && (old & 0xffffffffull) < rows) {
                    if (__hip_atomic_compare_exchange_strong(
                            &a.claim[slot], &old, old + per_claim, __ATOMIC_RELAXED,
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        first = old & 0xffffffffull;
                        break;
                    }
                }
                s_claim = first;
            }
            __syncthreads();
            const uint64_t c0 = s_claim;
            if (c0 == ~0ull) break;
            const uint64_t c1 = c0 + per_claim < rows ? c0 + per_claim : rows;
            more = c1 < rows;
            // Row j covers outputs [kFlatPerBlock j, kFlatPerBlock (j + 1)); lane l
            // owns x_b - 1 and x_b = kFlatPerBlock j + 2 l + 1, the states
            // base * (2^53)^(x_b) and base * (2^53)^(x_b + 1): the row's start
            // from the flat layout's two row tables, the lane's offset from t_lo
            // (all three loads independent), then one step per row.
            uint64_t xb = kFlatPerBlock * c0 + 2u * l + 1;
            const Mult hi = a.tabs[kFlatHiOffset + c0 / kFlatLoSize];
            const Mult lo = a.tabs[kFlatLoOffset + c0 % kFlatLoSize];
            const Mult ma = a.tabs[2u * l + 1], mb = a.tabs[2u * l + 2];
            const VarFP64::S S = VarFP64::mul(VarFP64::mul(VarFP64::load(E.base), hi), lo);
            VarFP64::S za = VarFP64::mul(S, ma);
            VarFP64::S zb = VarFP64::mul(S, mb);
            for (uint64_t j = c0; j < c1; ++j) {
                const global_ptr<uint64_t> p = out + (xb - 1);
                if (xb < E.count) {
                    u64x2 v;
                    v.x = out_bits<VarFP64, KIND>(za);
                    v.y = out_bits<VarFP64, KIND>(zb);
                    put<true>(reinterpret_cast<global_ptr<u64x2>>(p), v);
                } else if (xb - 1 < E.count) {
                    put<true>(p, out_bits<VarFP64, KIND>(za));
                }
                za = VarFP64::mul(za, a.JB);
                zb = VarFP64::mul(zb, a.JB);
                xb += kFlatPerBlock;
            }
            mine += c1 - c0;
        }
        if (mine) {
            // Each wave waits for its own stores to reach L2; then one
            // system-scope release by thread 0 writes this workgroup's outputs
            // back from the L2 before its rows are counted.  The workgroup whose
            // count completes the entry (acquiring the others' releases through
            // the counter) resets the slot and publishes seq + 1 to the host.
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (l == 0) {
                __threadfence_system();  // the release that the count carries
                const uint64_t before = __hip_atomic_fetch_add(&a.fin[slot], mine, __ATOMIC_ACQUIRE,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                if (before + mine == rows) {
                    __hip_atomic_store(&a.fin[slot], 0ull, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&a.claim[slot], (round + 1) << 32, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&a.done[slot], seq + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
        __syncthreads();  // s_go and s_e are rewritten by thread 0 next
    }
}

// Static batches (nn_generate_batch_static): the copied descriptors become
// the chunked kernel's BatchDescs.  Thread t takes the contiguous
// descriptors [t p, t p + p), p = ceil(n / 1024): it counts their chunk
// records, the workgroup scans the 1024 counts, and each thread writes its
// descriptors with their record offsets.
__global__ __launch_bounds__(1024) void k_static_descs(char* scratch, uint32_t n, uint64_t* out) {
    constexpr uint32_t T = 1024;
    constexpr uint64_t C = kChunkOuts;
    __shared__ uint64_t s_sum[T];
    const uint64_t* raw = reinterpret_cast<const uint64_t*>(scratch + kStaticRawOff);
    BatchDesc* dd = reinterpret_cast<BatchDesc*>(scratch + kStaticDescOff);
    const uint32_t t = threadIdx.x;
    const uint32_t p = (n + T - 1) / T;
    const uint32_t d0 = t * p < n ? t * p : n;
    const uint32_t d1 = d0 + p < n ? d0 + p : n;
    auto records = [](uint64_t len, uint64_t off) -> uint64_t {
        return len ? (len + (off & (C - 1)) + C - 1) / C : 0;
    };
    uint64_t mine = 0;
    for (uint32_t d = d0; d < d1; ++d) mine += records(raw[3 * d + 1], raw[3 * d + 2]);
    s_sum[t] = mine;
    __syncthreads();
    // inclusive scan of the counts (Hillis-Steele over the 1024 entries)
    for (uint32_t k = 1; k < T; k <<= 1) {
        const uint64_t add = t >= k ? s_sum[t - k] : 0;
        __syncthreads();
        s_sum[t] += add;
        __syncthreads();
    }
    uint64_t r = s_sum[t] - mine;  // exclusive prefix
    for (uint32_t d = d0; d < d1; ++d) {
        const uint64_t len = raw[3 * d + 1];
        BatchDesc D;
        D.src = raw[3 * d];
        D.pos = 0;
        D.len = len;
        D.out_off = len ? raw[3 * d + 2] : 0;  // an empty window gets no record
        D.row_start = r;
        dd[d] = D;
        r += records(len, D.out_off);
    }
    if (t == T - 1) {
        BatchHeader h;
        h.out = out;
        h.n_desc = n;
        h.mode = kChunkPerRecord;
        h.n_rows = s_sum[T - 1];
        h.states = nullptr;
        for (int i = 0; i < 4; ++i) h.pad[i] = 0;
        *reinterpret_cast<BatchHeader*>(scratch) = h;
    }
}

hipError_t launch_static_descs(hipStream_t s, void* scratch, uint32_t n, uint64_t* out) {
    k_static_descs<<<1, 1024, 0, s>>>(static_cast<char*>(scratch), n, out);
    return hipGetLastError();
}

hipError_t launch_queue(int kind, uint32_t grid, uint32_t block, hipStream_t s,
                        const QueueArgs& a) {
    if (block != kFlatBlock) return hipErrorInvalidValue;
    if (kind == 0)
        k_queue<0><<<grid, block, 0, s>>>(a);
    else
        k_queue<1><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

const void* batch_rec_kernel(bool indexed) {
    return indexed ? reinterpret_cast<const void*>(&k_batch_rec<true>)
                   : reinterpret_cast<const void*>(&k_batch_rec<false>);
}

const void* batch_chunks_kernel(int kind, bool nt) {
    if (kind == 0)
        return nt ? reinterpret_cast<const void*>(&k_batch_chunks<0, true>)
                  : reinterpret_cast<const void*>(&k_batch_chunks<0, false>);
    return nt ? reinterpret_cast<const void*>(&k_batch_chunks<1, true>)
              : reinterpret_cast<const void*>(&k_batch_chunks<1, false>);
}

const void* batch_rows_kernel(int kind, bool nt) {
    constexpr int P = kIlPairs, IL = kIlRows;
    if (kind == 0)
        return nt ? reinterpret_cast<const void*>(&k_batch_rows<0, true, P, IL>)
                  : reinterpret_cast<const void*>(&k_batch_rows<0, false, P, IL>);
    return nt ? reinterpret_cast<const void*>(&k_batch_rows<1, true, P, IL>)
              : reinterpret_cast<const void*>(&k_batch_rows<1, false, P, IL>);
}

template <class V, int KIND, bool NT>
static const void* kernel_kvn(bool indexed) {
    return indexed ? reinterpret_cast<const void*>(&k_batch<V, KIND, NT, true>)
                   : reinterpret_cast<const void*>(&k_batch<V, KIND, NT, false>);
}

template <class V, int KIND>
static const void* kernel_kv(bool nt, bool indexed) {
    return nt ? kernel_kvn<V, KIND, true>(indexed) : kernel_kvn<V, KIND, false>(indexed);
}

template <class V>
static const void* kernel_v(int kind, bool nt, bool indexed) {
    return kind == 0 ? kernel_kv<V, 0>(nt, indexed) : kernel_kv<V, 1>(nt, indexed);
}

const void* batch_kernel(int mulmod, int kind, bool nt, bool indexed) {
    switch (mulmod) {
        case 1: return kernel_v<VarFP64>(kind, nt, indexed);
        case 2: return kernel_v<VarBarrett>(kind, nt, indexed);
        case 3: return kernel_v<VarShoup>(kind, nt, indexed);
        case 4: return kernel_v<VarMontgomery>(kind, nt, indexed);
        default: return nullptr;
    }
}

template <class V, int KIND, bool NT>
static const void* inline_kvn(bool indexed) {
    return indexed ? reinterpret_cast<const void*>(&k_batch_inline<V, KIND, NT, true>)
                   : reinterpret_cast<const void*>(&k_batch_inline<V, KIND, NT, false>);
}

template <class V>
static const void* inline_v(int kind, bool nt, bool indexed) {
    if (kind == 0) return nt ? inline_kvn<V, 0, true>(indexed) : inline_kvn<V, 0, false>(indexed);
    return nt ? inline_kvn<V, 1, true>(indexed) : inline_kvn<V, 1, false>(indexed);
}

hipError_t launch_batch_inline(int mulmod, int kind, bool nt, bool indexed, uint32_t grid,
                               uint32_t block, hipStream_t s, const BatchArgs& a,
                               const BatchInline& in) {
    const void* k = nullptr;
    switch (mulmod) {
        case 1: k = inline_v<VarFP64>(kind, nt, indexed); break;
        case 2: k = inline_v<VarBarrett>(kind, nt, indexed); break;
        case 3: k = inline_v<VarShoup>(kind, nt, indexed); break;
        case 4: k = inline_v<VarMontgomery>(kind, nt, indexed); break;
        default: return hipErrorInvalidValue;
    }
    BatchArgs ca = a;
    BatchInline ci = in;
    void* params[] = {&ca, &ci};
    return hipLaunchKernel(k, dim3(grid), dim3(block), params, 0, s);
}

hipError_t launch_batch(int mulmod, int kind, bool nt, bool indexed, uint32_t grid,
                        uint32_t block, hipStream_t s, const BatchArgs& a) {
    const void* k = batch_kernel(mulmod, kind, nt, indexed);
    if (!k) return hipErrorInvalidValue;
    BatchArgs copy = a;
    void* params[] = {&copy};
    return hipLaunchKernel(k, dim3(grid), dim3(block), params, 0, s);
}

}  // namespace nn
