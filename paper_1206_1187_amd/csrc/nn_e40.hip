// nn_e40.hip -- the modulus-3^40 generator (Section 2's longer-period
// variant): host arithmetic, device tables, the row-layout kernel and the
// extern "C" entry points nn_e40_* of include/nn.h.
//
// Layout as the 3^33 row kernel: T = grid*block threads, two consecutive
// outputs per lane and row (one 16-byte store), row i covering elements
// [2 T i, 2 T (i+1)), IL rows in flight per thread, each chain advanced by
// (2^53)^(2 T IL) per trip.  A thread starts at element 2t by two table
// multiplications.  An output that is only 8-byte aligned gets its first
// element from lane 0 of workgroup 0 with an 8-byte store, the rest from
// the aligned row loop.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "nn.h"
#include "nn_device.hpp"
#include "nn_e40.hpp"
#include "nn_internal.hpp"

namespace nn {
namespace e40 {
namespace {

// ------------------------------------------------------------------ host --
inline uint64_t h_mul(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) % kMod); }

inline uint64_t h_pow(uint64_t base, uint64_t e) {
    uint64_t r = 1, b = base % kMod;
    while (e) {
        if (e & 1) r = h_mul(r, b);
        b = h_mul(b, b);
        e >>= 1;
    }
    return r;
}

inline bool valid_state(uint64_t s) { return s != 0 && s < kMod && s % 3 != 0; }

// (2^53)^k mod 3^40 through byte tables; k is reduced by the period first
// (2^53 has order exactly 2*3^39: 53 is prime to it).
class Powers {
  public:
    static const Powers& get() {
        static Powers p;
        return p;
    }
    uint64_t pow(uint64_t k) const {
        k %= kPeriod;
        uint64_t r = 1;
        for (int i = 0; k != 0; ++i, k >>= 8) {
            const uint32_t j = (uint32_t)(k & 0xff);
            if (j) r = h_mul(r, tab_[i][j]);
        }
        return r;
    }

  private:
    Powers() {
        uint64_t step = kMult;
        for (int i = 0; i < 8; ++i) {
            tab_[i][0] = 1;
            for (int j = 1; j < 256; ++j) tab_[i][j] = h_mul(tab_[i][j - 1], step);
            step = h_mul(tab_[i][255], step);
        }
    }
    uint64_t tab_[8][256];
};

inline Mult40 make_mult40(uint64_t v) {
    Mult40 f;
    f.v = v;
    f.mont = (uint64_t)(((u128)v << 64) % kMod);
    return f;
}

constexpr uint32_t kLo = 1024;      // t_lo[l] = (2^53)^l
constexpr uint32_t kHi = 1u << 15;  // t_hi[j] = (2^53)^(1024 j)
// Flat layout: t_flo[j] = (2^53)^(512 j), j < kFLo, and
// t_fhi[i] = (2^53)^(512 kFLo i), i < kFHi, after t_lo and t_hi.
constexpr uint32_t kFLo = 1024;
constexpr uint32_t kFHi = 2048;
constexpr uint64_t kFLoOff = (uint64_t)kLo + kHi;
constexpr uint64_t kFHiOff = kFLoOff + kFLo;
constexpr uint64_t kFlatMaxRows = (uint64_t)kFLo * kFHi;  // rows of 512 per launch (2^21)
// The tables' entries as Mult40, then the same entries as base-B limbs
// (Mult40L, the same size), so the FP64 step starts without Montgomery.
constexpr uint64_t kTabEntries = kFHiOff + kFHi;
static_assert(sizeof(Mult40L) == sizeof(Mult40), "limb entries follow at the same stride");
constexpr uint64_t kMaxThreads = (uint64_t)kLo * kHi / 2;
constexpr int kMaxDev = 64;

std::mutex g_mu;
Mult40* g_tab[kMaxDev];  // kLo + kHi + kFLo + kFHi entries per device

// The FP64 step's flat-layout multipliers as limbs, in a static device array
// of this module: the lane offsets (2^53)^k for k < 512, then t_flo and
// t_fhi.  Its address is a constant of the code, so a workgroup's table
// loads go out at its start.  Filled per device with the tables.
constexpr uint32_t kSymLo = 512;
constexpr uint32_t kSymHi = kSymLo + kFLo;
constexpr uint32_t kSymEntries = kSymHi + kFHi;
__device__ Mult40L e40_sym[kSymEntries];

int device_tables(const Mult40** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NN_ENODEV, "hipGetDevice: %s", hipGetErrorString(e));
    DeviceTables* d = nullptr;  // checks the architecture
    const int st = current_device(&d);
    if (st) return st;
    if (dev < 0 || dev >= kMaxDev) return fail(NN_ENODEV, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_tab[dev]) {
        static std::vector<Mult40> host = [] {
            std::vector<Mult40> t(2 * kTabEntries);
            uint64_t r = 1;
            for (uint32_t l = 0; l < kLo; ++l, r = h_mul(r, kMult)) t[l] = make_mult40(r);
            const uint64_t step = Powers::get().pow(kLo);
            r = 1;
            for (uint32_t j = 0; j < kHi; ++j, r = h_mul(r, step)) t[kLo + j] = make_mult40(r);
            const uint64_t row = Powers::get().pow(512);
            r = 1;
            for (uint32_t j = 0; j < kFLo; ++j, r = h_mul(r, row)) t[kFLoOff + j] = make_mult40(r);
            const uint64_t big = r;  // (2^53)^(512 kFLo)
            r = 1;
            for (uint32_t i = 0; i < kFHi; ++i, r = h_mul(r, big)) t[kFHiOff + i] = make_mult40(r);
            Mult40L* limbs = reinterpret_cast<Mult40L*>(t.data() + kTabEntries);
            for (uint64_t i = 0; i < kTabEntries; ++i) limbs[i] = make_mult40l(t[i].v);
            return t;
        }();
        void* mem = nullptr;
        e = hipMalloc(&mem, host.size() * sizeof(Mult40));
        if (e != hipSuccess) return fail(NN_ENOMEM, "hipMalloc e40 tables: %s", hipGetErrorString(e));
        e = hipMemcpy(mem, host.data(), host.size() * sizeof(Mult40), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            const Mult40L* limbs = reinterpret_cast<const Mult40L*>(host.data() + kTabEntries);
            std::vector<Mult40L> sym(limbs, limbs + kSymLo);  // t_lo's first 512
            sym.insert(sym.end(), limbs + kFLoOff, limbs + kFLoOff + kFLo);
            sym.insert(sym.end(), limbs + kFHiOff, limbs + kFHiOff + kFHi);
            e = hipMemcpyToSymbol(HIP_SYMBOL(e40_sym), sym.data(), sizeof(Mult40L) * kSymEntries,
                                  0, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return fail(NN_EHIP, "e40 table upload: %s", hipGetErrorString(e));
        }
        g_tab[dev] = (Mult40*)mem;
    }
    *out = g_tab[dev];
    return NN_OK;
}

// ---------------------------------------------------------------- device --
struct E40Args {
    uint64_t* out;  // 16-byte aligned: the row loop's first element
    uint64_t T;
    uint64_t e_full;
    uint32_t rem;
    uint64_t base;  // state of out[0]
    Mult40 J;       // (2^53)^(2T)
    Mult40 M1;      // 2^53
    Mult40 JI;      // J^IL
    Mult40L JL, M1L, JIL;  // the same multipliers as base-B limbs
    const Mult40* t_lo;
    const Mult40* t_hi;
    uint64_t* head;       // 8-byte aligned output's first element, or null
    uint64_t head_state;  // its state
};

// The two step reductions: MM 0 = Montgomery on 64-bit states, MM 1 = FP64
// on base-B limbs.
template <int MM>
struct Step;
template <>
struct Step<0> {
    typedef uint64_t S;
    static __device__ __forceinline__ S from(uint64_t z) { return z; }
    static __device__ __forceinline__ S mul(S z, const Mult40& v, const Mult40L&) {
        return mm40(z, v.mont);
    }
    template <int KIND>
    static __device__ __forceinline__ uint64_t bits(S z) {
        if constexpr (KIND == 0)
            return z;
        else
            return (uint64_t)__double_as_longlong(to_f64(z));
    }
};
template <>
struct Step<1> {
    typedef L2 S;
    static __device__ __forceinline__ S from(uint64_t z) { return limbs(z); }
    static __device__ __forceinline__ S mul(S z, const Mult40&, const Mult40L& v) {
        return mul40l(z, v);
    }
    template <int KIND>
    static __device__ __forceinline__ uint64_t bits(S z) {
        if constexpr (KIND == 0)
            return to_u64(z);
        else
            return (uint64_t)__double_as_longlong(to_f64(z));
    }
};

template <int KIND, int MM, int IL, int UNROLL, bool NT>
__global__ __launch_bounds__(1024) void k_e40(E40Args a) {
    typedef Step<MM> St;
    typedef typename St::S S;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0 && a.head) put<NT>(as_global(a.head), St::template bits<KIND>(St::from(a.head_state)));
    const uint32_t rem_pairs = a.rem >> 1;
    const bool extra_pair = t < rem_pairs;
    const bool extra_one = (a.rem & 1u) && t == rem_pairs;
    if (a.e_full == 0 && !extra_pair && !extra_one) return;
    const uint64_t k = 2ull * t;  // < 2^25
    // The thread's first pair by two table multiplications (Montgomery),
    // then the step's own representation.
    const uint64_t z0 = mm40(mm40(a.base, a.t_hi[k >> 10].mont), a.t_lo[k & (kLo - 1)].mont);
    S za[IL], zb[IL];
    za[0] = St::from(z0);
    zb[0] = St::from(mm40(z0, a.M1.mont));
#pragma unroll
    for (int r = 1; r < IL; ++r) {
        za[r] = St::mul(za[r - 1], a.J, a.JL);
        zb[r] = St::mul(zb[r - 1], a.J, a.JL);
    }
    const global_ptr<u64x2> out = reinterpret_cast<global_ptr<u64x2>>(as_global(a.out));
    global_ptr<u64x2> row = out;
    const uint64_t T = a.T;
    uint64_t i = 0;
#pragma unroll UNROLL
    for (; i + IL <= a.e_full; i += IL) {
        // each row: its store, then its two multiplications, kept in that
        // order so stores leave the wave evenly spaced
#pragma unroll
        for (int r = 0; r < IL; ++r) {
            u64x2 v;
            v.x = St::template bits<KIND>(za[r]);
            v.y = St::template bits<KIND>(zb[r]);
            put<NT>(row + r * T + t, v);
            za[r] = St::mul(za[r], a.JI, a.JIL);
            zb[r] = St::mul(zb[r], a.JI, a.JIL);
            __builtin_amdgcn_sched_barrier(0);
        }
        row += IL * T;
    }
    // Rows left over (fewer than IL): the states before the last advance.
    const uint32_t left = (uint32_t)(a.e_full - i);
    S pa = za[0], pb = zb[0];
#pragma unroll
    for (int r = 0; r < IL; ++r) {
        if ((uint32_t)r < left) {
            u64x2 v;
            v.x = St::template bits<KIND>(za[r]);
            v.y = St::template bits<KIND>(zb[r]);
            put<NT>(row + r * T + t, v);
        }
        if ((uint32_t)r == left) {
            pa = za[r];
            pb = zb[r];
        }
    }
    row += left * T;
    if (extra_pair) {
        u64x2 v;
        v.x = St::template bits<KIND>(pa);
        v.y = St::template bits<KIND>(pb);
        put<NT>(row + t, v);
    } else if (extra_one) {
        put<NT>(reinterpret_cast<global_ptr<uint64_t>>(row + t), St::template bits<KIND>(pa));
    }
}

// Flat layout at modulus 3^40: chunks of R rows of 512 outputs; lane l
// writes the pair 2l, 2l + 1 of each row with one 16-byte store.
// Workgroup b starts at chunk b (u = R b rows in) from
// base * t_fhi[u / kFLo] * t_flo[u % kFLo] * t_lo[2l] (Montgomery, then
// the step's representation) and takes chunks b, b + G, ... (G the grid):
// one step of (2^53)^512 per row, and from a chunk's last row to the next
// chunk one step of JN = (2^53)^(512 R G - 512 (R - 1)).  With G equal to
// the chunk count each workgroup writes one chunk and exits.
struct E40FlatArgs {
    uint64_t* out;       // 16-byte aligned
    uint64_t n_chunks;   // whole chunks, n_chunks * R <= kFlatMaxRows
    uint64_t base;       // state of out[0]
    Mult40 M1, J, JN;
    Mult40L M1L, JL, JNL;
    const Mult40* tabs;  // t_lo, t_hi, t_flo, t_fhi, then the same as limbs
    double base_lo, base_hi;  // base as base-B limbs (limbs())
};

// Workgroup w writes chunk w, then w + grid, ... (grid <= n_chunks, as the
// host launches it), or with G > 0 (one workgroup per chunk over whole XCD
// runs of kFlatXcds*G chunks) chunk x G + i of its run for the run's
// workgroup kFlatXcds i + x, so XCD x writes G consecutive chunks (4 MiB).
template <int KIND, int MM, int R, bool NT, int G>
__global__ __launch_bounds__(256) void k_e40_flat(E40FlatArgs a) {
    extern __shared__ char occupancy_cap[];
    (void)occupancy_cap;
    typedef Step<MM> St;
    typedef typename St::S S;
    uint64_t c = blockIdx.x;
    if constexpr (G > 0) {
        constexpr uint64_t run = (uint64_t)kFlatXcds * G;
        const uint64_t r = c % run;
        c = c - r + (r % kFlatXcds) * G + r / kFlatXcds;
    }
    const uint32_t l = threadIdx.x;
    const uint64_t u = c * R;
    S za, zb;
    if constexpr (MM == 1) {
        // in limbs throughout: the chunk's two row multipliers, then the
        // lane's two offsets (all four loads independent, from e40_sym), no
        // Montgomery
        const Mult40L hi = e40_sym[kSymHi + u / kFLo], lo = e40_sym[kSymLo + u % kFLo];
        const Mult40L la = e40_sym[2u * l], lb = e40_sym[2u * l + 1];
        const L2 S0 = mul40l(mul40l(L2{a.base_lo, a.base_hi}, hi), lo);
        za = mul40l(S0, la);
        zb = mul40l(S0, lb);
    } else {
        const uint64_t z0 = mm40(mm40(mm40(a.base, a.tabs[kFHiOff + u / kFLo].mont),
                                      a.tabs[kFLoOff + u % kFLo].mont),
                                 a.tabs[2u * l].mont);
        za = St::from(z0);
        zb = St::from(mm40(z0, a.M1.mont));
    }
    const global_ptr<uint64_t> out = as_global(a.out);
    for (;;) {
        const global_ptr<u64x2> p =
            reinterpret_cast<global_ptr<u64x2>>(out + (uint64_t)512 * R * c + 2u * l);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u64x2 v;
            v.x = St::template bits<KIND>(za);
            v.y = St::template bits<KIND>(zb);
            put<NT>(p + r * 256, v);
            if (r + 1 < R) {
                za = St::mul(za, a.J, a.JL);
                zb = St::mul(zb, a.J, a.JL);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        c += gridDim.x;
        if (c >= a.n_chunks) break;
        za = St::mul(za, a.JN, a.JNL);
        zb = St::mul(zb, a.JN, a.JNL);
    }
}

// The last, partial chunk (count < 512 R outputs, one workgroup), from its
// own base.
template <int KIND, int MM, int R, bool NT>
__global__ __launch_bounds__(256) void k_e40_flat_tail(E40FlatArgs a, uint64_t count) {
    typedef Step<MM> St;
    typedef typename St::S S;
    const uint32_t l = threadIdx.x;
    const uint64_t z0 = mm40(a.base, a.tabs[2u * l].mont);
    S za = St::from(z0);
    S zb = St::from(mm40(z0, a.M1.mont));
    const global_ptr<uint64_t> out = as_global(a.out);
    uint64_t k = 2u * l;
    for (int r = 0; r < R && k < count; ++r, k += 512) {
        if (k + 1 < count) {
            u64x2 v;
            v.x = St::template bits<KIND>(za);
            v.y = St::template bits<KIND>(zb);
            put<NT>(reinterpret_cast<global_ptr<u64x2>>(out + k), v);
        } else {
            put<NT>(out + k, St::template bits<KIND>(za));
        }
        za = St::mul(za, a.J, a.JL);
        zb = St::mul(zb, a.J, a.JL);
    }
}

// XCD runs of 4 MiB: chunks of 512 R outputs per XCD run.
template <int R>
constexpr int kE40Run = 1024 / R;

// Whole chunks of a launch of one workgroup per chunk that go to the
// XCD-run kernel.
inline uint64_t e40_run_chunks(int rows, uint64_t n_chunks) {
    const uint64_t run = (uint64_t)kFlatXcds * (1024 / rows);
    return n_chunks / run * run;
}

// a: the whole chunks (grid workgroups; grid == a.n_chunks: one per chunk,
// then mid takes the chunks after the XCD runs, mid.n_chunks of them, from
// its own base); tail: the partial last chunk.
template <int KIND, int MM, int R, bool NT>
hipError_t flat_launch(uint32_t grid, uint32_t lds, hipStream_t s, const E40FlatArgs& a,
                       const E40FlatArgs& mid, const E40FlatArgs& tail, uint64_t tail_count) {
    if (a.n_chunks) {
        if (grid == a.n_chunks && MM == 1) {
            const uint64_t runs = e40_run_chunks(R, a.n_chunks);
            if (runs) {
                E40FlatArgs r = a;
                r.n_chunks = runs;
                k_e40_flat<KIND, MM, R, NT, kE40Run<R>><<<(uint32_t)runs, 256, lds, s>>>(r);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            if (mid.n_chunks) {
                k_e40_flat<KIND, MM, R, NT, 0><<<(uint32_t)mid.n_chunks, 256, lds, s>>>(mid);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
        } else {
            k_e40_flat<KIND, MM, R, NT, 0><<<grid, 256, lds, s>>>(a);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    if (tail_count) {
        k_e40_flat_tail<KIND, MM, R, NT><<<1, 256, 0, s>>>(tail, tail_count);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <int KIND, int MM, bool NT>
hipError_t flat_r(int rows, uint32_t grid, uint32_t lds, hipStream_t s, const E40FlatArgs& a,
                  const E40FlatArgs& mid, const E40FlatArgs& tail, uint64_t tail_count) {
    switch (rows) {
        case 2: return flat_launch<KIND, MM, 2, NT>(grid, lds, s, a, mid, tail, tail_count);
        case 4: return flat_launch<KIND, MM, 4, NT>(grid, lds, s, a, mid, tail, tail_count);
        case 8: return flat_launch<KIND, MM, 8, NT>(grid, lds, s, a, mid, tail, tail_count);
        case 16: return flat_launch<KIND, MM, 16, NT>(grid, lds, s, a, mid, tail, tail_count);
        case 32: return flat_launch<KIND, MM, 32, NT>(grid, lds, s, a, mid, tail, tail_count);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_flat(int kind, int mm, int rows, bool nt, uint32_t grid, uint32_t lds,
                       hipStream_t s, const E40FlatArgs& a, const E40FlatArgs& mid,
                       const E40FlatArgs& tail, uint64_t tail_count) {
#define NN_E40_FLAT(K, M)                                                          \
    return nt ? flat_r<K, M, true>(rows, grid, lds, s, a, mid, tail, tail_count)    \
              : flat_r<K, M, false>(rows, grid, lds, s, a, mid, tail, tail_count);
    if (kind == 0) {
        if (mm) { NN_E40_FLAT(0, 1) } else { NN_E40_FLAT(0, 0) }
    }
    if (mm) { NN_E40_FLAT(1, 1) } else { NN_E40_FLAT(1, 0) }
#undef NN_E40_FLAT
}

template <int KIND, int MM, int IL, int U, bool NT>
hipError_t launch_one(uint32_t grid, uint32_t block, hipStream_t s, const E40Args& a) {
    k_e40<KIND, MM, IL, U, NT><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

template <int KIND, int MM, int IL, bool NT>
hipError_t launch_u(int unroll, uint32_t grid, uint32_t block, hipStream_t s, const E40Args& a) {
    switch (unroll) {
        case 1: return launch_one<KIND, MM, IL, 1, NT>(grid, block, s, a);
        case 2: return launch_one<KIND, MM, IL, 2, NT>(grid, block, s, a);
        case 4: return launch_one<KIND, MM, IL, 4, NT>(grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <int KIND, int MM, bool NT>
hipError_t launch_il(int ilp, int unroll, uint32_t grid, uint32_t block, hipStream_t s,
                     const E40Args& a) {
    switch (ilp) {
        case 1: return launch_u<KIND, MM, 1, NT>(unroll, grid, block, s, a);
        case 2: return launch_u<KIND, MM, 2, NT>(unroll, grid, block, s, a);
        case 4: return launch_u<KIND, MM, 4, NT>(unroll, grid, block, s, a);
        default: return hipErrorInvalidValue;
    }
}

template <int KIND, int MM>
hipError_t launch_nt(int ilp, int unroll, bool nt, uint32_t grid, uint32_t block, hipStream_t s,
                     const E40Args& a) {
    return nt ? launch_il<KIND, MM, true>(ilp, unroll, grid, block, s, a)
              : launch_il<KIND, MM, false>(ilp, unroll, grid, block, s, a);
}

hipError_t launch(int kind, int mm, int ilp, int unroll, bool nt, uint32_t grid, uint32_t block,
                  hipStream_t s, const E40Args& a) {
    if (kind == 0)
        return mm ? launch_nt<0, 1>(ilp, unroll, nt, grid, block, s, a)
                  : launch_nt<0, 0>(ilp, unroll, nt, grid, block, s, a);
    return mm ? launch_nt<1, 1>(ilp, unroll, nt, grid, block, s, a)
              : launch_nt<1, 0>(ilp, unroll, nt, grid, block, s, a);
}

}  // namespace

// The library's default layout at modulus 3^40 for a 16-byte aligned
// output with the FP64 step: the flat one, 16 rows of 512 per chunk, in XCD
// runs, its multipliers at a fixed address (2^30 f64 / 2^28 u64 outputs, one
// MI355X, medians of four interleaved rounds: f64 6.21-6.30 TB/s at caps 3-5
// against 5.98-6.11 with 8 rows, 5.81-5.96 with 32 rows and 6.12 for the row
// layout; u64 6.28-6.36 against 6.10-6.21 with 8 rows and 6.05 for the row
// layout).  The step is VALU-bound, so the longer chunk pays: a lane's
// start (four limb products) is spread over 32 outputs.
constexpr uint32_t kE40FlatDefaultRows = 16;

// nn_e40_generate_ex's flat layout (arguments already validated: a valid
// state, count > 0, an in-range pointer).  cfg: unroll = rows of 512
// outputs per chunk (2, 4, 8, 16, 32; default 16), grid = workgroups per launch
// (0: one per chunk), occupancy = residency cap (0: 4), store policy
// (default temporal).
int generate_flat(uint64_t* state, uint64_t count, void* out_dev, int kind, void* stream,
                  const nn_launch_cfg& c, int mm) {
    if ((c.block && c.block != 256) || c.ilp > 1)
        return fail(NN_EINVAL, "the flat layout has 256 threads per workgroup and no ilp");
    const uint32_t rows = c.unroll ? c.unroll : kE40FlatDefaultRows;
    if (rows != 2 && rows != 4 && rows != 8 && rows != 16 && rows != 32)
        return fail(NN_EINVAL, "unroll %u: the flat layout writes 2, 4, 8, 16 or 32 rows per chunk",
                    rows);
    const Mult40* tab = nullptr;
    int st = device_tables(&tab);
    if (st) return st;
    DeviceTables* d = nullptr;
    st = current_device(&d);
    if (st) return st;
    const uint32_t occ = c.occupancy ? c.occupancy : kFlatDefaultOccupancy;
    if (occ < 2 || occ > 16) return fail(NN_EINVAL, "occupancy %u: must be 0 or in [2, 16]", occ);
    const uint32_t lds = (d->lds_per_cu / (occ + 1) / 512 + 1) * 512;
    if (lds > d->lds_per_block || (uint64_t)lds * occ > d->lds_per_cu)
        return fail(NN_EINVAL, "occupancy %u not expressible on this device", occ);
    const bool nt = (c.flags & NN_CFG_NONTEMPORAL_STORES) != 0;
    const uint64_t s = *state;
    const uint64_t per = 512ull * rows;
    const uint64_t max_launch = kFlatMaxRows * 512;
    E40FlatArgs a;
    a.M1 = make_mult40(kMult);
    a.J = make_mult40(Powers::get().pow(512));
    a.M1L = make_mult40l(a.M1.v);
    a.JL = make_mult40l(a.J.v);
    a.tabs = tab;
    // an output that is only 8-byte aligned: its first element alone (the
    // tail kernel with one output), then the 16-byte aligned rest
    const uint64_t head = ((uintptr_t)out_dev % 16) ? 1 : 0;
    if (head) {
        E40FlatArgs h = a;
        h.n_chunks = 0;
        h.out = (uint64_t*)out_dev;
        h.base = h_mul(s, Powers::get().pow(1));
        const hipError_t e =
            launch_flat(kind, mm, (int)rows, nt, 1, lds, (hipStream_t)stream, h, h, h, 1);
        if (e != hipSuccess) return fail(NN_EHIP, "e40 launch: %s", hipGetErrorString(e));
    }
    for (uint64_t off = head; off < count; off += max_launch) {
        const uint64_t n = count - off < max_launch ? count - off : max_launch;
        a.out = (uint64_t*)out_dev + off;
        a.base = h_mul(s, Powers::get().pow(off + 1));  // the state of this slice's first output
        a.base_lo = limbs(a.base).lo;
        a.base_hi = limbs(a.base).hi;
        a.n_chunks = n / per;
        uint32_t grid = 1;
        if (a.n_chunks) {
            grid = c.grid && c.grid < a.n_chunks ? c.grid : (uint32_t)a.n_chunks;
            a.JN = make_mult40(Powers::get().pow(per * grid - 512ull * (rows - 1)));
            a.JNL = make_mult40l(a.JN.v);
        }
        // one workgroup per chunk with the FP64 step: XCD runs, then the
        // chunks after the last run from their own base
        E40FlatArgs m = a;
        m.n_chunks = 0;
        if (a.n_chunks && grid == a.n_chunks && mm == 1) {
            const uint64_t runs = e40_run_chunks((int)rows, a.n_chunks);
            m.n_chunks = a.n_chunks - runs;
            m.out = a.out + runs * per;
            m.base = h_mul(a.base, Powers::get().pow(runs * per));
            m.base_lo = limbs(m.base).lo;
            m.base_hi = limbs(m.base).hi;
        }
        E40FlatArgs t = a;
        const uint64_t tail = n - a.n_chunks * per;
        t.out = a.out + a.n_chunks * per;
        t.base = h_mul(a.base, Powers::get().pow(a.n_chunks * per));
        const hipError_t e = launch_flat(kind, mm, (int)rows, nt, grid, lds, (hipStream_t)stream,
                                         a, m, t, tail);
        if (e != hipSuccess) return fail(NN_EHIP, "e40 launch: %s", hipGetErrorString(e));
    }
    *state = h_mul(s, Powers::get().pow(count));
    return ok();
}

}  // namespace e40
}  // namespace nn

using namespace nn;

extern "C" {

int nn_e40_seed(uint64_t index, uint64_t* state_out) {
    if (!state_out) return fail(NN_EINVAL, "state_out is NULL");
    if (index < e40::kIndexMin)
        return fail(NN_EINVAL, "index %llu below 3^40+100", (unsigned long long)index);
    *state_out = e40::h_mul(e40::h_pow(2, index - e40::kMod), e40::kHalf);
    return ok();
}

int nn_e40_skip(uint64_t state, uint64_t k, uint64_t* state_out) {
    if (!state_out) return fail(NN_EINVAL, "state_out is NULL");
    if (!e40::valid_state(state))
        return fail(NN_EINVAL, "state %llu is not a unit modulo 3^40", (unsigned long long)state);
    *state_out = e40::h_mul(state, e40::Powers::get().pow(k));
    return ok();
}

int nn_e40_generate_ex(uint64_t* state, uint64_t count, void* out_dev, int kind, void* stream,
                       const nn_launch_cfg* cfg) {
    if (!state) return fail(NN_EINVAL, "state is NULL");
    if (kind != NN_OUT_U64 && kind != NN_OUT_F64) return fail(NN_EINVAL, "kind %d unknown", kind);
    const uint64_t s = *state;
    if (!e40::valid_state(s))
        return fail(NN_EINVAL, "state %llu is not a unit modulo 3^40", (unsigned long long)s);
    if (count == 0) return ok();
    if (count > UINT64_MAX / 8) return fail(NN_ERANGE, "count*8 overflows");
    if (!out_dev) return fail(NN_EINVAL, "output pointer is NULL");
    if ((uintptr_t)out_dev % 8) return fail(NN_EINVAL, "output pointer %p is not 8-byte aligned", out_dev);
    if ((uintptr_t)out_dev > UINTPTR_MAX - count * 8)
        return fail(NN_ERANGE, "output range wraps the address space");
    nn_launch_cfg c = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cfg) c = *cfg;
    const uint32_t known = NN_CFG_TEMPORAL_STORES | NN_CFG_NONTEMPORAL_STORES | NN_CFG_ROWS |
                           NN_CFG_FLAT;
    if ((c.flags & ~known) || (c.width && c.width != 2) ||
        (c.mulmod && c.mulmod != NN_MULMOD_MONTGOMERY && c.mulmod != NN_MULMOD_FP64))
        return fail(NN_EINVAL, "the 3^40 generator takes block, grid, unroll, ilp, occupancy, "
                               "mulmod (NN_MULMOD_FP64 or NN_MULMOD_MONTGOMERY), the store "
                               "policy flags and NN_CFG_ROWS / NN_CFG_FLAT (16-byte stores)");
    if ((c.flags & NN_CFG_ROWS) && (c.flags & NN_CFG_FLAT))
        return fail(NN_EINVAL, "the layout flags are exclusive");
    if ((c.flags & NN_CFG_TEMPORAL_STORES) && (c.flags & NN_CFG_NONTEMPORAL_STORES))
        return fail(NN_EINVAL, "NN_CFG_TEMPORAL_STORES and NN_CFG_NONTEMPORAL_STORES are exclusive");
    const int mm = c.mulmod == NN_MULMOD_MONTGOMERY ? 0 : 1;
    // No layout flag: the flat layout with the FP64 step unless the cfg sets
    // a row-layout field (block, ilp); an output that is only 8-byte aligned
    // gets its first element alone, by default from kFlatUnalignedMin
    // outputs on (below, the row layout's one launch is the cheaper).
    const bool aligned16 = ((uintptr_t)out_dev % 16) == 0;
    const bool flat = (c.flags & NN_CFG_FLAT) ||
                      (!(c.flags & NN_CFG_ROWS) && mm == 1 && !c.block && !c.ilp &&
                       (aligned16 || count >= kFlatUnalignedMin));
    if (flat) return e40::generate_flat(state, count, out_dev, kind, stream, c, mm);
    if (c.occupancy) return fail(NN_EINVAL, "occupancy applies to the flat layout only");
    const uint32_t block = c.block ? c.block : 256u;
    if (block < 64 || block > 1024 || block % 64)
        return fail(NN_EINVAL, "block %u: must be a multiple of 64 in [64, 1024]", block);
    // Defaults from sweeps on MI355X (2^30 f64 outputs, 256 threads):
    //  * FP64 limb step: one workgroup per CU, two rows in flight, no
    //    unrolling: 6.1-6.3 TB/s on two GPUs (ilp 4 within 2 %).  Grids that
    //    are not a multiple of the CU count lose badly (272 workgroups: 3.9
    //    TB/s), since every workgroup carries the same number of rows;
    //  * Montgomery: three workgroups per CU, four rows in flight, unroll 2:
    //    5.6 TB/s (it needs more waves to hide its 64-bit multiplies).
    const bool limb_step = mm == 1;
    const uint32_t unroll = c.unroll ? c.unroll : (limb_step ? 1u : 2u);
    if (unroll != 1 && unroll != 2 && unroll != 4)
        return fail(NN_EINVAL, "unroll %u: must be 1, 2 or 4", unroll);
    const uint32_t ilp = c.ilp ? c.ilp : (limb_step ? 2u : 4u);
    if (ilp != 1 && ilp != 2 && ilp != 4) return fail(NN_EINVAL, "ilp %u: must be 1, 2 or 4", ilp);
    const e40::Mult40* tab = nullptr;
    int st = e40::device_tables(&tab);
    if (st) return st;
    DeviceTables* d = nullptr;
    st = current_device(&d);
    if (st) return st;
    // An 8-byte aligned output: its first element separately, then rows.
    const uint64_t head = ((uintptr_t)out_dev % 16) ? 1 : 0;
    const uint64_t n = count - head;
    uint32_t grid = c.grid;
    if (!grid) {
        const uint64_t need = (n + 2ull * block - 1) / (2ull * block);
        const uint64_t cap = (uint64_t)(d->cus > 0 ? d->cus : 1) * (limb_step ? 1 : 3);
        grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
    }
    if ((uint64_t)grid * block > e40::kMaxThreads)
        return fail(NN_EINVAL, "grid*block exceeds %llu threads",
                    (unsigned long long)e40::kMaxThreads);
    e40::E40Args a;
    a.T = (uint64_t)grid * block;
    const uint64_t row = 2 * a.T;
    a.e_full = n / row;
    a.rem = (uint32_t)(n % row);
    a.head = head ? (uint64_t*)out_dev : nullptr;
    a.head_state = e40::h_mul(s, e40::kMult);  // element 0: z_1
    a.out = (uint64_t*)out_dev + head;
    a.base = head ? e40::h_mul(a.head_state, e40::kMult) : a.head_state;
    a.J = e40::make_mult40(e40::Powers::get().pow(row));
    a.M1 = e40::make_mult40(e40::kMult);
    a.JI = e40::make_mult40(e40::Powers::get().pow(row * ilp));
    a.JL = e40::make_mult40l(a.J.v);
    a.M1L = e40::make_mult40l(a.M1.v);
    a.JIL = e40::make_mult40l(a.JI.v);
    a.t_lo = tab;
    a.t_hi = tab + e40::kLo;
    hipError_t e = e40::launch(kind, mm, (int)ilp, (int)unroll, !(c.flags & NN_CFG_TEMPORAL_STORES),
                               grid, block, (hipStream_t)stream, a);
    if (e != hipSuccess) return fail(NN_EHIP, "e40 launch: %s", hipGetErrorString(e));
    *state = e40::h_mul(s, e40::Powers::get().pow(count));
    return ok();
}

int nn_e40_generate(uint64_t* state, uint64_t count, void* out_dev, int kind, void* stream) {
    return nn_e40_generate_ex(state, count, out_dev, kind, stream, nullptr);
}

int nn_e40_debug_mulmod_ex(int mulmod, const uint64_t* a, const uint64_t* b, uint64_t n,
                           uint64_t* out) {
    if (mulmod != NN_MULMOD_DEFAULT && mulmod != NN_MULMOD_FP64 && mulmod != NN_MULMOD_MONTGOMERY)
        return fail(NN_EINVAL, "mulmod %d: the 3^40 step is NN_MULMOD_FP64 or NN_MULMOD_MONTGOMERY",
                    mulmod);
    if (n && (!a || !b || !out)) return fail(NN_EINVAL, "NULL array");
    for (uint64_t i = 0; i < n; ++i)
        if (!e40::valid_state(a[i]) || !e40::valid_state(b[i]))
            return fail(NN_EINVAL, "pair %llu is not a pair of units modulo 3^40",
                        (unsigned long long)i);
    if (mulmod == NN_MULMOD_MONTGOMERY)
        for (uint64_t i = 0; i < n; ++i) out[i] = e40::mm40(a[i], e40::make_mult40(b[i]).mont);
    else
        for (uint64_t i = 0; i < n; ++i)
            out[i] = e40::to_u64(e40::mul40l(e40::limbs(a[i]), e40::make_mult40l(b[i])));
    return ok();
}

int nn_e40_debug_mulmod(const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t* out) {
    return nn_e40_debug_mulmod_ex(NN_MULMOD_MONTGOMERY, a, b, n, out);
}

}  // extern "C"
