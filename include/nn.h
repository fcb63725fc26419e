/*
 * nn.h -- C ABI of the MI355X (gfx950) alpha_{2,3} normal-number generator.
 *
 * The generator is the linear congruential form of Bailey and Borwein's
 * alpha_{2,3} digit generator studied by Beliakov, Johnstone, Creighton and
 * Wilkin, "Parallel random variates generator for GPUs based on normal
 * numbers" (Section 2, Algorithm BB):
 *
 *   seed     z_0 = 2^(a - 3^33) * floor(3^33 / 2)  mod 3^33      (Eq. 2)
 *   step     z_k = 2^53 * z_(k-1)                  mod 3^33      (Eq. 3)
 *   variate  u_k = z_k * 3^-33 in (0,1)                           (Alg. BB step 3)
 *
 * with period 2 * 3^32 (Section 2).  Every function is extern "C", takes
 * plain integers and pointers, never throws, and returns an nn_status
 * (0 = NN_OK).  On any error nothing is enqueued and no output argument is
 * written.  A failing call leaves a human-readable detail retrievable with
 * nn_last_error() on the same host thread.
 *
 * States.  A state is a unit modulo 3^33: 1 <= s < 3^33 and s mod 3 != 0.
 * Every unit lies on the single cycle of Eq. 3 (2^53 generates the unit
 * group), so any unit is a valid state; anything else is NN_EINVAL.
 *
 * Output convention.  A call that emits n values after state s emits
 * z_1..z_n (Eq. 3 applied before each output, as Algorithm BB returns z_k
 * for k >= 1) and leaves s = z_n, so consecutive calls concatenate to the
 * serial sequence.  F64 outputs are RN(double(z) * RN(1/3^33)), the product
 * with the rounded reciprocal that the paper's listings multiply by; U64
 * outputs are the raw states z.
 */
#ifndef NN_H
#define NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nn_status {
    NN_OK = 0,
    NN_EINVAL = 1, /* invalid argument: state, index, kind, pointer, config */
    NN_ERANGE = 2, /* count too large for the address space or a descriptor */
    NN_EHIP = 3,   /* a HIP runtime call or kernel launch failed */
    NN_ENOMEM = 4, /* device or host allocation failed */
    NN_ENODEV = 5, /* no usable gfx950 device */
    NN_ECANCELED = 6 /* a served request was cancelled before admission */
} nn_status;

typedef enum nn_out_kind {
    NN_OUT_U64 = 0, /* raw states z_k (uint64) */
    NN_OUT_F64 = 1  /* variates RN(z_k * RN(3^-33)) (IEEE binary64) */
} nn_out_kind;

/* 106-bit modular multiplication used by the step loop.  All are exact;
 * they differ only in speed (Section 3.1 discusses the paper's own
 * choices; these are the gfx950 candidates). */
typedef enum nn_mulmod {
    NN_MULMOD_DEFAULT = 0,
    NN_MULMOD_FP64 = 1,     /* FP64 FMA two-product, FP64 quotient estimate */
    NN_MULMOD_BARRETT = 2,  /* integer Barrett, k = 53, mu = floor(2^106/m) */
    NN_MULMOD_SHOUP = 3,    /* integer fixed-multiplier quotient (Shoup)    */
    NN_MULMOD_MONTGOMERY = 4, /* integer Montgomery, R = 2^64, pre-scaled  */
    NN_MULMOD_MODBARRETT = 5  /* Section 3.1's Modified Barrett: the step by
                                 exactly 2^53 only (consecutive layout)     */
} nn_mulmod;

#define NN_MODULUS 5559060566555523ULL   /* 3^33 */
#define NN_PERIOD 3706040377703682ULL    /* 2 * 3^32 */
#define NN_INDEX_MIN 5559060566555623ULL /* 3^33 + 100 (Algorithm BB step 1) */
#define NN_INDEX_MAX 9007199254740992ULL /* 2^53       (Algorithm BB step 1) */

/* Launch configuration.  Any field left 0 takes the library default.
 *
 * Three layouts write the same values (serial order in memory):
 *  - flat (NN_CFG_FLAT; the default for a cfg that sets none of block,
 *    grid, ilp or width 1, on an output that is 16-byte aligned or, with
 *    width 0, holds at least 2^22 outputs): every 256-thread workgroup writes `unroll` rows of 512
 *    consecutive outputs (one contiguous chunk), two per lane in one
 *    16-byte store per row, and exits; an output that is only 8-byte
 *    aligned gets its first element from a one-workgroup launch and the
 *    rest 16-byte aligned.  With 4 rows the chunks are
 *    taken in XCD runs: of every 2048 consecutive chunks, each of the 8
 *    XCDs (which take consecutive workgroups in turn) writes 256
 *    consecutive ones (4 MiB); chunks after the last full run, and every
 *    chunk with other row counts, in address order;
 *  - rows (NN_CFG_ROWS; the default otherwise): grid*block threads loop
 *    over rows of width*grid*block outputs, stepping by a jump multiplier;
 *  - consecutive (NN_CFG_CONSECUTIVE): the paper's per-thread loop (Section
 *    3.2): each thread makes `unroll` consecutive outputs with Eq. 3's own
 *    multiplier 2^53 and Section 3.1's Modified Barrett reduction; the
 *    workgroup's block*unroll outputs pass through LDS and leave in serial
 *    order with coalesced stores (the paper instead stored them strided,
 *    out of order).  Workgroup w takes tiles w, w + grid, ...
 *
 * block: threads per workgroup, a multiple of 64 in [64,1024] (rows,
 * consecutive).
 * grid: workgroups, block*grid <= 2^24 (rows); block*grid*unroll <= 2^25
 * (consecutive).
 * mulmod: an nn_mulmod; NN_MULMOD_MODBARRETT only, and only it, with the
 * consecutive layout (0 selects it there).
 * unroll: 1, 2, 4 or 8 iterations of the step loop per trip (rows); outputs
 * per thread and tile, 2, 4, 8, 16 or 32 (consecutive, default 4 with 512
 * threads per workgroup); rows per workgroup, 1, 2, 4, 8 or 16 (flat,
 * default 4).
 * flags: NN_CFG_TEMPORAL_STORES keeps stores cacheable and
 * NN_CFG_NONTEMPORAL_STORES makes them non-temporal streaming stores (at
 * most one of the two; default: non-temporal, except temporal for the flat
 * layout); NN_CFG_ROWS / NN_CFG_FLAT force a layout (see above for the
 * default).
 * width: outputs per lane and store, 1 (8-byte stores) or 2 (16-byte
 * stores, needs a 16-byte aligned output) (rows; flat is always 2).
 * occupancy: 0, or a cap in [2,16] on resident workgroups per compute unit
 * (flat; 0 there means 4), enforced through unused dynamic LDS.
 * Consecutive: width 2 (16-byte stores) on a 16-byte aligned output, else 1. 
 * ilp: rows each thread keeps in flight, 1, 2 or 4 (rows with width 2):
 * 2*ilp independent multiplication chains per lane. */
typedef struct nn_launch_cfg {
    uint32_t block;
    uint32_t grid;
    uint32_t mulmod; /* nn_mulmod */
    uint32_t unroll;
    uint32_t flags;
    uint32_t width;
    uint32_t occupancy;
    uint32_t ilp;
} nn_launch_cfg;
#define NN_CFG_TEMPORAL_STORES 1u
#define NN_CFG_ROWS 2u
#define NN_CFG_FLAT 4u
#define NN_CFG_CONSECUTIVE 8u
/* The paper's own layout (Section 3.2), for comparison: T = count / unroll
 * threads (block threads per workgroup, default 512), thread t makes
 * elements t*E .. t*E + E-1 (E = unroll, default 4096, must divide count)
 * with the Modified Barrett step and stores its i-th one at out[t + i*T]:
 * coalesced 8-byte stores, but the array holds the sequence TRANSPOSED,
 * out[t + i*T] = z_(t*E + i + 1), not in serial order.  mulmod 0 or
 * NN_MULMOD_MODBARRETT; grid, width, ilp and occupancy must be 0. */
#define NN_CFG_PAPER_STRIDED 16u
#define NN_CFG_NONTEMPORAL_STORES 32u
/* Flat layout with 4 rows: the whole chunks in address order (workgroup w
 * writes chunk w) instead of the default XCD runs; for comparison. */
#define NN_CFG_ADDRESS_ORDER 128u

/* ---------------------------------------------------------------- host -- */

/* nn_seed -- Eq. 2 (Algorithm BB steps 1-2): the state z_0 of starting index
 * `index`.  index must lie in [NN_INDEX_MIN, NN_INDEX_MAX] (inclusive, as
 * Algorithm BB step 1 states the range); otherwise NN_EINVAL.  state_out must
 * be non-NULL.  Pure host computation, thread-safe, no device needed. */
int nn_seed(uint64_t index, uint64_t *state_out);

/* nn_skip -- skip-ahead (Section 2, last paragraph: any iterate is computable
 * directly): *state_out = the state k steps after `state`, i.e.
 * state * (2^53)^k mod 3^33.  Any 64-bit k is accepted; it is reduced modulo
 * the period 2*3^32.  NN_EINVAL for an invalid state or NULL state_out.
 * Pure host computation, thread-safe, no device needed. */
int nn_skip(uint64_t state, uint64_t k, uint64_t *state_out);

/* --------------------------------------------------------------- device -- */

/* nn_init -- set up the library on HIP device `device` (uploads the
 * immutable skip-ahead tables, about 3.4 MB: 69 632 48-byte multipliers
 * and the 43 KB device-API table, owned by the library until process
 * exit).  Optional: the first generating call on a device does it.  The
 * caller's current device is left unchanged.  Thread-safe. */
int nn_init(int device);

/* nn_generate -- Algorithm BB step 3 for `count` outputs (Eq. 3 iterated).
 * Writes z_1..z_count after *state, in serial order, to out_dev[0..count)
 * as uint64 (NN_OUT_U64) or binary64 (NN_OUT_F64), then sets *state to
 * z_count.  out_dev: device memory owned by the caller on the current HIP
 * device, 8-byte aligned, holding count*8 bytes; the library keeps no
 * reference to it.  stream: a hipStream_t (NULL = the legacy default
 * stream).  Asynchronous: the kernel is enqueued on `stream` and the host
 * state is advanced by skip-ahead without waiting.  count == 0 is a no-op
 * (out_dev may then be NULL).  Errors: NN_EINVAL (state, kind, NULL or
 * misaligned pointers), NN_ERANGE (count*8 overflows), NN_EHIP (launch
 * failed; *state unchanged). */
int nn_generate(uint64_t *state, uint64_t count, void *out_dev, int kind, void *stream);

/* nn_generate_ex -- nn_generate with an explicit launch configuration
 * (cfg may be NULL for the defaults).  The output is identical for every
 * valid configuration.  NN_EINVAL for an invalid configuration. */
int nn_generate_ex(uint64_t *state, uint64_t count, void *out_dev, int kind, void *stream,
                   const nn_launch_cfg *cfg);

/* nn_default_cfg -- the configuration nn_generate would use for `count`
 * outputs of `kind` on the current device (fields all filled in). */
int nn_default_cfg(int kind, uint64_t count, nn_launch_cfg *cfg_out);

/* nn_consume -- the fused consumer: generates the `count` outputs after
 * *state exactly as nn_generate would, but reduces them in registers
 * instead of storing them (variates usually feed a simulation directly,
 * Section 3.2; Table 2 measures generation with the memory traffic
 * removed).  Adds to *result_dev (device memory, 8-byte aligned, one
 * value the caller initialises): for NN_OUT_U64 the sum of the raw states
 * z_1..z_count modulo 2^64 (exact, independent of the launch shape); for
 * NN_OUT_F64 the binary64 sum of the variates (summation order depends on
 * the launch shape).  Sets *state to z_count.  cfg: block, grid and mulmod
 * only (NULL for the defaults).  Asynchronous on `stream`. */
int nn_consume(uint64_t *state, uint64_t count, int kind, void *result_dev, void *stream,
               const nn_launch_cfg *cfg);

/* ------------------------------------------------ device-side generation --
 * For consumer kernels that make variates where they use them (nn_device.h,
 * the header-only device functions built on these two calls). */

/* A multiplier v = (2^53)^k mod 3^33 in the form nn_dev_mulmod takes: v as a
 * double (exact, v < 2^53) and v / 3^33 as the double-double qh + ql. */
typedef struct nn_dev_mult {
    double v;
    double qh;
    double ql;
} nn_dev_mult;

#define NN_DEV_SKIP_LEVELS 7u
#define NN_DEV_SKIP_SIZE 256u

/* nn_dev_mult_pow -- (2^53)^k mod 3^33 (Eq. 3 applied k times; k is taken
 * modulo the period) as an nn_dev_mult.  Host only, pure, thread-safe.
 * NN_EINVAL if out is NULL. */
int nn_dev_mult_pow(uint64_t k, nn_dev_mult *out);

/* nn_dev_skip_table -- device pointer, on the current HIP device, of the
 * skip table nn_dev_skip reads: NN_DEV_SKIP_LEVELS x NN_DEV_SKIP_SIZE
 * entries, entry [lvl][j] = (2^53)^(j * 256^lvl) as an nn_dev_mult.  Owned
 * by the library, immutable, valid until the process ends; set up as by
 * nn_init.  NN_EINVAL if table_out is NULL; NN_ENODEV / NN_ENOMEM / NN_EHIP
 * as nn_init. */
int nn_dev_skip_table(const nn_dev_mult **table_out);

/* nn_fill -- the paper's "Constant" measurement kernel (Section 4.2,
 * Tables 1-2): writes `value` to out_dev[0..count) with exactly the store
 * pattern nn_generate_ex uses for the same cfg and NN_OUT_F64 (the same
 * layout, launch shape, rows per workgroup, store policy and residency cap,
 * fields left 0 resolving as they do for F64 output), with the arithmetic
 * taken out: the write-bandwidth ceiling of that pattern.  Same pointer
 * rules and errors as nn_generate. */
int nn_fill(uint64_t count, void *out_dev, uint64_t value, void *stream,
            const nn_launch_cfg *cfg);
/* nn_fill only, flat layout: also make the generator's start in each
 * workgroup -- its table loads, with a comparison in place of its
 * multiplications -- before the stores, so the fill is the generator minus
 * its arithmetic (Table 2 removes the memory-access time from the
 * generation time; on MI355X a fill of bare back-to-back stores in the
 * generator's pattern writes slower than the generator itself). */
#define NN_FILL_WITH_START 64u

/* -------------------------------------------------------------- batch -- */

/* One stream of a batch: a window of the sequence.  The call writes the
 * `length` outputs that follow `state` (z_1..z_length after it) to
 * out[out_offset .. out_offset + length).  Windows of one batch must not
 * overlap in the output (overlapping windows leave the overlap undefined). */
typedef struct nn_stream_desc {
    uint64_t state;
    uint64_t length;
    uint64_t out_offset;
} nn_stream_desc;

/* Batch configuration (0 = default).  The batch is cut into rows of
 * 2*block outputs handed to `grid` persistent workgroups; a workgroup steps
 * its states while a stream continues and skips ahead afresh where a new
 * one starts.  By default the workgroups form clusters of `cluster`
 * consecutive workgroups: each cluster takes a contiguous range of rows and
 * its members take every cluster-th row of it (cluster 1: each workgroup a
 * contiguous range).
 * block: threads per workgroup (a multiple of 64 in [64,1024]); grid:
 * workgroups (a multiple of cluster); cluster: 1..64 (interleaved: up to
 * grid; 0 = grid); mulmod: an
 * nn_mulmod; flags: NN_CFG_TEMPORAL_STORES, NN_BATCH_NO_GRAPH (enqueue a
 * copy and a kernel launch instead of replaying the plan's graph),
 * NN_BATCH_INTERLEAVED; occupancy: NN_BATCH_CHUNKS only, 0 (4) or a cap in
 * [2,16] on the chunk kernel's resident workgroups per compute unit (as
 * nn_launch_cfg's occupancy caps the plain flat layout's). */
typedef struct nn_batch_cfg {
    uint32_t block;
    uint32_t grid;
    uint32_t cluster;
    uint32_t mulmod;
    uint32_t flags;
    uint32_t occupancy;
} nn_batch_cfg;
#define NN_BATCH_NO_GRAPH 8u
/* Interleaved kernel: a pre-pass writes one record per row of 2*block
 * outputs (its first state and output index; rows aligned to the output),
 * so a workgroup enters a stream at no cost and rows can be dealt out
 * freely: clusters of `cluster` consecutive workgroups take contiguous
 * ranges of rows and interleave them (cluster 0: one range for all, i.e.
 * workgroup w writes rows w, w + grid, ..., one region of the output at a
 * time, as the plain generator does).  Needs the FP64 reduction, block 64,
 * 128 or 256, a grid that cluster divides, and output indices below 2^51
 * (NN_ERANGE otherwise).  Batches of at most 16 windows travel in the
 * kernel arguments and run the blocked kernel in either case. */
#define NN_BATCH_INTERLEAVED 16u
/* Chunked kernel: the plain generator's flat layout over a batch.  The
 * output is cut into aligned chunks of 2048 outputs (16 KiB); a pre-pass
 * writes the chunks' records (the state of the chunk's first element as if
 * the window covered it, and the window's part of the chunk), and
 * 256-thread workgroups write the records' chunks as four rows of 512
 * outputs with one 16-byte store per lane and row.  The plan sorts the
 * windows by output offset (they are independent) and gives each chunk one
 * record and one workgroup, which writes every window's part of it; windows
 * that overlap each other get a record per chunk and window instead.
 * grid 0 (the default): one workgroup per record, the records taken in
 * the plain flat layout's XCD runs (the plan's graph gets the batch's
 * record count as its grid before each replay); a nonzero grid: that many
 * persistent workgroups taking the records round-robin in the same order.  Needs
 * the FP64 reduction, block 0 or 256, cluster 0 or 1 and output indices
 * below 2^51 (NN_ERANGE otherwise).  Exclusive with NN_BATCH_INTERLEAVED.
 * Batches of at most 16 windows travel in the kernel arguments (the FP64
 * reduction's flat inline kernel). */
#define NN_BATCH_CHUNKS 32u

/* Opaque batch plan: device workspace, pinned staging and a hipGraph of
 * (staging -> workspace copy, persistent kernel) whose arguments never
 * change, owned by the library until nn_batch_plan_destroy.  A chunked
 * plan (NN_BATCH_CHUNKS) also owns a stream (non-blocking, default
 * priority) that carries each batch's descriptor upload and record
 * pre-pass, so they run during the previous batch's kernel; its graph holds
 * the chunk kernel alone. */
typedef struct nn_batch_plan nn_batch_plan;

/* nn_batch_plan_create -- a plan on the current device for batches of at
 * most `max_streams` streams and `max_outputs` outputs in total, writing
 * `kind` outputs.  Allocates two slots (batches alternate between them),
 * each a workspace of 40 bytes per descriptor (one per stream, plus one per
 * 2^24 outputs for the split of long streams) in device and pinned host
 * memory; the interleaved and chunked kernels add 16 bytes of device
 * memory per record (one per row of 2*block outputs or chunk of 2048, plus
 * two per descriptor, and for chunks one more per descriptor).
 * Errors: NN_EINVAL (kind, cfg), NN_ERANGE (capacity), NN_ENOMEM, NN_EHIP. */
int nn_batch_plan_create(int kind, uint32_t max_streams, uint64_t max_outputs,
                         const nn_batch_cfg *cfg, nn_batch_plan **plan_out);
/* Waits for the plan's last batch, then frees it (NULL is a no-op). */
int nn_batch_plan_destroy(nn_batch_plan *plan);
/* The plan's resolved configuration. */
int nn_batch_plan_cfg(const nn_batch_plan *plan, nn_batch_cfg *cfg_out);

/* nn_generate_batch -- the batched form of Algorithm BB step 3: every
 * stream of `descs` (host array of n) is generated by one persistent kernel
 * launch on `stream` (a hipStream_t), replayed from the plan's hipGraph.
 * It takes a plan rather than (descs, n, out, kind, stream) alone because a
 * hipGraph is replayed with fixed kernel arguments: the plan owns the
 * instantiated graphs and the device workspace their arguments point to
 * (descriptors, records), and fixes the output kind and kernel shape, so a
 * call uploads descriptors and replays without allocating or capturing.
 * nn_generate_batch_static below is the plan-free form of the same call.
 * out_dev: device memory of the plan's device, 16-byte aligned, holding
 * every window.  Streams longer than 2^24 outputs are split internally.
 * Outputs are identical to nn_generate on each stream alone.  final_states
 * (host array of n, or NULL) receives each stream's state after its window.
 * Asynchronous; the call blocks only while the plan's previous batch is
 * still copying its descriptors.  In a chunked plan the upload and the
 * pre-pass go to the plan's own stream and `stream` waits for them through
 * an event before the chunk kernel, so the call is not meant for a stream
 * under capture (the plan replays graphs of its own).  A plan serves one
 * call at a time (calls on one plan are serialised).  Errors: NN_EINVAL (states, pointers, wrong
 * device), NN_ERANGE (more streams or outputs than the plan holds; nothing
 * is enqueued), NN_EHIP. */
int nn_generate_batch(nn_batch_plan *plan, const nn_stream_desc *descs, uint32_t n,
                      void *out_dev, void *stream, uint64_t *final_states);

/* nn_generate_batch_static -- nn_generate_batch for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no plan, and no allocation of any kind.  The
 * workspace (descriptors and chunk records) is a fixed static array of
 * about 23 MB that every device loading the library holds until the
 * process ends.  Every stream of `descs` (host array of n) is written to
 * out_dev (device memory of the current device, 16-byte aligned) with the
 * chunked batch kernel (NN_BATCH_CHUNKS, non-temporal stores); outputs are
 * identical to nn_generate on each stream alone.  kind: nn_out_kind.
 * final_states (host array of n, or NULL) receives each stream's state
 * after its window.  Limits: at most 65 536 streams and 2^31 outputs per
 * call, output indices below 2^51 (NN_ERANGE otherwise; nothing is
 * enqueued).  Asynchronous on `stream`: descs is read by an asynchronous
 * host-to-device copy on that stream, so keep it unchanged until the stream
 * has passed this call's work.  All calls on one device share the one
 * workspace, which keeps the last call's contents: calls that overlap on
 * one device (different streams, or different host threads, without
 * ordering between them) race and may write wrong outputs; calls ordered on
 * one stream are safe.  Errors: NN_EINVAL (kind, states, pointers),
 * NN_ERANGE, NN_EHIP. */
int nn_generate_batch_static(const nn_stream_desc *descs, uint32_t n, void *out_dev, int kind,
                             void *stream, uint64_t *final_states);

/* ------------------------------------------------------------- server -- */

/* The served form: continuous batching of variate requests.  Each client
 * stream has a state at position 0, held in a device table.  A request
 * (stream, count) receives the next `count` outputs of its stream in
 * submission order (its window is fixed at submission), so its bytes are
 * the same whether it runs alone or with any other traffic.  Requests are
 * admitted from the head of the arrival queue while the output pool has
 * room and slots are free, and launched as batches on `lanes` concurrent
 * HIP streams, each replaying a batch plan's graph. */
typedef struct nn_server nn_server;

typedef struct nn_server_cfg {
    void *pool;                  /* caller-owned output pool (device memory of the
                                    current device, 256-byte aligned), or NULL for
                                    one owned by the server */
    uint64_t pool_bytes;         /* output pool size in bytes, > 0 */
    uint64_t max_batch_outputs;  /* outputs per batch and per request; 0 = 2^27 */
    uint32_t max_batch_requests; /* requests per batch; 0 = 4096 */
    uint32_t max_slots;          /* admitted, unreleased requests; 0 = 65536 */
    uint32_t lanes;              /* concurrent batches; 0 = 2, at most 64 */
    uint32_t kind;               /* nn_out_kind */
    uint32_t flags;              /* NN_SERVER_FAKE_DEVICE */
    nn_batch_cfg batch;          /* kernel shape of every lane's plan */
    double fake_latency_s;       /* fake device: seconds per batch */
    double fake_bytes_per_s;     /* fake device: write rate (0 = instant) */
    /* NN_SERVER_DEVICE_QUEUE only: */
    uint64_t queue_max_outputs;  /* requests of at most this many outputs go to
                                    the device queue; 0 = 2^18 */
    uint32_t queue_workgroups;   /* workgroups of the queue kernel; 0 = 16 */
    uint32_t queue_capacity;     /* ring entries, a power of two; 0 = 1024 */
    double queue_idle_s;         /* the queue kernel leaves after this long
                                    without work (and is relaunched on demand);
                                    0 = 0.05 */
} nn_server_cfg;
/* Fake device: host memory pool, outputs computed on the host by the
 * library's exact host arithmetic, completions on a clock set by the caller
 * (nn_server_set_clock), launch failures injectable.  For testing the
 * scheduler without a GPU. */
#define NN_SERVER_FAKE_DEVICE 1u
/* Device request queue: admitted requests up to queue_max_outputs skip the
 * batch launch.  A persistent kernel on its own stream serves them from a
 * ring in host-mapped memory that the server publishes into, so such a
 * request costs no launch; its workgroups claim the request's rows as they
 * reach it.  Larger requests, and small ones while two per queue workgroup
 * are already in flight or the ring is full, take the batch lanes.  Outputs are the same either way (windows are fixed at
 * submission).  GPU only. */
#define NN_SERVER_DEVICE_QUEUE 2u

typedef struct nn_completion {
    uint64_t ticket;
    uint64_t count;
    uint64_t position; /* window start within the stream (modulo the period) */
    void *data;        /* the outputs: device pointer into the pool (host
                          pointer on the fake device); valid until release */
    double t_submit, t_admit, t_launch, t_done; /* seconds on the server clock */
    uint32_t stream_id;
    int32_t status;    /* NN_OK, NN_EHIP (launch failed) or NN_ECANCELED */
} nn_completion;

typedef struct nn_server_stats {
    uint64_t submitted, completed, failed, released;
    uint64_t in_flight, batches, queued, pending;
    uint64_t pool_used, pool_peak, slots_used;
    double now;
} nn_server_stats;

/* nn_server_create -- a server on the current device for n_streams client
 * streams whose states at position 0 are stream_states (host array of
 * units).  Allocates the pool, the state table and `lanes` batch plans.
 * Errors: NN_EINVAL, NN_ENOMEM, NN_EHIP. */
int nn_server_create(const nn_server_cfg *cfg, const uint64_t *stream_states, uint32_t n_streams,
                     nn_server **out);
/* Waits for in-flight batches and frees everything (NULL is a no-op). */
int nn_server_destroy(nn_server *srv);
/* Queues a request; *ticket_out identifies it.  NN_ERANGE if it can never
 * be admitted (larger than the pool or than max_batch_outputs). */
int nn_server_submit(nn_server *srv, uint32_t stream_id, uint64_t count, uint64_t *ticket_out);
/* Makes progress (harvest finished batches, admit, launch) and reports up
 * to max_out finished requests, oldest first, into out (host array). */
int nn_server_poll(nn_server *srv, nn_completion *out, uint32_t max_out, uint32_t *n_out);
/* Returns a reported request's pool region and slot to the server. */
int nn_server_release(nn_server *srv, uint64_t ticket);
/* Cancels a request still in the queue (it finishes with NN_ECANCELED). */
int nn_server_cancel(nn_server *srv, uint64_t ticket);
int nn_server_stats_get(nn_server *srv, nn_server_stats *out);
/* Fake device only: advance the server clock; inject n launch failures. */
int nn_server_set_clock(nn_server *srv, double now);
int nn_server_inject_failures(nn_server *srv, uint32_t n);

/* ------------------------------------------------------------- replay -- */

/* Native load generators for measuring the served form against one launch
 * per request on the same arrival trace (host arrays of n requests, arrival
 * times in seconds, non-decreasing, divided by time_scale).  Both run in
 * real time on the calling thread, release every output as soon as it is
 * finished, and write each request's latency (seconds from its arrival to
 * the moment its completion was observed) to latency_out[i].  timeout_s > 0
 * bounds the run (NN_ERANGE when exceeded). */
typedef struct nn_replay_stats {
    double wall_s;
    uint64_t requests, variates, failed;
    /* Each request's latency in three stages (seconds, p50 and p99 over the
     * requests): `seen`, from its arrival to the moment the loop submitted
     * it; `launch`, from there until its work was enqueued on the GPU (the
     * server's admission and batching included); `done`, from the enqueue
     * until its completion was observed. */
    double seen_p50, seen_p99, launch_p50, launch_p99, done_p50, done_p99;
} nn_replay_stats;

/* The trace through `srv` (nn_server_submit / _poll / _release). */
int nn_server_replay(nn_server *srv, const double *t_arrive, const uint32_t *stream_id,
                     const uint64_t *count, uint64_t n, double time_scale, double timeout_s,
                     double *latency_out, nn_replay_stats *stats_out);

/* The trace with one nn_generate launch per request on `stream`: window
 * positions per stream in arrival order as in the server, outputs in a ring
 * over pool_dev (pool_elems outputs of `kind`, caller-owned device memory);
 * a request waits while the ring is full. */
int nn_replay_per_request(const uint64_t *stream_states, uint32_t n_streams,
                          const double *t_arrive, const uint32_t *stream_id,
                          const uint64_t *count, uint64_t n, double time_scale, double timeout_s,
                          void *pool_dev, uint64_t pool_elems, int kind, void *stream,
                          double *latency_out, nn_replay_stats *stats_out);

/* ------------------------------------------------------------- status -- */

/* Static description of a status code (never NULL). */
const char *nn_strerror(int status);
/* Detail of the last failing call on this host thread ("" if none). */
const char *nn_last_error(void);
/* Library version string. */
const char *nn_version(void);

/* ------------------------------------------------------ modulus 3^40 -- */
/* The larger modulus Section 2 names for a longer period: the same
 * generator with m = 3^40 (period 2*3^39), the multiplier 2^53 of Eq. 3
 * (53 bits of alpha_{2,3} per step, now at positions 3^40 and above) and
 * Eq. 2 with 3^40 in place of 3^33.  A state is a unit modulo 3^40 (all 64
 * bits are used).  F64 outputs are RN(RN(z) * RN(1/3^40)), RN(z) being the
 * rounding of the 64-bit state to binary64; they lie in (0,1).  Same output
 * convention as above (step-then-emit, *state left at the last output). */
#define NN_E40_MODULUS 12157665459056928801ULL   /* 3^40 */
#define NN_E40_PERIOD 8105110306037952534ULL     /* 2 * 3^39 */
#define NN_E40_INDEX_MIN 12157665459056928901ULL /* 3^40 + 100 */
#define NN_E40_INDEX_MAX 18446744073709551615ULL /* 2^64 - 1 (the index type) */

/* Eq. 2 at modulus 3^40: the state of starting index `index` in
 * [NN_E40_INDEX_MIN, NN_E40_INDEX_MAX]; NN_EINVAL otherwise.  Host, pure. */
int nn_e40_seed(uint64_t index, uint64_t *state_out);

/* The state k steps after `state` at modulus 3^40 (k reduced modulo the
 * period).  NN_EINVAL for a non-unit state or NULL state_out.  Host, pure. */
int nn_e40_skip(uint64_t state, uint64_t k, uint64_t *state_out);

/* nn_generate at modulus 3^40: writes z_1..z_count after *state to out_dev
 * (device memory, 8-byte aligned, count*8 bytes, owned by the caller) as
 * uint64 or binary64 and sets *state to z_count; asynchronous on `stream`.
 * cfg (NULL for the defaults) may set block, grid, unroll (1, 2, 4), ilp
 * (1, 2, 4), NN_CFG_TEMPORAL_STORES and mulmod: NN_MULMOD_FP64 (the
 * default: states as two base-3^20 limbs, since 3^40 = (3^20)^2 the step is
 * three exact FP64 products modulo 3^20; defaults 256 threads, one
 * workgroup per CU, ilp 2, unroll 1) or NN_MULMOD_MONTGOMERY (64-bit
 * states, R = 2^64; defaults 256 threads, three workgroups per CU, ilp 4,
 * unroll 2).  Layouts: the row layout, or (NN_CFG_FLAT, and the default for
 * either kind with the FP64 step) the flat layout: one 256-thread workgroup
 * per chunk of `unroll` rows of 512 outputs (2, 4, 8, 16, 32; default 16),
 * residency capped by `occupancy` (default 4); with one workgroup per chunk
 * (grid 0) the chunks are taken in XCD runs of 4 MiB per XCD as in the 3^33
 * flat layout; an output that is only 8-byte aligned gets its first element
 * alone (by default from 2^22 outputs on); NN_CFG_ROWS forces the row
 * layout.  16-byte stores in both.  Both
 * reductions give the same bits.  Errors as nn_generate_ex. */
int nn_e40_generate_ex(uint64_t *state, uint64_t count, void *out_dev, int kind, void *stream,
                       const nn_launch_cfg *cfg);
int nn_e40_generate(uint64_t *state, uint64_t count, void *out_dev, int kind, void *stream);

/* ---------------------------------------------------------- diagnostic -- */

/* nn_debug_mulmod -- runs the host build of a step-loop modular
 * multiplication (the same source the device compiles) on n pairs:
 * out[i] = a[i] * b[i] mod 3^33, with b[i] taking the role of the fixed
 * multiplier.  Every a[i] and b[i] must be a valid state;
 * NN_MULMOD_MODBARRETT multiplies by 2^53 itself and needs every b[i] to be
 * 2^53 mod 3^33.  NN_DEBUG_DEVICE_MULMOD selects the public device header's
 * nn_dev_mulmod (include/nn_device.h), the FP64 reduction without the
 * two-product of q 3^33 that the library's storing kernels use.  For testing
 * the arithmetic on a CPU; host pointers. */
#define NN_DEBUG_DEVICE_MULMOD 100
int nn_debug_mulmod(int mulmod, const uint64_t *a, const uint64_t *b, uint64_t n,
                    uint64_t *out);

/* nn_e40_debug_mulmod -- the host build of the 3^40 step's Montgomery
 * reduction: out[i] = a[i] * b[i] mod 3^40 for units a[i], b[i]; host
 * pointers.  nn_e40_debug_mulmod_ex selects the reduction: NN_MULMOD_FP64
 * (or NN_MULMOD_DEFAULT; the base-3^20 limb step) or NN_MULMOD_MONTGOMERY;
 * NN_EINVAL for any other, a NULL array or a non-unit operand. */
int nn_e40_debug_mulmod(const uint64_t *a, const uint64_t *b, uint64_t n, uint64_t *out);
int nn_e40_debug_mulmod_ex(int mulmod, const uint64_t *a, const uint64_t *b, uint64_t n,
                           uint64_t *out);

#ifdef __cplusplus
}
#endif

#endif /* NN_H */
