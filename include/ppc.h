/*
 * ppc.h -- positional population count (pospopcnt) on AMD Instinct MI355X.
 *
 * The operation (Clausecker, Lemire, Schintke, "Faster Positional-Population
 * Counts for AVX2, AVX-512, and ASIMD", Section 1, Fig. 2): for an array of
 * w-bit words, counts[j] += number of words whose bit j is set, j < w,
 * w in {8, 16, 32, 64}.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory.  `buf` and `counts` are DEVICE pointers (memory of the current
 *    HIP device).  The caller owns both.  `counts` holds w uint64 values and
 *    must be 8-byte aligned.  `buf` may have any byte alignment.
 *  - Words.  Word i is the little-endian integer of bytes buf[i*s .. i*s+s-1],
 *    s = w/8.  Bit positions are relative to `buf`, not to absolute
 *    addresses: byte buf[b] feeds counters 8*(b mod s) .. 8*(b mod s)+7.
 *    A trailing partial word is counted as if zero-padded; `nbytes` may be
 *    any value.  Bytes outside [buf, buf+nbytes) are never read.
 *  - Accumulation.  Counts are ADDED to `counts`, never cleared (Section 4,
 *    step 1 and its footnote: this is what streamed input needs).  Counters
 *    wrap modulo 2^64.
 *  - Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Every call only enqueues work and returns; results are valid
 *    once the stream has reached that point.
 *  - Errors.  Every call returns a ppc_status.  Invalid arguments return
 *    PPC_EINVAL and enqueue nothing; a failed HIP call returns PPC_EDEVICE.
 *    No call aborts the process.  nbytes == 0 is a successful no-op (buf may
 *    then be NULL).
 *  - Aliasing.  `counts` must not overlap `buf`.
 */
#ifndef PPC_H
#define PPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ppc_status {
    PPC_OK = 0,      /* success                                            */
    PPC_EINVAL = 1,  /* invalid argument (bad width, NULL, misaligned ...)  */
    PPC_ENOMEM = 2,  /* a host or device allocation failed                 */
    PPC_EDEVICE = 3, /* a HIP runtime call or kernel launch failed         */
    PPC_EBUSY = 4,   /* not admitted now (serving); retry later            */
    PPC_ETIMEDOUT = 5 /* a host wait passed its deadline (serving)         */
} ppc_status;

/* Human-readable name of a status code.  Never NULL. */
const char *ppc_status_string(int status);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int ppc_version(void);

/* ------------------------------------------------------------------------
 * Plain calls, one per width (Section 4; the width only changes the final
 * accumulation function f_w, Section 5).  counts[0..w) += pospopcnt_w of
 * buf[0..nbytes).  The kernel counts 64 bit positions relative to absolute
 * addresses mod 8 and then folds them to w positions relative to `buf`.
 * No scratch memory: per-block partial counts live in LDS and are added to
 * `counts` with 64-bit device atomics (order-independent, so exact).
 * ---------------------------------------------------------------------- */
ppc_status ppc_pospopcnt8(uint64_t *counts, const void *buf, size_t nbytes, void *stream);
ppc_status ppc_pospopcnt16(uint64_t *counts, const void *buf, size_t nbytes, void *stream);
ppc_status ppc_pospopcnt32(uint64_t *counts, const void *buf, size_t nbytes, void *stream);
ppc_status ppc_pospopcnt64(uint64_t *counts, const void *buf, size_t nbytes, void *stream);

/* The same with the width as an argument (8, 16, 32 or 64). */
ppc_status ppc_pospopcnt(unsigned width, uint64_t *counts, const void *buf, size_t nbytes,
                         void *stream);

/* The plain call with kernel timing: `start_event` / `stop_event` (hipEvent_t
 * as void*, created by the caller, either may be NULL) are recorded by the
 * kernel dispatch itself (AMD's extended launch), so the interval between
 * them is the kernel's execution time, without the gaps that events
 * recorded separately on the stream would add.  If the call needs several
 * launches (more than the per-launch limit of bytes), start is recorded by
 * the first and stop by the last.  If nothing is launched (nbytes == 0) the
 * events are not recorded.  Measured with ROCm 7.2, a dispatch that records
 * events leaves the queue idle for about 5 us after the kernel: use the
 * untimed call for throughput. */
ppc_status ppc_pospopcnt_timed(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, void *stream,
                               void *start_event, void *stop_event);

/* Streamed input (Section 4, step 1 and its footnote: counts of several
 * pieces of one stream add up).  Like ppc_pospopcnt, but bit positions are
 * relative to a stream that starts `stream_offset` bytes before `buf`:
 * byte buf[b] feeds counters 8*((stream_offset + b) mod s) .. +7.  Counting
 * consecutive pieces of a stream, each with its own offset, cut anywhere,
 * gives exactly the counts of one call over the whole stream. */
ppc_status ppc_pospopcnt_at(unsigned width, uint64_t *counts, const void *buf, size_t nbytes,
                            uint64_t stream_offset, void *stream);

/* Conventional population count (the quantity the Harley-Seal scheme of
 * Section 3.3 computes), on the same carry-save front end: *total (device,
 * one uint64) += number of set bits in buf[0..nbytes).  Same argument rules
 * as the plain call. */
ppc_status ppc_popcount(uint64_t *total, const void *buf, size_t nbytes, void *stream);

/* Accumulation-schedule variants of the plain call, for measurement: the
 * same exact counts computed three ways.  0 = the library path (carry-save
 * front end + bit-parallel accumulation of the weight-16 plane, Sections
 * 4.2-4.5); 1 = carry-save front end + per-position accumulation of the
 * weight-16 plane (the O(w) schedule of Klarqvist et al., Algorithm 2);
 * 2 = no carry-save front end (every bit added to its position counter, the
 * loop of Fig. 2 across lanes).  Same argument rules as ppc_pospopcnt;
 * variants 1 and 2 reject (PPC_EINVAL) inputs that would give a wave more
 * than 2^20 tiles of 16 KiB in one launch. */
ppc_status ppc_pospopcnt_variant(unsigned variant, unsigned width, uint64_t *counts, const void *buf,
                                 size_t nbytes, void *stream);

/* ------------------------------------------------------------------------
 * Launch geometry of the plain call.  `waves` caps the number of wavefronts
 * the grid holds (0 = the library default: one 8-wave block on each of 3/4
 * of the compute units, which streams faster than a block on every one);
 * `waves_per_block` is 2, 4 or 8 (default 8).  Applies to later plain calls
 * from any thread on any device.  Returns PPC_EINVAL for values out of range.
 * ---------------------------------------------------------------------- */
ppc_status ppc_set_plain_geometry(unsigned waves, unsigned waves_per_block);
ppc_status ppc_get_plain_geometry(unsigned *waves, unsigned *waves_per_block);

/* ------------------------------------------------------------------------
 * Read roofline: the "dummy" kernel of the paper's benchmark (Section 5,
 * Table "Benchmarked algorithms"), which sums the input and adds the sum to
 * an output.  *sink (device, one uint64) += sum of the little-endian 64-bit
 * words of buf[0..nbytes) mod 2^64; `buf` must be 16-byte aligned and
 * nbytes a multiple of 16 KiB (whole tiles).  Same load pattern and launch
 * geometry as the plain pospopcnt call: it measures the bandwidth that call
 * can reach.
 * ---------------------------------------------------------------------- */
ppc_status ppc_read_roofline(uint64_t *sink, const void *buf, size_t nbytes, void *stream);

/* The same, with events recorded by the kernel dispatch (see
 * ppc_pospopcnt_timed). */
ppc_status ppc_read_roofline_timed(uint64_t *sink, const void *buf, size_t nbytes, void *stream,
                                   void *start_event, void *stop_event);


/* ------------------------------------------------------------------------
 * Batched form: thousands of arrays of uneven length and mixed width in one
 * persistent launch (a plan runs arrays shorter than one 16 KiB tile in a
 * second kernel of its own, captured in the same graph).  Same arithmetic
 * as the plain call for every array (the width only selects the final
 * accumulation, Section 5), so each array's counts are exactly what
 * ppc_pospopcnt would add.
 * ---------------------------------------------------------------------- */
typedef struct ppc_desc {
    const void *buf;   /* device pointer, any alignment                     */
    uint64_t nbytes;   /* bytes to count (0 allowed)                        */
    uint64_t *counts;  /* device pointer to `width` uint64, 8-byte aligned  */
    uint32_t width;    /* 8, 16, 32 or 64                                   */
    uint32_t reserved; /* must be 0                                         */
} ppc_desc;

typedef struct ppc_plan_opts {
    uint32_t tiles_per_item; /* 16 KiB tiles per work item; 0 = tuned        */
    uint32_t waves;          /* wavefronts in the persistent grid; 0 = tuned */
    uint32_t autotune;       /* 1: time candidates when not cached/given    */
    uint32_t use_graph;      /* 1: replay a captured hipGraph on run         */
    uint32_t reserved;       /* must be 0                                    */
} ppc_plan_opts;

typedef struct ppc_plan_info {
    uint64_t n_arrays, n_items, total_bytes;
    uint32_t tiles_per_item, waves;
    uint32_t tuned; /* 0 = given or default, 1 = measured now, 2 = from cache */
    uint32_t graph; /* 1 if runs replay a hipGraph                            */
} ppc_plan_info;

typedef struct ppc_plan ppc_plan;

/* Builds a plan for `n` arrays described by the HOST array `descs` (the
 * descriptors are copied; the buffers and counters they point to must stay
 * valid while the plan is used).  Validates every descriptor (PPC_EINVAL if
 * any is bad: same rules as the plain call), splits arrays into work items
 * (an array shorter than one 16 KiB tile, of at most 14 16-byte chunks per
 * lane, goes whole to the small-array kernel instead), picks tiles per item
 * and grid size (opts NULL: autotuned for batches of 64 MiB or more with an
 * array of a tile or more, a default setting otherwise; runs replay a
 * graph), uploads the tables and captures the launches.  Autotuning times candidate settings
 * on `stream` with the counters redirected to scratch memory, so the
 * caller's counters are untouched; the choice is cached in the text file
 * $PPC_TUNE_CACHE (default ~/.cache/ppc_tune.txt) keyed by device and batch
 * shape.  Blocks until the plan is ready.  *plan is owned by the caller and
 * released with ppc_plan_destroy. */
ppc_status ppc_plan_create(ppc_plan **plan, const ppc_desc *descs, size_t n, const ppc_plan_opts *opts,
                           void *stream);

/* Enqueues one pass over every array of the plan on `stream`: each array's
 * counts are added to its counters.  Runs of one plan must not overlap
 * (they share the plan's work cursor): order them on one stream. */
ppc_status ppc_plan_run(ppc_plan *plan, void *stream);

/* Fills *info with the plan's shape and chosen settings.  PPC_EINVAL if
 * either pointer is NULL. */
ppc_status ppc_plan_get_info(const ppc_plan *plan, ppc_plan_info *info);

/* Waits for the device to be idle, then frees the plan. */
ppc_status ppc_plan_destroy(ppc_plan *plan);

/* ------------------------------------------------------------------------
 * Batched count that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Each array's counts are exactly what
 * the plain call (and a plan over the same descriptors) adds.
 *
 * `descs` is a DEVICE array of `n` ppc_desc (8-byte aligned), read by the
 * kernels when the stream reaches the call; the buffers and counters it
 * points to follow the plain call's rules.  n <= PPC_NOALLOC_MAX_ARRAYS,
 * else PPC_EINVAL (nothing enqueued).  If any descriptor is invalid (bad
 * width, NULL or misaligned counters, NULL buf with nbytes > 0, reserved
 * != 0) nothing is counted, and if `n_invalid` (device, one uint32,
 * optional) is given the kernels write there the number of invalid
 * descriptors (0 when the batch was counted).
 *
 * Memory.  Every table the kernels use (array table, block sums, work
 * items, work cursor) lives in one static device array of
 * PPC_NOALLOC_SCRATCH_BYTES (about 8 MiB) per GPU, held until the process
 * ends; the call enqueues three kernels (five for more than 256 arrays)
 * and no copy, and calls no allocating routine.  Calls that
 * overlap on one GPU (other streams, other host threads) share that array
 * and race: order them on one stream.  PPC_EDEVICE if a launch fails.
 * ---------------------------------------------------------------------- */
#define PPC_NOALLOC_MAX_ARRAYS 65536u
#define PPC_NOALLOC_SCRATCH_BYTES (512u + 64u * 65536u + 128u * 256u + 16u * 262144u)

ppc_status ppc_batch_noalloc(const ppc_desc *descs, uint32_t n, uint32_t *n_invalid, void *stream);

/* ------------------------------------------------------------------------
 * Serving form: count queries over device-resident columns.  A pool of
 * equal columns (pool_bytes = n_columns * column_bytes, device memory owned
 * by the caller) is counted by requests (column, width, offset, nbytes).
 * Admission is by memory: a request is admitted when a result slot is free
 * and the bytes of all admitted, unfinished requests stay within
 * `inflight_bytes` (a request larger than the budget is admitted only when
 * nothing else is in flight).  Admitted requests are batched continuously:
 * whenever one of `n_streams` streams is idle and requests are pending,
 * the pending ones (up to `max_batch`, in arrival order) go out as one
 * persistent batched launch, so batches overlap on the device.  Results are
 * exactly the plain call's counts for the same bytes and width.  A server
 * is used from one host thread at a time.
 * ---------------------------------------------------------------------- */
typedef struct ppc_server_cfg {
    uint32_t n_streams;      /* batches in flight at once (0 = 3)             */
    uint32_t max_batch;      /* requests per batch (0 = 4096)                 */
    uint32_t max_inflight;   /* result slots = admitted requests (0 = 16384)  */
    uint32_t tiles_per_item; /* 16 KiB tiles per work item (0 = 16)           */
    uint64_t inflight_bytes; /* admission budget in bytes (0 = 16 GiB)        */
    uint32_t waves;          /* persistent grid per batch (0 = 8 per CU)      */
    uint32_t batch_timeout_us; /* deadline of a batch on the device, from its
                                  launch, in microseconds (0 = 10 s)          */
} ppc_server_cfg;

typedef struct ppc_request {
    uint32_t column; /* column index                         */
    uint32_t width;  /* 8, 16, 32 or 64                      */
    uint64_t offset; /* byte offset inside the column        */
    uint64_t nbytes; /* byte length; offset+nbytes <= column */
    uint64_t tag;    /* caller's id, returned in the result  */
} ppc_request;

typedef struct ppc_result {
    uint64_t tag;
    uint32_t width;
    uint32_t status;      /* PPC_OK, or PPC_EDEVICE if its batch failed */
    uint64_t t_submit_ns; /* admission time (steady clock)            */
    uint64_t t_done_ns;   /* time the host saw the counts             */
    uint64_t counts[64];  /* counts[0..width) valid                   */
} ppc_result;

typedef struct ppc_server_stats {
    uint64_t inflight, pending, inflight_bytes;
    uint64_t batches, batched_requests, max_batch_seen;
    uint64_t host_dispatch_ns, host_retire_ns; /* host time enqueuing / retiring */
} ppc_server_stats;

typedef struct ppc_trace_stats {
    uint64_t n_requests, total_bytes, makespan_ns;
    uint64_t p50_ns, p99_ns, max_ns, mean_ns; /* arrival -> counts on host */
    uint64_t batches, busy_rejections;
    uint64_t host_dispatch_ns, host_retire_ns; /* host time enqueuing / retiring */
    double mean_batch;
    double gbps; /* total_bytes / makespan, 1 GB = 1e9 B */
} ppc_trace_stats;

typedef struct ppc_server ppc_server;

/* Creates a server over the device pool [pool, pool + pool_bytes), cut into
 * columns of `column_bytes` (pool_bytes must be a positive multiple of it;
 * the pool must stay valid and unchanged while requests are in flight).
 * `cfg` may be NULL (all defaults); zero fields take their defaults.  The
 * server allocates, per stream, pinned host staging and result buffers and
 * device tables, and captures one graph; *server is owned by the caller and
 * released with ppc_server_destroy.  PPC_EINVAL for bad arguments or a
 * field out of range (n_streams <= 64, max_batch <= 2^20, max_inflight <=
 * 2^24, tiles_per_item <= 2^20), PPC_EDEVICE if no device
 * is current, PPC_ENOMEM if an allocation, a stream or the graph capture
 * fails (nothing is leaked). */
ppc_status ppc_server_create(ppc_server **server, const void *pool, uint64_t pool_bytes, uint64_t column_bytes,
                             const ppc_server_cfg *cfg);

/* Admits one request (PPC_EBUSY if slots or the byte budget are exhausted:
 * poll and retry; PPC_EINVAL if it lies outside its column, the width is
 * bad, or it exceeds what one batch's item table holds: max(4096,
 * 16*max_batch)/4 items of 2^20 tiles of 16 KiB, at least 16 TiB) and makes
 * progress (retires finished batches, launches pending).
 *
 * Deadlines.  Every host wait of the server is a poll with a deadline: a
 * batch still running `batch_timeout_us` after its launch turns the
 * server's status into PPC_ETIMEDOUT (a failed batch into PPC_EDEVICE).
 * From then on submit, poll and run_trace return that status and admit
 * nothing; the batch itself stays in flight, so the only way on is
 * ppc_server_destroy, which waits for the device. */
ppc_status ppc_server_submit(ppc_server *server, const ppc_request *req);

/* Makes progress and returns up to `cap` finished results in *out.
 * Returns PPC_OK, or the server's error status (see Deadlines above);
 * results finished before the error are still returned. */
ppc_status ppc_server_poll(ppc_server *server, ppc_result *out, size_t cap, size_t *n_out);

/* Snapshot of the server's counters (no progress is made).  PPC_EINVAL if
 * either pointer is NULL. */
ppc_status ppc_server_get_stats(const ppc_server *server, ppc_server_stats *stats);

/* Open-loop driver: request i arrives arrival_ns[i] nanoseconds after the
 * start (non-decreasing); requests not admitted wait in arrival order.
 * results[i] receives request i's result (its tag is i) and *stats the
 * latency percentiles (arrival -> counts on host) and throughput.  The
 * server must be idle (nothing admitted, nothing unpolled).  Returns
 * PPC_ETIMEDOUT or PPC_EDEVICE as soon as the server's status becomes one
 * of them (see Deadlines above), so it never waits without bound. */
ppc_status ppc_server_run_trace(ppc_server *server, const ppc_request *reqs, const uint64_t *arrival_ns, size_t n,
                                ppc_result *results, ppc_trace_stats *stats);

/* Waits for the server's streams, then frees it.  This is the one wait
 * without a deadline: the device must be done with the server's buffers
 * before they are freed. */
ppc_status ppc_server_destroy(ppc_server *server);

#ifdef __cplusplus
}
#endif

#endif /* PPC_H */
