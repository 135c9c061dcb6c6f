/*
 * gace.h -- C ABI of the MI355X probe library for the Measurement Engine of
 * GACE (Chang, "Risk-Aware GPU-Assisted Cardinality Estimation for Cost-Based
 * Query Optimizers", arXiv 2512.19750).
 *
 * What is computed (Sec. III-B): the engine measures, on a sample of a table,
 * how many rows satisfy each of many candidate conjunctive conditions (the
 * selectivities S_probe = count / n that Eq. 2 compares with the optimizer's
 * estimate, and the joint and marginal frequencies of Eq. 3), and builds
 * key-only frequency tables of join keys, which give the number of distinct
 * values (the NDV of Eq. 1) and the equi-join size sum_k f_R(k) * f_S(k).
 * All results are exact unsigned 64-bit integers on a deterministic sample.
 *
 * Sampling (block-level dynamic sampling, Sec. II-A item 5 and Sec. III-B):
 * rows are grouped into blocks of `block_rows` rows; block b is kept iff
 * word 0 of Philox4x32-10 (Salmon et al., SC'11) with key = seed (low word
 * first) and counter = (b low 32 bits, b high 32 bits, table_id, 0) is below
 * thr = floor(rate * 2^32); rate 1 keeps every block, rate 0 none.  A partial
 * last block is kept or dropped as a unit.  With one seed and table_id the
 * samples are nested by rate.
 *
 * Memory and ownership: column and key pointers are DEVICE pointers owned by
 * the caller (the library never frees or writes them) and must stay valid and
 * unmodified until the call returns (for served requests: until
 * gace_server_wait reports the request done).  Column base addresses must be
 * 16-byte aligned.  Output pointers are HOST pointers owned by the caller.
 * The library owns a device workspace sized at gace_create.  `stream` is a
 * hipStream_t (may be NULL for the default stream).  Plain calls are
 * synchronous: they return after the results are in host memory.
 *
 * Errors: every call returns a gace_status; a negative value is a failure,
 * no exception crosses the ABI, outputs are left untouched on failure and
 * gace_last_error() gives a message (thread-local, valid until the next call
 * on the same thread).
 *   GACE_EINVAL    bad argument (NULL pointer with a nonzero count, column
 *                  index >= n_cols, unknown dtype or op, a predicate with 0 or
 *                  more than 16 terms, RANGE without exactly 2 values, EQ
 *                  without exactly 1, IN with 0 or more than 8 values, a NaN
 *                  float bound, rate NaN or outside [0,1], block_rows not a
 *                  power of two in [1, 2^20], misaligned column, more than
 *                  2^32 - 1 keys on one join side, or more than 65536
 *                  predicates in one request)
 *   GACE_ENOMEM    the workspace is too small for the request (the message
 *                  states the bytes needed)
 *   GACE_EOVERFLOW reserved, never returned: each join side is limited to
 *                  2^32 - 1 keys (GACE_EINVAL beyond), so n_R * n_S, which
 *                  bounds sum f_R f_S, stays below 2^64
 *   GACE_EDEVICE   a HIP runtime error (the message carries HIP's text), or a
 *                  bounded wait inside a kernel that gave up
 *   GACE_EBUSY     the server queue is full
 *   GACE_ETIMEOUT  gace_server_wait timed out; the request is still running
 */
#ifndef GACE_H
#define GACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gace_status;
#define GACE_OK 0
#define GACE_EINVAL (-1)
#define GACE_ENOMEM (-2)
#define GACE_EOVERFLOW (-3)
#define GACE_EDEVICE (-4)
#define GACE_EBUSY (-5)
#define GACE_ETIMEOUT (-6)

/* column storage types */
#define GACE_I32 1u
#define GACE_I64 2u
#define GACE_F32 3u

/* term operators */
#define GACE_RANGE 1u /* v[0] <= x < v[1]          */
#define GACE_EQ 2u    /* x == v[0]                 */
#define GACE_IN 3u    /* x == v[i] for some i < n  */

/* request kinds */
#define GACE_REQ_SELECTIVITY 1u
#define GACE_REQ_JOIN 2u

typedef struct gace_ctx gace_ctx;
typedef struct gace_server gace_server;

/* One column: device pointer to n_rows values of `dtype`, 16-byte aligned. */
typedef struct {
    const void* data;
    uint32_t dtype;
    uint32_t reserved;
} gace_column;

/* A column-major table; table_id enters the sampler's counter. */
typedef struct {
    uint64_t n_rows;
    const gace_column* cols; /* host array of n_cols descriptors */
    uint32_t n_cols;
    uint32_t table_id;
} gace_table;

/* One atomic condition on one column (80 bytes).  Integer columns compare
   in int64 with int32 values sign-extended.  Float columns take the float
   whose IEEE binary32 bit pattern is the low 32 bits of v[i] and compare
   with IEEE semantics: NaN never matches, -0.0 == +0.0. */
typedef struct {
    uint32_t col;
    uint32_t op;
    uint32_t n_vals;
    uint32_t reserved;
    int64_t v[8];
} gace_term;

/* Candidate conditions in CSR form: predicate p is the conjunction of
   terms[pred_off[p] .. pred_off[p+1]); pred_off has n_preds + 1 entries,
   pred_off[0] == 0, 1..16 terms per predicate (host arrays). */
typedef struct {
    const gace_term* terms;
    const uint32_t* pred_off;
    uint32_t n_preds;
    uint32_t reserved;
} gace_predicates;

/* Block-Bernoulli sample: rate in [0,1], block_rows a power of two in
   [1, 2^20] (1 is row-level sampling).  A NULL spec means rate 1. */
typedef struct {
    uint64_t seed;
    double rate;
    uint32_t block_rows;
    uint32_t reserved;
} gace_sample_spec;

typedef struct {
    uint64_t sampled_rows; /* n of Eq. 2: rows in kept blocks */
    uint64_t kept_blocks;
} gace_probe_info;

/* One side of a join-frequency probe: device array of n int64 keys. */
typedef struct {
    const int64_t* keys;
    uint64_t n;
    uint32_t table_id;
    uint32_t reserved;
    gace_sample_spec spec;
} gace_keys;

typedef struct {
    uint64_t join_card; /* sum_k f_R(k) * f_S(k) over the samples */
    uint64_t ndv_R;     /* distinct sampled keys of R */
    uint64_t ndv_S;
    uint64_t n_R;       /* sampled keys of R */
    uint64_t n_S;
    uint64_t f1_R, f1_S; /* distinct sampled keys seen exactly once (the f_1 of
                            NDV scale-up estimators such as GEE) */
    uint64_t f2_R, f2_S; /* ... exactly twice */
} gace_join_result;

/* A request for gace_batch_run / gace_server_submit.  kind selects which
   half is read; outputs are host pointers written when the request ends. */
typedef struct {
    uint32_t kind;
    uint32_t reserved;
    /* GACE_REQ_SELECTIVITY */
    gace_table table;
    gace_predicates preds;
    gace_sample_spec spec;
    uint64_t* counts;      /* n_preds entries */
    gace_probe_info* info; /* may be NULL */
    /* GACE_REQ_JOIN */
    gace_keys R;
    gace_keys S;
    gace_join_result* join;
} gace_request;

/* Launch schedule of the batched path (chosen by gace_autotune). */
typedef struct {
    uint32_t wg_threads;       /* 256 or 512 */
    uint32_t wgs_per_cu;       /* scan kernel grid = CUs * wgs_per_cu (CUs * 1 in batches with joins) */
    uint32_t item_rows;        /* target sampled rows per work item */
    uint32_t count_mode;       /* 0 auto (ballot for <= 6 active predicates, else 2), 1 ballot,
                                  2 carry-save adder tree over 16 rows + a wave transpose per bit plane */
    uint32_t join_part_keys;   /* expected sampled keys per join hash partition (power of two) */
    uint32_t join_wgs_per_cu;  /* join partitioning kernel grid = CUs * join_wgs_per_cu */
    uint32_t agg_wgs_per_cu;   /* join aggregation kernel grid = CUs * agg_wgs_per_cu */
    uint32_t reserved;
} gace_schedule;

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `hip_device` with a device workspace of
   workspace_bytes (0 = a default of 1/8 of free device memory). */
gace_status gace_create(int hip_device, uint64_t workspace_bytes, gace_ctx** out);
gace_status gace_destroy(gace_ctx* ctx);
const char* gace_last_error(void);
const char* gace_version(void);

/* Validate a request on the host only (no device access, no context):
   the checks listed under GACE_EINVAL above. */
gace_status gace_check_request(const gace_request* req);

/* ---------------------------------------------------------------- plain path */
/* Count, for each predicate, the sampled rows of `table` that satisfy it
   (Sec. III-B; S_probe of Eq. 2 is counts[p] / info->sampled_rows).  Only
   the columns the predicates reference are read.  counts: n_preds host
   entries; info may be NULL. */
gace_status gace_probe_selectivity(gace_ctx* ctx, const gace_table* table, const gace_predicates* preds,
                                   const gace_sample_spec* spec, uint64_t* counts, gace_probe_info* info,
                                   void* stream);

/* Key-only frequency tables of the sampled keys of R and S; returns
   sum_k f_R(k) f_S(k), the NDVs and the sampled key counts (Sec. III-B
   "Key-Only" aggregations; Eq. 1 NDV; Eq. 3 joint frequencies). */
gace_status gace_join_freq(gace_ctx* ctx, const gace_keys* R, const gace_keys* S, gace_join_result* out,
                           void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   probe as gace_probe_selectivity, with the same results, on the calling
   thread's current HIP device and without a context.  Its device scratch is
   a static array of the library (about 4 MiB per GPU the process runs on,
   held until the process ends): a plan of at most 2 MiB, at most 32,768
   work items and 131,072 counters; larger requests fail with GACE_ENOMEM
   before any device work and leave counts untouched.  It calls no hipMalloc,
   hipHostMalloc or hipFree (the host compiles into reused per-thread
   buffers).  All calls on one GPU share that GPU's scratch: calls that
   overlap on one GPU, from several threads or on several streams, race.
   Returns once the results are in counts / info (host memory).  Errors as
   gace_probe_selectivity, plus GACE_EDEVICE if the scratch's device address
   cannot be found (counts untouched) or if a scan workgroup's bounded wait
   gave up (counts unspecified). */
gace_status gace_probe_selectivity_noalloc(const gace_table* table, const gace_predicates* preds,
                                           const gace_sample_spec* spec, uint64_t* counts, gace_probe_info* info,
                                           void* stream);

/* ---------------------------------------------------------------- batched path */
/* Run n requests of either kind in one launch of the persistent kernels: the
   scan kernel and the join stage run concurrently, each replayed from its
   captured graph.
   Selectivity requests on the same table, seed and block size share one
   scan (their samples are nested by rate).  per_req (n entries, may be NULL)
   receives each request's status; an invalid request fails alone.  Returns
   GACE_OK if every request succeeded, else the first failing status. */
gace_status gace_batch_run(gace_ctx* ctx, const gace_request* reqs, uint32_t n, gace_status* per_req,
                           void* stream);

/* Time candidate schedules on this request mix, in the context's launch
   mode (gace_set_graph), and keep the fastest for its shape bucket in the
   context; cache_path (may be NULL) is a JSON file read before and written
   after the search, keyed by device, kernels, launch mode and shape. */
gace_status gace_autotune(gace_ctx* ctx, const gace_request* reqs, uint32_t n, const char* cache_path,
                          void* stream);
gace_status gace_get_schedule(gace_ctx* ctx, gace_schedule* out);
gace_status gace_set_schedule(gace_ctx* ctx, const gace_schedule* s);

/* Timing of the last gace_batch_run: device time of the persistent kernel
   in milliseconds, measured with HIP events on the call's stream, and the
   algorithmic HBM bytes it moved (kept rows x referenced column widths of
   each shared scan + 8 bytes per sampled join key + 16 bytes per distinct
   key and side). */
gace_status gace_last_batch_stats(gace_ctx* ctx, double* kernel_ms, uint64_t* alg_bytes,
                                  uint64_t* rows_preds);

/* Per-kernel timing of the last gace_batch_run: device time of the scan kernel, measured with HIP
   events on the call's stream, and of the join stage (the partitioning
   kernel followed by the aggregation kernel), measured on the context's side
   stream where it runs concurrently; with the algorithmic HBM bytes of each
   (scan: kept rows x referenced column widths per shared scan; join: 8 bytes
   per sampled key + 16 bytes per distinct key and side).
   Both launch modes time the kernels: graph replay captures one graph per
   branch (the scan kernel; the join stage) and records the same timing
   events around each graph launch (timed = 1 once a batch ran).  compile_ms is
   the host time spent validating and compiling the batch's requests into
   the device plan (either launch mode). */
typedef struct {
    double scan_ms, join_ms;
    uint64_t scan_alg_bytes, join_alg_bytes;
    uint32_t timed;
    float compile_ms;
    uint64_t zones_skipped;   /* zones the batch's scans skipped by attached zone maps (gace_zone.h) */
} gace_kernel_stats;

gace_status gace_last_kernel_stats(gace_ctx* ctx, gace_kernel_stats* out);

/* Select how gace_batch_run launches: graph replay (enable != 0, the
   default) or direct launches.  Both time each kernel branch; results are
   identical. */
gace_status gace_set_graph(gace_ctx* ctx, int enable);

/* Bound on a join's phase waits on the device.  Each join phase waits for
   the join's items of the phase before it, all queued ahead of it (and a
   merge of a split partition for that partition's chunks), so the waits
   always end; as a guard each gives up after `polls` polls of its counter,
   and the join then fails with GACE_EDEVICE instead of hanging the kernel.
   0 makes every such wait give up at once (this is how the failure path is
   tested from the host; every kernel still exits normally).  Default 2^24
   polls, many seconds.  The other requests of the batch are unaffected.
   Errors: GACE_EINVAL (NULL context). */
gace_status gace_set_spin_limit(gace_ctx* ctx, uint64_t polls);

/* Per-item device trace of the last batch (for profiling the batched path).
   Item kinds: 1 scan, 2 join histogram, 3 join offsets, 4 join partition
   starts, 5 join scatter (first pass), 6 join aggregation, 7 join scatter
   (second pass).  Timestamps are ticks of the
   device's constant-rate counter (ticks_per_us of them per microsecond):
   t_begin when a workgroup took the item, t_ready when its dependencies were
   met, t_end when it finished.  Tracing costs one store per item. */
typedef struct {
    uint32_t kind;
    uint32_t index;   /* scan or join index within the batch */
    uint32_t wg;      /* workgroup id */
    uint32_t xcc;     /* XCD (accelerator complex die) the workgroup ran on */
    uint64_t t_begin, t_ready, t_end;
    uint64_t work;    /* join aggregation: units taken << 32 | LDS table passes; else 0 */
} gace_trace_rec;

gace_status gace_set_trace(gace_ctx* ctx, int enable);
/* Copies up to cap records of the last batch; *n receives the total. */
gace_status gace_get_trace(gace_ctx* ctx, gace_trace_rec* out, uint32_t cap, uint32_t* n, double* ticks_per_us);

/* ---------------------------------------------------------------- measurement */
/* The GPU's HBM read ceiling, reported beside the probe kernels' bandwidth:
   reads n_bytes (a nonzero multiple of 16) of device memory at `data`
   (16-byte aligned) with 16-byte nontemporal loads, 64 KiB per workgroup,
   and returns the kernel's device time in *ms, measured with HIP events on
   `stream` (the call waits for it).  `sink`: one device word that the kernel
   writes only if a thread's XOR of its words is all ones (never, for
   zero-filled memory).  Errors: GACE_EINVAL (NULL pointer, misaligned or
   empty range), GACE_EDEVICE. */
gace_status gace_read_ceiling(const void* data, uint64_t n_bytes, uint32_t* sink, double* ms, void* stream);

/* ---------------------------------------------------------------- serving */
typedef struct {
    uint32_t max_inflight;       /* batches on the device at once (>= 1) */
    uint32_t max_batch;          /* requests per batch */
    uint32_t queue_capacity;     /* submitted but not finished requests */
    uint32_t flags;              /* GACE_SERVER_* bits; 0 by default */
    uint64_t workspace_bytes;    /* device memory for admitted requests (admission budget) */
} gace_server_cfg;

/* finish a request only when its whole batch does (no per-request publishing) */
#define GACE_SERVER_BATCH_COMPLETION 1u

typedef struct {
    uint64_t submitted, completed, rejected, batches;
    uint64_t queued, inflight;
    uint64_t workspace_in_use, workspace_peak;
    uint64_t completed_early;    /* of completed: finished as their own scan or join did, before their batch */
} gace_server_stats;

/* The server owns a worker thread, its own streams and workspace on
   hip_device.  Requests are admitted while their workspace fits the budget,
   batched with whatever else is waiting, and launched while earlier batches
   still run (continuous batching).  A request is done when its own scan or
   join finishes on the device, not when its whole batch does: the kernels
   publish each finished scan's and join's results to pinned host memory and
   the worker writes that request's outputs and wakes its waiter at once. */
gace_status gace_server_create(int hip_device, const gace_server_cfg* cfg, gace_server** out);
/* Enqueue a copy of *req (its host arrays are copied; device buffers and
   output pointers must stay valid until done).  GACE_EBUSY if the queue is
   full; GACE_EINVAL if the request is invalid; GACE_ENOMEM if its workspace
   estimate exceeds one slot's share of the budget. */
gace_status gace_server_submit(gace_server* srv, const gace_request* req, uint64_t* ticket);
/* Wait until request `ticket` is done (timeout_ns < 0: forever).  Its status
   goes to *req_status; GACE_ETIMEOUT if still running; GACE_EINVAL for an
   unknown ticket or one another wait has already collected. */
gace_status gace_server_wait(gace_server* srv, uint64_t ticket, int64_t timeout_ns, gace_status* req_status);
/* As gace_server_wait, and also returns when the request was submitted and
   when the server saw it finish, in nanoseconds of CLOCK_MONOTONIC (either
   pointer may be NULL).  Latency = done - arrival. */
gace_status gace_server_wait_times(gace_server* srv, uint64_t ticket, int64_t timeout_ns, gace_status* req_status,
                                   uint64_t* submit_ns, uint64_t* done_ns);
gace_status gace_server_stats_get(gace_server* srv, gace_server_stats* out);
gace_status gace_server_destroy(gace_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* GACE_H */
