/*
 * mdrq.h -- C ABI of libmdrq: exact multidimensional range queries (MDRQ) over
 * column-stored float32 data on an AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Sprenger, Schaefer & Leser, "Multidimensional Range Queries on
 * Modern Hardware", section 2.1): a data set holds n objects with m attributes each.
 * A query gives a closed interval [lb_j, ub_j] for some or all dimensions j; a
 * dimension without an interval behaves as [-inf, +inf] (a partial-match query).
 * An object qualifies iff lb_j <= value_j <= ub_j holds on every queried dimension.
 * The answer is the set of identifiers of the qualifying objects; the identifier of
 * an object is its 0-based index in the column arrays (section 2.2.4).  Data are
 * 32-bit floats (section 7.2) stored one array per dimension, as in the vertically
 * partitioned scan of section 5.5.
 *
 * Conventions for every call:
 *  - Return value: MDRQ_OK (0) or a negative MDRQ_E* code.  After a failure,
 *    mdrq_last_error() returns a message for the calling thread.
 *  - Identifiers are uint32 (so n_rows <= 2^32 - 1) and are always written in
 *    ascending order.  Result sets are exact: no approximation anywhere.
 *  - NaN is not a value: a NaN in the data makes mdrq_load_columns fail with
 *    MDRQ_EINVAL, and a NaN bound makes the query invalid.  -0.0 equals +0.0;
 *    infinities and subnormal numbers are ordinary values.
 *  - lo > hi is a valid, empty interval.  A dimension may appear at most once per
 *    query (one interval per dimension, section 2.1).  A query without predicates
 *    selects every object.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls return only when
 *    their results are complete and `count` is valid on the host.
 *  - Calls on one dataset are serialised by the library; different datasets may be
 *    used from different threads.
 */
#ifndef MDRQ_H
#define MDRQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDRQ_MAX_DIMS 128          /* dimensions per dataset, predicates per query */
#define MDRQ_MAX_BATCH 1024        /* queries per mdrq_query_batch call */

/* Status codes. */
enum {
  MDRQ_OK = 0,
  MDRQ_EINVAL = -1,     /* invalid argument (see each call) */
  MDRQ_ENOMEM = -2,     /* device or host allocation failed */
  MDRQ_EOVERFLOW = -3,  /* result larger than the caller's buffer; count is exact */
  MDRQ_EDEVICE = -4,    /* a HIP call or kernel failed */
  MDRQ_EBUSY = -5,      /* serving: request could not be admitted */
  MDRQ_ENOTSUP = -6     /* valid request this build cannot serve */
};

/* mdrq_load_columns flags. */
enum {
  MDRQ_MEM_HOST = 0,    /* cols[] are host pointers: copied into library-owned HBM */
  MDRQ_MEM_DEVICE = 1,  /* cols[] are device pointers: copied device to device */
  MDRQ_BORROW = 2       /* with MDRQ_MEM_DEVICE: use the caller's device arrays in place */
};

/* Result modes. */
enum {
  MDRQ_OUT_IDS = 0,     /* ascending uint32 identifiers */
  MDRQ_OUT_BITMAP = 1,  /* uint64 words: bit (i % 64) of word i / 64 <=> object i qualifies */
  MDRQ_OUT_COUNT = 2,   /* the count only */
  MDRQ_OUT_AUTO = 3     /* IDS or BITMAP, whichever is smaller for the exact count and fits
                           buf_bytes (decided on the device); the choice is reported */
};

/* Query flags. */
enum {
  MDRQ_Q_ORDER_GIVEN = 0,      /* evaluate predicates in the order given */
  MDRQ_Q_ORDER_ESTIMATED = 1,  /* most selective first, by the attached estimator */
  MDRQ_Q_NO_EARLYOUT = 2,      /* read every queried column in full (measurement) */
  MDRQ_Q_SIZE_ESTIMATED = 4    /* batches and serving: size this query's share of the
                                  shared scan's scratch by the attached estimator's joint
                                  estimate instead of the worst case (a bitmap row of
                                  ceil(n_rows / 64) words): only the chunks of rows with a
                                  hit are kept, in room for about MDRQ_OPT_RESERVE_FACTOR
                                  times the estimated count; when the estimate was too
                                  low the query is answered again by the single-query
                                  scan.  Needs an attached estimator (else the worst case
                                  is reserved); results never depend on it */
};

typedef struct mdrq_dataset mdrq_dataset;  /* opaque, owned by the library */

/* One predicate: closed interval [lo, hi] on dimension `dim`. */
typedef struct {
  uint32_t dim;
  float lo;
  float hi;
} mdrq_pred;

typedef struct {
  const mdrq_pred* preds;  /* n_preds entries; read only during the call */
  uint32_t n_preds;
  uint32_t flags;          /* MDRQ_Q_* */
} mdrq_query_t;

/* Output of one query.  `buf` is owned by the caller and lives in host memory
 * (mem = MDRQ_MEM_HOST) or device memory (mem = MDRQ_MEM_DEVICE).  IDS mode holds
 * buf_bytes / 4 identifiers; BITMAP mode needs ceil(n_rows / 64) words to hold the
 * full bitmap.  If the result does not fit, the first identifiers (or words) that
 * fit are written, `count` is still exact and status is MDRQ_EOVERFLOW. */
typedef struct {
  uint32_t mode;       /* in: MDRQ_OUT_*; out: the mode used (AUTO resolved) */
  uint32_t mem;        /* MDRQ_MEM_HOST or MDRQ_MEM_DEVICE */
  void* buf;           /* may be NULL when buf_bytes == 0 */
  uint64_t buf_bytes;
  uint64_t count;      /* out: exact number of qualifying objects */
  uint64_t written;    /* out: identifiers (IDS) or words (BITMAP) written */
  int32_t status;      /* out: MDRQ_OK or MDRQ_EOVERFLOW */
  uint32_t reserved;
} mdrq_result_t;

/*
 * Load n_dims columns of n_rows float32 values (paper section 5.5: one array per
 * dimension).  cols[j] points to column j.  With MDRQ_MEM_HOST or MDRQ_MEM_DEVICE
 * the data are copied into one library-owned HBM allocation (each column 256-byte
 * aligned); with MDRQ_MEM_DEVICE | MDRQ_BORROW the caller's device arrays are used in
 * place (each must be 16-byte aligned and must stay alive and unchanged until
 * mdrq_free).  Every value is checked on the device: a NaN makes the call fail with
 * MDRQ_EINVAL.  Per-column minima and maxima are kept (mdrq_column_range).
 * Errors: MDRQ_EINVAL (NULL pointers, n_dims == 0 or > MDRQ_MAX_DIMS,
 * n_rows > 2^32 - 1, misaligned borrowed column, NaN data), MDRQ_ENOMEM,
 * MDRQ_EDEVICE.  On success *out receives the dataset.
 */
int mdrq_load_columns(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                      uint32_t flags, void* stream, mdrq_dataset** out);

/*
 * Answer one query (paper section 2.1) with a full columnar scan: each tile of rows
 * is tested against the predicates one dimension at a time (section 5.5), the
 * per-dimension results are ANDed (section 3.2), and rows already rejected are not
 * read again for later dimensions (the early break of section 2.2.4).  Identifiers
 * are compacted in ascending order.
 * Errors: MDRQ_EINVAL (NULL ds/q/r, n_preds > n_dims, dim >= n_dims, repeated dim,
 * NaN bound, unknown mode or mem, buf == NULL with buf_bytes > 0),
 * MDRQ_EOVERFLOW (result truncated, r->count exact), MDRQ_EDEVICE.
 */
int mdrq_query(mdrq_dataset* ds, const mdrq_query_t* q, mdrq_result_t* r, void* stream);

/*
 * Answer n_queries queries (1 .. MDRQ_MAX_BATCH) with one shared scan: each column
 * tile is read from HBM once and tested against every query of the batch.  Each
 * query's result is exactly what mdrq_query returns for it alone.  rs[i] is the
 * result of qs[i]; a per-query overflow sets rs[i].status and makes the call return
 * MDRQ_EOVERFLOW after all results are written.
 * Errors: as mdrq_query, for any query of the batch (nothing is run then).
 */
int mdrq_query_batch(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n_queries,
                     mdrq_result_t* rs, void* stream);

/*
 * mdrq_query without allocation, for callers that cannot allocate device memory during
 * a call (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as mdrq_query, but the scan's
 * workspace (staged bitmap, per-tile and per-workgroup counts, scan state) is a fixed
 * 32 MiB array compiled into the library, one per GPU, held until the process ends;
 * the call allocates no device memory (no hipMalloc or hipFree) and builds its launch
 * parameters without the host heap.  Calls on one GPU share
 * that array and are serialised by a process-wide lock per device; the array keeps the
 * last call's contents, and each call clears what must start at zero.  Limits:
 * results must be count-only or in device memory (host buf: MDRQ_EINVAL), predicates
 * are evaluated in the order given (MDRQ_Q_ORDER_ESTIMATED: MDRQ_ENOTSUP), and the
 * dataset must fit the array (about n_rows / 8 + n_rows / 512 bytes at the default tile
 * height, i.e. up to about 2.6e8 rows; larger: MDRQ_ENOTSUP).
 */
int mdrq_query_noalloc(mdrq_dataset* ds, const mdrq_query_t* q, mdrq_result_t* r, void* stream);

/* Serving configuration.  n_streams workers each own a device stream and an equal share
 * of result_budget_bytes of device memory for the scans' scratch: a request whose result
 * needs identifiers or a bitmap reserves one bitmap row of ceil(n_rows / 64) words and
 * its chunk marks (its result can never need more), or, with use_estimator bit 1, the
 * room its estimated result needs in the scan's sparse scratch (MDRQ_Q_SIZE_ESTIMATED;
 * about four times the estimate, and never more than the row); a count-only request
 * reserves none.
 * A worker that is idle takes the oldest waiting requests, at most max_batch and as many
 * as its share holds, and answers them with one batched shared scan (as
 * mdrq_query_batch); requests that arrive meanwhile wait for the next idle worker
 * (continuous batching), and the workers' scans overlap on the device.
 * With segments > 0 each worker runs a circular shared scan instead (the shared scan of
 * section 3.2 kept running over the data, which late arrivals join): the rows are cut
 * into `segments` parts of whole 4096-row tiles (at most one per tile), and the worker
 * scans one part per step, in order and wrapping around, for all its active requests.
 * Between steps it admits waiting requests, oldest first, into free query slots (as many
 * as its share holds, at most max_batch; each slot is a bitmap row, its chunk marks and
 * a row of tile counts, whatever the output mode) while the union of their columns fits
 * one scan; a request is complete, and finished exactly as in a shared scan, once it has
 * seen every part.  So a request waits at most about one step before its scan starts,
 * instead of a whole scan (two with pipelined steps, MDRQ_OPT_CIRCULAR).  Optionally
 * (MDRQ_OPT_CIRCULAR) a worker with no pass running whose waiting requests are few
 * enough that separate single-query scans cost less than a pass (the batched path's
 * cost model) answers them that way instead.  Results are the same as in the other
 * mode. */
typedef struct {
  uint64_t result_budget_bytes;
  uint32_t max_batch;       /* 1 .. MDRQ_MAX_BATCH */
  uint32_t n_streams;       /* 1 .. 8 */
  uint32_t use_estimator;   /* bit 0: every request evaluates its predicates in
                               estimated order (MDRQ_Q_ORDER_ESTIMATED); bit 1: every
                               request has its scratch sized by its estimate and is
                               admitted by that size (MDRQ_Q_SIZE_ESTIMATED); either
                               needs an attached estimator */
  uint32_t max_queue;       /* live server: requests allowed to wait; a submission
                               beyond it fails with MDRQ_EBUSY (admission control).
                               0 = unbounded.  The replay ignores it. */
  uint32_t segments;        /* 0: continuous batching; 1 .. 4096: circular scan with
                               this many parts per pass (use_estimator bit 1 is then
                               MDRQ_EINVAL; bit 0 changes nothing: predicates are
                               walked in the given order) */
} mdrq_serve_config_t;

/* One request: the query, and its arrival time in ns after the start of the run. */
typedef struct {
  uint64_t arrival_ns;
  mdrq_query_t query;
} mdrq_request_t;

typedef struct {
  uint64_t completed;       /* requests answered */
  uint64_t scans;           /* shared scans launched */
  double wall_s;            /* first arrival to last completion */
  double qps;               /* completed / wall_s */
  double p50_us, p99_us, mean_us, max_us;  /* arrival -> result complete in device memory */
  double mean_batch;        /* requests per worker batch (circular scan: active
                               requests per step) */
  double hbm_gbps;          /* column bytes covered by the scans (each union column in
                               full) / wall_s */
  uint64_t overflow_reruns; /* requests answered again by the single-query scan because
                               their estimate-sized scratch was too small */
  uint64_t sized_by_estimate; /* requests whose scratch was sized by their estimate */
} mdrq_serve_stats_t;

/*
 * Replay n_reqs arrival-stamped requests through the serving loop: request i is
 * queued when the run's clock reaches reqs[i].arrival_ns.  The call first waits until
 * the device is idle (work queued on any stream before the call is complete before
 * the first scan).  rs[i] receives request i's
 * result exactly as mdrq_query would give it; results that are not count-only must be
 * in device memory.  latency_ns (optional, n_reqs entries) receives each request's
 * arrival-to-completion time; stats (optional) the summary.  The call returns when
 * every request is answered.
 * Errors: MDRQ_EINVAL (bad config or request, host-memory result buffer, use_estimator
 * without an estimator), MDRQ_EBUSY (one bitmap row exceeds a stream's share of the
 * budget), MDRQ_EOVERFLOW (some rs[i] truncated; all others complete), MDRQ_ENOMEM,
 * MDRQ_EDEVICE.
 */
int mdrq_serve(mdrq_dataset* ds, const mdrq_serve_config_t* cfg, const mdrq_request_t* reqs,
               uint32_t n_reqs, mdrq_result_t* rs, uint64_t* latency_ns,
               mdrq_serve_stats_t* stats);

/*
 * Live serving: the same workers and continuous batching as mdrq_serve, fed by
 * submissions instead of a replayed arrival list.
 *
 * mdrq_serve_open starts a server on ds (workers, streams and each worker's share of
 * result_budget_bytes are allocated here, nothing later).  The server does not hold
 * the dataset's call lock: mdrq_query and mdrq_query_batch on the same dataset may run
 * meanwhile from other threads; options must not be changed while it is open.
 * mdrq_free closes any server still open on the dataset (its handle is invalid then).
 *
 * mdrq_serve_submit queues one request and returns its ticket (0, 1, 2, ... in
 * submission order).  The query is copied; *r is the caller's: it must stay valid,
 * with its device buffer, until the ticket is reported by mdrq_serve_poll, and the
 * server writes the complete result into it (count, mode, written, status exactly as
 * mdrq_query would) before reporting the ticket.  Results that are not count-only must
 * be in device memory.  `stream` (a hipStream_t, NULL = the default stream) is the
 * stream of the caller's work on the result buffer: the server records an event on it
 * at submission and the request's scan runs only after that event, so writes the
 * caller queued before submitting (a fill, a pending read of a reused buffer) complete
 * first.  Latency counts from the submission.
 * Errors: MDRQ_EINVAL (bad request, host-memory result, server closing), MDRQ_EBUSY
 * (max_queue requests already waiting, or one bitmap row exceeds a stream's share),
 * or a device error that stopped the server.
 *
 * mdrq_serve_poll writes up to max_tickets completed tickets (each reported once, in
 * completion order) to tickets[] and their number to *n_out; with wait_ns > 0 it
 * waits up to that long for at least one.  It returns the server's error, if a scan
 * failed (the requests of that scan carry it in their status).
 *
 * mdrq_serve_close answers every request already submitted, stops the workers, frees
 * the server and writes the summary over all its requests to *stats (optional).
 * Returns MDRQ_EOVERFLOW if some result was truncated, a scan's error if one failed.
 */
typedef struct mdrq_server mdrq_server;   /* opaque */
int mdrq_serve_open(mdrq_dataset* ds, const mdrq_serve_config_t* cfg, mdrq_server** out);
int mdrq_serve_submit(mdrq_server* s, const mdrq_query_t* q, mdrq_result_t* r, void* stream,
                      uint64_t* ticket);
int mdrq_serve_poll(mdrq_server* s, uint64_t* tickets, uint32_t max_tickets, uint32_t* n_out,
                    uint64_t wait_ns);
int mdrq_serve_close(mdrq_server* s, mdrq_serve_stats_t* stats);

/* Release a dataset and everything the library allocated for it (closing any server
 * still open on it first). */
void mdrq_free(mdrq_dataset* ds);

/* Message of the calling thread's last failure ("" if none); valid until its next call. */
const char* mdrq_last_error(void);

/* Shape of a dataset. */
int mdrq_dataset_info(const mdrq_dataset* ds, uint64_t* n_rows, uint32_t* n_dims);

/* Minimum and maximum of column `dim`, found at load. */
int mdrq_column_range(const mdrq_dataset* ds, uint32_t dim, float* min_out, float* max_out);

/* Kernel timing: when enabled, a dataset's query launches are bracketed by HIP events
 * on the stream they run on.  mdrq_get_profile returns the number of timed queries,
 * the summed duration of their scan kernels alone (scan_ms: predicate evaluation and
 * bitmap/count output) and of the whole device work of each query (total_ms: scan plus
 * ordered compaction), in milliseconds. */
int mdrq_set_profiling(mdrq_dataset* ds, int enable);
int mdrq_get_profile(const mdrq_dataset* ds, uint64_t* launches, double* scan_ms,
                     double* total_ms);
int mdrq_reset_profile(mdrq_dataset* ds);
/* Shared scans run by mdrq_query_batch and mdrq_serve since the last reset, and their
 * summed device time (scan and finishing launches) in milliseconds. */
int mdrq_get_batch_profile(const mdrq_dataset* ds, uint64_t* scans, double* ms);
/* Work of the shared scans since the last reset: rank lookups (rows times the (group of
 * up to 128 queries, column) pairs with a predicate, each one bucket word, a search
 * within the bucket and one row of query bitsets read from LDS; 0 for the other
 * variants), the column bytes read (4 per row and (group, column) pair of the rank
 * variant, per row and union column otherwise), and the device time of the scan kernels
 * alone in milliseconds (without the finishing launches). */
int mdrq_get_batch_work(const mdrq_dataset* ds, uint64_t* lookups, uint64_t* column_bytes, double* scan_ms);
/* Queries of mdrq_query_batch and mdrq_serve since the last reset whose scratch was
 * sized by their estimate (MDRQ_Q_SIZE_ESTIMATED), and how many of them were answered
 * again by the single-query scan because their result outgrew it. */
int mdrq_get_sizing_profile(const mdrq_dataset* ds, uint64_t* sized, uint64_t* reruns);

/* Tuning options of a dataset's scans (results never depend on them). */
enum {
  MDRQ_OPT_UNROLL = 1,  /* 16-byte loads per lane per column in one tile: 1, 2, 4, 8
                           or 16 (one wave scans 256 x value rows per tile); 0 (default):
                           by the table's rows per CU, 2 below 6144, 4 below 65536,
                           else 8 */
  MDRQ_OPT_GRID = 2,    /* workgroups per scan launch; 0 = MDRQ_OPT_BLOCKS_PER_CU per CU */
  MDRQ_OPT_BLOCKS_PER_CU = 3, /* default launch width: workgroups per CU, 1..8
                                 (capped by occupancy); default 3 */
  MDRQ_OPT_BATCH_WAVES = 4,   /* shared scans: waves per workgroup, 4 or 8; 0 = autotune */
  MDRQ_OPT_BATCH_GROUP = 5,   /* shared scans: queries per workgroup group (each group
                                 re-reads the tile); 0 = autotune */
  MDRQ_OPT_AUTOTUNE = 6,      /* 1 (default): on the first batch of a new shape (rows,
                                 union columns, batch size), time each candidate launch
                                 configuration and keep the fastest; 0: fixed defaults */
  MDRQ_OPT_BATCH_ROWS = 7,    /* shared scans: 64-row groups each lane holds per chunk,
                                 1, 2, 4, 8 or 16 (tile height 64 x value rows per wave);
                                 0 = autotune */
  MDRQ_OPT_BATCH_VARIANT = 8, /* shared scans: 1 = the union's keys in registers (unions
                                 of up to 16 columns; wider ones use LDS), 2 = keys
                                 staged in LDS (any union, up to MDRQ_MAX_DIMS columns),
                                 3 = keys in registers with each query's predicates
                                 evaluated in column order, 4 = keys in registers with
                                 fixed-size query records (a slot mask and the bounds of
                                 every slot), 5 = per group of up to 128 queries, each
                                 row's rank among the group's interval ends and per-rank
                                 query bitsets; 0 = autotune (default) */
  MDRQ_OPT_RANK_BUCKETS = 9,  /* rank variant: how a column's keys map to the search's
                                 buckets: 0 = per column the map that leaves the fewest
                                 ends in the fullest bucket (default), 1 = by key,
                                 2 = by float value (by key where the ends' finite values
                                 do not span a finite range); results never depend on it */
  MDRQ_OPT_GRAPHS = 10,       /* bit 0: the launch sequence of a single query (scan,
                                 compaction), bit 1: that of a shared scan (query-table
                                 copy, zeroing, scan, finish), is built once per launch
                                 shape as a HIP graph and replayed with each call's
                                 arguments; a clear bit launches each kernel directly.
                                 Default 0 */
  MDRQ_OPT_RESERVE_FACTOR = 11, /* MDRQ_Q_SIZE_ESTIMATED: room reserved per estimated
                                 result row, in millionths (default 4000000: four times
                                 the estimate, plus 64 chunks); 1..10^9.  Small values
                                 force the fallback (tests) */
  MDRQ_OPT_CIRCULAR = 12      /* circular-scan servers opened from now on (segments > 0):
                                 bit 0: steps pipelined (the host prepares the next step
                                 while the device runs one; a request then joins up to
                                 two steps later), bit 1: an idle worker answers up to
                                 four waiting requests by separate single-query scans
                                 when those cost less than a pass, bit 2: a step whose
                                 requests are few enough that single-query scans of its
                                 rows cost less than the shared scan (the batched path's
                                 cost model) runs those instead, into the same slots.
                                 Default 4 */
};
int mdrq_set_option(mdrq_dataset* ds, uint32_t option, int64_t value);
/* The value an option takes now into *value (MDRQ_OPT_UNROLL: the tile height in use,
 * also when chosen by size).  MDRQ_EINVAL for an unknown option or a NULL argument. */
int mdrq_get_option(const mdrq_dataset* ds, uint32_t option, int64_t* value);

/* Streaming-read ceiling: read the listed columns in full (k entries of dims[],
 * no predicate, no output) with the scan kernels' launch shape, `iters` times, and
 * return the mean duration of one pass in *ms.  The read rate 4 * n_rows * k / ms is
 * the achievable bandwidth the scans are compared against.
 * Errors: MDRQ_EINVAL (NULL pointers, k == 0, dim out of range), MDRQ_EDEVICE. */
int mdrq_probe_bandwidth(mdrq_dataset* ds, const uint32_t* dims, uint32_t k, uint32_t iters,
                         void* stream, double* ms);

/* Column bytes the scan of query q must read from HBM (a measurement of the method's
 * own traffic, for rooflines; q is not answered).  With the early break (section 2.2.4)
 * a later predicate needs only the rows that every earlier one accepted; memory is read
 * in 128-byte lines (32 rows of a column), so the figure is 128 times the number of
 * (predicate, line) pairs where the line holds such a row, predicates taken in the
 * query's evaluation order (given, or estimated with MDRQ_Q_ORDER_ESTIMATED); with
 * MDRQ_Q_NO_EARLYOUT every queried column is read in full.  Lines are counted from each
 * column's first row (library-owned columns start on 256-byte boundaries).  Writes of
 * the result are not included.  An empty query reads nothing.
 * Errors: as mdrq_query for q; MDRQ_EDEVICE. */
int mdrq_query_read_bytes(mdrq_dataset* ds, const mdrq_query_t* q, uint64_t* bytes, void* stream);

/* ---------------------------------------------------------------- learned estimator
 *
 * Evaluating the most selective dimension first lets the early break skip more rows,
 * but needs selectivity estimates (paper section 2.2.4); learning them is left to
 * future work (section 8).  An estimator holds, per column, an equi-depth histogram
 * of MDRQ_EST_BINS bins built on the device from a strided sample, and a small
 * network (features -> hidden -> hidden -> n_dims + 1, GELU) whose matrix products run
 * on the matrix cores with bfloat16 operands and float32 accumulation, trained with
 * Adam on float32 master weights.  Estimates only choose the order of evaluation
 * (MDRQ_Q_ORDER_ESTIMATED) and reservations in serving: results never depend on them.
 *
 * Selectivities s are handled on the log scale y(s) = -ln(max(s, 1/N)) / ln N, s = N^-y.
 * Features of a query (n_dims * (MDRQ_EST_BINS + 3) values, bfloat16): per dimension,
 * the histogram CDF H at lo and at hi, the histogram estimate y(H(hi) - H(lo)) and the
 * covered fraction of each bin; a dimension without a predicate (or with [-inf, +inf])
 * gives (-1, -1, 0, 1, ..., 1).  The network's n_dims + 1 outputs correct a base
 * estimate: the histogram estimate of each dimension's predicate alone and, last, of
 * the whole query as the independence product min(1, sum of the per-dimension y)
 * (section 2.1).  The output layer starts at zero, so an untrained estimator returns
 * the base estimate.
 *
 * Selectivity arrays (sel) hold n_queries rows of n_dims + 1 floats: entry j < n_dims
 * is the selectivity of the query's predicate on dimension j alone (-1 if the query
 * has none there), the last entry the selectivity of the whole query.
 * Parameters (get/set) are float32 in the order W1 [F x H], b1 [H], W2 [H x H], b2 [H],
 * W3 [H x O], b3 [O] (row-major, F features, H hidden, O = n_dims + 1).
 * Estimator calls run on the null stream and return when their results are on the
 * host.  Free an estimator before its dataset.
 */
#define MDRQ_EST_BINS 16
#define MDRQ_EST_MAX_QUERIES (1u << 22)  /* queries per estimator call */

typedef struct mdrq_estimator mdrq_estimator;  /* opaque, owned by the library */

typedef struct {
  uint32_t hidden;       /* width of both hidden layers: multiple of 16 in 16..256; 0 = 64 */
  uint32_t sample_rows;  /* rows sampled per column: 2..16384; 0 = min(16384, n_rows) */
  uint64_t seed;         /* initial hidden weights (Glorot-uniform, counter-based generator) */
} mdrq_estimator_config_t;

typedef struct {
  uint32_t epochs;       /* passes over the training queries, >= 1 */
  uint32_t batch;        /* queries per Adam step: 1..65536 */
  float lr;              /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
  uint32_t reserved;
  uint64_t seed;         /* shuffling of each epoch */
} mdrq_train_config_t;

/* Build the histograms of every column of ds (a strided sample of sample_rows rows,
 * sorted on the device) and initialise the network.
 * Errors: MDRQ_EINVAL (NULL, bad config, empty dataset), MDRQ_ENOMEM, MDRQ_EDEVICE. */
int mdrq_estimator_create(mdrq_dataset* ds, const mdrq_estimator_config_t* cfg,
                          mdrq_estimator** out);
/* Detach (if attached) and release. */
void mdrq_estimator_free(mdrq_estimator* e);
/* Histogram boundaries: n_dims rows of MDRQ_EST_BINS + 1 floats (host). */
int mdrq_estimator_histograms(const mdrq_estimator* e, float* bounds);
/* Features of n queries (1 .. MDRQ_EST_MAX_QUERIES) as bfloat16 bit patterns, n rows of
 * n_dims * (MDRQ_EST_BINS + 3) (host).  Errors: as mdrq_query for each query. */
int mdrq_estimator_features(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n,
                            uint16_t* out);
/* Number of float32 parameters; copy them out / in (set also clears Adam's moments). */
int mdrq_estimator_param_count(const mdrq_estimator* e, uint64_t* count);
int mdrq_estimator_get_params(const mdrq_estimator* e, float* out);
int mdrq_estimator_set_params(mdrq_estimator* e, const float* in);

/* Exact selectivities of n queries (training labels), measured with shared count-only
 * scans: for each query, each predicate alone and the whole query.  sel: n rows of
 * n_dims + 1 (host).  Errors: as mdrq_query_batch. */
int mdrq_label_selectivities(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, float* sel);

/* Loss (mean squared error of the outputs against the present targets y(s)) of the
 * current parameters on n queries taken as one batch (n <= 65536), and its gradient
 * with respect to the parameters (param_count floats, host).  Nothing is updated. */
int mdrq_estimator_gradient(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n,
                            const float* sel, float* loss, float* grad);

/* Train on n labelled queries; epoch_loss (optional, epochs entries) receives the mean
 * minibatch loss of each epoch.  Errors: MDRQ_EINVAL (bad config, query or label). */
int mdrq_estimator_train(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n,
                         const float* sel, const mdrq_train_config_t* cfg, float* epoch_loss);

/* Estimated selectivities of n queries (same layout as sel; 1 for a dimension the
 * query does not restrict). */
int mdrq_estimator_predict(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, float* sel);

/* The network's intermediate values for n queries (1 .. 65536), as the prediction computes
 * them: h1 and h2 receive the two hidden layers' bfloat16 activations (n rows of `hidden`
 * bit patterns each), y the output layer (n rows of n_dims + 1 floats: the network's
 * correction plus the base estimate, on the log scale y(s), before clamping to [0, 1]).
 * Any of the three may be NULL.  For checking the matrix products against a reference
 * fed the same bfloat16 operands.  Errors: as mdrq_estimator_predict. */
int mdrq_estimator_activations(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, uint16_t* h1,
                               uint16_t* h2, float* y);

/* Keep each output's learned correction only where it helps: on n labelled queries
 * (1 .. MDRQ_EST_MAX_QUERIES; a held-out split, not the training queries) compare, for
 * every output, the mean squared and the mean absolute error on the log scale of the
 * network's estimate and of the base estimate alone (the histogram estimate of a
 * dimension's predicate, or the independence product for the whole query), over the
 * targets present.  An output whose correction does not lower both gets its correction removed (its column of W3 and its entry
 * of b3 set to zero, with their Adam moments), so it returns the base estimate from then
 * on.  kept (optional, n_dims + 1 entries) receives 1 for each output kept, 0 for each
 * removed.  Errors: as mdrq_estimator_gradient. */
int mdrq_estimator_gate(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, const float* sel,
                        uint32_t* kept);

/* Let queries flagged MDRQ_Q_ORDER_ESTIMATED on ds evaluate their predicates in order of
 * ascending estimated selectivity (e = NULL detaches; such queries then keep the order
 * given).  e must have been created on ds. */
int mdrq_attach_estimator(mdrq_dataset* ds, mdrq_estimator* e);

/* Library version as "major.minor.patch". */
const char* mdrq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDRQ_H */
