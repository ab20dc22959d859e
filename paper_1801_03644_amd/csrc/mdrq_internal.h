// Internal declarations shared by the library's HIP sources (never by the oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <exception>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "mdrq.h"

namespace mdrq {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;

// Output modes of the kernels.  kStage is internal: the bitmap goes to scratch and
// the per-tile counts are kept, ready for the ordered compaction into identifiers.
enum Mode : uint32_t { kIds = 0, kBitmap = 1, kCount = 2, kStage = 3 };

// One predicate as the kernels see it: column base pointer and closed interval.
struct DevPred {
  const float* col;
  float lo;
  float hi;
};

// Cross-workgroup bookkeeping of one scan launch.  Zero between launches: the last
// workgroup of a launch resets it, so launches on one stream need no memset.
// The device copy holds `total`; the kernels write `count_out` and `kind` straight into
// the pinned host copy, which the host reads after the stream has completed.
struct ScanState {
  uint64_t total;      // finished workgroups (bits 40..63) and their count (bits 0..39)
  uint64_t count_out;  // exact result size, written at the end of a launch
  uint32_t pad;
  uint32_t kind;       // output chosen for MDRQ_OUT_AUTO: 1 bitmap, 0 identifiers
};

struct ScanParams {
  uint64_t n_rows;
  uint64_t n_tiles;       // wave tiles of 256 * unroll rows (the end of the tile range)
  uint64_t tile_begin;    // first tile of the launch's segments (0: the whole table)
  uint32_t n_preds;
  uint32_t early_out;     // 1: rows rejected by earlier predicates are not re-read
  uint64_t* bitmap;       // kBitmap / kStage: output words
  uint64_t capacity;      // words the bitmap output holds
  uint64_t seg_tiles;     // tiles per workgroup segment
  uint32_t* tile_counts;  // kStage: qualifying rows per tile
  uint32_t* block_sums;   // kStage: qualifying rows per workgroup segment
  ScanState* state;       // device: the workgroups' running total
  uint64_t* count_out;    // pinned host memory: exact result size (count, bitmap modes)
  const uint32_t* order;  // device: evaluation order of preds (null: as given)
  DevPred preds[MDRQ_MAX_DIMS];
};

// Ordered compaction of a staged bitmap into ascending identifiers.
struct CompactParams {
  uint64_t n_tiles;
  uint64_t n_words;
  uint64_t seg_tiles;          // as in the scan that staged the bitmap
  const uint64_t* bitmap;
  const uint32_t* tile_counts;
  const uint32_t* block_sums;
  uint32_t* ids;
  uint64_t capacity;           // identifiers the output holds
  uint64_t* count_out;         // exact result size (written by the last workgroup;
                               // pinned host memory)
  uint32_t auto_mode;          // 1: bitmap or identifiers, whichever is smaller and fits
  uint32_t pad;
  uint64_t buf_bytes;          // output bytes (auto_mode)
  uint32_t* kind_out;          // auto_mode: 1 bitmap, 0 identifiers (pinned host memory)
};

// Launch one single-query scan.  `unroll` selects the tile height (float4 loads per
// lane per column: 1, 2, 4 or 8).  Returns a hipError_t.
hipError_t launch_scan(const ScanParams& p, uint32_t mode, int unroll, int grid,
                       hipStream_t stream);
hipError_t launch_compact(const CompactParams& c, int unroll, int grid, hipStream_t stream);
int scan_tile_rows(int unroll);
// The kernels behind launch_scan / launch_compact (for graph kernel nodes).
const void* scan_kernel_fn(uint32_t mode, int unroll);
const void* compact_kernel_fn(int unroll);
// Workgroups per CU the scan kernel can keep resident (occupancy).
int scan_blocks_per_cu(uint32_t mode, int unroll);

struct ProbeParams {
  uint64_t n_rows;
  uint32_t n_cols;
  uint32_t pad;
  uint32_t* sink;
  const float* cols[MDRQ_MAX_DIMS];
};
hipError_t launch_probe(const ProbeParams& p, int unroll, int grid, hipStream_t stream);

// Early-break read measurement: 128-byte column lines one query's scan must read.
struct LinesParams {
  uint64_t n_rows;
  uint32_t n_preds;
  uint32_t early_out;
  const uint32_t* order;        // device evaluation order (null: as given)
  unsigned long long* lines;    // device: incremented by the line count
  DevPred preds[MDRQ_MAX_DIMS];
};
hipError_t launch_lines(const LinesParams& p, int grid, hipStream_t stream);

// ---------------------------------------------------------------- batched scan

constexpr int kMaxSlots = 16;   // union columns the register variant holds
constexpr int kMaxUnion = MDRQ_MAX_DIMS;   // union columns of one shared scan (LDS variant)

// Output kind of one query in a shared scan.
enum BatchKind : uint32_t { kBatchCount = 0, kBatchBitmap = 1, kBatchIds = 2, kBatchAuto = 3 };

struct BatchParams {
  uint64_t n_rows;
  uint64_t n_tiles;             // 4096-row tiles
  uint64_t n_words;             // bitmap words per query
  uint32_t n_slots;             // union columns held by the scan
  uint32_t pad;
  const uint32_t* table;        // per group: [offsets of records][records]
  const uint32_t* group_first;  // first query of each group (+ end)
  const uint32_t* group_table;  // first table word of each group (+ end)
  uint64_t* words;              // bitmap scratch, one row of n_words per output query
  uint64_t n_out;               // rows of the scratch in use
  uint32_t* tile_counts;        // [count row][tile]
  // Tiles [tile_begin, tile_end) are scanned (all of them: 0 and n_tiles).  count_row
  // maps a query of the batch to its row of tile_counts (null: the query's own index),
  // so that a query can keep its rows over several scans of different tile ranges.
  uint64_t tile_begin, tile_end;
  const uint32_t* count_row;
  // Null: the scratch rows are zeroed before the scan, which stores the non-zero words.
  // Otherwise (slot-mask variant with at most 8 register slots, rank variant) one
  // 16-bit mark per (output row, chunk of at most 16 words) is zeroed instead; the scan
  // stores the non-zero words of a chunk and sets bit g of its mark for each stored
  // word g, and the finish takes unmarked words as zero.
  uint16_t* flags;
  uint64_t n_chunks;            // chunks per output row
  uint64_t n_zero;              // with flags: 64-bit words zeroed from flags on (marks,
                                // then slot tables and slot counters)
  // Sparse scratch (rank variant): a query whose table word has bit 2 set stores only
  // its chunks with a hit, each in a slot of 64-row words taken from its own region of
  // the pool; output row r of such a query is its sparse index.  slot_next[r] counts
  // the slots taken (zeroed before the scan); slots[r * n_chunks + chunk] is the slot
  // + 1 of a stored chunk, 0 otherwise (zeroed); a chunk past sparse_cap[r] slots is
  // not stored, and the query is answered again by the single-query scan.
  uint64_t* pool;               // sparse words, sparse_base[r] + slot slots of RG words
  uint32_t* slots;
  uint32_t* slot_next;
  const uint32_t* sparse_base;  // first pool slot of each sparse query
  const uint32_t* sparse_cap;   // pool slots of each sparse query
  const float* slot_cols[kMaxUnion];
};

struct BatchOut {
  uint32_t kind;                // BatchKind; kBatchAuto is resolved on the device
  uint32_t out_index;           // row of the bitmap scratch, or the sparse index
  void* buf;                    // ids or bitmap words (device)
  uint64_t buf_bytes;
  uint32_t sparse;              // 1: the scratch of this query is sparse (BatchParams)
  uint32_t pad;
};

struct BatchFinish {
  uint64_t n_tiles;
  uint64_t n_words;
  const uint64_t* words;
  const uint16_t* flags;        // as BatchParams::flags (null: every word is valid)
  uint64_t n_chunks;
  uint32_t chunk_shift;         // log2 of the bitmap words per chunk (4, 8 or 16 words)
  uint32_t pad;
  const uint32_t* tile_counts;  // [count row][tile]
  uint32_t* chunk_pos;          // [count row][emit chunk of 128 tiles]: the chunk's count,
                                // then, for identifiers, its first output position
  const uint32_t* count_row;    // per query its row of tile_counts and chunk_pos (null: its index)
  const BatchOut* outs;
  uint64_t* counts_out;         // [query] exact count
  uint32_t* kind_out;           // [query] kind used (kBatchAuto resolved)
  // Sparse scratch (see BatchParams); over_out[query] = 1 when its slots ran out (its
  // output is then not written: the host answers it again).
  const uint64_t* pool;
  const uint32_t* slots;
  const uint32_t* slot_next;
  const uint32_t* sparse_base;
  const uint32_t* sparse_cap;
  uint32_t* over_out;
};

uint32_t batch_key(float x);
int batch_rows_per_lane(int n_slots, int waves, int rg);
int batch_blocks_per_cu(int n_slots, int waves, int rg, int lds_variant, size_t lds_bytes, int sw = 1);
// Shared-scan launch.  lds_variant 0: union keys in registers (n_slots <= kMaxSlots,
// query table in LDS), each predicate's slot searched; 2: the same with each query's
// predicates sorted by slot and the slots walked in order; 3: union keys in registers,
// fixed-size query records (slot mask, bounds per slot) read with scalar loads and the
// range test as a median of three; 4: per group of 32 * sw queries, each row's rank
// among the group's interval ends and per-rank query bitsets (tables in LDS, any union
// that fits); 5: the same with sparse scratch for the queries flagged so (rg 8); 1: union
// keys staged in LDS (n_slots <= kMaxUnion, query table read with scalar loads).
// lds_bytes: the dynamic LDS of the launch.
hipError_t launch_batch_scan(const BatchParams& bp, int n_slots, int waves, int rg, int lds_variant,
                             dim3 grid, size_t lds_bytes, hipStream_t stream, int sw = 1);
// Register slots of the slot-mask variant for a union of n_slots columns (4, 8, 12 or 16):
// its query records hold 2 + 2 x that many words.
int batch_reg_slots(int n_slots);
// Whether the slot-mask variant with that many register slots marks stored chunks
// (BatchParams::flags) instead of relying on zeroed scratch rows.
constexpr bool batch_reg_uses_marks(int reg_slots) { return reg_slots <= 8; }
// LDS bytes the LDS variant stages keys in: waves x slots x rows per lane x 64 x 4.
size_t batch_lds_key_bytes(int n_slots, int waves, int rg);
// Emit chunks (of 128 tiles) of a row of n_tiles tiles: the length of a chunk_pos row.
uint64_t batch_emit_chunks(uint64_t n_tiles);
hipError_t launch_batch_finish(const BatchFinish& f, uint32_t n_queries, hipStream_t stream);
// Zero n 64-bit words with a fill kernel (no memset node, so capturable).
hipError_t launch_zero_words(uint64_t* w, uint64_t n, hipStream_t stream);
// p[0, n) = v (16-bit words).
hipError_t launch_fill_u16(uint16_t* p, uint64_t n, uint16_t v, hipStream_t stream);
// Zero n_rows rows of row_words 64-bit words: row rows[i] (device array) at
// base + rows[i] * row_words.
hipError_t launch_zero_rows(uint64_t* base, uint64_t row_words, const uint32_t* rows, uint32_t n_rows,
                            hipStream_t stream);
// The kernel launches of one shared scan (zeroing, scan, count, emit) as graph kernel
// node parameters, whose arguments point into *L (kept alive while they are used).
struct BatchLaunches {
  uint64_t* zero_ptr;
  uint64_t zero_n;
  BatchParams bp;
  BatchFinish fin;
  void* zero_args[2];
  void* scan_args[1];
  void* fin_args[1];
  hipKernelNodeParams zero, scan, chunk, count, emit;
};
hipError_t batch_launches(const BatchParams& bp, const BatchFinish& f, uint32_t n_queries, int n_slots, int waves,
                          int rg, int lds_variant, dim3 grid, size_t lds_bytes, int sw, BatchLaunches* L);


// ---------------------------------------------------------------- learned estimator

constexpr int kBins = MDRQ_EST_BINS;
constexpr int kFeatPerDim = kBins + 3;  // H(lo), H(hi), histogram estimate, bins
constexpr uint32_t kSampleMax = 16384;   // sample rows sorted in LDS per column

struct HistArgs {
  uint64_t n_rows;
  uint32_t m;                  // sample size
  uint32_t m_pow2;             // power of two >= m (sorting network width)
  float* bounds;               // [column][kBins + 1]
  const float* cols[MDRQ_MAX_DIMS];
};

struct FeatureArgs {
  const float* qd;             // [query][dim] (lo, hi, restricted)
  const float* bounds;         // [dim][kBins + 1]
  uint16_t* x;                 // [query][dim * kFeatPerDim] bfloat16 bits
  float* base;                 // [query][dim + 1] histogram estimates (log scale)
  uint32_t n, d;
  float inv_rows;              // 1 / N
  float inv_ln_rows;           // 1 / ln N
};

// C = A * B (+ bias) with bfloat16 operands read through element strides.
struct GemmArgs {
  const uint16_t* a;
  const uint16_t* b;
  uint64_t a_m, a_k, b_k, b_n;
  uint32_t M, N, K;
  uint32_t c_ld;
  const float* bias;           // [N] or null
  const float* add;            // [M][c_ld] added to the result, or null
  float* c;                    // float32 result or null
  uint16_t* act;               // bfloat16 of the result (GELU applied if gelu) or null
  uint32_t gelu;
  uint32_t pad;
};

struct LossArgs {
  const float* y;              // [rows][cols] network output
  const float* t;              // targets
  const float* mask;           // 1 where a target is present
  float* dy;                   // gradient of the loss
  uint16_t* dyb;               // the same in bfloat16
  float* loss;                 // += loss of this batch
  uint32_t rows, cols;
  float inv_count;             // 1 / present targets in the batch
  uint32_t pad;
};

hipError_t launch_sample_sort(const HistArgs& a, uint32_t n_cols, hipStream_t s);
hipError_t launch_features(const FeatureArgs& f, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_loss_grad(const LossArgs& l, hipStream_t s);
hipError_t launch_gelu_back(const float* dh, const float* z, float* dz, uint16_t* dzb, uint64_t n,
                            hipStream_t s);
hipError_t launch_colsum(const float* in, uint32_t rows, uint32_t cols, float* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint64_t n, float lr, int step,
                       hipStream_t s);
hipError_t launch_to_bf16(const float* src, uint64_t n, uint16_t* dst, hipStream_t s);
hipError_t launch_gather_rows(const void* src, const uint32_t* idx, uint32_t n, uint32_t row_bytes,
                              void* dst, hipStream_t s);
hipError_t launch_targets(const float* sel, uint32_t n, uint32_t o, uint64_t n_rows, float* t,
                          float* mask, hipStream_t s);
hipError_t launch_to_selectivity(const float* y, const float* qd, uint32_t n, uint32_t d,
                                 uint64_t n_rows, float* sel, hipStream_t s);

// Load-time validation: NaN count and per-column min/max (order-preserving keys).
struct ColumnStats {
  uint32_t nan_count;
  uint32_t pad;
  uint32_t min_key[MDRQ_MAX_DIMS];
  uint32_t max_key[MDRQ_MAX_DIMS];
};
hipError_t launch_validate(const float* const* cols_dev, uint32_t n_dims, uint64_t n_rows,
                           ColumnStats* stats, hipStream_t stream);
float key_to_float(uint32_t key);

// A canonical query: predicates that can change the result, in evaluation order.
struct Plan {
  std::vector<DevPred> preds;
  std::vector<uint32_t> dims;  // dimension of each entry of preds
  bool empty = false;          // some interval is empty: no row qualifies
  uint32_t mode = kIds;
  uint64_t capacity = 0;
  bool early_out = true;
  bool auto_mode = false;          // MDRQ_OUT_AUTO: identifiers or bitmap, decided on device
  const uint32_t* order = nullptr;  // device evaluation order, written by the estimator
};

// Thread-local error reporting.
int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
void clear_error();

// Body of a C entry point: a C++ exception (a failed host allocation) becomes a status
// instead of crossing the C boundary.
template <typename F>
int guarded(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(MDRQ_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    return fail(MDRQ_EDEVICE, std::string("unexpected host error: ") + e.what());
  } catch (...) {
    return fail(MDRQ_EDEVICE, "unexpected host error");
  }
}

struct Device {
  int id = 0;
  int cus = 0;
  size_t lds = 0;
};
const Device& device();

}  // namespace mdrq

struct mdrq_dataset;

namespace mdrq {
// Host runtime pieces shared by the single-query and batched paths (runtime.cpp).
int check_query(const mdrq_dataset* ds, const mdrq_query_t* q);
int check_result(const mdrq_result_t* r);
Plan make_plan(const mdrq_dataset* ds, const mdrq_query_t* q, const mdrq_result_t* r);
uint64_t n_words(const mdrq_dataset* ds);
// Tile height of the dataset's single-query scans: MDRQ_OPT_UNROLL, else chosen from
// its rows per CU.
int scan_unroll(const mdrq_dataset* ds);
int finish_empty(mdrq_dataset* ds, const Plan& plan, mdrq_result_t* r, hipStream_t stream);
struct SingleScratch;
int run_query(mdrq_dataset* ds, const Plan& plan, mdrq_result_t* r, hipStream_t stream);
// The same on a worker's own scratch (no lock; falls back to run_query when the launch
// shape does not fit it or the scratch is not allocated).
int run_query_on(mdrq_dataset* ds, const Plan& plan, mdrq_result_t* r, hipStream_t stream,
                 const SingleScratch& s);
// Allocate a worker's single-query scratch for this dataset; freed by free_single.
int reserve_single(const mdrq_dataset* ds, SingleScratch& s);
void free_single(SingleScratch& s);
}  // namespace mdrq

namespace mdrq {
// Estimator hooks (estimator_host.cpp): estimated selectivities of the queries that
// ask for estimated order (rows of n_dims + 1; empty if no estimator is attached),
// and the reordering of a plan by them.
int estimate_for_order(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n,
                       std::vector<float>& est);
void order_plan(Plan& plan, const float* est_row);
// Queue, on `stream`, the estimator's prediction for one query and the permutation of
// the plan's predicates by ascending estimated selectivity into a device buffer
// (plan.order); no host round trip.  The estimator stays locked through `hold` until
// the caller's launches that read plan.order have completed.
int order_on_device(mdrq_dataset* ds, const mdrq_query_t* q, Plan& plan, hipStream_t stream,
                    std::unique_lock<std::mutex>& hold);

// One query's evaluation order computed in one launch (features, network, ranking).
struct OrderArgs {
  const float* bounds;         // [dim][kBins + 1]
  const uint16_t* wb;          // bfloat16 weights (W1, W2, W3 at their parameter offsets)
  const float* params;         // float32 parameters (biases)
  uint64_t oW1, ob1, oW2, ob2, oW3, ob3;
  uint32_t d, H, k, pad;
  float inv_rows, inv_ln_rows, ln_rows, pad2;
  uint32_t* order;             // out: order[rank] = position in the plan
  uint32_t restricted[MDRQ_MAX_DIMS / 32];  // bit j: dimension j is restricted
  float lo[MDRQ_MAX_DIMS], hi[MDRQ_MAX_DIMS];
  uint32_t dims[MDRQ_MAX_DIMS];             // the plan's dimensions, in plan order
};
hipError_t launch_order_fused(const OrderArgs& a, hipStream_t s);
void detach_estimator(mdrq_dataset* ds);
}  // namespace mdrq

namespace mdrq {
struct BatchWorkspace;
// What a batched call did: shared scans launched, the column bytes they cover (every
// union column in full) and their device time.
struct BatchRunStats {
  uint64_t scans = 0;
  uint64_t column_bytes = 0;
  double device_ms = 0.0;
  uint64_t alone = 0;          // queries answered by their own scan (cheaper for few)
  uint64_t sparse = 0;         // queries whose scratch was sized by their estimate
  uint64_t reruns = 0;         // of those, answered again (the estimate was too low)
};
// Scratch of one query in a shared scan with estimated sizing: pool slots (chunks with a
// hit) reserved for an estimated result of est_rows rows, 0 when the worst case (a full
// bitmap row) is no larger.  chunk_rows: rows per chunk.
uint64_t sparse_slots(const mdrq_dataset* ds, double est_rows, uint64_t chunk_rows);
// Bytes of scratch a request reserves in serving (an upper bound on what the shared
// scan lays out for it): a bitmap row and its chunk marks, or, sized by an estimate,
// the slot table and pool slots; 0 for count-only requests.
uint64_t request_scratch_bytes(const mdrq_dataset* ds, const mdrq_result_t& r, double est_rows);
// Batched path (batch_host.cpp).  ws: the workspace to use (null: the dataset's own);
// tune: a new batch shape may be autotuned (otherwise a known or default configuration
// is used).  Calls with different workspaces may run concurrently.
// est_in (optional): the attached estimator's estimates of the n queries (rows of
// n_dims + 1), computed by the caller; otherwise they are computed here when a query
// asks for estimated order or sizing.
int run_batch(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, mdrq_result_t* rs,
              hipStream_t stream, BatchWorkspace* ws = nullptr, bool tune = true,
              BatchRunStats* st = nullptr, const float* est_in = nullptr);
// Circular shared scan (batch_host.cpp).  The rows are cut into segments of whole
// tiles; each step scans the next segment, wrapping around, for every active query, so
// a query joins at whatever segment comes next and is complete once it has seen each
// segment once.  Each active query holds a slot (a bitmap row, its chunk marks and a row
// of tile counts) from its first step to its last.
struct CircularScan;
// Bytes of device memory one query slot takes.
uint64_t circular_slot_bytes(const mdrq_dataset* ds);
// A circular scan with `slots` query slots and `segments` segments per circle (at most
// one per tile).
int circular_create(mdrq_dataset* ds, uint32_t slots, uint32_t segments, CircularScan** out);
void circular_destroy(CircularScan* c);
uint32_t circular_free_slots(const CircularScan* c);
uint32_t circular_active(const CircularScan* c);
// Active queries, a step in flight, or requests answered at admission not yet reported.
bool circular_busy(const CircularScan* c);
// Admit a query whose result goes to *r (count-only or device memory; checked by the
// caller).  *answered = true: it needed no shared scan (an empty result, or more
// predicates than a scan's union may hold) and was answered on `stream`; its tag is
// reported by a later circular_step, once the stream has done that work.  Otherwise it
// joins at the next step.  MDRQ_EBUSY: no free slot, or its columns would make the
// active queries' union too wide for one scan; nothing was done.
int circular_admit(CircularScan* c, const mdrq_query_t* q, mdrq_result_t* r, void* tag, hipStream_t stream,
                   bool* answered);
// One call: enqueue the next step (the next segment for every active query) on `stream`,
// then wait for the step enqueued by the previous call (pipelined steps) or for this one
// and report the queries it completed (their results written, their tags appended to
// `done`).  Call while circular_busy.  `active_out`: the
// queries the enqueued step scans.  On an error every query in flight or active is
// dropped, its tag appended to `done` and the error put in its result record.
int circular_step(CircularScan* c, hipStream_t stream, std::vector<void*>& done, BatchRunStats* st,
                  uint64_t* active_out);
// Answer queries one after another, each by its own single-query scan, exactly as
// mdrq_query does (estimated order ranked on the device when asked; AUTO decided
// exactly on the device).  Allocates nothing once the dataset's single-query buffers
// exist.
int run_separately(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, mdrq_result_t* rs, hipStream_t stream,
                   const SingleScratch* scratch = nullptr);
// Whether separate single-query scans answer these queries sooner than one shared scan
// (the cost model of the batched path).
bool separate_scans_cheaper(const mdrq_dataset* ds, const mdrq_query_t* qs, const mdrq_result_t* rs, uint32_t n);
// Grow a workspace so that batches of up to max_queries queries whose requests'
// request_scratch_bytes sum to at most scratch_bytes run without allocating.
int reserve_batch(const mdrq_dataset* ds, BatchWorkspace& ws, uint32_t max_queries,
                  uint64_t scratch_bytes);
void free_batch(BatchWorkspace& ws);
// Close every live server still open on the dataset (serve.cpp), before it is freed.
void close_servers(mdrq_dataset* ds);
// Exact count of each single predicate (label.hip): one sort of each queried column's
// keys, then two binary searches per predicate.
int count_single_predicates(const mdrq_dataset* ds, const std::vector<mdrq_pred>& preds,
                            std::vector<uint64_t>& counts);
}  // namespace mdrq

namespace mdrq {
// Device and pinned buffers of the batched path, grown on demand.
// Single-query scratch of one serving worker: its own scan state, staged bitmap, tile
// and workgroup counts and pinned result record, so workers' single-query scans run
// side by side (the dataset's own scratch serialises its callers by a lock).
struct SingleScratch {
  ScanState* state = nullptr;        // device, zero between launches
  uint64_t* stage_bitmap = nullptr;  // ceil(n_rows / 64) words
  uint32_t* tile_counts = nullptr;   // one per wave tile of the smallest height
  uint64_t tile_counts_len = 0;
  uint32_t* block_sums = nullptr;    // one per workgroup
  uint64_t block_sums_len = 0;
  ScanState* host = nullptr;         // pinned, mapped: the count and AUTO's choice
  ScanState* host_dev = nullptr;
};

struct BatchWorkspace {
  SingleScratch single;          // serving workers: scratch of their single-query scans
  void* d_blob = nullptr;        // table words, group arrays, BatchOut records
  uint64_t d_blob_bytes = 0;
  void* h_blob = nullptr;        // pinned staging of the same
  uint64_t h_blob_bytes = 0;
  uint64_t* d_words = nullptr;   // bitmap scratch: rows, sparse pools, marks, slot tables
  uint64_t d_words_len = 0;
  uint32_t* d_tile_counts = nullptr;
  uint64_t d_tile_counts_len = 0;
  void* h_res = nullptr;         // counts (u64) and kinds (u32) per query: mapped pinned
  void* h_res_dev = nullptr;     // its device address
  uint64_t res_len = 0;          // queries the two hold
  void* d_stage = nullptr;       // device staging for host-memory outputs
  uint64_t d_stage_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  // Shared scans replayed from graphs (query-table copy, zeroing, scan, finish, and the
  // events around them), one per scan kernel, arguments updated per batch.
  struct Graph {
    const void* scan_fn = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr, zero = nullptr, scan = nullptr, chunk = nullptr, count = nullptr, emit = nullptr;
  };
  std::vector<Graph> graphs;
};

// A single-query launch sequence (scan, compaction for identifiers, and the profiling
// events when enabled) instantiated once per launch shape and replayed with each
// query's kernel arguments.
struct QueryGraph {
  uint32_t mode = 0;
  int unroll = 0;
  uint64_t grid = 0;
  bool profiling = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t scan = nullptr, compact = nullptr;
};

// Launch configuration of a shared scan.
struct BatchConfig {
  int waves = 4;                 // waves per workgroup (4 or 8)
  uint32_t group = 0;            // queries per workgroup group (0 = all)
  int rows_per_lane = 16;        // 64-row groups per lane per chunk: 2, 4, 8 or 16
  int lds = 0;                   // 1: keys staged in LDS (any union up to kMaxUnion);
                                 // 2: keys in registers, predicates walked in slot order;
                                 // 3: keys in registers, slot-mask records;
                                 // 4: ranks among interval ends, query bitsets
};
}  // namespace mdrq

// Dataset: columns in HBM plus the workspace of its scans.
struct mdrq_dataset {
  uint64_t n_rows = 0;
  uint32_t n_dims = 0;
  bool owned = true;
  float* base = nullptr;                 // owned allocation (all columns)
  uint64_t stride = 0;                   // owned: floats between columns
  std::vector<const float*> cols;        // device pointer of each column
  std::vector<float> col_min, col_max;

  // Calls on a dataset are serialised by `mu`; inside a call, `single_mu` guards the
  // single-query workspace and `stat_mu` the counters and the tuned configurations (the
  // serving loop's workers run batches concurrently).
  std::mutex mu;
  std::mutex single_mu;
  std::mutex stat_mu;
  // Single-query workspace.
  mdrq::ScanState* state = nullptr;      // device
  uint64_t* stage_bitmap = nullptr;      // device, ceil(n_rows / 64) words
  uint32_t* tile_counts = nullptr;       // device, tiles at the smallest tile height
  uint32_t* block_sums = nullptr;        // device, block_sums_len entries
  uint64_t block_sums_len = 0;
  uint64_t max_tiles = 0;
  mdrq::ScanState* host_state = nullptr; // pinned: results the kernels write for the host
  mdrq::ScanState* host_state_dev = nullptr;  // its device address
  void* staging = nullptr;               // device staging for host-resident outputs
  uint64_t staging_bytes = 0;

  // Profiling.
  bool profiling = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  uint64_t prof_launches = 0;
  double prof_scan_ms = 0.0;
  double prof_total_ms = 0.0;
  int unroll = 0;                        // tile height of single-query scans (x 256 rows); 0: by size
  // Launch sequences replayed from graphs (MDRQ_OPT_GRAPHS): single queries (one graph
  // per launch shape) and shared scans (one per scan kernel and workspace), arguments
  // updated per call.
  bool graph_single = false;
  bool graph_batch = false;
  int circular_mode = 4;                 // MDRQ_OPT_CIRCULAR bits
  int64_t reserve_ppm = 4000000;         // MDRQ_Q_SIZE_ESTIMATED: reserved rows per estimate (1e-6)
  std::vector<mdrq::QueryGraph> graphs;
  // Batched path.
  mdrq::BatchWorkspace batch;
  int batch_waves = 0;                   // 0: autotuned
  uint32_t batch_group = 0;              // 0: autotuned
  int batch_rows = 0;                    // 64-row groups per lane (2, 4, 8, 16); 0: autotuned
  int batch_variant = 0;                 // 1: keys in registers, 2: in LDS, 3: registers and
                                         // slot-order walk, 4: registers and slot-mask
                                         // records, 5: ranks and query bitsets;
                                         // 0: autotuned
  int rank_buckets = 0;                  // rank variant's bucket map: 0 fewest steps,
                                         // 1 by key, 2 by value
  bool autotune = true;
  std::vector<std::pair<uint64_t, mdrq::BatchConfig>> tuned;  // shape key -> config
  uint64_t batch_launches = 0;
  double batch_ms = 0.0;
  uint64_t batch_lookups = 0;            // rank variant: rows x (group, column) pairs looked up
  uint64_t batch_column_bytes = 0;       // column bytes the shared scans read
  double batch_scan_ms = 0.0;            // device time of the shared-scan kernels alone
  uint64_t sized_queries = 0;            // MDRQ_Q_SIZE_ESTIMATED queries with sparse scratch
  uint64_t sized_reruns = 0;             // of those, answered again (estimate too low)

  mdrq_estimator* estimator = nullptr;   // attached estimator (MDRQ_Q_ORDER_ESTIMATED)
  std::vector<mdrq_server*> servers;     // live servers open on the dataset (stat_mu)

  int64_t grid = 0;                      // workgroups per launch (0 = blocks_per_cu per CU)
  int blocks_per_cu = 3;                 // default launch width, capped by occupancy
};
