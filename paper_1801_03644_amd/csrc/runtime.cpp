// Host runtime behind the C ABI: dataset load and validation, query checks and
// canonicalisation, output planning, launch and completion of single-query scans.
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>

#include "mdrq_internal.h"

namespace mdrq {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return MDRQ_EDEVICE;
}

void clear_error() { g_err.clear(); }

const Device& device() {
  static std::mutex mu;
  static std::vector<Device> cache;
  int id = 0;
  if (hipGetDevice(&id) != hipSuccess) id = 0;
  std::lock_guard<std::mutex> lock(mu);
  for (const Device& d : cache)
    if (d.id == id) return d;
  Device d;
  d.id = id;
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, id) == hipSuccess) {
    d.cus = prop.multiProcessorCount;
    d.lds = prop.sharedMemPerBlock;
  }
  if (d.cus <= 0) d.cus = 256;
  cache.push_back(d);
  return cache.back();
}

}  // namespace mdrq

using namespace mdrq;

namespace {

constexpr uint64_t kMaxRows = 0xFFFFFFFFull;

#define MDRQ_HIP(call, what)                  \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return fail_hip(e_, what); \
  } while (0)

void destroy_graph(QueryGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

void free_dataset(mdrq_dataset* ds) {
  if (!ds) return;
  if (ds->owned && ds->base) (void)hipFree(ds->base);
  if (ds->state) (void)hipFree(ds->state);
  if (ds->stage_bitmap) (void)hipFree(ds->stage_bitmap);
  if (ds->tile_counts) (void)hipFree(ds->tile_counts);
  if (ds->block_sums) (void)hipFree(ds->block_sums);
  if (ds->host_state) (void)hipHostFree(ds->host_state);
  if (ds->staging) (void)hipFree(ds->staging);
  for (QueryGraph& g : ds->graphs) destroy_graph(g);
  if (ds->ev0) (void)hipEventDestroy(ds->ev0);
  if (ds->ev1) (void)hipEventDestroy(ds->ev1);
  if (ds->ev2) (void)hipEventDestroy(ds->ev2);
  free_batch(ds->batch);
  delete ds;
}

int alloc_workspace(mdrq_dataset* ds) {
  const uint64_t min_tile = static_cast<uint64_t>(scan_tile_rows(1));
  ds->max_tiles = (ds->n_rows + min_tile - 1) / min_tile + 1;
  const uint64_t words = (ds->n_rows + 63) / 64 + 1;
  MDRQ_HIP(hipMalloc(&ds->state, sizeof(ScanState)), "hipMalloc(scan state)");
  MDRQ_HIP(hipMemset(ds->state, 0, sizeof(ScanState)), "hipMemset(scan state)");
  MDRQ_HIP(hipMalloc(&ds->stage_bitmap, words * sizeof(uint64_t)), "hipMalloc(stage bitmap)");
  MDRQ_HIP(hipMalloc(&ds->tile_counts, ds->max_tiles * sizeof(uint32_t)), "hipMalloc(tile counts)");
  // Mapped and coherent: the kernels' stores reach it without a copy.
  MDRQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&ds->host_state), sizeof(ScanState),
                         hipHostMallocMapped | hipHostMallocCoherent),
           "hipHostMalloc(scan state)");
  memset(ds->host_state, 0, sizeof(ScanState));
  MDRQ_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&ds->host_state_dev), ds->host_state, 0),
           "hipHostGetDevicePointer(scan state)");
  return MDRQ_OK;
}

}  // namespace

namespace mdrq {

int check_query(const mdrq_dataset* ds, const mdrq_query_t* q) {
  if (!q) return fail(MDRQ_EINVAL, "query is NULL");
  if (q->n_preds > 0 && !q->preds) return fail(MDRQ_EINVAL, "query has predicates but preds is NULL");
  if (q->n_preds > ds->n_dims) return fail(MDRQ_EINVAL, "more predicates than dimensions");
  if (q->flags & ~static_cast<uint32_t>(MDRQ_Q_ORDER_ESTIMATED | MDRQ_Q_NO_EARLYOUT | MDRQ_Q_SIZE_ESTIMATED))
    return fail(MDRQ_EINVAL, "unknown query flags");
  uint64_t seen[MDRQ_MAX_DIMS / 64] = {0, 0};
  for (uint32_t i = 0; i < q->n_preds; ++i) {
    const mdrq_pred& p = q->preds[i];
    if (p.dim >= ds->n_dims) return fail(MDRQ_EINVAL, "predicate dimension out of range");
    if (std::isnan(p.lo) || std::isnan(p.hi)) return fail(MDRQ_EINVAL, "NaN bound");
    uint64_t& w = seen[p.dim / 64];
    const uint64_t bit = uint64_t{1} << (p.dim % 64);
    if (w & bit) return fail(MDRQ_EINVAL, "dimension appears twice in one query");
    w |= bit;
  }
  return MDRQ_OK;
}

int check_result(const mdrq_result_t* r) {
  if (!r) return fail(MDRQ_EINVAL, "result is NULL");
  if (r->mode > MDRQ_OUT_AUTO) return fail(MDRQ_EINVAL, "unknown result mode");
  if (r->mem > MDRQ_MEM_DEVICE) return fail(MDRQ_EINVAL, "unknown result memory kind");
  if (!r->buf && r->buf_bytes > 0) return fail(MDRQ_EINVAL, "buf is NULL but buf_bytes > 0");
  return MDRQ_OK;
}

Plan make_plan(const mdrq_dataset* ds, const mdrq_query_t* q, const mdrq_result_t* r) {
  Plan plan;
  const float inf = std::numeric_limits<float>::infinity();
  plan.preds.reserve(q->n_preds);
  plan.dims.reserve(q->n_preds);
  for (uint32_t i = 0; i < q->n_preds; ++i) {
    const mdrq_pred& p = q->preds[i];
    if (p.lo > p.hi) plan.empty = true;
    if (p.lo == -inf && p.hi == inf) continue;  // the partial-match [-inf, +inf]
    plan.preds.push_back(DevPred{ds->cols[p.dim], p.lo, p.hi});
    plan.dims.push_back(p.dim);
  }
  plan.mode = r->mode == MDRQ_OUT_BITMAP ? kBitmap : r->mode == MDRQ_OUT_COUNT ? kCount : kIds;
  plan.auto_mode = r->mode == MDRQ_OUT_AUTO;
  plan.capacity = plan.mode == kIds ? r->buf_bytes / 4 : plan.mode == kBitmap ? r->buf_bytes / 8 : 0;
  plan.early_out = !(q->flags & MDRQ_Q_NO_EARLYOUT);
  return plan;
}

uint64_t n_words(const mdrq_dataset* ds) { return (ds->n_rows + 63) / 64; }

// Small tables leave most CUs idle with tall tiles, and short tiles cost more per row:
// measured over 2.5e5 .. 1.6e7 rows of three columns, two 16-byte loads per lane were
// fastest below about 6k rows per CU, four below 64k, eight above (within 2% at 64k).
int scan_unroll(const mdrq_dataset* ds) {
  if (ds->unroll) return ds->unroll;
  const uint64_t per_cu = ds->n_rows / std::max<uint64_t>(1, device().cus);
  return per_cu < 6144 ? 2 : per_cu < 65536 ? 4 : 8;
}

// Result of an empty answer (no launch): zero the bitmap words the buffer holds.
int finish_empty(mdrq_dataset* ds, const Plan& plan, mdrq_result_t* r, hipStream_t stream) {
  r->count = 0;
  r->written = 0;
  r->status = MDRQ_OK;
  if (plan.mode == kBitmap) {
    const uint64_t words = std::min(plan.capacity, n_words(ds));
    if (words) {
      if (r->mem == MDRQ_MEM_DEVICE) {
        MDRQ_HIP(hipMemsetAsync(r->buf, 0, words * 8, stream), "hipMemsetAsync(bitmap)");
        MDRQ_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
      } else {
        memset(r->buf, 0, words * 8);
      }
    }
    r->written = words;
    if (plan.capacity < n_words(ds)) r->status = MDRQ_EOVERFLOW;
  }
  return r->status;
}

int ensure_staging(mdrq_dataset* ds, uint64_t bytes) {
  if (bytes <= ds->staging_bytes) return MDRQ_OK;
  if (ds->staging) (void)hipFree(ds->staging);
  ds->staging = nullptr;
  ds->staging_bytes = 0;
  if (hipMalloc(&ds->staging, bytes) != hipSuccess) return fail(MDRQ_ENOMEM, "staging buffer");
  ds->staging_bytes = bytes;
  return MDRQ_OK;
}

int recover_state(ScanState* state) {
  (void)hipDeviceSynchronize();
  (void)hipMemset(state, 0, sizeof(ScanState));
  (void)hipDeviceSynchronize();
  return MDRQ_OK;
}

// Device buffers of one single-query scan, and the pinned record its kernels write the
// count and AUTO's choice into (null: the dataset's).
struct ScanWork {
  ScanState* state;        // zero between launches
  uint64_t* stage_bitmap;  // ceil(n_rows / 64) words
  uint32_t* tile_counts;   // one per wave tile
  uint32_t* block_sums;    // one per workgroup
  ScanState* host = nullptr;
  ScanState* host_dev = nullptr;
};

// Launch shape of a single-query scan: grid and tiles per workgroup segment.
void scan_shape(const mdrq_dataset* ds, uint32_t kmode, uint64_t n_tiles, uint64_t max_grid, uint64_t* grid_out,
                uint64_t* seg_out) {
  const int U = scan_unroll(ds);
  const uint64_t tile = static_cast<uint64_t>(scan_tile_rows(U));
  const Device& dev = device();
  const uint64_t per_cu = std::min<uint64_t>(scan_blocks_per_cu(kmode, U), ds->blocks_per_cu);
  const uint64_t resident = per_cu * dev.cus;
  uint64_t want = ds->grid > 0 ? static_cast<uint64_t>(ds->grid) : resident;
  want = std::min(want, max_grid);
  const uint64_t blocks_needed = (n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  uint64_t grid = std::min<uint64_t>(blocks_needed, want);
  // Segments of whole 4096-row compaction chunks.
  const uint64_t align = std::max<uint64_t>(1, 4096 / tile);
  const uint64_t seg = ((n_tiles + grid - 1) / grid + align - 1) / align * align;
  *grid_out = (n_tiles + seg - 1) / seg;
  *seg_out = seg;
}

constexpr size_t kMaxQueryGraphs = 16;

// Launch a single query's scan (and compaction) by replaying the dataset's graph for
// this launch shape, built on first use; each replay carries this query's arguments.
// With profiling on, the graph records the dataset's three events around the kernels.
hipError_t launch_query_graph(mdrq_dataset* ds, const ScanParams& p, const CompactParams& c, uint32_t kmode,
                              uint64_t grid, bool compact, hipStream_t stream) {
  const int U = scan_unroll(ds);
  void* sargs[] = {const_cast<ScanParams*>(&p)};
  void* cargs[] = {const_cast<CompactParams*>(&c)};
  hipKernelNodeParams ks{};
  ks.func = const_cast<void*>(scan_kernel_fn(kmode, U));
  ks.gridDim = dim3(static_cast<uint32_t>(grid));
  ks.blockDim = dim3(kBlock);
  ks.sharedMemBytes = 0;
  ks.kernelParams = sargs;
  ks.extra = nullptr;
  hipKernelNodeParams kc = ks;
  kc.func = const_cast<void*>(compact_kernel_fn(U));
  kc.kernelParams = cargs;
  if (!ks.func || !kc.func) return hipErrorInvalidValue;
  QueryGraph* qg = nullptr;
  for (QueryGraph& g : ds->graphs)
    if (g.mode == kmode && g.unroll == U && g.grid == grid && g.profiling == ds->profiling) qg = &g;
  hipError_t e = hipSuccess;
  if (qg) {
    e = hipGraphExecKernelNodeSetParams(qg->exec, qg->scan, &ks);
    if (e == hipSuccess && compact) e = hipGraphExecKernelNodeSetParams(qg->exec, qg->compact, &kc);
    if (e == hipSuccess) return hipGraphLaunch(qg->exec, stream);
    // An update the instantiated graph does not take: build it anew below.
    destroy_graph(*qg);
    ds->graphs.erase(ds->graphs.begin() + (qg - ds->graphs.data()));
  }
  if (ds->graphs.size() >= kMaxQueryGraphs) {
    destroy_graph(ds->graphs.front());
    ds->graphs.erase(ds->graphs.begin());
  }
  QueryGraph g;
  g.mode = kmode;
  g.unroll = U;
  g.grid = grid;
  g.profiling = ds->profiling;
  e = hipGraphCreate(&g.graph, 0);
  hipGraphNode_t last = nullptr;
  auto chain = [&](hipGraphNode_t n) { last = n; };
  if (e == hipSuccess && g.profiling) {
    hipGraphNode_t n = nullptr;
    e = hipGraphAddEventRecordNode(&n, g.graph, nullptr, 0, ds->ev0);
    chain(n);
  }
  if (e == hipSuccess) {
    e = hipGraphAddKernelNode(&g.scan, g.graph, last ? &last : nullptr, last ? 1 : 0, &ks);
    chain(g.scan);
  }
  if (e == hipSuccess && g.profiling) {
    hipGraphNode_t n = nullptr;
    e = hipGraphAddEventRecordNode(&n, g.graph, &last, 1, ds->ev1);
    chain(n);
  }
  if (e == hipSuccess && compact) {
    e = hipGraphAddKernelNode(&g.compact, g.graph, &last, 1, &kc);
    chain(g.compact);
  }
  if (e == hipSuccess && g.profiling) {
    hipGraphNode_t n = nullptr;
    e = hipGraphAddEventRecordNode(&n, g.graph, &last, 1, ds->ev2);
    chain(n);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    destroy_graph(g);
    return e;
  }
  ds->graphs.push_back(g);
  return hipGraphLaunch(ds->graphs.back().exec, stream);
}

// Scan (and compaction) of one planned query, whose predicates are preds[0 .. n_preds),
// into `out` (device memory, out_elems elements) with the workspace `w`; waits for
// completion.  With host_out, `out` is device staging copied to r->buf at the end.
int scan_query(mdrq_dataset* ds, const Plan& plan, const DevPred* preds, uint32_t n_preds, mdrq_result_t* r,
               hipStream_t stream, const ScanWork& w, void* out, uint64_t out_elems, uint64_t grid, uint64_t seg,
               bool host_out) {
  const int U = scan_unroll(ds);
  const uint64_t tile = static_cast<uint64_t>(scan_tile_rows(U));
  const uint32_t kmode = plan.mode == kIds ? kStage : plan.mode;
  const uint64_t n_tiles = (ds->n_rows + tile - 1) / tile;
  const uint64_t elem = plan.mode == kIds ? 4 : 8;
  ScanParams p{};
  p.n_rows = ds->n_rows;
  p.n_tiles = n_tiles;
  p.n_preds = n_preds;
  p.early_out = plan.early_out ? 1u : 0u;
  p.bitmap = plan.mode == kIds ? w.stage_bitmap
             : plan.mode == kBitmap ? static_cast<uint64_t*>(out) : nullptr;
  p.capacity = plan.mode == kIds ? n_words(ds) : plan.mode == kBitmap ? out_elems : 0;
  p.seg_tiles = seg;
  p.tile_counts = w.tile_counts;
  p.block_sums = w.block_sums;
  p.state = w.state;
  ScanState* const host_dev = w.host_dev ? w.host_dev : ds->host_state_dev;
  const volatile ScanState* const host = w.host ? w.host : ds->host_state;
  // The dataset's profiling events and graphs serve its own scratch only.
  const bool profiling = ds->profiling && !w.host;
  p.count_out = &host_dev->count_out;
  p.order = plan.order;
  for (uint32_t i = 0; i < n_preds; ++i) p.preds[i] = preds[i];
  CompactParams c{};
  c.n_tiles = n_tiles;
  c.n_words = n_words(ds);
  c.seg_tiles = seg;
  c.bitmap = w.stage_bitmap;
  c.tile_counts = w.tile_counts;
  c.block_sums = w.block_sums;
  c.ids = static_cast<uint32_t*>(out);
  c.capacity = plan.mode == kIds ? out_elems : 0;
  c.count_out = &host_dev->count_out;
  c.auto_mode = plan.auto_mode ? 1u : 0u;
  c.buf_bytes = r->buf_bytes;
  c.kind_out = &host_dev->kind;

  if (profiling) {
    if (!ds->ev0) MDRQ_HIP(hipEventCreate(&ds->ev0), "hipEventCreate");
    if (!ds->ev1) MDRQ_HIP(hipEventCreate(&ds->ev1), "hipEventCreate");
    if (!ds->ev2) MDRQ_HIP(hipEventCreate(&ds->ev2), "hipEventCreate");
  }
  hipError_t e = hipSuccess;
  if (ds->graph_single && w.state == ds->state) {
    e = launch_query_graph(ds, p, c, kmode, grid, plan.mode == kIds, stream);
  } else {
    if (profiling) e = hipEventRecord(ds->ev0, stream);
    if (e == hipSuccess) e = launch_scan(p, kmode, U, static_cast<int>(grid), stream);
    if (e == hipSuccess && profiling) e = hipEventRecord(ds->ev1, stream);
    if (e == hipSuccess && plan.mode == kIds) e = launch_compact(c, U, static_cast<int>(grid), stream);
    if (e == hipSuccess && profiling) e = hipEventRecord(ds->ev2, stream);
  }
  if (e != hipSuccess) {
    recover_state(w.state);
    return fail_hip(e, "scan kernel launch");
  }
  // The last workgroup wrote the count (and AUTO's choice) into pinned host memory.
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    recover_state(w.state);
    return fail_hip(e, "scan completion");
  }
  if (profiling) {
    float ms1 = 0.f, ms2 = 0.f;
    MDRQ_HIP(hipEventElapsedTime(&ms1, ds->ev0, ds->ev1), "hipEventElapsedTime");
    MDRQ_HIP(hipEventElapsedTime(&ms2, ds->ev0, ds->ev2), "hipEventElapsedTime");
    ds->prof_scan_ms += ms1;
    ds->prof_total_ms += ms2;
    ds->prof_launches += 1;
  }
  const volatile ScanState* hs = host;
  const uint64_t count = hs->count_out;
  r->count = count;
  if (plan.auto_mode && hs->kind == 1) {  // AUTO chose the bitmap
    r->mode = MDRQ_OUT_BITMAP;
    r->written = n_words(ds);
    r->status = MDRQ_OK;
    if (host_out) MDRQ_HIP(hipMemcpy(r->buf, out, r->written * 8, hipMemcpyDeviceToHost),
                           "copy result to host");
    return r->status;
  }
  if (plan.mode == kIds) {
    r->written = std::min(count, plan.capacity);
    r->status = count > plan.capacity ? MDRQ_EOVERFLOW : MDRQ_OK;
  } else if (plan.mode == kBitmap) {
    r->written = out_elems;
    r->status = plan.capacity < n_words(ds) ? MDRQ_EOVERFLOW : MDRQ_OK;
  } else {
    r->written = 0;
    r->status = MDRQ_OK;
  }
  if (host_out && r->written)
    MDRQ_HIP(hipMemcpy(r->buf, out, r->written * elem, hipMemcpyDeviceToHost), "copy result to host");
  return r->status;
}

int run_query(mdrq_dataset* ds, const Plan& plan, mdrq_result_t* r, hipStream_t stream) {
  if (plan.empty || ds->n_rows == 0) return finish_empty(ds, plan, r, stream);
  std::lock_guard<std::mutex> single(ds->single_mu);
  const bool host_out = r->mem == MDRQ_MEM_HOST && plan.mode != kCount;
  const uint64_t elem = plan.mode == kIds ? 4 : 8;
  const uint64_t out_elems = plan.mode == kBitmap ? std::min(plan.capacity, n_words(ds)) : plan.capacity;
  void* out = r->buf;
  if (host_out) {
    if (out_elems) {
      int rc = ensure_staging(ds, out_elems * elem);
      if (rc) return rc;
    }
    out = ds->staging;
  }
  const uint64_t tile = static_cast<uint64_t>(scan_tile_rows(scan_unroll(ds)));
  const uint32_t kmode = plan.mode == kIds ? kStage : plan.mode;
  const uint64_t n_tiles = (ds->n_rows + tile - 1) / tile;
  uint64_t grid = 0, seg = 0;
  scan_shape(ds, kmode, n_tiles, UINT64_MAX, &grid, &seg);
  if (plan.mode == kIds && grid > ds->block_sums_len) {
    if (ds->block_sums) (void)hipFree(ds->block_sums);
    ds->block_sums = nullptr;
    ds->block_sums_len = 0;
    if (hipMalloc(&ds->block_sums, grid * sizeof(uint32_t)) != hipSuccess)
      return fail(MDRQ_ENOMEM, "workgroup count buffer");
    ds->block_sums_len = grid;
  }
  const ScanWork w{ds->state, ds->stage_bitmap, ds->tile_counts, ds->block_sums};
  return scan_query(ds, plan, plan.preds.data(), static_cast<uint32_t>(plan.preds.size()), r, stream, w, out,
                    out_elems, grid, seg, host_out);
}

int run_query_on(mdrq_dataset* ds, const Plan& plan, mdrq_result_t* r, hipStream_t stream, const SingleScratch& s) {
  if (plan.empty || ds->n_rows == 0) return finish_empty(ds, plan, r, stream);
  const bool host_out = r->mem == MDRQ_MEM_HOST && plan.mode != kCount;
  const uint64_t tile = static_cast<uint64_t>(scan_tile_rows(scan_unroll(ds)));
  const uint32_t kmode = plan.mode == kIds ? kStage : plan.mode;
  const uint64_t n_tiles = (ds->n_rows + tile - 1) / tile;
  uint64_t grid = 0, seg = 0;
  scan_shape(ds, kmode, n_tiles, UINT64_MAX, &grid, &seg);
  // Host outputs need the dataset's staging; a launch wider than this scratch holds, or
  // a scratch not allocated, takes the dataset's own path.
  if (host_out || !s.state || grid > s.block_sums_len || n_tiles > s.tile_counts_len) return run_query(ds, plan, r, stream);
  const uint64_t out_elems = plan.mode == kBitmap ? std::min(plan.capacity, n_words(ds)) : plan.capacity;
  ScanWork w{s.state, s.stage_bitmap, s.tile_counts, s.block_sums};
  w.host = s.host;
  w.host_dev = s.host_dev;
  return scan_query(ds, plan, plan.preds.data(), static_cast<uint32_t>(plan.preds.size()), r, stream, w, r->buf,
                    out_elems, grid, seg, false);
}

void free_single(SingleScratch& s) {
  if (s.state) (void)hipFree(s.state);
  if (s.stage_bitmap) (void)hipFree(s.stage_bitmap);
  if (s.tile_counts) (void)hipFree(s.tile_counts);
  if (s.block_sums) (void)hipFree(s.block_sums);
  if (s.host) (void)hipHostFree(s.host);
  s = SingleScratch{};
}

int reserve_single(const mdrq_dataset* ds, SingleScratch& s) {
  free_single(s);
  const uint64_t min_tile = static_cast<uint64_t>(scan_tile_rows(1));
  const uint64_t tiles = (ds->n_rows + min_tile - 1) / min_tile + 1;
  const uint64_t words = (ds->n_rows + 63) / 64 + 1;
  // Workgroups: at most every CU's occupancy limit of the widest scan kernel.
  uint64_t grid = 1;
  for (int u : {1, 2, 4, 8, 16})
    for (uint32_t m : {static_cast<uint32_t>(kStage), static_cast<uint32_t>(kBitmap), static_cast<uint32_t>(kCount)})
      grid = std::max<uint64_t>(grid, static_cast<uint64_t>(scan_blocks_per_cu(m, u)) * device().cus);
  grid = std::max<uint64_t>(grid, ds->grid > 0 ? static_cast<uint64_t>(ds->grid) : 0);
  auto fail_free = [&](const char* what) {
    free_single(s);
    return fail(MDRQ_ENOMEM, what);
  };
  if (hipMalloc(&s.state, sizeof(ScanState)) != hipSuccess) return fail_free("worker scan state");
  if (hipMemset(s.state, 0, sizeof(ScanState)) != hipSuccess) return fail_free("worker scan state");
  if (hipMalloc(&s.stage_bitmap, words * 8) != hipSuccess) return fail_free("worker stage bitmap");
  if (hipMalloc(&s.tile_counts, tiles * 4) != hipSuccess) return fail_free("worker tile counts");
  if (hipMalloc(&s.block_sums, grid * 4) != hipSuccess) return fail_free("worker workgroup counts");
  s.tile_counts_len = tiles;
  s.block_sums_len = grid;
  if (hipHostMalloc(reinterpret_cast<void**>(&s.host), sizeof(ScanState), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&s.host_dev), s.host, 0) != hipSuccess)
    return fail_free("worker result record");
  memset(s.host, 0, sizeof(ScanState));
  return MDRQ_OK;
}

// ---------------------------------------------------------------- fixed scratch

// mdrq_query_noalloc's workspace: one array per GPU, part of the library's code object
// (so nothing is allocated at call time), kept until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host it names a host-side stand-in): it
// uses the device address that hipGetSymbolAddress returns for the current device.
constexpr uint64_t kScratchBytes = uint64_t{32} << 20;
constexpr uint64_t kScratchMaxGrid = 4096;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];   // one call at a time per GPU
unsigned char* g_scratch_ptr[kMaxDevices] = {};

struct ScratchLayout {
  uint64_t state, block_sums, tile_counts, bitmap, end;
};
ScratchLayout scratch_layout(uint64_t n_rows, uint64_t n_tiles, uint64_t grid) {
  auto up = [](uint64_t x) { return (x + 255) / 256 * 256; };
  ScratchLayout l{};
  l.state = 0;
  l.block_sums = up(sizeof(ScanState));
  l.tile_counts = l.block_sums + up(grid * 4);
  l.bitmap = l.tile_counts + up(n_tiles * 4);
  l.end = l.bitmap + ((n_rows + 63) / 64 + 1) * 8;
  return l;
}

// Device address of this GPU's scratch, looked up once per device (the current one).
int scratch_address(int dev, unsigned char** out) {
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(MDRQ_EDEVICE, "scratch has no device address");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return MDRQ_OK;
}

}  // namespace mdrq

extern "C" {

int mdrq_load_columns(const float* const* cols, uint32_t n_dims, uint64_t n_rows, uint32_t flags,
                      void* stream_, mdrq_dataset** out) {
  return guarded([&]() -> int {
    clear_error();
    if (!out) return fail(MDRQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cols) return fail(MDRQ_EINVAL, "cols is NULL");
    if (n_dims == 0 || n_dims > MDRQ_MAX_DIMS) return fail(MDRQ_EINVAL, "n_dims must be 1..128");
    if (n_rows > kMaxRows) return fail(MDRQ_EINVAL, "n_rows exceeds 2^32 - 1");
    const bool dev_in = flags & MDRQ_MEM_DEVICE;
    const bool borrow = flags & MDRQ_BORROW;
    if (flags & ~static_cast<uint32_t>(MDRQ_MEM_DEVICE | MDRQ_BORROW))
      return fail(MDRQ_EINVAL, "unknown load flags");
    if (borrow && !dev_in) return fail(MDRQ_EINVAL, "MDRQ_BORROW requires MDRQ_MEM_DEVICE");
    for (uint32_t j = 0; j < n_dims; ++j) {
      if (!cols[j] && n_rows > 0) return fail(MDRQ_EINVAL, "column pointer is NULL");
      if (borrow && (reinterpret_cast<uintptr_t>(cols[j]) & 15u))
        return fail(MDRQ_EINVAL, "borrowed column is not 16-byte aligned");
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    mdrq_dataset* ds = new mdrq_dataset();
    ds->n_rows = n_rows;
    ds->n_dims = n_dims;
    ds->owned = !borrow;
    ds->cols.resize(n_dims);
    int rc = MDRQ_OK;
    ColumnStats* st_dev = nullptr;
    ColumnStats st_host{};
    if (borrow) {
      for (uint32_t j = 0; j < n_dims; ++j) ds->cols[j] = cols[j];
    } else {
      ds->stride = (n_rows + 63) / 64 * 64;
      const uint64_t bytes = std::max<uint64_t>(1, ds->stride * n_dims * sizeof(float));
      if (hipMalloc(reinterpret_cast<void**>(&ds->base), bytes) != hipSuccess) {
        free_dataset(ds);
        return fail(MDRQ_ENOMEM, "device allocation of the columns failed");
      }
      for (uint32_t j = 0; j < n_dims; ++j) {
        float* dst = ds->base + ds->stride * j;
        ds->cols[j] = dst;
        if (n_rows) {
          hipError_t e = hipMemcpyAsync(dst, cols[j], n_rows * sizeof(float),
                                        dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                        stream);
          if (e != hipSuccess) {
            free_dataset(ds);
            return fail_hip(e, "column copy");
          }
        }
      }
    }
    rc = alloc_workspace(ds);
    if (rc) {
      free_dataset(ds);
      return rc;
    }
    // Validation on the device: NaN check, min and max per column.
    st_host.nan_count = 0;
    for (uint32_t j = 0; j < MDRQ_MAX_DIMS; ++j) {
      st_host.min_key[j] = 0xFFFFFFFFu;
      st_host.max_key[j] = 0u;
    }
    hipError_t e = hipMalloc(&st_dev, sizeof(ColumnStats));
    if (e == hipSuccess)
      e = hipMemcpyAsync(st_dev, &st_host, sizeof(ColumnStats), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && n_rows) e = launch_validate(ds->cols.data(), n_dims, n_rows, st_dev, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&st_host, st_dev, sizeof(ColumnStats), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (st_dev) (void)hipFree(st_dev);
    if (e != hipSuccess) {
      free_dataset(ds);
      return fail_hip(e, "column validation");
    }
    if (st_host.nan_count) {
      free_dataset(ds);
      return fail(MDRQ_EINVAL, "NaN in the data");
    }
    ds->col_min.resize(n_dims);
    ds->col_max.resize(n_dims);
    for (uint32_t j = 0; j < n_dims; ++j) {
      if (n_rows) {
        ds->col_min[j] = key_to_float(st_host.min_key[j]);
        ds->col_max[j] = key_to_float(st_host.max_key[j]);
      } else {
        ds->col_min[j] = std::numeric_limits<float>::infinity();
        ds->col_max[j] = -std::numeric_limits<float>::infinity();
      }
    }
    *out = ds;
    return MDRQ_OK;
  });
}

int mdrq_query(mdrq_dataset* ds, const mdrq_query_t* q, mdrq_result_t* r, void* stream) {
  return guarded([&]() -> int {
    clear_error();
    if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
    int rc = check_query(ds, q);
    if (rc) return rc;
    rc = check_result(r);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(ds->mu);
    Plan plan = make_plan(ds, q, r);
    // Estimated order: the estimator's graph ranks the predicates on the device, ahead of
    // the scan on the same stream (no host round trip); it stays locked until the scan
    // has completed.
    std::unique_lock<std::mutex> est_hold;
    if ((q->flags & MDRQ_Q_ORDER_ESTIMATED) && !plan.empty) {
      rc = order_on_device(ds, q, plan, static_cast<hipStream_t>(stream), est_hold);
      if (rc) return rc;
    }
    r->mode = plan.mode == kBitmap ? MDRQ_OUT_BITMAP : plan.mode == kCount ? MDRQ_OUT_COUNT : MDRQ_OUT_IDS;
    return run_query(ds, plan, r, static_cast<hipStream_t>(stream));
  });
}

void mdrq_free(mdrq_dataset* ds) {
  if (!ds) return;
  close_servers(ds);
  (void)hipDeviceSynchronize();
  free_dataset(ds);
}

const char* mdrq_last_error(void) { return g_err.c_str(); }

int mdrq_dataset_info(const mdrq_dataset* ds, uint64_t* n_rows, uint32_t* n_dims) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (n_rows) *n_rows = ds->n_rows;
  if (n_dims) *n_dims = ds->n_dims;
  return MDRQ_OK;
}

int mdrq_column_range(const mdrq_dataset* ds, uint32_t dim, float* min_out, float* max_out) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (dim >= ds->n_dims) return fail(MDRQ_EINVAL, "dimension out of range");
  if (min_out) *min_out = ds->col_min[dim];
  if (max_out) *max_out = ds->col_max[dim];
  return MDRQ_OK;
}

int mdrq_set_profiling(mdrq_dataset* ds, int enable) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  std::lock_guard<std::mutex> lock(ds->mu);
  // The events are created here, so that timed calls (mdrq_query_noalloc too) allocate
  // nothing.
  if (enable) {
    if (!ds->ev0) MDRQ_HIP(hipEventCreate(&ds->ev0), "hipEventCreate");
    if (!ds->ev1) MDRQ_HIP(hipEventCreate(&ds->ev1), "hipEventCreate");
    if (!ds->ev2) MDRQ_HIP(hipEventCreate(&ds->ev2), "hipEventCreate");
  }
  ds->profiling = enable != 0;
  return MDRQ_OK;
}

int mdrq_get_profile(const mdrq_dataset* ds, uint64_t* launches, double* scan_ms,
                     double* total_ms) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (launches) *launches = ds->prof_launches;
  if (scan_ms) *scan_ms = ds->prof_scan_ms;
  if (total_ms) *total_ms = ds->prof_total_ms;
  return MDRQ_OK;
}

int mdrq_reset_profile(mdrq_dataset* ds) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  std::lock_guard<std::mutex> lock(ds->mu);
  ds->prof_launches = 0;
  ds->prof_scan_ms = 0.0;
  ds->prof_total_ms = 0.0;
  ds->batch_launches = 0;
  ds->batch_ms = 0.0;
  ds->sized_queries = 0;
  ds->sized_reruns = 0;
  ds->batch_lookups = 0;
  ds->batch_column_bytes = 0;
  ds->batch_scan_ms = 0.0;
  return MDRQ_OK;
}

int mdrq_set_option(mdrq_dataset* ds, uint32_t option, int64_t value) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  std::lock_guard<std::mutex> lock(ds->mu);
  switch (option) {
    case MDRQ_OPT_RESERVE_FACTOR:
      if (value < 1 || value > 1000000000) return fail(MDRQ_EINVAL, "reserve factor must be 1..10^9 millionths");
      ds->reserve_ppm = value;
      return MDRQ_OK;
    case MDRQ_OPT_CIRCULAR:
      if (value < 0 || value > 7) return fail(MDRQ_EINVAL, "circular mode must be 0..7");
      ds->circular_mode = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_GRAPHS:
      if (value < 0 || value > 3) return fail(MDRQ_EINVAL, "graphs must be 0..3");
      ds->graph_single = (value & 1) != 0;
      ds->graph_batch = (value & 2) != 0;
      return MDRQ_OK;
    case MDRQ_OPT_UNROLL:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
        return fail(MDRQ_EINVAL, "unroll must be 0, 1, 2, 4, 8 or 16");
      ds->unroll = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_BATCH_WAVES:
      if (value != 0 && value != 4 && value != 8) return fail(MDRQ_EINVAL, "batch waves must be 0, 4 or 8");
      ds->batch_waves = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_BATCH_GROUP:
      if (value < 0 || value > MDRQ_MAX_BATCH) return fail(MDRQ_EINVAL, "batch group out of range");
      ds->batch_group = static_cast<uint32_t>(value);
      return MDRQ_OK;
    case MDRQ_OPT_BATCH_ROWS:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
        return fail(MDRQ_EINVAL, "batch rows per lane must be 0, 1, 2, 4, 8 or 16");
      ds->batch_rows = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_BATCH_VARIANT:
      if (value < 0 || value > 5) return fail(MDRQ_EINVAL, "batch variant must be 0 .. 5");
      ds->batch_variant = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_RANK_BUCKETS:
      if (value < 0 || value > 2) return fail(MDRQ_EINVAL, "rank buckets must be 0, 1 or 2");
      ds->rank_buckets = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_AUTOTUNE:
      ds->autotune = value != 0;
      if (!ds->autotune) ds->tuned.clear();
      return MDRQ_OK;
    case MDRQ_OPT_BLOCKS_PER_CU:
      if (value < 1 || value > 8) return fail(MDRQ_EINVAL, "blocks per CU must be 1..8");
      ds->blocks_per_cu = static_cast<int>(value);
      return MDRQ_OK;
    case MDRQ_OPT_GRID:
      if (value < 0 || value > (int64_t{1} << 20)) return fail(MDRQ_EINVAL, "grid out of range");
      ds->grid = value;
      return MDRQ_OK;
    default:
      return fail(MDRQ_EINVAL, "unknown option");
  }
}

int mdrq_get_option(const mdrq_dataset* ds, uint32_t option, int64_t* value) {
  clear_error();
  if (!ds || !value) return fail(MDRQ_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(const_cast<mdrq_dataset*>(ds)->mu);
  switch (option) {
    case MDRQ_OPT_UNROLL: *value = scan_unroll(ds); return MDRQ_OK;
    case MDRQ_OPT_GRID: *value = static_cast<int64_t>(ds->grid); return MDRQ_OK;
    case MDRQ_OPT_BLOCKS_PER_CU: *value = ds->blocks_per_cu; return MDRQ_OK;
    case MDRQ_OPT_BATCH_WAVES: *value = ds->batch_waves; return MDRQ_OK;
    case MDRQ_OPT_BATCH_GROUP: *value = ds->batch_group; return MDRQ_OK;
    case MDRQ_OPT_AUTOTUNE: *value = ds->autotune ? 1 : 0; return MDRQ_OK;
    case MDRQ_OPT_BATCH_ROWS: *value = ds->batch_rows; return MDRQ_OK;
    case MDRQ_OPT_BATCH_VARIANT: *value = ds->batch_variant; return MDRQ_OK;
    case MDRQ_OPT_RANK_BUCKETS: *value = ds->rank_buckets; return MDRQ_OK;
    case MDRQ_OPT_GRAPHS: *value = (ds->graph_single ? 1 : 0) | (ds->graph_batch ? 2 : 0); return MDRQ_OK;
    case MDRQ_OPT_RESERVE_FACTOR: *value = static_cast<int64_t>(ds->reserve_ppm); return MDRQ_OK;
    case MDRQ_OPT_CIRCULAR: *value = ds->circular_mode; return MDRQ_OK;
    default:
      return fail(MDRQ_EINVAL, "unknown option");
  }
}

int mdrq_probe_bandwidth(mdrq_dataset* ds, const uint32_t* dims, uint32_t k, uint32_t iters,
                         void* stream_, double* ms) {
  clear_error();
  if (!ds || !dims || !ms) return fail(MDRQ_EINVAL, "NULL argument");
  if (k == 0 || k > ds->n_dims) return fail(MDRQ_EINVAL, "k must be 1..n_dims");
  if (iters == 0) iters = 1;
  std::lock_guard<std::mutex> lock(ds->mu);
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  ProbeParams p{};
  p.n_rows = ds->n_rows;
  p.n_cols = k;
  for (uint32_t i = 0; i < k; ++i) {
    if (dims[i] >= ds->n_dims) return fail(MDRQ_EINVAL, "dimension out of range");
    p.cols[i] = ds->cols[dims[i]];
  }
  p.sink = reinterpret_cast<uint32_t*>(ds->state) + offsetof(ScanState, kind) / 4;  // a sink no query reads before writing
  const Device& dev = device();
  const int grid = static_cast<int>(static_cast<uint64_t>(scan_blocks_per_cu(kCount, scan_unroll(ds))) * dev.cus);
  hipEvent_t e0, e1;
  MDRQ_HIP(hipEventCreate(&e0), "hipEventCreate");
  MDRQ_HIP(hipEventCreate(&e1), "hipEventCreate");
  hipError_t e = launch_probe(p, scan_unroll(ds), grid, stream);  // warm-up pass
  if (e == hipSuccess) e = hipEventRecord(e0, stream);
  for (uint32_t i = 0; e == hipSuccess && i < iters; ++i) e = launch_probe(p, scan_unroll(ds), grid, stream);
  if (e == hipSuccess) e = hipEventRecord(e1, stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail_hip(e, "bandwidth probe");
  *ms = static_cast<double>(t) / iters;
  return MDRQ_OK;
}

int mdrq_query_read_bytes(mdrq_dataset* ds, const mdrq_query_t* q, uint64_t* bytes, void* stream_) {
  return guarded([&]() -> int {
    clear_error();
    if (!ds || !bytes) return fail(MDRQ_EINVAL, "NULL argument");
    int rc = check_query(ds, q);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(ds->mu);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const mdrq_result_t count_only{MDRQ_OUT_COUNT, MDRQ_MEM_HOST, nullptr, 0, 0, 0, 0, 0};
    Plan plan = make_plan(ds, q, &count_only);
    *bytes = 0;
    if (plan.empty || ds->n_rows == 0 || plan.preds.empty()) return MDRQ_OK;
    std::unique_lock<std::mutex> est_hold;
    if (q->flags & MDRQ_Q_ORDER_ESTIMATED) {
      rc = order_on_device(ds, q, plan, stream, est_hold);
      if (rc) return rc;
    }
    std::lock_guard<std::mutex> single(ds->single_mu);
    LinesParams p{};
    p.n_rows = ds->n_rows;
    p.n_preds = static_cast<uint32_t>(plan.preds.size());
    p.early_out = plan.early_out ? 1u : 0u;
    p.order = plan.order;
    for (size_t i = 0; i < plan.preds.size(); ++i) p.preds[i] = plan.preds[i];
    // The running sum lives in the dataset's scan state word, which is zero between
    // scans and is set back to zero here.
    p.lines = reinterpret_cast<unsigned long long*>(&ds->state->total);
    const int grid = static_cast<int>(std::min<uint64_t>((ds->n_rows + kBlock - 1) / kBlock,
                                                         static_cast<uint64_t>(device().cus) * 8));
    unsigned long long lines = 0;
    hipError_t e = launch_lines(p, grid, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&lines, p.lines, sizeof lines, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemsetAsync(p.lines, 0, sizeof lines, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      recover_state(ds->state);
      return fail_hip(e, "read-bytes measurement");
    }
    *bytes = static_cast<uint64_t>(lines) * 128;
    return MDRQ_OK;
  });
}

const char* mdrq_version(void) { return "0.1.0"; }

int mdrq_query_noalloc(mdrq_dataset* ds, const mdrq_query_t* q, mdrq_result_t* r, void* stream_) {
  return guarded([&]() -> int {
    clear_error();
    if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
    int rc = check_query(ds, q);
    if (rc) return rc;
    rc = check_result(r);
    if (rc) return rc;
    if (q->flags & MDRQ_Q_ORDER_ESTIMATED)
      return fail(MDRQ_ENOTSUP, "mdrq_query_noalloc evaluates predicates in the order given");
    if (r->mem == MDRQ_MEM_HOST && r->mode != MDRQ_OUT_COUNT)
      return fail(MDRQ_EINVAL, "mdrq_query_noalloc writes results to device memory only");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MDRQ_ENOTSUP, "device index beyond the scratch table");
    // No heap use from here on: the plan is built in the launch parameters directly.
    std::lock_guard<std::mutex> lock(ds->mu);
    std::lock_guard<std::mutex> single(ds->single_mu);
    std::lock_guard<std::mutex> gpu(g_scratch_mu[dev]);
    unsigned char* base = nullptr;
    rc = scratch_address(dev, &base);
    if (rc) return rc;
    Plan plan;  // empty vectors: no allocation
    const float inf = std::numeric_limits<float>::infinity();
    plan.mode = r->mode == MDRQ_OUT_BITMAP ? kBitmap : r->mode == MDRQ_OUT_COUNT ? kCount : kIds;
    plan.auto_mode = r->mode == MDRQ_OUT_AUTO;
    plan.capacity = plan.mode == kIds ? r->buf_bytes / 4 : plan.mode == kBitmap ? r->buf_bytes / 8 : 0;
    plan.early_out = !(q->flags & MDRQ_Q_NO_EARLYOUT);
    r->mode = plan.mode == kBitmap ? MDRQ_OUT_BITMAP : plan.mode == kCount ? MDRQ_OUT_COUNT : MDRQ_OUT_IDS;
    for (uint32_t i = 0; i < q->n_preds; ++i) plan.empty |= q->preds[i].lo > q->preds[i].hi;
    if (plan.empty || ds->n_rows == 0) {
      r->count = 0;
      r->written = 0;
      r->status = MDRQ_OK;
      if (plan.mode == kBitmap) {
        const uint64_t words = std::min(plan.capacity, n_words(ds));
        if (words) {
          e = launch_zero_words(static_cast<uint64_t*>(r->buf), words, stream);
          if (e == hipSuccess) e = hipStreamSynchronize(stream);
          if (e != hipSuccess) return fail_hip(e, "clearing the bitmap");
        }
        r->written = words;
        if (plan.capacity < n_words(ds)) r->status = MDRQ_EOVERFLOW;
      }
      return r->status;
    }
    const uint64_t tile = static_cast<uint64_t>(scan_tile_rows(scan_unroll(ds)));
    const uint32_t kmode = plan.mode == kIds ? kStage : plan.mode;
    const uint64_t n_tiles = (ds->n_rows + tile - 1) / tile;
    uint64_t grid = 0, seg = 0;
    scan_shape(ds, kmode, n_tiles, kScratchMaxGrid, &grid, &seg);
    const ScratchLayout L = scratch_layout(ds->n_rows, n_tiles, grid);
    if (L.end > kScratchBytes)
      return fail(MDRQ_ENOTSUP, "dataset too large for mdrq_query_noalloc's fixed 32 MiB scratch "
                                "(bitmap of n_rows / 8 bytes plus tile counts; about 2.6e8 rows at "
                                "the default tile height)");
    // The scan state must start at zero; the last call may have been cut short.
    ScanWork w{reinterpret_cast<ScanState*>(base + L.state), reinterpret_cast<uint64_t*>(base + L.bitmap),
               reinterpret_cast<uint32_t*>(base + L.tile_counts), reinterpret_cast<uint32_t*>(base + L.block_sums)};
    e = launch_zero_words(reinterpret_cast<uint64_t*>(w.state), sizeof(ScanState) / 8, stream);
    if (e != hipSuccess) return fail_hip(e, "clearing the scan state");
    // Predicates that can change the result, in the order given.
    DevPred preds[MDRQ_MAX_DIMS];
    uint32_t k = 0;
    for (uint32_t i = 0; i < q->n_preds; ++i) {
      const mdrq_pred& pr = q->preds[i];
      if (pr.lo == -inf && pr.hi == inf) continue;
      preds[k++] = DevPred{ds->cols[pr.dim], pr.lo, pr.hi};
    }
    const uint64_t out_elems = plan.mode == kBitmap ? std::min(plan.capacity, n_words(ds)) : plan.capacity;
    return scan_query(ds, plan, preds, k, r, stream, w, r->buf, out_elems, grid, seg, false);
  });
}

int mdrq_query_batch(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n_queries,
                     mdrq_result_t* rs, void* stream) {
  return guarded([&]() -> int {
    clear_error();
    if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
    if (!qs || !rs) return fail(MDRQ_EINVAL, "queries or results is NULL");
    if (n_queries == 0 || n_queries > MDRQ_MAX_BATCH)
      return fail(MDRQ_EINVAL, "n_queries must be 1..MDRQ_MAX_BATCH");
    for (uint32_t i = 0; i < n_queries; ++i) {
      int rc = check_query(ds, &qs[i]);
      if (!rc) rc = check_result(&rs[i]);
      if (rc) return fail(rc, "query " + std::to_string(i) + ": " + mdrq_last_error());
    }
    std::lock_guard<std::mutex> lock(ds->mu);
    int rc = run_batch(ds, qs, n_queries, rs, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    for (uint32_t i = 0; i < n_queries; ++i)
      if (rs[i].status == MDRQ_EOVERFLOW) return MDRQ_EOVERFLOW;
    return MDRQ_OK;
  });
}

int mdrq_get_batch_profile(const mdrq_dataset* ds, uint64_t* scans, double* ms) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (scans) *scans = ds->batch_launches;
  if (ms) *ms = ds->batch_ms;
  return MDRQ_OK;
}

int mdrq_get_batch_work(const mdrq_dataset* ds, uint64_t* lookups, uint64_t* column_bytes, double* scan_ms) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (lookups) *lookups = ds->batch_lookups;
  if (column_bytes) *column_bytes = ds->batch_column_bytes;
  if (scan_ms) *scan_ms = ds->batch_scan_ms;
  return MDRQ_OK;
}

int mdrq_get_sizing_profile(const mdrq_dataset* ds, uint64_t* sized, uint64_t* reruns) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (sized) *sized = ds->sized_queries;
  if (reruns) *reruns = ds->sized_reruns;
  return MDRQ_OK;
}


}  // extern "C"
