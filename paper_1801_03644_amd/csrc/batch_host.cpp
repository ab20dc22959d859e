// Host side of the batched shared scan: query validation and canonicalisation,
// grouping of queries into shared scans, the query table, the launch configuration
// autotuner, and completion.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <system_error>
#include <thread>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>

#include "mdrq_internal.h"
#include "rank_buckets.h"

namespace mdrq {
namespace {

#define MDRQ_HIP(call, what)                         \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return fail_hip(e_, what); \
  } while (0)

constexpr uint64_t kTileRows = 4096;
constexpr uint64_t kMaxLdsTable = 60 * 1024;   // bytes of query table per workgroup
constexpr uint64_t kMaxRegGroup = 4096;         // queries per workgroup, slot-mask variant
constexpr uint64_t kRankLdsWords = 72 * 256;    // group tables up to which it is tried

template <typename T>
int grow_device(T** p, uint64_t* have, uint64_t need, const char* what) {
  if (need <= *have) return MDRQ_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipMalloc(reinterpret_cast<void**>(p), need * sizeof(T)) != hipSuccess)
    return fail(MDRQ_ENOMEM, std::string("device allocation failed: ") + what);
  *have = need;
  return MDRQ_OK;
}

int grow_pinned(void** p, uint64_t* have, uint64_t need) {
  if (need <= *have) return MDRQ_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipHostMalloc(p, need, hipHostMallocDefault) != hipSuccess)
    return fail(MDRQ_ENOMEM, "pinned host allocation failed");
  *have = need;
  return MDRQ_OK;
}

// Per-query counts (u64), kinds (u32) and sparse-scratch overflow marks (u32) of a
// batch, in mapped pinned memory that the finish kernel writes directly (no copy back).
int grow_results(BatchWorkspace& ws, uint64_t nq) {
  if (nq <= ws.res_len) return MDRQ_OK;
  if (ws.h_res) (void)hipHostFree(ws.h_res);
  ws.h_res = ws.h_res_dev = nullptr;
  ws.res_len = 0;
  if (hipHostMalloc(&ws.h_res, nq * 16, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(&ws.h_res_dev, ws.h_res, 0) != hipSuccess)
    return fail(MDRQ_ENOMEM, "batch result buffers");
  ws.res_len = nq;
  return MDRQ_OK;
}

// One query of a shared scan.
struct Item {
  uint32_t index;         // position in the caller's arrays
  Plan plan;
  uint32_t kind;          // BatchKind
  mdrq_result_t* r;
  std::vector<float> sel; // estimated selectivity of each plan predicate alone
  double est_rows = -1.0; // MDRQ_Q_SIZE_ESTIMATED: estimated result rows (< 0: none)
};

// Rows per chunk of the rank variant when some query's scratch is sized by estimate.
constexpr uint64_t kSparseChunkRows = 512;

uint32_t kind_of(uint32_t mode) {
  switch (mode) {
    case MDRQ_OUT_COUNT: return kBatchCount;
    case MDRQ_OUT_BITMAP: return kBatchBitmap;
    case MDRQ_OUT_AUTO: return kBatchAuto;
    default: return kBatchIds;
  }
}

// Autotuner key of a batch shape: log2 rows, union columns, log2 queries, and whether
// any query writes ids or a bitmap (storing output words changes which launch shape is
// fastest: a count-only batch does not predict an output batch's choice).
uint64_t shape_key(uint64_t n_rows, size_t n_slots, size_t n_queries, bool writes) {
  const uint64_t lr = n_rows ? 64 - __builtin_clzll(n_rows) : 0;
  const uint64_t lq = n_queries ? 64 - __builtin_clzll(n_queries) : 0;
  return (static_cast<uint64_t>(writes) << 24) | (lr << 16) | (static_cast<uint64_t>(n_slots) << 8) | lq;
}


void destroy_graph(BatchWorkspace::Graph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = BatchWorkspace::Graph{};
}

// Queue one shared scan by replaying the workspace's graph for its scan kernel (built on
// first use): the query-table copy, the zeroing, the scan and the finish, with the
// workspace's events after the copy, after the scan and at the end, every node updated
// with this batch's arguments, grid and buffers.
hipError_t launch_shared_graph(BatchWorkspace& ws, const BatchParams& bp, const BatchFinish& fin, uint32_t nq,
                               int n_slots, int waves, int rg, int variant, dim3 grid, size_t lds, int sw,
                               uint64_t blob, hipStream_t stream) {
  BatchLaunches L;
  hipError_t e = batch_launches(bp, fin, nq, n_slots, waves, rg, variant, grid, lds, sw, &L);
  if (e != hipSuccess) return e;
  BatchWorkspace::Graph* g = nullptr;
  for (BatchWorkspace::Graph& c : ws.graphs)
    if (c.scan_fn == L.scan.func) g = &c;
  if (g) {
    e = hipGraphExecMemcpyNodeSetParams1D(g->exec, g->copy, ws.d_blob, ws.h_blob, blob, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(g->exec, g->zero, &L.zero);
    if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(g->exec, g->scan, &L.scan);
    if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(g->exec, g->chunk, &L.chunk);
    if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(g->exec, g->count, &L.count);
    if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(g->exec, g->emit, &L.emit);
    if (e == hipSuccess) return hipGraphLaunch(g->exec, stream);
    // An update the instantiated graph does not take: build it anew below.
    destroy_graph(*g);
    ws.graphs.erase(ws.graphs.begin() + (g - ws.graphs.data()));
  }
  if (ws.graphs.size() >= 8) {
    destroy_graph(ws.graphs.front());
    ws.graphs.erase(ws.graphs.begin());
  }
  BatchWorkspace::Graph n;
  n.scan_fn = L.scan.func;
  hipGraphNode_t prev = nullptr, ev = nullptr;
  e = hipGraphCreate(&n.graph, 0);
  if (e == hipSuccess)
    e = hipGraphAddMemcpyNode1D(&n.copy, n.graph, nullptr, 0, ws.d_blob, ws.h_blob, blob, hipMemcpyHostToDevice);
  prev = n.copy;
  if (e == hipSuccess) e = hipGraphAddEventRecordNode(&ev, n.graph, &prev, 1, ws.ev0);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n.zero, n.graph, &ev, 1, &L.zero);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n.scan, n.graph, &n.zero, 1, &L.scan);
  if (e == hipSuccess) e = hipGraphAddEventRecordNode(&ev, n.graph, &n.scan, 1, ws.ev2);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n.chunk, n.graph, &ev, 1, &L.chunk);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n.count, n.graph, &n.chunk, 1, &L.count);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&n.emit, n.graph, &n.count, 1, &L.emit);
  if (e == hipSuccess) e = hipGraphAddEventRecordNode(&ev, n.graph, &n.emit, 1, ws.ev1);
  if (e == hipSuccess) e = hipGraphInstantiate(&n.exec, n.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    destroy_graph(n);
    return e;
  }
  ws.graphs.push_back(n);
  return hipGraphLaunch(ws.graphs.back().exec, stream);
}

// Run one shared scan over `items` (union of at most kMaxUnion columns; unions of more
// than kMaxSlots columns take the LDS variant).
// ms_out receives the device time of the scan and finish launches.
// Union of the items' queried columns in register-slot order: numbered by the columns'
// mean relative position in the queries' evaluation orders (given or estimated), so that
// a walk over the slots in order follows those orders as closely as one order can.
std::vector<uint32_t> union_columns(const mdrq_dataset* ds, const std::vector<Item>& items) {
  std::vector<uint32_t> slot_dim;
  std::vector<bool> seen(ds->n_dims, false);
  std::vector<double> pos_sum(ds->n_dims, 0.0);
  std::vector<uint32_t> uses(ds->n_dims, 0);
  for (const Item& it : items) {
    const size_t k = it.plan.dims.size();
    for (size_t i = 0; i < k; ++i) {
      const uint32_t d = it.plan.dims[i];
      pos_sum[d] += (i + 0.5) / static_cast<double>(k);
      uses[d] += 1;
      if (!seen[d]) {
        seen[d] = true;
        slot_dim.push_back(d);
      }
    }
  }
  std::stable_sort(slot_dim.begin(), slot_dim.end(), [&](uint32_t a, uint32_t b) {
    return pos_sum[a] / uses[a] < pos_sum[b] / uses[b];
  });
  return slot_dim;
}

// LDS words that bound the rank tables of a group of S queries over n_slots columns:
// its per-query counts and headers (4-word aligned), 4 header words per slot and each
// slot's tables.  Tables with up to kRankBuckets buckets are only built when the whole
// group stays within kRankLdsWords, else at most 256 buckets, whose size
// slot_table_words_bound caps for any 2 S interval ends.
uint64_t rank_group_words(uint64_t S, int n_slots) {
  const uint32_t sw = S <= 32 ? 1 : S <= 64 ? 2 : 4;
  const uint64_t bound = 2 * align4(S) + 4 * static_cast<uint64_t>(n_slots) +
                         static_cast<uint64_t>(n_slots) *
                             slot_table_words_bound(static_cast<uint32_t>(2 * S), 256, sw);
  return std::max<uint64_t>(bound, kRankLdsWords);
}

// Dynamic LDS a rank group may use (the rest is the kernel's own).
size_t rank_lds_room() { return device().lds > 4096 ? device().lds - 4096 : 0; }

// Rank-variant tables of the items, in groups of rank_group consecutive queries: per
// group, per query (kind | sparse << 2 | output row << 8), per slot a header (offset of
// the ends; M | d << 12 | log2(nb) << 16 | shift << 24 | by value << 31; kmin or vlo;
// scale), then per slot the tables of append_slot_tables (offsets relative to the
// group's start, 4-word aligned).  The bucket words hold the range of each bucket's
// ends, and no bucket holds more than 2^d - 1 ends (M <= 2 x 128 fits the header's 12
// bits and the bucket words' 16).  Appends to table, group_first and group_table;
// pairs_out: the (group, column) pairs with a predicate.
// The groups' tables are independent: each is built into its own vector, on several
// host threads when there are 24 or more slot tables (about 10 us each), then appended
// in group order.
// Host threads that build rank tables: started on first use and kept until the process
// ends (starting threads for every batch cost a few hundred microseconds).  One caller
// at a time uses them, a concurrent caller builds alone; the calling thread always takes
// part, so work finishes even where no helper thread could be started.
class TablePool {
 public:
  static TablePool& get() {
    static TablePool pool;
    return pool;
  }
  // f(i) for every i in [0, n); false if a call threw (the calls after it are skipped).
  bool run(size_t n, const std::function<void(size_t)>& f) {
    std::unique_lock<std::mutex> use(use_mu_, std::try_to_lock);
    if (!use.owns_lock() || helpers_.empty() || n < 2) {
      try {
        for (size_t i = 0; i < n; ++i) f(i);
      } catch (...) {
        return false;
      }
      return true;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      f_ = &f;
      n_ = n;
      next_ = 0;
      failed_ = false;
      busy_ = helpers_.size();
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return busy_ == 0; });
    f_ = nullptr;
    return !failed_;
  }

 private:
  TablePool() {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned n = std::min(15u, hw - 1);
    for (unsigned t = 0; t < n; ++t) {
      try {
        helpers_.emplace_back([this] { loop(); });
      } catch (...) {
        break;
      }
    }
  }
  ~TablePool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (std::thread& t : helpers_) t.join();
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      lk.unlock();
      work();
      lk.lock();
      if (--busy_ == 0) done_cv_.notify_all();
    }
  }
  void work() {
    try {
      for (size_t i = next_++; i < n_ && !failed_; i = next_++) (*f_)(i);
    } catch (...) {
      failed_ = true;
    }
  }
  std::mutex use_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  std::vector<std::thread> helpers_;
  const std::function<void(size_t)>* f_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0};
  std::atomic<bool> failed_{false};
  size_t busy_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

int build_rank_tables(const mdrq_dataset* ds, const std::vector<Item>& items, const std::vector<BatchOut>& outs,
                      const std::vector<int>& slot_of, int n_slots, uint64_t rank_group, int rank_sw,
                      std::vector<uint32_t>& table, std::vector<uint32_t>& group_first,
                      std::vector<uint32_t>& group_table, uint64_t* pairs_out) {
  const uint64_t nq = items.size();
  std::vector<uint64_t> rank_q0;
  for (uint64_t q0 = 0; q0 < nq; q0 += rank_group) rank_q0.push_back(q0);
  std::vector<std::vector<uint32_t>> rank_tables(rank_q0.size());
  std::atomic<uint64_t> used_pairs{0};   // (group, column) pairs with a predicate
  auto build_rank_group = [&](size_t gi) {
    const uint64_t q0 = rank_q0[gi];
    const uint64_t q1 = std::min<uint64_t>(nq, q0 + rank_group);
    const uint32_t gq = static_cast<uint32_t>(q1 - q0);
    std::vector<uint32_t>& table = rank_tables[gi];
    const uint32_t hq = static_cast<uint32_t>(align4(gq));  // headers, 16-byte aligned
    table.assign(hq + 4 * static_cast<uint64_t>(n_slots), 0u);
    for (uint64_t q = q0; q < q1; ++q)
      table[q - q0] = outs[q].kind | (outs[q].out_index << 8) | (outs[q].sparse ? 4u : 0u);
    // Per slot and query: (key(lo), key(hi)) of its predicate, if any; a query without
    // predicates carries the always-true [key(-inf), key(+inf)] on slot 0.
    std::vector<std::vector<KeyInterval>> iv(n_slots, std::vector<KeyInterval>(gq));
    for (uint64_t q = q0; q < q1; ++q) {
      const Plan& pl = items[q].plan;
      for (size_t i = 0; i < pl.preds.size(); ++i)
        iv[slot_of[pl.dims[i]]][q - q0] = rank_interval(pl.preds[i].lo, pl.preds[i].hi);
      if (pl.preds.empty())
        iv[0][q - q0] = rank_interval(-std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity());
    }
    // Per slot the sorted distinct interval ends and their buckets: up to kRankBuckets
    // buckets where the group's tables then stay within kRankLdsWords (two workgroups
    // of 8 waves per CU, the most the kernel's registers allow), else up to 256.
    std::vector<std::vector<uint32_t>> ends_of(n_slots);
    std::vector<RankBuckets> buckets_of(n_slots);
    for (int sl = 0; sl < n_slots; ++sl) {
      std::vector<uint32_t>& ends = ends_of[sl];
      ends.reserve(2 * static_cast<size_t>(gq));
      for (const KeyInterval& k : iv[sl])
        if (k.has) {
          ends.push_back(k.klo);
          ends.push_back(k.khi + 1);  // keys of non-NaN floats stay below 0xFFFFFFFF
        }
      std::sort(ends.begin(), ends.end());
      ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
    }
    // A slot's candidate maps for a lower bucket limit are the same list when no
    // candidate had more buckets than that limit (few ends: the walk starts at about 4
    // buckets per end), so they are found again only where one had.
    std::vector<std::vector<RankBuckets>> cands(n_slots);
    auto choose = [&](uint32_t max_nb) {
      uint64_t words = hq + 4 * static_cast<uint64_t>(n_slots);
      for (int sl = 0; sl < n_slots; ++sl) {
        const uint32_t M = static_cast<uint32_t>(ends_of[sl].size());
        if (M == 0) continue;
        bool again = cands[sl].empty();
        for (const RankBuckets& m : cands[sl]) again |= m.nb > max_nb;
        if (again) cands[sl] = bucket_candidates(ends_of[sl], ds->rank_buckets, max_nb);
        buckets_of[sl] = pick_buckets(cands[sl], max_nb);
        words += slot_table_words(M, buckets_of[sl], rank_sw);
      }
      return words;
    };
    if (choose(kRankBuckets) + hq > kRankLdsWords) choose(256);
    {
      uint64_t words = table.size();
      for (int sl = 0; sl < n_slots; ++sl)
        if (!ends_of[sl].empty())
          words += slot_table_words(static_cast<uint32_t>(ends_of[sl].size()), buckets_of[sl], rank_sw) + 4;
      table.reserve(words);
    }
    uint64_t used = 0;
    for (int sl = 0; sl < n_slots; ++sl) used += ends_of[sl].empty() ? 0 : 1;
    used_pairs += used;
    for (int sl = 0; sl < n_slots; ++sl) {
      const std::vector<uint32_t>& ends = ends_of[sl];
      const uint32_t M = static_cast<uint32_t>(ends.size());
      if (M == 0) continue;  // header all zero
      RankBuckets& rb = buckets_of[sl];
      fill_starts(ends, rb);
      const uint32_t at = append_slot_tables(table, ends, rb, iv[sl], rank_sw);
      uint32_t vlo_bits, scale_bits;
      std::memcpy(&vlo_bits, &rb.vlo, 4);
      std::memcpy(&scale_bits, &rb.scale, 4);
      table[hq + 4 * sl] = at;
      table[hq + 4 * sl + 1] = M | (rb.d << 12) | (static_cast<uint32_t>(__builtin_ctz(rb.nb)) << 16) |
                               (rb.shift << 24) | (rb.by_value ? 0x80000000u : 0u);
      table[hq + 4 * sl + 2] = rb.by_value ? vlo_bits : ends[0];
      table[hq + 4 * sl + 3] = rb.by_value ? scale_bits : 0u;
    }
  };
  const size_t slot_tables = rank_q0.size() * static_cast<size_t>(n_slots);
  bool built = true;
  if (slot_tables >= 24) {
    built = TablePool::get().run(rank_q0.size(), build_rank_group);
  } else {
    try {
      for (size_t gi = 0; gi < rank_q0.size(); ++gi) build_rank_group(gi);
    } catch (...) {
      built = false;
    }
  }
  if (!built) return fail(MDRQ_ENOMEM, "shared scan: host memory for the rank tables");
  if (pairs_out) *pairs_out = used_pairs.load();
  size_t total = table.size();
  for (const std::vector<uint32_t>& t : rank_tables) total += t.size();
  table.reserve(total);
  for (size_t gi = 0; gi < rank_q0.size(); ++gi) {
    group_first.push_back(static_cast<uint32_t>(rank_q0[gi]));
    group_table.push_back(static_cast<uint32_t>(table.size()));
    table.insert(table.end(), rank_tables[gi].begin(), rank_tables[gi].end());
  }
  return MDRQ_OK;
}

int run_shared(mdrq_dataset* ds, BatchWorkspace& ws, std::vector<Item>& items,
               const BatchConfig& cfg_in, hipStream_t stream, float* ms_out, BatchRunStats* st = nullptr,
               std::vector<uint32_t>* redo = nullptr) {
  const uint64_t nq = items.size();
  // Scratch sized by estimate: pool slots per query (0: a full bitmap row).  Any such
  // query makes the scan a rank-variant scan of 512-row chunks, the layout the serving
  // loop's admission reserves for.
  std::vector<uint64_t> cap_of(nq, 0);
  bool any_sparse = false;
  for (uint64_t q = 0; q < nq; ++q)
    if (items[q].kind != kBatchCount && items[q].est_rows >= 0.0) {
      cap_of[q] = sparse_slots(ds, items[q].est_rows, kSparseChunkRows);
      any_sparse |= cap_of[q] > 0;
    }
  BatchConfig cfg = cfg_in;
  if (any_sparse) {
    cfg.lds = 4;
    cfg.rows_per_lane = 8;
  }
  const uint64_t n_rows = ds->n_rows;
  const uint64_t nw = n_words(ds);
  const uint64_t n_tiles = (n_rows + kTileRows - 1) / kTileRows;

  std::vector<uint32_t> slot_dim = union_columns(ds, items);
  // The slot-mask, rank and LDS variants give a query without predicates an always-true
  // one on slot 0 (it rejects only the rows past the end), so the union has at least one
  // column.
  if ((cfg.lds == 1 || cfg.lds == 3 || cfg.lds == 4) && slot_dim.empty()) slot_dim.push_back(0);
  std::vector<int> slot_of(ds->n_dims, -1);
  for (size_t i = 0; i < slot_dim.size(); ++i) slot_of[slot_dim[i]] = static_cast<int>(i);
  const int n_slots = static_cast<int>(slot_dim.size());

  // Rank variant: queries per group (32 x sw) such that the tables of any group fit LDS.
  const size_t lds_room = rank_lds_room();
  auto rank_words = [&](uint64_t S) { return rank_group_words(S, n_slots); };
  uint64_t rank_group = std::min<uint64_t>(128, cfg.group ? cfg.group : nq);
  while (rank_group > 32 && rank_words(rank_group) * 4 > lds_room) rank_group /= 2;
  const bool rank = cfg.lds == 4 && rank_words(rank_group) * 4 <= lds_room;
  const int rank_sw = rank_group <= 32 ? 1 : rank_group <= 64 ? 2 : 4;
  const bool use_lds = !rank && (cfg.lds == 1 || n_slots > kMaxSlots);
  const bool walk = cfg.lds == 2 && !use_lds;
  const bool reg = cfg.lds == 3 && !use_lds;
  int variant = rank ? 4 : use_lds ? 1 : walk ? 2 : reg ? 3 : 0;
  // Queries per group: what the configuration asks for, and no more than fits LDS.
  uint64_t group = cfg.group ? cfg.group : nq;
  std::vector<uint32_t> group_first, group_table, table;
  std::vector<BatchOut> outs(nq);
  uint32_t n_out = 0, n_sparse = 0;
  if (rank && any_sparse) variant = 5;   // the rank kernel with sparse scratch (512-row chunks)
  std::vector<uint32_t> sparse_base, sparse_cap;
  uint64_t pool_slots = 0;
  for (uint64_t q = 0; q < nq; ++q) {
    outs[q].kind = items[q].kind;
    outs[q].sparse = 0;
    if (items[q].kind == kBatchCount) {
      outs[q].out_index = 0;
    } else if (rank && cap_of[q] > 0) {
      outs[q].sparse = 1;
      outs[q].out_index = n_sparse++;
      sparse_base.push_back(static_cast<uint32_t>(pool_slots));
      sparse_cap.push_back(static_cast<uint32_t>(cap_of[q]));
      pool_slots += cap_of[q];
    } else {
      outs[q].out_index = n_out++;
    }
  }
  // Slot-mask variant: fixed-size records (header, slot mask, then key(lo), key(hi)
  // for every register slot), read by scalar loads, so a group is not limited by LDS.
  const uint32_t reg_slots = static_cast<uint32_t>(batch_reg_slots(std::max(1, n_slots)));
  for (uint64_t q0 = 0; reg && q0 < nq;) {
    const uint64_t q1 = std::min<uint64_t>(nq, q0 + std::min<uint64_t>(group, kMaxRegGroup));
    group_first.push_back(static_cast<uint32_t>(q0));
    group_table.push_back(static_cast<uint32_t>(table.size()));
    for (uint64_t q = q0; q < q1; ++q) {
      const Plan& pl = items[q].plan;
      const uint64_t base = table.size();
      table.resize(base + 2 + 2 * reg_slots, 0u);
      table[base] = static_cast<uint32_t>(pl.preds.size()) | (outs[q].kind << 8) |
                    (outs[q].out_index << 16);
      if (pl.preds.empty()) {
        table[base + 1] = 1u;
        table[base + 2] = batch_key(-std::numeric_limits<float>::infinity());
        table[base + 3] = batch_key(std::numeric_limits<float>::infinity());
      }
      for (size_t i = 0; i < pl.preds.size(); ++i) {
        const uint32_t s = static_cast<uint32_t>(slot_of[pl.dims[i]]);
        table[base + 1] |= 1u << s;
        table[base + 2 + 2 * s] = batch_key(pl.preds[i].lo);
        table[base + 3 + 2 * s] = batch_key(pl.preds[i].hi);
      }
      // Early-break tests, placed by the estimated chance that the whole chunk is
      // rejected: with s the product of the selectivities so far (slot order), a chunk
      // of R rows survives with probability about 1 - exp(-R s).  A test (five vector
      // instructions) follows a predicate when that chance has grown by a third since
      // the last test and predicates remain; none follows the last one.
      std::vector<float> s_of(reg_slots, 1.0f);
      for (size_t i = 0; i < pl.preds.size(); ++i)
        s_of[slot_of[pl.dims[i]]] = items[q].sel[i];
      const double chunk_rows = 64.0 * cfg.rows_per_lane;
      double cum = 1.0, p_tested = 0.0;
      uint32_t seen = 0;
      for (uint32_t s = 0; s < reg_slots; ++s)
        if ((table[base + 1] >> s) & 1u) {
          ++seen;
          cum *= std::max(0.0f, std::min(1.0f, s_of[s]));
          const double p_dead = std::exp(-chunk_rows * cum);
          if (seen < pl.preds.size() && p_dead - p_tested > 1.0 / 3.0) {
            table[base + 1] |= 0x10000u << s;
            p_tested = p_dead;
          }
        }
    }
    q0 = q1;
  }
  // Rank variant: the groups' tables (build_rank_tables).
  uint64_t used_pairs = 0;
  if (rank) {
    uint64_t pairs = 0;
    const int rc_tables = build_rank_tables(ds, items, outs, slot_of, n_slots, rank_group, rank_sw, table, group_first,
                                  group_table, &pairs);
    if (rc_tables) return rc_tables;
    used_pairs = pairs;
  }
  // Group table: record offsets (padded to 4 words), then per query a 4-word header
  // and one 4-word entry (slot, key(lo), key(hi) - key(lo) or, for the LDS variant,
  // key(hi), 0) per predicate.
  for (uint64_t q0 = 0; !reg && !rank && q0 < nq;) {
    // Grow the group while its table and counts fit LDS.
    uint64_t words = 0, q1 = q0;
    while (q1 < nq && q1 - q0 < group) {
      const uint64_t add = 8 + 4 * items[q1].plan.preds.size() + 2;  // record, offset, count
      if ((words + add + 8) * 4 > kMaxLdsTable && q1 > q0) break;
      words += add;
      ++q1;
    }
    group_first.push_back(static_cast<uint32_t>(q0));
    group_table.push_back(static_cast<uint32_t>(table.size()));
    const uint64_t base = table.size();
    table.resize(base + ((q1 - q0 + 3) & ~uint64_t{3}), 0u);
    for (uint64_t q = q0; q < q1; ++q) {
      table[base + (q - q0)] = static_cast<uint32_t>(table.size() - base);
      const Plan& pl = items[q].plan;
      const bool always = use_lds && pl.preds.empty();   // the always-true predicate
      table.push_back(static_cast<uint32_t>(always ? 1 : pl.preds.size()) | (outs[q].kind << 8) |
                      (outs[q].out_index << 16));
      table.push_back(0u);
      table.push_back(0u);
      table.push_back(0u);
      if (always) {
        table.push_back(0u);
        table.push_back(batch_key(-std::numeric_limits<float>::infinity()));
        table.push_back(batch_key(std::numeric_limits<float>::infinity()));
        table.push_back(0u);
      }
      // The slot walk needs each query's predicates in ascending slot order.
      std::vector<size_t> ord(pl.preds.size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
      if (walk)
        std::sort(ord.begin(), ord.end(),
                  [&](size_t a, size_t b) { return slot_of[pl.dims[a]] < slot_of[pl.dims[b]]; });
      for (size_t i : ord) {
        const uint32_t klo = batch_key(pl.preds[i].lo);
        const uint32_t khi = batch_key(pl.preds[i].hi);
        table.push_back(static_cast<uint32_t>(slot_of[pl.dims[i]]));
        table.push_back(klo);
        table.push_back(use_lds ? khi : khi - klo);   // the LDS variant takes key(hi)
        table.push_back(0u);
      }
    }
    q0 = q1;
  }
  const uint32_t n_groups = static_cast<uint32_t>(group_first.size());
  group_first.push_back(static_cast<uint32_t>(nq));
  group_table.push_back(static_cast<uint32_t>(table.size()));
  uint64_t max_group_words = 0;
  for (uint32_t g = 0; g < n_groups; ++g)
    max_group_words = std::max<uint64_t>(
        max_group_words, (reg ? 0 : group_table[g + 1] - group_table[g]) +
                             ((group_first[g + 1] - group_first[g] + 3) & ~uint64_t{3}));
  if (rank && max_group_words > rank_words(rank_group)) {
    // Cannot happen (rank_words bounds every group's tables); answered by the
    // LDS-staged variant rather than failing if it ever did.
    BatchConfig other = cfg;
    other.lds = 1;
    for (Item& it : items) it.est_rows = -1.0;
    return run_shared(ds, ws, items, other, stream, ms_out, st, redo);
  }

  // Outputs: device buffers directly, host buffers through device staging.
  uint64_t stage_need = 0;
  std::vector<uint64_t> stage_off(nq, 0);
  for (uint64_t q = 0; q < nq; ++q) {
    mdrq_result_t* r = items[q].r;
    if (items[q].kind != kBatchCount && r->mem == MDRQ_MEM_HOST) {
      stage_off[q] = stage_need;
      const uint64_t cap = std::min<uint64_t>(r->buf_bytes, std::max<uint64_t>(4 * n_rows, 8 * nw));
      stage_need += (cap + 255) / 256 * 256;
    }
  }
  int rc = grow_device(reinterpret_cast<uint8_t**>(&ws.d_stage), &ws.d_stage_bytes,
                       std::max<uint64_t>(stage_need, 1), "batch staging");
  if (rc) return rc;
  for (uint64_t q = 0; q < nq; ++q) {
    mdrq_result_t* r = items[q].r;
    if (items[q].kind == kBatchCount) {
      outs[q].buf = nullptr;
      outs[q].buf_bytes = 0;
    } else if (r->mem == MDRQ_MEM_HOST) {
      outs[q].buf = static_cast<uint8_t*>(ws.d_stage) + stage_off[q];
      outs[q].buf_bytes = std::min<uint64_t>(r->buf_bytes, std::max<uint64_t>(4 * n_rows, 8 * nw));
    } else {
      outs[q].buf = r->buf;
      outs[q].buf_bytes = r->buf_bytes;
    }
  }

  // Device buffers (the bitmap scratch is laid out below, once the chunk size is known).
  const int rank_rg = cfg.rows_per_lane >= 8 ? 8 : 4;
  rc = grow_device(&ws.d_tile_counts, &ws.d_tile_counts_len, nq * (n_tiles + batch_emit_chunks(n_tiles)) + 1,
                   "batch tile counts");
  if (rc) return rc;
  rc = grow_results(ws, nq);
  if (rc) return rc;
  // Blob: table, group_first, group_table (uint32), then BatchOut records (8-aligned).
  const uint64_t words_u32 = table.size() + group_first.size() + group_table.size() + 2 * n_sparse;
  const uint64_t outs_off = (words_u32 * 4 + 15) / 16 * 16;
  const uint64_t blob = outs_off + nq * sizeof(BatchOut);
  rc = grow_pinned(&ws.h_blob, &ws.h_blob_bytes, blob);
  if (rc) return rc;
  rc = grow_device(reinterpret_cast<uint8_t**>(&ws.d_blob), &ws.d_blob_bytes, blob, "batch table");
  if (rc) return rc;
  uint32_t* hb = static_cast<uint32_t*>(ws.h_blob);
  std::memcpy(hb, table.data(), table.size() * 4);
  std::memcpy(hb + table.size(), group_first.data(), group_first.size() * 4);
  std::memcpy(hb + table.size() + group_first.size(), group_table.data(), group_table.size() * 4);
  uint32_t* hsp = hb + table.size() + group_first.size() + group_table.size();
  if (n_sparse) {
    std::memcpy(hsp, sparse_base.data(), n_sparse * 4);
    std::memcpy(hsp + n_sparse, sparse_cap.data(), n_sparse * 4);
  }
  std::memcpy(static_cast<uint8_t*>(ws.h_blob) + outs_off, outs.data(), nq * sizeof(BatchOut));
  const uint32_t* db = static_cast<const uint32_t*>(ws.d_blob);

  BatchParams bp{};
  bp.n_rows = n_rows;
  bp.n_tiles = n_tiles;
  bp.tile_begin = 0;
  bp.tile_end = n_tiles;
  bp.count_row = nullptr;
  bp.n_words = nw;
  bp.n_slots = static_cast<uint32_t>(n_slots);
  bp.table = db;
  bp.group_first = db + table.size();
  bp.group_table = db + table.size() + group_first.size();
  bp.words = ws.d_words;
  bp.flags = nullptr;
  bp.n_chunks = 0;
  bp.n_out = n_out;
  bp.tile_counts = ws.d_tile_counts;
  const uint32_t* dsp = db + table.size() + group_first.size() + group_table.size();
  bp.sparse_base = dsp;
  bp.sparse_cap = dsp + n_sparse;
  for (int s = 0; s < n_slots; ++s) bp.slot_cols[s] = ds->cols[slot_dim[s]];
  BatchFinish fin{};
  fin.n_tiles = n_tiles;
  fin.n_words = nw;
  fin.words = ws.d_words;
  fin.flags = nullptr;
  fin.n_chunks = 0;
  fin.chunk_shift = 0;
  fin.tile_counts = ws.d_tile_counts;
  fin.chunk_pos = ws.d_tile_counts + nq * n_tiles;
  fin.count_row = nullptr;
  fin.outs = reinterpret_cast<const BatchOut*>(static_cast<const uint8_t*>(ws.d_blob) + outs_off);
  fin.counts_out = static_cast<uint64_t*>(ws.h_res_dev);
  fin.kind_out = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(ws.h_res_dev) + nq * 8);
  fin.over_out = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(ws.h_res_dev) + nq * 12);
  fin.sparse_base = bp.sparse_base;
  fin.sparse_cap = bp.sparse_cap;

  int waves = cfg.waves == 8 ? 8 : 4;
  int rg;
  size_t lds;
  if (use_lds) {
    uint64_t max_nq = 0;
    for (uint32_t g = 0; g < n_groups; ++g)
      max_nq = std::max<uint64_t>(max_nq, group_first[g + 1] - group_first[g]);
    rg = cfg.rows_per_lane >= 8 ? 8 : cfg.rows_per_lane >= 4 ? 4 : cfg.rows_per_lane >= 2 ? 2 : 1;
    auto need = [&](int r) {
      return ((max_nq + 3) & ~uint64_t{3}) * 4 + batch_lds_key_bytes(std::max(1, n_slots), waves, r);
    };
    while (need(rg) > device().lds && rg > 1) rg /= 2;
    if (need(rg) > device().lds && waves == 8) {
      waves = 4;
      rg = 1;
    }
    lds = need(rg);
    if (lds > device().lds) return fail(MDRQ_ENOTSUP, "shared scan: union keys do not fit LDS");
  } else if (rank) {
    rg = rank_rg;
    lds = max_group_words * 4;
  } else {
    rg = batch_rows_per_lane(std::max(1, n_slots), waves, cfg.rows_per_lane);
    lds = max_group_words * 4;
  }
  // Bitmap scratch, one allocation: the dense queries' rows, the sparse queries' pool
  // slots, then (variants with marks) the dense rows' chunk marks, the sparse queries'
  // slot tables and slot counters, which are zeroed before the scan.  The serving loop
  // admits requests by these sizes (request_scratch_bytes bounds each query's part).
  const bool marks = rank || (reg && batch_reg_uses_marks(static_cast<int>(reg_slots)));
  const uint64_t rows_words = static_cast<uint64_t>(n_out) * nw + pool_slots * static_cast<uint64_t>(rg);
  const uint64_t chunk_rows = 64 * static_cast<uint64_t>(rg);
  const uint64_t n_chunks = (n_rows + chunk_rows - 1) / chunk_rows;
  const uint64_t marks_words = marks ? (n_chunks * n_out + 3) / 4 : 0;
  const uint64_t slots_words = (n_chunks * n_sparse + 1) / 2;
  const uint64_t next_words = (static_cast<uint64_t>(n_sparse) + 1) / 2;
  rc = grow_device(&ws.d_words, &ws.d_words_len, rows_words + marks_words + slots_words + next_words + 1,
                   "batch bitmaps");
  if (rc) return rc;
  bp.words = ws.d_words;
  fin.words = ws.d_words;
  bp.pool = ws.d_words + static_cast<uint64_t>(n_out) * nw;
  fin.pool = bp.pool;
  if ((n_out || n_sparse) && marks) {
    uint64_t* fl = ws.d_words + rows_words;
    bp.flags = reinterpret_cast<uint16_t*>(fl);
    bp.n_chunks = n_chunks;
    bp.slots = reinterpret_cast<uint32_t*>(fl + marks_words);
    bp.slot_next = reinterpret_cast<uint32_t*>(fl + marks_words + slots_words);
    bp.n_zero = marks_words + slots_words + next_words;
    fin.flags = bp.flags;
    fin.n_chunks = n_chunks;
    fin.chunk_shift = static_cast<uint32_t>(__builtin_ctz(static_cast<unsigned>(rg)));
    fin.slots = bp.slots;
    fin.slot_next = bp.slot_next;
  }
  const int per_cu = batch_blocks_per_cu(std::max(1, n_slots), waves, rg, variant, lds, rank_sw);
  const uint64_t resident = static_cast<uint64_t>(per_cu) * device().cus;
  const uint64_t gx = std::max<uint64_t>(1, std::min<uint64_t>(n_tiles, resident / n_groups));

  if (!ws.ev0) MDRQ_HIP(hipEventCreate(&ws.ev0), "hipEventCreate");
  if (!ws.ev1) MDRQ_HIP(hipEventCreate(&ws.ev1), "hipEventCreate");
  if (!ws.ev2) MDRQ_HIP(hipEventCreate(&ws.ev2), "hipEventCreate");
  if (ds->graph_batch && n_tiles > 0) {
    MDRQ_HIP(launch_shared_graph(ws, bp, fin, static_cast<uint32_t>(nq), std::max(1, n_slots), waves, rg, variant,
                                 dim3(static_cast<uint32_t>(gx), n_groups), lds, rank_sw, blob, stream),
             "shared scan graph");
  } else {
    MDRQ_HIP(hipMemcpyAsync(ws.d_blob, ws.h_blob, blob, hipMemcpyHostToDevice, stream),
             "copy query table");
    MDRQ_HIP(hipEventRecord(ws.ev0, stream), "hipEventRecord");
    if (n_tiles > 0)
      MDRQ_HIP(launch_batch_scan(bp, std::max(1, n_slots), waves, rg, variant,
                                 dim3(static_cast<uint32_t>(gx), n_groups), lds, stream, rank_sw),
               "shared scan launch");
    MDRQ_HIP(hipEventRecord(ws.ev2, stream), "hipEventRecord");
    MDRQ_HIP(launch_batch_finish(fin, static_cast<uint32_t>(nq), stream), "batch finish launch");
    MDRQ_HIP(hipEventRecord(ws.ev1, stream), "hipEventRecord");
  }
  MDRQ_HIP(hipStreamSynchronize(stream), "shared scan completion");
  float ms = 0.f, scan_ms = 0.f;
  MDRQ_HIP(hipEventElapsedTime(&ms, ws.ev0, ws.ev1), "hipEventElapsedTime");
  MDRQ_HIP(hipEventElapsedTime(&scan_ms, ws.ev0, ws.ev2), "hipEventElapsedTime");
  if (ms_out) *ms_out = ms;
  {
    // Work of the scan: rows looked up per (group, column) in the rank variant, column
    // bytes read (each group reads its own columns in the rank variant).
    std::lock_guard<std::mutex> lock(ds->stat_mu);
    const uint64_t pairs = rank ? used_pairs : static_cast<uint64_t>(n_slots);
    ds->batch_lookups += rank ? n_rows * pairs : 0;
    ds->batch_column_bytes += 4 * n_rows * pairs;
    ds->batch_scan_ms += scan_ms;
  }

  // The finish kernel wrote the counts and kinds into the mapped pinned buffer.
  const volatile uint64_t* counts = static_cast<const volatile uint64_t*>(ws.h_res);
  const volatile uint32_t* kinds =
      reinterpret_cast<const volatile uint32_t*>(static_cast<const uint8_t*>(ws.h_res) + nq * 8);
  for (uint64_t q = 0; q < nq; ++q) {
    mdrq_result_t* r = items[q].r;
    const uint64_t count = counts[q];
    const uint32_t kind = kinds[q];
    r->count = count;
    r->status = MDRQ_OK;
    r->written = 0;
    uint64_t bytes = 0;
    if (kind == kBatchCount) {
      r->mode = MDRQ_OUT_COUNT;
    } else if (kind == kBatchBitmap) {
      r->mode = MDRQ_OUT_BITMAP;
      const uint64_t cap = outs[q].buf_bytes / 8;
      r->written = std::min(cap, nw);
      if (cap < nw) r->status = MDRQ_EOVERFLOW;
      bytes = r->written * 8;
    } else {
      r->mode = MDRQ_OUT_IDS;
      const uint64_t cap = outs[q].buf_bytes / 4;
      r->written = std::min(cap, count);
      if (count > cap) r->status = MDRQ_EOVERFLOW;
      bytes = r->written * 4;
    }
    if (kind != kBatchCount && r->mem == MDRQ_MEM_HOST && bytes)
      MDRQ_HIP(hipMemcpy(r->buf, outs[q].buf, bytes, hipMemcpyDeviceToHost), "copy result to host");
  }
  // Queries whose estimate was too low for their scratch: handed back in `redo` (the
  // caller answers them again together, with worst-case scratch), or without it
  // answered again here, each alone (the count above was exact already).
  const volatile uint32_t* over =
      reinterpret_cast<const volatile uint32_t*>(static_cast<const uint8_t*>(ws.h_res) + nq * 12);
  uint64_t n_reruns = 0;
  for (uint64_t q = 0; q < nq; ++q) {
    if (!outs[q].sparse || !over[q]) continue;
    Item& it = items[q];
    ++n_reruns;
    if (redo) {
      redo->push_back(it.index);
      continue;
    }
    it.r->mode = it.plan.mode == kBitmap ? MDRQ_OUT_BITMAP : it.plan.mode == kCount ? MDRQ_OUT_COUNT : MDRQ_OUT_IDS;
    rc = run_query(ds, it.plan, it.r, stream);
    if (rc != MDRQ_OK && rc != MDRQ_EOVERFLOW) return rc;
  }
  if (st) {
    st->sparse += n_sparse;
    st->reruns += n_reruns;
  }
  if (n_sparse) {
    std::lock_guard<std::mutex> lock(ds->stat_mu);
    ds->sized_queries += n_sparse;
    ds->sized_reruns += n_reruns;
  }
  return MDRQ_OK;
}

// Widest union of columns one shared scan can stage in LDS (4 waves, one 64-row group
// per lane, 1024-query counts), at most kMaxUnion.
int max_union() {
  const size_t per_slot = batch_lds_key_bytes(1, 4, 1);
  const size_t room = device().lds > 4096 ? device().lds - 4096 : 0;
  return static_cast<int>(std::min<size_t>(kMaxUnion, std::max<size_t>(kMaxSlots, room / per_slot)));
}

// Best-fit decreasing grouping of the items listed in `which` into sets whose union of
// columns has at most `limit` columns and which hold at most MDRQ_MAX_BATCH items.  Each
// group lists item positions in ascending order.
std::vector<std::vector<size_t>> group_by_columns(const std::vector<Item>& items,
                                                  const std::vector<size_t>& which,
                                                  uint32_t n_dims, int limit) {
  struct Group {
    std::vector<bool> in;
    int used = 0;
    std::vector<size_t> members;
  };
  std::vector<size_t> order(which);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return items[a].plan.dims.size() > items[b].plan.dims.size();
  });
  std::vector<Group> groups;
  for (size_t i : order) {
    const std::vector<uint32_t>& dims = items[i].plan.dims;
    Group* best = nullptr;
    int best_add = limit + 1;
    for (Group& g : groups) {
      if (g.members.size() >= MDRQ_MAX_BATCH) continue;
      int add = 0;
      for (uint32_t d : dims) add += g.in[d] ? 0 : 1;
      if (g.used + add <= limit && add < best_add) {
        best = &g;
        best_add = add;
        if (add == 0) break;
      }
    }
    if (!best) {
      groups.push_back(Group{std::vector<bool>(n_dims, false), 0, {}});
      best = &groups.back();
    }
    for (uint32_t d : dims)
      if (!best->in[d]) {
        best->in[d] = true;
        ++best->used;
      }
    best->members.push_back(i);
  }
  std::vector<std::vector<size_t>> out;
  out.reserve(groups.size());
  for (Group& g : groups) {
    std::sort(g.members.begin(), g.members.end());
    out.push_back(std::move(g.members));
  }
  return out;
}

// Unions wider than the register slots take the LDS variant, which tests about half as
// fast.  When a batch's queries would share such a union, also try grouping them into
// register-sized unions (queries with more predicates than slots stay in wide groups)
// and keep whichever grouping a simple cost model prefers: per scan, the larger of its
// column bytes at streaming bandwidth and its row tests at the variant's rate.
std::vector<std::vector<size_t>> plan_groups(const std::vector<Item>& items, uint32_t n_dims,
                                             uint64_t n_rows) {
  std::vector<size_t> all(items.size());
  for (size_t i = 0; i < all.size(); ++i) all[i] = i;
  std::vector<std::vector<size_t>> wide = group_by_columns(items, all, n_dims, max_union());
  auto union_of = [&](const std::vector<size_t>& g) {
    std::vector<bool> in(n_dims, false);
    int u = 0;
    for (size_t m : g)
      for (uint32_t d : items[m].plan.dims)
        if (!in[d]) {
          in[d] = true;
          ++u;
        }
    return u;
  };
  bool any_wide = false;
  for (const auto& g : wide) any_wide |= union_of(g) > kMaxSlots;
  if (!any_wide) return wide;
  std::vector<size_t> narrow_items, wide_items;
  for (size_t i = 0; i < items.size(); ++i)
    (items[i].plan.dims.size() <= static_cast<size_t>(kMaxSlots) ? narrow_items : wide_items).push_back(i);
  if (narrow_items.empty()) return wide;   // the split grouping would be the same
  std::vector<std::vector<size_t>> split = group_by_columns(items, narrow_items, n_dims, kMaxSlots);
  for (auto& g : group_by_columns(items, wide_items, n_dims, max_union())) split.push_back(std::move(g));
  auto cost = [&](const std::vector<std::vector<size_t>>& groups) {
    constexpr double kBytesPerS = 6e12, kRegTests = 8e12, kLdsTests = 4e12, kLaunchS = 30e-6;
    double t = 0.0;
    for (const auto& g : groups) {
      const int u = union_of(g);
      double tests = 0.0;
      for (size_t m : g) tests += static_cast<double>(n_rows) * items[m].plan.dims.size();
      t += std::max(4.0 * n_rows * u / kBytesPerS, tests / (u > kMaxSlots ? kLdsTests : kRegTests)) +
           kLaunchS;
    }
    return t;
  };
  return cost(split) < cost(wide) ? split : wide;
}

// A shared scan reads every column of its union in full and tests each query on every
// row; one scan per query reads only that query's columns, and its early break skips
// the groups of rows already rejected (about a quarter of the bytes on c2's mix).  For a
// few queries the separate scans are cheaper.  Model: shared = max(union column bytes
// at 4.5 TB/s, row tests at 8e12/s in registers or 4e12/s in LDS) + 30 us; separate =
// sum over queries of 3/4 of its column bytes at 6 TB/s + 25 us.  (Measured on 2·10^8
// rows x 12 columns, batches of 1..32 queries: the shared scan, rank variant with its
// finish, took 1.05 / 1.72 / 2.25 / 2.97 ms at 2 / 4 / 8 / 32 queries, separate scans
// about 0.37 ms per query; the two meet at 4 to 5 queries.)
bool plain_is_cheaper(const std::vector<Item>& items, const std::vector<size_t>& members, int used,
                      uint64_t n_rows) {
  constexpr double kBytesPerS = 6e12, kSharedBytesPerS = 4.5e12, kRegTests = 8e12, kLdsTests = 4e12;
  const double n = static_cast<double>(n_rows);
  double tests = 0.0, plain = 0.0;
  for (size_t m : members) {
    const double k = static_cast<double>(items[m].plan.dims.size());
    tests += n * k;
    plain += 0.75 * 4.0 * n * k / kBytesPerS + 25e-6;
  }
  const double shared =
      std::max(4.0 * n * used / kSharedBytesPerS, tests / (used > kMaxSlots ? kLdsTests : kRegTests)) + 30e-6;
  return plain < shared;
}

// Candidate configurations the autotuner tries on a new batch shape.
std::vector<BatchConfig> candidates(uint64_t nq, int n_slots, int variant) {
  std::vector<BatchConfig> c;
  auto add = [&](const BatchConfig& b) {
    for (const BatchConfig& o : c)
      if (o.waves == b.waves && o.group == b.group && o.rows_per_lane == b.rows_per_lane && o.lds == b.lds)
        return;
    c.push_back(b);
  };
  for (uint64_t g : {nq, (nq + 1) / 2, (nq + 3) / 4}) {
    if (g < 16 && g != nq) continue;
    for (int w : {4, 8}) {
      if (n_slots <= kMaxSlots && variant != 2 && variant != 5)
        for (int rg : {16, 8, 4})
          for (int v : {0, 2, 3}) {
            if ((variant == 1 && v != 0) || (variant == 3 && v != 2) || (variant == 4 && v != 3))
              continue;
            BatchConfig b;
            b.waves = w;
            b.group = static_cast<uint32_t>(g);
            b.rows_per_lane = batch_rows_per_lane(n_slots, w, rg);
            b.lds = v;
            add(b);
          }
      if (variant == 0 || variant == 5)
        for (int rg : {8, 4}) {
          BatchConfig b;
          b.waves = w;
          b.group = static_cast<uint32_t>(std::min<uint64_t>(g, 128));
          b.rows_per_lane = rg;
          b.lds = 4;
          add(b);
        }
      if (variant == 0 || variant == 2 || n_slots > kMaxSlots) {
        bool any = false;
        for (int rg : {8, 4, 2, 1}) {
          // one 64-row group per lane only where nothing larger fits (it is slower)
          if (rg == 1 && any) break;
          if (((g + 3) & ~uint64_t{3}) * 4 + batch_lds_key_bytes(std::max(1, n_slots), w, rg) > device().lds)
            continue;
          BatchConfig b;
          b.waves = w;
          b.group = static_cast<uint32_t>(g);
          b.rows_per_lane = rg;
          b.lds = 1;
          add(b);
          any = true;
        }
      }
    }
  }
  if (c.empty()) {  // the smallest LDS configuration: run_shared shrinks it to fit
    BatchConfig b;
    b.rows_per_lane = 1;
    b.lds = 1;
    c.push_back(b);
  }
  return c;
}

}  // namespace

uint64_t sparse_slots(const mdrq_dataset* ds, double est_rows, uint64_t chunk_rows) {
  if (!(est_rows >= 0.0)) return 0;
  const uint64_t n_chunks = (ds->n_rows + chunk_rows - 1) / chunk_rows;
  // A chunk with a hit holds at least one result row: chunks <= rows.
  const double want = std::ceil(est_rows * static_cast<double>(ds->reserve_ppm) * 1e-6) + 64.0;
  const uint64_t slots = want >= static_cast<double>(n_chunks) ? n_chunks : static_cast<uint64_t>(want);
  const uint64_t sparse_bytes = n_chunks * 4 + slots * (chunk_rows / 64) * 8;
  const uint64_t dense_bytes = n_words(ds) * 8 + n_chunks * 2;
  return sparse_bytes < dense_bytes ? slots : 0;
}

uint64_t request_scratch_bytes(const mdrq_dataset* ds, const mdrq_result_t& r, double est_rows) {
  if (r.mode == MDRQ_OUT_COUNT) return 0;
  const uint64_t slots = sparse_slots(ds, est_rows, kSparseChunkRows);
  const uint64_t n_chunks = (ds->n_rows + kSparseChunkRows - 1) / kSparseChunkRows;
  if (slots) return n_chunks * 4 + slots * (kSparseChunkRows / 64) * 8 + 16;
  // A bitmap row and its chunk marks at the smallest chunk (256 rows).
  return n_words(ds) * 8 + ((ds->n_rows + 255) / 256) * 2 + 16;
}

// Answer a batch: canonicalise each query, answer empty ones without a launch, run
// queries that cannot share a scan (more than max_union() predicates) alone, and group
// the rest into shared scans whose union of columns fits the register slots.
int run_batch(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, mdrq_result_t* rs,
              hipStream_t stream, BatchWorkspace* wsp, bool tune, BatchRunStats* st, const float* est_in) {
  BatchWorkspace& ws = wsp ? *wsp : ds->batch;
  // Estimated selectivities, for MDRQ_Q_ORDER_ESTIMATED and MDRQ_Q_SIZE_ESTIMATED.
  std::vector<float> est;
  if (est_in) {
    est.assign(est_in, est_in + static_cast<size_t>(n) * (ds->n_dims + 1));
  } else {
    int erc = estimate_for_order(ds, qs, n, est);
    if (erc) return erc;
  }
  auto plan_of = [&](uint32_t i) {
    Plan plan = make_plan(ds, &qs[i], &rs[i]);
    if (!est.empty() && (qs[i].flags & MDRQ_Q_ORDER_ESTIMATED))
      order_plan(plan, &est[static_cast<size_t>(i) * (ds->n_dims + 1)]);
    return plan;
  };
  std::vector<Item> shared;
  std::vector<uint32_t> alone;
  std::vector<uint32_t> redo;   // queries whose estimate-sized scratch was too small
  std::vector<uint32_t> asked(n);
  for (uint32_t i = 0; i < n; ++i) asked[i] = rs[i].mode;
  for (uint32_t i = 0; i < n; ++i) {
    Plan plan = plan_of(i);
    if (plan.empty || ds->n_rows == 0) {
      if (rs[i].mode == MDRQ_OUT_AUTO) {
        plan.mode = kIds;
        rs[i].mode = MDRQ_OUT_IDS;
      }
      int rc = finish_empty(ds, plan, &rs[i], stream);
      if (rc != MDRQ_OK && rc != MDRQ_EOVERFLOW) return rc;
      continue;
    }
    if (plan.preds.size() > static_cast<size_t>(max_union())) {
      alone.push_back(i);
      continue;
    }
    // Per-predicate selectivities for placing the early-break tests: the estimator's,
    // when the batch was estimated, else the interval's share of the column's range.
    std::vector<float> sel(plan.preds.size());
    const float* row = est.empty() ? nullptr : &est[static_cast<size_t>(i) * (ds->n_dims + 1)];
    for (size_t j = 0; j < sel.size(); ++j) {
      const uint32_t d = plan.dims[j];
      if (row) {
        sel[j] = row[d];
      } else {
        const double lo = std::max<double>(plan.preds[j].lo, ds->col_min[d]);
        const double hi = std::min<double>(plan.preds[j].hi, ds->col_max[d]);
        const double range = static_cast<double>(ds->col_max[d]) - ds->col_min[d];
        sel[j] = range > 0 && std::isfinite(range) ? static_cast<float>(std::max(0.0, hi - lo) / range) : 1.0f;
      }
    }
    shared.push_back(Item{i, std::move(plan), kind_of(rs[i].mode), &rs[i], std::move(sel)});
    if (row && (qs[i].flags & MDRQ_Q_SIZE_ESTIMATED))
      shared.back().est_rows = static_cast<double>(row[ds->n_dims]) * static_cast<double>(ds->n_rows);
  }
  // Grouping into shared scans whose union of columns fits the register slots:
  // best-fit decreasing -- queries with the most columns first, each into the open
  // group it adds the fewest new columns to (a new group if none has room).  Queries
  // on overlapping columns share a scan, so each column is read by few scans.
  std::vector<std::vector<size_t>> groups = plan_groups(shared, ds->n_dims, ds->n_rows);
  const bool fixed = ds->batch_waves || ds->batch_group || ds->batch_rows || ds->batch_variant ||
                     !ds->autotune;
  for (const std::vector<size_t>& members : groups) {
    std::vector<Item> batch;
    std::vector<bool> in(ds->n_dims, false);
    int used = 0;
    for (size_t m : members)
      for (uint32_t d : shared[m].plan.dims)
        if (!in[d]) {
          in[d] = true;
          ++used;
        }
    if (!fixed && plain_is_cheaper(shared, members, used, ds->n_rows)) {
      for (size_t m : members) {
        Item& it = shared[m];
        it.r->mode = it.plan.mode == kBitmap ? MDRQ_OUT_BITMAP
                     : it.plan.mode == kCount ? MDRQ_OUT_COUNT : MDRQ_OUT_IDS;
        int rc = wsp ? run_query_on(ds, it.plan, it.r, stream, wsp->single) : run_query(ds, it.plan, it.r, stream);
        if (rc != MDRQ_OK && rc != MDRQ_EOVERFLOW) return rc;
      }
      if (st) st->alone += members.size();
      continue;
    }
    for (size_t m : members) batch.push_back(std::move(shared[m]));
    BatchConfig cfg;
    cfg.waves = ds->batch_waves ? ds->batch_waves : 4;
    cfg.group = ds->batch_group;
    cfg.rows_per_lane = ds->batch_rows ? ds->batch_rows : used > 8 ? 4 : 8;
    // Untuned default: the rank variant (fastest on every measured shape, c3 and c5).
    cfg.lds = ds->batch_variant == 1 ? 0 : ds->batch_variant == 2 ? 1 : ds->batch_variant == 3 ? 2
              : ds->batch_variant == 4 ? 3 : 4;
    if (used > kMaxSlots && !ds->batch_rows) cfg.rows_per_lane = used > 32 ? 1 : 2;
    // The rank variant untuned: 8 waves and 512-row chunks (on 2*10^8 rows x 12 columns,
    // 256 queries with ids or bitmap output: 8.7 ms against 10.1 ms with 4 waves and
    // 256-row chunks; count-only 5.8 against 6.3 ms).
    if (cfg.lds == 4) {
      if (!ds->batch_waves) cfg.waves = 8;
      if (!ds->batch_rows) cfg.rows_per_lane = 8;
    }
    float ms = 0.f;
    if (fixed) {
      int rc = run_shared(ds, ws, batch, cfg, stream, &ms, st, &redo);
      if (rc) return rc;
    } else {
      bool writes = false;
      for (const Item& it : batch) writes |= it.kind != kBatchCount;
      const uint64_t key = shape_key(ds->n_rows, static_cast<size_t>(used), batch.size(), writes);
      BatchConfig known_cfg;
      bool known = false;
      {
        std::lock_guard<std::mutex> lock(ds->stat_mu);
        for (const auto& kv : ds->tuned)
          if (kv.first == key) {
            known_cfg = kv.second;
            known = true;
          }
        // Without tuning, take a configuration tuned for the same rows and columns.
        if (!known && !tune)
          for (const auto& kv : ds->tuned)
            if ((kv.first >> 8) == (key >> 8)) {
              known_cfg = kv.second;
              known = true;
            }
      }
      if (known || !tune) {
        int rc = run_shared(ds, ws, batch, known ? known_cfg : cfg, stream, &ms, st, &redo);
        if (rc) return rc;
      } else {
        // Every candidate computes the same exact results; keep the fastest.  One timing
        // per candidate is noisy (a kernel's first launch also loads its code), so the
        // three fastest are timed once more and each keeps its better time.
        std::vector<std::pair<float, BatchConfig>> timed;
        for (const BatchConfig& c : candidates(batch.size(), used, ds->batch_variant)) {
          int rc = run_shared(ds, ws, batch, c, stream, &ms);
          if (rc) return rc;
          timed.emplace_back(ms, c);
        }
        if (timed.empty()) {
          int rc = run_shared(ds, ws, batch, cfg, stream, &ms);
          if (rc) return rc;
          timed.emplace_back(ms, cfg);
        }
        std::stable_sort(timed.begin(), timed.end(),
                         [](const auto& a, const auto& b) { return a.first < b.first; });
        const size_t again = std::min<size_t>(3, timed.size());
        for (size_t i = 0; i < again; ++i) {
          int rc = run_shared(ds, ws, batch, timed[i].second, stream, &ms);
          if (rc) return rc;
          timed[i].first = std::min(timed[i].first, ms);
        }
        BatchConfig best = timed[0].second;
        float best_ms = timed[0].first;
        for (size_t i = 1; i < again; ++i)
          if (timed[i].first < best_ms) {
            best_ms = timed[i].first;
            best = timed[i].second;
          }
        std::lock_guard<std::mutex> lock(ds->stat_mu);
        ds->tuned.emplace_back(key, best);
        ms = best_ms;
      }
    }
    {
      std::lock_guard<std::mutex> lock(ds->stat_mu);
      ds->batch_launches += 1;
      ds->batch_ms += ms;
    }
    if (st) {
      st->scans += 1;
      st->column_bytes += 4 * ds->n_rows * static_cast<uint64_t>(used);
      st->device_ms += ms;
    }
  }
  for (uint32_t i : alone) {
    Plan plan = plan_of(i);
    if (rs[i].mode == MDRQ_OUT_AUTO) {
      plan.mode = kIds;
      rs[i].mode = MDRQ_OUT_IDS;
    }
    int rc = run_query(ds, plan, &rs[i], stream);
    if (rc != MDRQ_OK && rc != MDRQ_EOVERFLOW) return rc;
  }
  if (!redo.empty()) {
    // Answered again together, with worst-case scratch: one shared scan for many, the
    // single-query scan for a few (as any batch).
    std::sort(redo.begin(), redo.end());
    std::vector<mdrq_query_t> q2(redo.size());
    std::vector<mdrq_result_t> r2(redo.size());
    std::vector<float> e2;
    for (size_t k = 0; k < redo.size(); ++k) {
      const uint32_t i = redo[k];
      q2[k] = qs[i];
      q2[k].flags &= ~static_cast<uint32_t>(MDRQ_Q_SIZE_ESTIMATED);
      r2[k] = rs[i];
      r2[k].mode = asked[i];
      if (!est.empty())
        e2.insert(e2.end(), est.begin() + static_cast<size_t>(i) * (ds->n_dims + 1),
                  est.begin() + static_cast<size_t>(i + 1) * (ds->n_dims + 1));
    }
    int rc = run_batch(ds, q2.data(), static_cast<uint32_t>(q2.size()), r2.data(), stream, wsp, tune, st,
                       e2.empty() ? nullptr : e2.data());
    if (rc != MDRQ_OK) return rc;
    for (size_t k = 0; k < redo.size(); ++k) rs[redo[k]] = r2[k];
  }
  return MDRQ_OK;
}

int reserve_batch(const mdrq_dataset* ds, BatchWorkspace& ws, uint32_t max_queries, uint64_t scratch_bytes) {
  const uint64_t n_tiles = (ds->n_rows + kTileRows - 1) / kTileRows;
  const uint64_t nq = max_queries;
  // The bitmap scratch: dense rows, sparse pools, marks and slot tables of a batch whose
  // requests' request_scratch_bytes sum to at most scratch_bytes.
  int rc = grow_device(&ws.d_words, &ws.d_words_len, (scratch_bytes + 7) / 8 + 8, "batch bitmaps");
  if (rc) return rc;
  rc = grow_device(&ws.d_tile_counts, &ws.d_tile_counts_len, nq * (n_tiles + batch_emit_chunks(n_tiles)) + 1,
                   "batch tile counts");
  if (rc) return rc;
  rc = grow_results(ws, nq);
  if (rc) return rc;
  // Query table: at most a 4-word header and 4 words per predicate per query, record
  // offsets and group arrays; then the output records.
  const uint64_t blob = (nq * (8 + 4 * kMaxUnion) + 64) * 4 + nq * sizeof(BatchOut) + 16;
  rc = grow_pinned(&ws.h_blob, &ws.h_blob_bytes, blob);
  if (rc) return rc;
  rc = grow_device(reinterpret_cast<uint8_t**>(&ws.d_blob), &ws.d_blob_bytes, blob, "batch table");
  if (rc) return rc;
  rc = grow_device(reinterpret_cast<uint8_t**>(&ws.d_stage), &ws.d_stage_bytes, 1, "batch staging");
  if (rc) return rc;
  if (!ws.ev0) MDRQ_HIP(hipEventCreate(&ws.ev0), "hipEventCreate");
  if (!ws.ev1) MDRQ_HIP(hipEventCreate(&ws.ev1), "hipEventCreate");
  return MDRQ_OK;
}

void free_batch(BatchWorkspace& ws) {
  free_single(ws.single);
  if (ws.d_blob) (void)hipFree(ws.d_blob);
  if (ws.h_blob) (void)hipHostFree(ws.h_blob);
  if (ws.d_words) (void)hipFree(ws.d_words);
  if (ws.d_tile_counts) (void)hipFree(ws.d_tile_counts);
  if (ws.h_res) (void)hipHostFree(ws.h_res);
  if (ws.d_stage) (void)hipFree(ws.d_stage);
  if (ws.ev0) (void)hipEventDestroy(ws.ev0);
  if (ws.ev1) (void)hipEventDestroy(ws.ev1);
  if (ws.ev2) (void)hipEventDestroy(ws.ev2);
  for (BatchWorkspace::Graph& g : ws.graphs) destroy_graph(g);
  ws = BatchWorkspace{};
}


// ---------------------------------------------------------------- circular scan

namespace {
constexpr int kCircRg = 8;                          // rows per lane: 512-row chunks
constexpr int kCircWaves = 8;                       // waves per workgroup of a shared step
constexpr uint64_t kCircChunkRows = 64 * kCircRg;
constexpr int kCircPlainUnroll = 16;                // single-query steps: 4096-row tiles
}  // namespace

// Steps may be pipelined: the host builds and enqueues step k + 1 while the device runs
// step k, then waits for step k and reads its results.  Two step buffers alternate
// (query table, result records, events); a buffer is refilled only after its step is
// complete, and a slot freed by a step can be taken at the next one because the stream
// runs the next step's clearing and scan after this step's finish.  Otherwise each step
// is waited for before the next is built, so requests admitted meanwhile join it.
struct CircularScan {
  mdrq_dataset* ds = nullptr;
  uint64_t* rows = nullptr;          // slot rows, then the slots' chunk marks
  uint64_t rows_len = 0;
  uint32_t* tile_counts = nullptr;   // per slot a row of tile counts
  uint64_t tile_counts_len = 0;
  uint32_t n_slots = 0;              // query slots
  uint32_t max_union = 0;            // widest union of columns a step may scan
  uint64_t n_tiles = 0, seg_tiles = 0, n_segs = 0;
  uint64_t marks_stride = 0;         // marks per slot: the row's chunks, 4-aligned
  uint64_t cur = 0;                  // segment of the next step
  // Active queries, in admission order, and per query its slot, the steps it still
  // needs, whether its marks still have to be cleared, and the caller's tag.
  std::vector<Item> items;
  struct Meta {
    uint32_t slot;
    uint64_t left;
    bool fresh;
    void* tag;
  };
  std::vector<Meta> meta;
  std::vector<uint32_t> free_slots;
  std::vector<uint32_t> dim_uses;    // per dimension: active queries restricting it
  uint32_t union_size = 0;
  std::vector<void*> answered;       // answered at admission: complete with the next step
  struct Step {
    void* h_blob = nullptr;
    uint64_t h_blob_bytes = 0;
    void* d_blob = nullptr;
    uint64_t d_blob_bytes = 0;
    void* h_res = nullptr;           // counts (u64), then kinds (u32): mapped pinned
    void* h_res_dev = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool inflight = false;
    std::vector<std::pair<mdrq_result_t*, void*>> fin;   // finished by this step, in order
    std::vector<void*> extra;        // answered at admission before this step
    uint64_t seg_rows = 0, pairs = 0;
    uint64_t plain_cols = 0;         // single-query steps: the requests' columns
  };
  Step steps[2];
  int next = 0;                      // buffer of the next step
  bool pipelined = false;            // else each step is waited for before the next
  bool plain_steps = false;          // steps of few requests by single-query scans
  uint64_t n_chunks = 0;             // 512-row chunks of a row
  uint32_t* block_sums = nullptr;    // single-query steps: per-workgroup counts (unused)
  uint64_t block_sums_len = 0;
};

uint64_t circular_slot_bytes(const mdrq_dataset* ds) {
  const uint64_t n_chunks = (ds->n_rows + kCircChunkRows - 1) / kCircChunkRows;
  const uint64_t n_tiles = (ds->n_rows + kTileRows - 1) / kTileRows;
  return n_words(ds) * 8 + align4(n_chunks) * 2 + (n_tiles + batch_emit_chunks(n_tiles)) * 4;
}

void circular_destroy(CircularScan* c) {
  if (!c) return;
  if (c->rows) (void)hipFree(c->rows);
  if (c->tile_counts) (void)hipFree(c->tile_counts);
  if (c->block_sums) (void)hipFree(c->block_sums);
  for (CircularScan::Step& s : c->steps) {
    if (s.h_blob) (void)hipHostFree(s.h_blob);
    if (s.d_blob) (void)hipFree(s.d_blob);
    if (s.h_res) (void)hipHostFree(s.h_res);
    if (s.ev0) (void)hipEventDestroy(s.ev0);
    if (s.ev1) (void)hipEventDestroy(s.ev1);
  }
  delete c;
}

int circular_create(mdrq_dataset* ds, uint32_t slots, uint32_t segments, CircularScan** out) {
  *out = nullptr;
  if (slots == 0 || segments == 0) return fail(MDRQ_EINVAL, "circular scan: no slots or no segments");
  std::unique_ptr<CircularScan, void (*)(CircularScan*)> c(new CircularScan(), circular_destroy);
  c->ds = ds;
  c->n_slots = slots;
  c->pipelined = (ds->circular_mode & 1) != 0;
  c->plain_steps = (ds->circular_mode & 4) != 0;
  c->n_tiles = (ds->n_rows + kTileRows - 1) / kTileRows;
  const uint64_t segs = std::max<uint64_t>(1, std::min<uint64_t>(segments, c->n_tiles));
  c->seg_tiles = std::max<uint64_t>(1, (c->n_tiles + segs - 1) / segs);
  c->n_segs = c->n_tiles ? (c->n_tiles + c->seg_tiles - 1) / c->seg_tiles : 1;
  const uint64_t n_chunks = (ds->n_rows + kCircChunkRows - 1) / kCircChunkRows;
  c->n_chunks = n_chunks;
  c->marks_stride = align4(n_chunks);
  // The widest union whose smallest rank group (32 queries) fits LDS.
  uint32_t mu = 0;
  while (mu < static_cast<uint32_t>(kMaxUnion) && rank_group_words(32, static_cast<int>(mu) + 1) * 4 <= rank_lds_room())
    ++mu;
  if (mu == 0) return fail(MDRQ_ENOTSUP, "circular scan: no rank group fits LDS");
  c->max_union = mu;
  c->dim_uses.assign(ds->n_dims, 0);
  for (uint32_t i = slots; i-- > 0;) c->free_slots.push_back(i);
  const uint64_t nw = n_words(ds);
  int rc = grow_device(&c->rows, &c->rows_len, slots * nw + slots * c->marks_stride / 4 + 1, "circular scan rows");
  if (rc) return rc;
  // Per slot a row of tile counts, then per slot a row of emit-chunk sums.
  rc = grow_device(&c->tile_counts, &c->tile_counts_len,
                   slots * (std::max<uint64_t>(1, c->n_tiles) + batch_emit_chunks(c->n_tiles)),
                   "circular scan tile counts");
  if (rc) return rc;
  // One count per workgroup of a single-query step (at most one workgroup per 4 tiles
  // and resident workgroups).
  rc = grow_device(&c->block_sums, &c->block_sums_len,
                   static_cast<uint64_t>(scan_blocks_per_cu(kStage, kCircPlainUnroll)) * device().cus + 1,
                   "circular scan workgroup counts");
  if (rc) return rc;
  // Per step buffer: the query tables of all groups (at most one per 32 slots), the
  // per-query arrays, two sets of output records, and the result records.
  const uint64_t groups = (slots + 31) / 32;
  const uint64_t blob = groups * rank_group_words(128, static_cast<int>(mu)) * 4 + slots * (16 + 2 * sizeof(BatchOut)) +
                        (2 * groups + 16) * 4 + 64;
  for (CircularScan::Step& s : c->steps) {
    rc = grow_pinned(&s.h_blob, &s.h_blob_bytes, blob);
    if (rc) return rc;
    rc = grow_device(reinterpret_cast<uint8_t**>(&s.d_blob), &s.d_blob_bytes, blob, "circular scan table");
    if (rc) return rc;
    if (hipHostMalloc(&s.h_res, static_cast<uint64_t>(slots) * 16, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer(&s.h_res_dev, s.h_res, 0) != hipSuccess)
      return fail(MDRQ_ENOMEM, "circular scan result records");
    MDRQ_HIP(hipEventCreate(&s.ev0), "hipEventCreate");
    MDRQ_HIP(hipEventCreate(&s.ev1), "hipEventCreate");
  }
  *out = c.release();
  return MDRQ_OK;
}

uint32_t circular_free_slots(const CircularScan* c) { return static_cast<uint32_t>(c->free_slots.size()); }
uint32_t circular_active(const CircularScan* c) { return static_cast<uint32_t>(c->items.size()); }
bool circular_busy(const CircularScan* c) {
  return !c->items.empty() || c->steps[0].inflight || c->steps[1].inflight || !c->answered.empty();
}

int circular_admit(CircularScan* c, const mdrq_query_t* q, mdrq_result_t* r, void* tag, hipStream_t stream,
                   bool* answered) {
  *answered = false;
  mdrq_dataset* ds = c->ds;
  // Predicates in the given order: a step's early break needs a whole 512-row chunk to
  // die for every query of a group, which estimated order was not measured to bring
  // about any sooner (its estimates cost a host round trip per step).
  Plan plan = make_plan(ds, q, r);
  const bool no_scan = plan.empty || ds->n_rows == 0;
  if (no_scan || plan.preds.size() > c->max_union) {
    if (r->mode == MDRQ_OUT_AUTO) {
      plan.mode = kIds;
      r->mode = MDRQ_OUT_IDS;
    }
    const int rc = no_scan ? finish_empty(ds, plan, r, stream) : run_query(ds, plan, r, stream);
    if (rc != MDRQ_OK && rc != MDRQ_EOVERFLOW) return rc;
    c->answered.push_back(tag);
    *answered = true;
    return MDRQ_OK;
  }
  uint32_t added = 0;
  for (uint32_t d : plan.dims) added += c->dim_uses[d] == 0 ? 1 : 0;
  if (c->free_slots.empty() || c->union_size + std::max<uint32_t>(added, c->union_size ? 0 : 1) > c->max_union)
    return MDRQ_EBUSY;
  for (uint32_t d : plan.dims) c->dim_uses[d] += 1;
  c->union_size += added;
  const uint32_t slot = c->free_slots.back();
  c->free_slots.pop_back();
  c->items.push_back(Item{0, std::move(plan), kind_of(r->mode), r, {}});
  c->meta.push_back(CircularScan::Meta{slot, c->n_segs, true, tag});
  return MDRQ_OK;
}

namespace {
// Drop the active query at position i: its slot is free again.
void circular_drop(CircularScan* c, size_t i) {
  for (uint32_t d : c->items[i].plan.dims)
    if (--c->dim_uses[d] == 0) c->union_size -= 1;
  c->free_slots.push_back(c->meta[i].slot);
  c->items.erase(c->items.begin() + static_cast<std::ptrdiff_t>(i));
  c->meta.erase(c->meta.begin() + static_cast<std::ptrdiff_t>(i));
}

// Build and enqueue the next step into its buffer (not waited for).  The queries that
// see their last segment in it leave the active list now; their results are read when
// the step is complete.
int circular_enqueue(CircularScan* c, CircularScan::Step& sb, hipStream_t stream) {
  mdrq_dataset* ds = c->ds;
  const uint64_t nq = c->items.size();
  const uint64_t nw = n_words(ds);
  const uint64_t t0 = c->cur * c->seg_tiles;
  const uint64_t t1 = std::min<uint64_t>(c->n_tiles, t0 + c->seg_tiles);

  std::vector<uint32_t> slot_dim = union_columns(ds, c->items);
  if (slot_dim.empty()) slot_dim.push_back(0);   // only queries without predicates
  std::vector<int> slot_of(ds->n_dims, -1);
  for (size_t i = 0; i < slot_dim.size(); ++i) slot_of[slot_dim[i]] = static_cast<int>(i);
  const int n_cols = static_cast<int>(slot_dim.size());
  uint64_t rank_group = std::min<uint64_t>(128, std::max<uint64_t>(nq, 1));
  while (rank_group > 32 && rank_group_words(rank_group, n_cols) * 4 > rank_lds_room()) rank_group /= 2;
  if (rank_group_words(rank_group, n_cols) * 4 > rank_lds_room())
    return fail(MDRQ_ENOTSUP, "circular scan: the union of columns does not fit LDS");
  const int rank_sw = rank_group <= 32 ? 1 : rank_group <= 64 ? 2 : 4;

  // Output records: every query writes its own slot's row, marks and tile counts.
  std::vector<BatchOut> outs(nq);
  std::vector<uint32_t> count_row(nq), fresh, fin_q;
  for (uint64_t q = 0; q < nq; ++q) {
    const CircularScan::Meta& m = c->meta[q];
    const Item& it = c->items[q];
    outs[q].kind = it.kind;
    outs[q].out_index = m.slot;
    outs[q].sparse = 0;
    outs[q].pad = 0;
    outs[q].buf = it.kind == kBatchCount ? nullptr : it.r->buf;
    outs[q].buf_bytes = it.kind == kBatchCount ? 0 : it.r->buf_bytes;
    count_row[q] = m.slot;
    if (m.fresh) fresh.push_back(m.slot);
    if (m.left == 1) fin_q.push_back(static_cast<uint32_t>(q));
  }
  // Few requests: each scans the step's tiles with the single-query scan (its early
  // break works per 4-row group, where the shared scan's needs a whole 512-row chunk to
  // die for every query), writing the same slot row, tile counts and marks; chosen by
  // the batched path's cost model for the step's rows.
  const uint64_t seg_rows =
      std::min<uint64_t>(ds->n_rows, t1 * kTileRows) - std::min<uint64_t>(ds->n_rows, t0 * kTileRows);
  bool plain = false;
  if (c->plain_steps) {
    std::vector<size_t> all(nq);
    for (uint64_t q = 0; q < nq; ++q) all[q] = q;
    plain = plain_is_cheaper(c->items, all, n_cols, seg_rows);
  }
  std::vector<uint32_t> table, group_first, group_table;
  uint64_t pairs = 0;
  int rc = MDRQ_OK;
  if (!plain) {
    rc = build_rank_tables(ds, c->items, outs, slot_of, n_cols, rank_group, rank_sw, table, group_first,
                           group_table, &pairs);
    if (rc) return rc;
  }
  const uint32_t n_groups = static_cast<uint32_t>(group_first.size());
  group_first.push_back(static_cast<uint32_t>(nq));
  group_table.push_back(static_cast<uint32_t>(table.size()));
  uint64_t max_group_words = 0;
  for (uint32_t g = 0; g < n_groups; ++g)
    max_group_words = std::max<uint64_t>(max_group_words, (group_table[g + 1] - group_table[g]) +
                                                              align4(group_first[g + 1] - group_first[g]));
  const uint32_t n_fin = static_cast<uint32_t>(fin_q.size());
  std::vector<uint32_t> fin_row(n_fin);
  std::vector<BatchOut> fin_outs(n_fin);
  for (uint32_t k = 0; k < n_fin; ++k) {
    fin_row[k] = count_row[fin_q[k]];
    fin_outs[k] = outs[fin_q[k]];
  }

  // Blob: table, group_first, group_table, count rows, fresh slots, finishing count
  // rows (uint32), then the output records of the scan and of the finish (16-aligned).
  const uint64_t o_gf = table.size(), o_gt = o_gf + group_first.size(), o_cr = o_gt + group_table.size();
  const uint64_t o_fr = o_cr + nq, o_fn = o_fr + fresh.size(), words_u32 = o_fn + n_fin;
  const uint64_t outs_off = (words_u32 * 4 + 15) / 16 * 16;
  const uint64_t fin_off = outs_off + nq * sizeof(BatchOut);
  const uint64_t blob = fin_off + n_fin * sizeof(BatchOut);
  rc = grow_pinned(&sb.h_blob, &sb.h_blob_bytes, blob);
  if (rc) return rc;
  rc = grow_device(reinterpret_cast<uint8_t**>(&sb.d_blob), &sb.d_blob_bytes, blob, "circular scan table");
  if (rc) return rc;
  uint32_t* hb = static_cast<uint32_t*>(sb.h_blob);
  std::memcpy(hb, table.data(), table.size() * 4);
  std::memcpy(hb + o_gf, group_first.data(), group_first.size() * 4);
  std::memcpy(hb + o_gt, group_table.data(), group_table.size() * 4);
  std::memcpy(hb + o_cr, count_row.data(), nq * 4);
  if (!fresh.empty()) std::memcpy(hb + o_fr, fresh.data(), fresh.size() * 4);
  if (n_fin) std::memcpy(hb + o_fn, fin_row.data(), n_fin * 4);
  std::memcpy(static_cast<uint8_t*>(sb.h_blob) + outs_off, outs.data(), nq * sizeof(BatchOut));
  if (n_fin) std::memcpy(static_cast<uint8_t*>(sb.h_blob) + fin_off, fin_outs.data(), n_fin * sizeof(BatchOut));
  const uint32_t* db = static_cast<const uint32_t*>(sb.d_blob);
  const uint8_t* dbb = static_cast<const uint8_t*>(sb.d_blob);

  uint64_t* marks = c->rows + static_cast<uint64_t>(c->n_slots) * nw;
  BatchParams bp{};
  bp.n_rows = ds->n_rows;
  bp.n_tiles = c->n_tiles;
  bp.tile_begin = t0;
  bp.tile_end = t1;
  bp.count_row = db + o_cr;
  bp.n_words = nw;
  bp.n_slots = static_cast<uint32_t>(n_cols);
  bp.table = db;
  bp.group_first = db + o_gf;
  bp.group_table = db + o_gt;
  bp.words = c->rows;
  bp.n_out = c->n_slots;
  bp.tile_counts = c->tile_counts;
  bp.flags = reinterpret_cast<uint16_t*>(marks);
  bp.n_chunks = c->marks_stride;
  bp.n_zero = 0;   // each slot's marks are cleared once, before its first step
  for (int sl = 0; sl < n_cols; ++sl) bp.slot_cols[sl] = ds->cols[slot_dim[sl]];
  BatchFinish fin{};
  fin.n_tiles = c->n_tiles;
  fin.n_words = nw;
  fin.words = c->rows;
  fin.flags = bp.flags;
  fin.n_chunks = c->marks_stride;
  fin.chunk_shift = static_cast<uint32_t>(__builtin_ctz(static_cast<unsigned>(kCircRg)));
  fin.tile_counts = c->tile_counts;
  fin.chunk_pos = c->tile_counts + static_cast<uint64_t>(c->n_slots) * std::max<uint64_t>(1, c->n_tiles);
  fin.count_row = db + o_fn;
  fin.outs = reinterpret_cast<const BatchOut*>(dbb + fin_off);
  fin.counts_out = static_cast<uint64_t*>(sb.h_res_dev);
  fin.kind_out = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(sb.h_res_dev) + static_cast<uint64_t>(c->n_slots) * 8);
  fin.over_out = nullptr;

  const size_t lds = max_group_words * 4;
  uint64_t gx = 1;
  if (!plain) {
    const int per_cu = batch_blocks_per_cu(n_cols, kCircWaves, kCircRg, 4, lds, rank_sw);
    const uint64_t resident = static_cast<uint64_t>(per_cu) * device().cus;
    gx = std::max<uint64_t>(1, std::min<uint64_t>(t1 - t0, resident / n_groups));
  }
  MDRQ_HIP(hipMemcpyAsync(sb.d_blob, sb.h_blob, blob, hipMemcpyHostToDevice, stream), "copy query table");
  MDRQ_HIP(hipEventRecord(sb.ev0, stream), "hipEventRecord");
  if (!fresh.empty())
    MDRQ_HIP(launch_zero_rows(marks, c->marks_stride / 4, db + o_fr, static_cast<uint32_t>(fresh.size()), stream),
             "clear chunk marks");
  if (t1 > t0 && plain) {
    // Per request one single-query scan over tiles [t0, t1) (4096-row tiles, as the
    // shared scan's), staging its bitmap words and tile counts straight into its slot;
    // then its marks for the step's chunks are set (every word of them was written).
    const uint64_t tiles = t1 - t0;
    const uint64_t per_cu = std::min<uint64_t>(static_cast<uint64_t>(scan_blocks_per_cu(kStage, kCircPlainUnroll)),
                                               static_cast<uint64_t>(std::max(1, ds->blocks_per_cu)));
    const uint64_t resident = per_cu * device().cus;
    const uint64_t want = std::min<uint64_t>((tiles + kWavesPerBlock - 1) / kWavesPerBlock, resident);
    const uint64_t seg = (tiles + want - 1) / want;
    const uint64_t grid = (tiles + seg - 1) / seg;
    const uint64_t c_beg = t0 * (kTileRows / kCircChunkRows);
    const uint64_t c_end = std::min<uint64_t>(t1 * (kTileRows / kCircChunkRows), c->n_chunks);
    for (uint64_t q = 0; q < nq; ++q) {
      const Plan& pl = c->items[q].plan;
      const uint32_t slot = c->meta[q].slot;
      ScanParams sp{};
      sp.n_rows = ds->n_rows;
      sp.n_tiles = t1;
      sp.tile_begin = t0;
      sp.n_preds = static_cast<uint32_t>(pl.preds.size());
      sp.early_out = pl.early_out ? 1u : 0u;
      sp.bitmap = c->rows + static_cast<uint64_t>(slot) * nw;
      sp.capacity = nw;
      sp.seg_tiles = seg;
      sp.tile_counts = c->tile_counts + static_cast<uint64_t>(slot) * c->n_tiles;
      sp.block_sums = c->block_sums;
      sp.order = nullptr;
      for (size_t i = 0; i < pl.preds.size(); ++i) sp.preds[i] = pl.preds[i];
      MDRQ_HIP(launch_scan(sp, kStage, kCircPlainUnroll, static_cast<int>(grid), stream), "circular scan: single-query step");
      MDRQ_HIP(launch_fill_u16(bp.flags + static_cast<uint64_t>(slot) * c->marks_stride + c_beg, c_end - c_beg,
                               static_cast<uint16_t>((1u << (kCircChunkRows / 64)) - 1), stream),
               "circular scan: chunk marks");
    }
  } else if (t1 > t0) {
    MDRQ_HIP(launch_batch_scan(bp, n_cols, kCircWaves, kCircRg, 4, dim3(static_cast<uint32_t>(gx), n_groups), lds, stream,
                               rank_sw),
             "circular scan launch");
  }
  if (n_fin) MDRQ_HIP(launch_batch_finish(fin, n_fin, stream), "circular scan finish");
  MDRQ_HIP(hipEventRecord(sb.ev1, stream), "hipEventRecord");

  sb.inflight = true;
  sb.seg_rows = seg_rows;
  sb.pairs = pairs;
  sb.plain_cols = 0;
  if (plain)
    for (const Item& it : c->items) sb.plain_cols += it.plan.preds.size();
  sb.fin.clear();
  for (uint32_t k = 0; k < n_fin; ++k) sb.fin.emplace_back(c->items[fin_q[k]].r, c->meta[fin_q[k]].tag);
  sb.extra.swap(c->answered);
  c->answered.clear();
  for (uint32_t k = n_fin; k-- > 0;) circular_drop(c, fin_q[k]);
  for (CircularScan::Meta& m : c->meta) {
    m.left -= 1;
    m.fresh = false;
  }
  c->cur = (c->cur + 1) % c->n_segs;
  return MDRQ_OK;
}

// Wait for an enqueued step and read the results of the queries it finished.
int circular_collect(CircularScan* c, CircularScan::Step& sb, std::vector<void*>& done, BatchRunStats* st) {
  mdrq_dataset* ds = c->ds;
  MDRQ_HIP(hipEventSynchronize(sb.ev1), "circular scan step");
  sb.inflight = false;
  float ms = 0.f;
  MDRQ_HIP(hipEventElapsedTime(&ms, sb.ev0, sb.ev1), "hipEventElapsedTime");
  {
    std::lock_guard<std::mutex> lock(ds->stat_mu);
    ds->batch_lookups += sb.seg_rows * sb.pairs;
    ds->batch_column_bytes += 4 * sb.seg_rows * (sb.pairs + sb.plain_cols);
    ds->batch_scan_ms += ms;
  }
  if (st) {
    st->scans += 1;
    st->column_bytes += 4 * sb.seg_rows * (sb.pairs + sb.plain_cols);
    st->device_ms += ms;
  }
  const uint64_t nw = n_words(ds);
  const volatile uint64_t* counts = static_cast<const volatile uint64_t*>(sb.h_res);
  const volatile uint32_t* kinds = reinterpret_cast<const volatile uint32_t*>(
      static_cast<const uint8_t*>(sb.h_res) + static_cast<uint64_t>(c->n_slots) * 8);
  for (size_t k = 0; k < sb.fin.size(); ++k) {
    mdrq_result_t* r = sb.fin[k].first;
    const uint64_t count = counts[k];
    const uint32_t kind = kinds[k];
    r->count = count;
    r->status = MDRQ_OK;
    r->written = 0;
    if (kind == kBatchCount) {
      r->mode = MDRQ_OUT_COUNT;
    } else if (kind == kBatchBitmap) {
      r->mode = MDRQ_OUT_BITMAP;
      const uint64_t cap = r->buf_bytes / 8;
      r->written = std::min(cap, nw);
      if (cap < nw) r->status = MDRQ_EOVERFLOW;
    } else {
      r->mode = MDRQ_OUT_IDS;
      const uint64_t cap = r->buf_bytes / 4;
      r->written = std::min(cap, count);
      if (count > cap) r->status = MDRQ_EOVERFLOW;
    }
    done.push_back(sb.fin[k].second);
  }
  for (void* t : sb.extra) done.push_back(t);
  sb.fin.clear();
  sb.extra.clear();
  return MDRQ_OK;
}
}  // namespace

int circular_step(CircularScan* c, hipStream_t stream, std::vector<void*>& done, BatchRunStats* st,
                  uint64_t* active_out) {
  if (active_out) *active_out = c->items.size();
  int rc = MDRQ_OK;
  bool enqueued = false;
  try {
    CircularScan::Step& mine = c->steps[c->next];
    CircularScan::Step& prev = c->steps[c->next ^ 1];
    if (!c->items.empty()) {
      rc = circular_enqueue(c, mine, stream);
      enqueued = rc == MDRQ_OK;
    }
    if (rc == MDRQ_OK && prev.inflight) rc = circular_collect(c, prev, done, st);
    if (rc == MDRQ_OK && enqueued && !c->pipelined) {
      rc = circular_collect(c, mine, done, st);
      enqueued = false;   // complete: the same buffer serves the next step
    }
    if (rc == MDRQ_OK && !enqueued && !c->answered.empty()) {
      // Answered at admission with no step to complete them: wait for the stream.
      const hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) {
        rc = fail_hip(e, "circular scan: stream synchronisation");
      } else {
        for (void* t : c->answered) done.push_back(t);
        c->answered.clear();
      }
    }
    if (enqueued) c->next ^= 1;
  } catch (...) {
    rc = fail(MDRQ_ENOMEM, "circular scan: host memory");
  }
  if (rc != MDRQ_OK) {
    // The slots are in an unknown state: wait for what was enqueued, then every query
    // in flight or active is dropped with the error in its result record.
    (void)hipStreamSynchronize(stream);
    for (CircularScan::Step& sb : c->steps) {
      for (auto& f : sb.fin) {
        f.first->status = rc;
        done.push_back(f.second);
      }
      for (void* t : sb.extra) done.push_back(t);
      sb.fin.clear();
      sb.extra.clear();
      sb.inflight = false;
    }
    for (void* t : c->answered) done.push_back(t);
    c->answered.clear();
    for (size_t i = 0; i < c->items.size(); ++i) {
      c->items[i].r->status = rc;
      done.push_back(c->meta[i].tag);
    }
    while (!c->items.empty()) circular_drop(c, c->items.size() - 1);
  }
  return rc;
}

int run_separately(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, mdrq_result_t* rs, hipStream_t stream,
                   const SingleScratch* scratch) {
  for (uint32_t i = 0; i < n; ++i) {
    Plan plan = make_plan(ds, &qs[i], &rs[i]);
    int rc;
    if (plan.empty || ds->n_rows == 0) {
      if (rs[i].mode == MDRQ_OUT_AUTO) {
        plan.mode = kIds;
        rs[i].mode = MDRQ_OUT_IDS;
      }
      rc = finish_empty(ds, plan, &rs[i], stream);
    } else {
      // Estimated order as mdrq_query takes it: ranked on the device ahead of the scan.
      std::unique_lock<std::mutex> est_hold;
      if (qs[i].flags & MDRQ_Q_ORDER_ESTIMATED) {
        rc = order_on_device(ds, &qs[i], plan, stream, est_hold);
        if (rc) return rc;
      }
      rs[i].mode = plan.mode == kBitmap ? MDRQ_OUT_BITMAP : plan.mode == kCount ? MDRQ_OUT_COUNT : MDRQ_OUT_IDS;
      rc = scratch ? run_query_on(ds, plan, &rs[i], stream, *scratch) : run_query(ds, plan, &rs[i], stream);
    }
    if (rc != MDRQ_OK && rc != MDRQ_EOVERFLOW) return rc;
  }
  return MDRQ_OK;
}

// Whether separate single-query scans answer these queries sooner than one shared scan
// (the model run_batch chooses by).
bool separate_scans_cheaper(const mdrq_dataset* ds, const mdrq_query_t* qs, const mdrq_result_t* rs, uint32_t n) {
  std::vector<Item> items;
  std::vector<size_t> members;
  std::vector<bool> in(ds->n_dims, false);
  int used = 0;
  for (uint32_t i = 0; i < n; ++i) {
    Plan plan = make_plan(ds, &qs[i], &rs[i]);
    if (plan.empty) continue;
    for (uint32_t d : plan.dims)
      if (!in[d]) {
        in[d] = true;
        ++used;
      }
    members.push_back(items.size());
    items.push_back(Item{i, std::move(plan), kind_of(rs[i].mode), nullptr, {}});
  }
  return members.empty() || plain_is_cheaper(items, members, std::max(used, 1), ds->n_rows);
}

}  // namespace mdrq
