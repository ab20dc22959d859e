// Serving loop: replay arrival-stamped requests with continuous batching.
//
// Requests are queued as they arrive.  Each of n_streams workers owns a device stream
// and a preallocated batch workspace holding an equal share of the result-memory
// budget.  Whenever a worker is idle and requests are waiting, the dispatcher hands it
// the oldest waiting requests, as many as max_batch allows and as fit in the worker's
// share (a request that needs a bitmap reserves one full bitmap row: its result can
// never need more), and the worker answers them with one call of the batched shared
// scan.  Requests that arrive while scans run wait for the next idle worker, so scans
// of different workers overlap on the device.  Every request's answer is exactly what
// mdrq_query gives for it alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <string>
#include <thread>
#include <vector>

#include "mdrq_internal.h"

using namespace mdrq;

namespace {

using Clock = std::chrono::steady_clock;

struct Worker {
  hipStream_t stream = nullptr;
  BatchWorkspace ws;
  std::thread th;
  std::vector<uint32_t> batch;  // request indices handed to this worker
  bool busy = false;
  uint64_t rows_cap = 0;        // bitmap rows the worker's share holds
};

struct Shared {
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  int error = MDRQ_OK;
  std::string error_msg;
  uint32_t done = 0;
  BatchRunStats st;
  uint64_t batches = 0;
};

uint64_t elapsed_ns(Clock::time_point t0) {
  return static_cast<uint64_t>(
      std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count());
}

bool needs_row(const mdrq_result_t& r) { return r.mode != MDRQ_OUT_COUNT; }

}  // namespace

extern "C" int mdrq_serve(mdrq_dataset* ds, const mdrq_serve_config_t* cfg, const mdrq_request_t* reqs,
                          uint32_t n_reqs, mdrq_result_t* rs, uint64_t* latency_ns,
                          mdrq_serve_stats_t* stats) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (!cfg || !reqs || !rs) return fail(MDRQ_EINVAL, "NULL argument");
  if (n_reqs == 0) return fail(MDRQ_EINVAL, "no requests");
  if (cfg->max_batch == 0 || cfg->max_batch > MDRQ_MAX_BATCH)
    return fail(MDRQ_EINVAL, "max_batch must be in 1..MDRQ_MAX_BATCH");
  if (cfg->n_streams == 0 || cfg->n_streams > 8) return fail(MDRQ_EINVAL, "n_streams must be in 1..8");
  for (uint32_t i = 0; i < n_reqs; ++i) {
    int rc = check_query(ds, &reqs[i].query);
    if (rc) return rc;
    rc = check_result(&rs[i]);
    if (rc) return rc;
    if (needs_row(rs[i]) && rs[i].mem != MDRQ_MEM_DEVICE)
      return fail(MDRQ_EINVAL, "serving writes results to device memory only (mem = MDRQ_MEM_DEVICE)");
  }
  std::lock_guard<std::mutex> lock(ds->mu);
  if (cfg->use_estimator && !ds->estimator)
    return fail(MDRQ_EINVAL, "use_estimator needs an attached estimator");

  const uint64_t row_bytes = 8 * n_words(ds);
  const uint64_t share = cfg->result_budget_bytes / cfg->n_streams;
  const uint64_t rows_cap = row_bytes ? share / row_bytes : cfg->max_batch;
  bool any_row = false;
  for (uint32_t i = 0; i < n_reqs; ++i) any_row |= needs_row(rs[i]);
  if (any_row && rows_cap == 0)
    return fail(MDRQ_EBUSY, "a request's bitmap row does not fit in one stream's share of the result budget");

  // Arrival order (stable for equal stamps).
  std::vector<uint32_t> order(n_reqs);
  for (uint32_t i = 0; i < n_reqs; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return reqs[a].arrival_ns < reqs[b].arrival_ns; });

  // Workers with their own stream and preallocated workspace.
  std::vector<Worker> workers(cfg->n_streams);
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto cleanup = [&]() {
    for (Worker& w : workers) {
      free_batch(w.ws);
      if (w.stream) (void)hipStreamDestroy(w.stream);
    }
  };
  for (Worker& w : workers) {
    w.rows_cap = std::min<uint64_t>(rows_cap, cfg->max_batch);
    hipError_t e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      cleanup();
      return fail_hip(e, "serving stream");
    }
    int rc = reserve_batch(ds, w.ws, cfg->max_batch, any_row ? w.rows_cap : 0);
    if (rc) {
      cleanup();
      return rc;
    }
  }

  std::vector<uint64_t> done_ns(n_reqs, 0);
  std::vector<mdrq_query_t> qcopy(n_reqs);
  for (uint32_t i = 0; i < n_reqs; ++i) {
    qcopy[i] = reqs[i].query;
    if (cfg->use_estimator) qcopy[i].flags |= MDRQ_Q_ORDER_ESTIMATED;
  }
  Shared sh;
  const Clock::time_point t0 = Clock::now();

  auto work = [&](Worker* w) {
    (void)hipSetDevice(dev);
    std::vector<mdrq_query_t> qs;
    std::vector<mdrq_result_t> out;
    for (;;) {
      std::vector<uint32_t> batch;
      {
        std::unique_lock<std::mutex> lk(sh.mu);
        sh.cv.wait(lk, [&] { return sh.stop || !w->batch.empty(); });
        if (w->batch.empty()) return;
        batch.swap(w->batch);
      }
      qs.clear();
      out.clear();
      for (uint32_t i : batch) {
        qs.push_back(qcopy[i]);
        out.push_back(rs[i]);
      }
      BatchRunStats st;
      int rc = run_batch(ds, qs.data(), static_cast<uint32_t>(qs.size()), out.data(), w->stream,
                         &w->ws, false, &st);
      const uint64_t t = elapsed_ns(t0);
      std::string msg = rc ? mdrq_last_error() : "";
      std::lock_guard<std::mutex> lk(sh.mu);
      if (rc && rc != MDRQ_EOVERFLOW && sh.error == MDRQ_OK) {
        sh.error = rc;
        sh.error_msg = msg;
      }
      for (size_t k = 0; k < batch.size(); ++k) {
        rs[batch[k]] = out[k];
        done_ns[batch[k]] = t;
      }
      sh.done += static_cast<uint32_t>(batch.size());
      sh.st.scans += st.scans;
      sh.st.column_bytes += st.column_bytes;
      sh.st.device_ms += st.device_ms;
      sh.batches += 1;
      w->busy = false;
      sh.cv.notify_all();
    }
  };
  for (Worker& w : workers) w.th = std::thread(work, &w);

  // Dispatcher.
  {
    std::deque<uint32_t> ready;
    uint32_t next = 0;
    std::unique_lock<std::mutex> lk(sh.mu);
    while (sh.done < n_reqs && sh.error == MDRQ_OK) {
      const uint64_t now = elapsed_ns(t0);
      while (next < n_reqs && reqs[order[next]].arrival_ns <= now) ready.push_back(order[next++]);
      Worker* idle = nullptr;
      for (Worker& w : workers)
        if (!w.busy) {
          idle = &w;
          break;
        }
      if (idle && !ready.empty()) {
        uint64_t rows = 0;
        while (!ready.empty() && idle->batch.size() < cfg->max_batch) {
          const uint32_t i = ready.front();
          const uint64_t need = needs_row(rs[i]) ? 1 : 0;
          if (rows + need > idle->rows_cap) break;
          rows += need;
          idle->batch.push_back(i);
          ready.pop_front();
        }
        idle->busy = true;
        sh.cv.notify_all();
        continue;
      }
      if (next < n_reqs && (idle || ready.empty())) {
        const auto wake = t0 + std::chrono::nanoseconds(reqs[order[next]].arrival_ns);
        sh.cv.wait_until(lk, wake);
      } else {
        sh.cv.wait(lk);
      }
    }
    // Drain: let running batches finish, then stop the workers.
    sh.cv.wait(lk, [&] {
      for (Worker& w : workers)
        if (w.busy) return false;
      return true;
    });
    sh.stop = true;
    sh.cv.notify_all();
  }
  for (Worker& w : workers) w.th.join();
  cleanup();
  if (sh.error != MDRQ_OK) return fail(sh.error, "serving: " + sh.error_msg);

  // Latencies and statistics.
  std::vector<uint64_t> lat(n_reqs);
  uint64_t first = UINT64_MAX, last = 0;
  bool overflow = false;
  for (uint32_t i = 0; i < n_reqs; ++i) {
    lat[i] = done_ns[i] > reqs[i].arrival_ns ? done_ns[i] - reqs[i].arrival_ns : 0;
    if (latency_ns) latency_ns[i] = lat[i];
    first = std::min(first, reqs[i].arrival_ns);
    last = std::max(last, done_ns[i]);
    overflow |= rs[i].status == MDRQ_EOVERFLOW;
  }
  if (stats) {
    std::vector<uint64_t> sorted = lat;
    std::sort(sorted.begin(), sorted.end());
    auto pct = [&](double p) {
      const size_t k = static_cast<size_t>(std::min<double>(n_reqs - 1, std::floor(p * (n_reqs - 1) + 0.5)));
      return sorted[k] * 1e-3;
    };
    double sum = 0.0;
    for (uint64_t v : lat) sum += static_cast<double>(v);
    std::memset(stats, 0, sizeof(*stats));
    stats->completed = n_reqs;
    stats->scans = sh.st.scans;
    stats->wall_s = static_cast<double>(last > first ? last - first : 0) * 1e-9;
    stats->qps = stats->wall_s > 0 ? n_reqs / stats->wall_s : 0.0;
    stats->p50_us = pct(0.50);
    stats->p99_us = pct(0.99);
    stats->mean_us = sum / n_reqs * 1e-3;
    stats->max_us = sorted.back() * 1e-3;
    stats->mean_batch = sh.batches ? static_cast<double>(n_reqs) / sh.batches : 0.0;
    stats->hbm_gbps = stats->wall_s > 0 ? sh.st.column_bytes / stats->wall_s * 1e-9 : 0.0;
    stats->overflow_reruns = 0;
  }
  return overflow ? MDRQ_EOVERFLOW : MDRQ_OK;
}
