// Serving loop with continuous batching: a live server (open / submit / poll / close)
// and the replay of arrival-stamped requests built on it.
//
// Requests wait in a queue in submission order.  Each of n_streams workers owns a
// device stream and a preallocated batch workspace holding an equal share of the
// result-memory budget.  Whenever a worker is idle and requests are waiting, the
// dispatcher hands it the oldest waiting requests, as many as max_batch allows and as
// fit in the worker's share of scratch memory, and the worker answers them with one
// call of the batched shared scan.  A request that needs identifiers or a bitmap
// reserves a full bitmap row (its result can never need more), or, with estimated sizing
// (use_estimator bit 1), room for about four times its estimated result in the scan's sparse
// scratch: the dispatcher estimates waiting requests in bulk before admitting them, and
// a request whose result outgrows its room is answered again by the single-query scan.
// Requests that arrive while scans run wait for the next idle worker, so scans of
// different workers overlap on the device.  In circular-scan mode each worker instead
// keeps one shared scan running over the data, a segment of rows per step, and admits
// waiting requests between steps (circular_worker_loop).  Every request's answer is
// exactly what mdrq_query gives for it alone.
#include <algorithm>
#include <chrono>
#include <cmath>
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

// One queued request: a private copy of the query, the caller's result record, and an
// event recorded on the caller's stream at submission (null for the replay): the
// worker's stream waits for it, so the scan writes the result buffer only after the
// work the caller queued before submitting.
struct Pending {
  uint64_t ticket = 0;
  mdrq_query_t q{};
  std::vector<mdrq_pred> preds;
  mdrq_result_t* r = nullptr;
  Clock::time_point arrival;
  hipEvent_t ready = nullptr;
  std::vector<float> est;       // the estimator's estimates (n_dims + 1), when used
  bool estimated = false;
  mdrq_result_t res{};          // circular scan: the result, copied to *r when complete
};

struct Worker {
  hipStream_t stream = nullptr;
  BatchWorkspace ws;
  std::thread th;
  std::vector<Pending*> batch;  // handed to this worker by the dispatcher
  bool busy = false;
  CircularScan* circ = nullptr; // circular-scan mode: this worker's scan
};

bool needs_row(const mdrq_result_t& r) { return r.mode != MDRQ_OUT_COUNT; }

// Circular scan: most waiting requests an idle worker answers by separate scans.
constexpr size_t kSeparateMax = 4;

}  // namespace

struct mdrq_server {
  mdrq_dataset* ds = nullptr;
  mdrq_serve_config_t cfg{};
  uint64_t share = 0;           // scratch bytes of one worker's share of the budget
  int dev = 0;
  std::vector<Worker> workers;
  std::thread dispatcher;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending*> ready;
  bool closing = false;         // no more submissions; drain, then stop
  bool stop = false;            // workers exit
  int error = MDRQ_OK;
  std::string error_msg;
  uint64_t next_ticket = 0;
  uint64_t completed = 0;
  std::vector<uint64_t> done;   // completed tickets not yet polled
  std::vector<uint64_t> lat_ns; // per ticket: arrival -> completion
  Clock::time_point first_arrival{}, last_done{};
  BatchRunStats st;
  uint64_t batches = 0;
  uint64_t active_sum = 0;      // circular scan: active requests summed over steps
  bool separate_when_idle = false;  // circular scan: MDRQ_OPT_CIRCULAR bit 1
  bool overflow = false;
  std::vector<hipEvent_t> free_events;  // submission events for reuse (mu)
};

namespace {

// Under the server's lock: the first error is kept for the callers.
void record_error(mdrq_server* s, int rc, const std::string& msg) {
  if (s->error != MDRQ_OK) return;
  s->error = rc;
  s->error_msg = msg;
}

// Under the server's lock: request p is answered with `res` at time t.
void complete(mdrq_server* s, Pending* p, const mdrq_result_t& res, Clock::time_point t) {
  *p->r = res;
  s->overflow |= res.status == MDRQ_EOVERFLOW;
  if (s->lat_ns.size() <= p->ticket) s->lat_ns.resize(p->ticket + 1, 0);
  s->lat_ns[p->ticket] = static_cast<uint64_t>(
      std::max<int64_t>(0, std::chrono::duration_cast<std::chrono::nanoseconds>(t - p->arrival).count()));
  s->done.push_back(p->ticket);
  if (p->ready) s->free_events.push_back(p->ready);
  delete p;
  s->completed += 1;
  s->last_done = t;
}

void worker_loop(mdrq_server* s, Worker* w) {
  (void)hipSetDevice(s->dev);
  std::vector<mdrq_query_t> qs;
  std::vector<mdrq_result_t> out;
  std::vector<float> est;
  for (;;) {
    std::vector<Pending*> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !w->batch.empty(); });
      if (w->batch.empty()) return;
      batch.swap(w->batch);
    }
    qs.clear();
    out.clear();
    est.clear();
    int rc = MDRQ_OK;
    bool all_est = true;
    for (Pending* p : batch) all_est &= !p->est.empty();
    for (Pending* p : batch) {
      qs.push_back(p->q);
      out.push_back(*p->r);
      if (all_est) est.insert(est.end(), p->est.begin(), p->est.end());
      if (p->ready && rc == MDRQ_OK) {
        const hipError_t e = hipStreamWaitEvent(w->stream, p->ready, 0);
        if (e != hipSuccess) rc = fail_hip(e, "serving: wait for the submitting stream");
      }
    }
    BatchRunStats st;
    if (rc == MDRQ_OK) {
      try {
        rc = run_batch(s->ds, qs.data(), static_cast<uint32_t>(qs.size()), out.data(), w->stream,
                       &w->ws, false, &st, est.empty() ? nullptr : est.data());
      } catch (...) {
        rc = fail(MDRQ_ENOMEM, "serving: host memory");
      }
    }
    const Clock::time_point t = Clock::now();
    std::string msg = rc ? mdrq_last_error() : "";
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc && rc != MDRQ_EOVERFLOW) record_error(s, rc, msg);
    for (size_t k = 0; k < batch.size(); ++k) {
      if (rc && rc != MDRQ_EOVERFLOW) out[k].status = rc;
      complete(s, batch[k], out[k], t);
    }
    s->st.scans += st.scans;
    s->st.column_bytes += st.column_bytes;
    s->st.device_ms += st.device_ms;
    s->st.sparse += st.sparse;
    s->st.reruns += st.reruns;
    s->batches += 1;
    w->busy = false;
    s->cv.notify_all();
  }
}

// Circular-scan worker: between steps it admits waiting requests (oldest first, as many
// as it has free slots and as keep the union of columns within one scan), then runs the
// next step and completes the requests whose pass it closed (with pipelined steps: those
// of the step before).  A request waits about one step (two) before its scan starts, and
// its scan takes one pass.  Optionally (MDRQ_OPT_CIRCULAR bit 1), when the worker is idle
// and the waiting requests are few enough that separate single-query scans are cheaper
// than a pass (the batched path's cost model), it answers them that way instead of
// starting a pass.  The worker ends once the server is closing and nothing waits or is
// in flight.
void circular_worker_loop(mdrq_server* s, Worker* w) {
  (void)hipSetDevice(s->dev);
  CircularScan* c = w->circ;
  std::vector<Pending*> take, answered;
  std::vector<void*> done;
  std::vector<mdrq_query_t> qs;
  std::vector<mdrq_result_t> rs;
  for (;;) {
    take.clear();
    bool separate = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (!circular_busy(c)) {
        s->cv.wait(lk, [&] { return s->closing || !s->ready.empty(); });
        if (s->ready.empty()) return;
        // Idle: up to kSeparateMax waiting requests by separate scans if that is cheaper
        // than a pass for them.  (The cost model prices a scan's column bytes, not its
        // output; capped so, a run of large-result scans cannot hold the others long.)
        const size_t n = s->separate_when_idle && s->ready.size() <= kSeparateMax ? s->ready.size() : 0;
        qs.clear();
        rs.clear();
        for (size_t i = 0; i < n; ++i) {
          qs.push_back(s->ready[i]->q);
          rs.push_back(s->ready[i]->res);
        }
        try {
          separate = n && separate_scans_cheaper(s->ds, qs.data(), rs.data(), static_cast<uint32_t>(n));
        } catch (...) {
        }
        if (separate)
          for (size_t i = 0; i < n; ++i) {
            take.push_back(s->ready.front());
            s->ready.pop_front();
          }
      }
      const uint32_t room = separate ? 0 : circular_free_slots(c);
      while (!s->ready.empty() && take.size() < room) {
        take.push_back(s->ready.front());
        s->ready.pop_front();
      }
    }
    if (separate) {
      int rc = MDRQ_OK;
      for (Pending* p : take)
        if (p->ready && rc == MDRQ_OK) {
          const hipError_t e = hipStreamWaitEvent(w->stream, p->ready, 0);
          if (e != hipSuccess) rc = fail_hip(e, "serving: wait for the submitting stream");
        }
      if (rc == MDRQ_OK) {
        // Each alone (not through the batched path, whose shared scans would grow this
        // worker's batch workspace, unused in circular mode, by allocating).
        try {
          rc = run_separately(s->ds, qs.data(), static_cast<uint32_t>(qs.size()), rs.data(), w->stream,
                              &w->ws.single);
        } catch (...) {
          rc = fail(MDRQ_ENOMEM, "serving: host memory");
        }
      }
      const Clock::time_point t = Clock::now();
      const std::string msg = rc ? mdrq_last_error() : "";
      std::lock_guard<std::mutex> lk(s->mu);
      if (rc && rc != MDRQ_EOVERFLOW) record_error(s, rc, msg);
      for (size_t k = 0; k < take.size(); ++k) {
        if (rc && rc != MDRQ_EOVERFLOW) rs[k].status = rc;
        complete(s, take[k], rs[k], t);
      }
      s->st.alone += take.size();
      s->cv.notify_all();
      continue;
    }
    answered.clear();
    size_t k = 0;
    for (; k < take.size(); ++k) {
      Pending* p = take[k];
      int rc = MDRQ_OK;
      if (p->ready) {
        const hipError_t e = hipStreamWaitEvent(w->stream, p->ready, 0);
        if (e != hipSuccess) rc = fail_hip(e, "serving: wait for the submitting stream");
      }
      bool now = false;
      if (rc == MDRQ_OK) {
        try {
          rc = circular_admit(c, &p->q, &p->res, p, w->stream, &now);
        } catch (...) {
          rc = fail(MDRQ_ENOMEM, "serving: host memory");
        }
        if (rc == MDRQ_EBUSY) break;   // its columns would widen the union too far: it waits
      }
      if (rc != MDRQ_OK) {
        const std::string msg = mdrq_last_error();
        p->res.status = rc;
        std::lock_guard<std::mutex> lk(s->mu);
        record_error(s, rc, msg);
      }
      // (one answered at admission is reported by a later step, with the stream's work)
      if (rc != MDRQ_OK) answered.push_back(p);
    }
    if (k < take.size()) {
      std::lock_guard<std::mutex> lk(s->mu);
      for (size_t j = take.size(); j-- > k;) s->ready.push_front(take[j]);
    }
    done.clear();
    uint64_t active = 0;
    BatchRunStats st;
    const int rc = circular_step(c, w->stream, done, &st, &active);
    const std::string msg = rc ? mdrq_last_error() : "";
    const Clock::time_point t = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc) record_error(s, rc, msg);
    for (Pending* p : answered) complete(s, p, p->res, t);
    for (void* tag : done) {
      Pending* p = static_cast<Pending*>(tag);
      complete(s, p, p->res, t);
    }
    s->st.scans += st.scans;
    s->st.column_bytes += st.column_bytes;
    s->st.device_ms += st.device_ms;
    if (active) {
      s->batches += 1;
      s->active_sum += active;
    }
    s->cv.notify_all();
  }
}

// Estimates of the waiting requests not yet estimated, in one call (the server's lock is
// released meanwhile; only the dispatcher takes requests off the queue).
void estimate_waiting(mdrq_server* s, std::unique_lock<std::mutex>& lk) {
  std::vector<Pending*> todo;
  for (Pending* p : s->ready)
    if (!p->estimated) todo.push_back(p);
  if (todo.empty()) return;
  std::vector<mdrq_query_t> qs;
  for (Pending* p : todo) qs.push_back(p->q);
  lk.unlock();
  std::vector<float> est;
  const int rc = estimate_for_order(s->ds, qs.data(), static_cast<uint32_t>(qs.size()), est);
  lk.lock();
  const size_t o = s->ds->n_dims + 1;
  for (size_t i = 0; i < todo.size(); ++i) {
    todo[i]->estimated = true;
    if (rc == MDRQ_OK && est.size() == todo.size() * o)
      todo[i]->est.assign(est.begin() + i * o, est.begin() + (i + 1) * o);
  }
}

void dispatch_loop(mdrq_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  const double n_rows = static_cast<double>(s->ds->n_rows);
  for (;;) {
    Worker* idle = nullptr;
    bool any_busy = false;
    for (Worker& w : s->workers) {
      if (!w.busy && !idle) idle = &w;
      any_busy |= w.busy;
    }
    if (idle && !s->ready.empty()) {
      if (s->cfg.use_estimator & 2u) estimate_waiting(s, lk);
      uint64_t bytes = 0;
      while (!s->ready.empty() && idle->batch.size() < s->cfg.max_batch) {
        Pending* p = s->ready.front();
        const double est_rows = p->est.empty() ? -1.0 : p->est[s->ds->n_dims] * n_rows;
        const uint64_t need = request_scratch_bytes(s->ds, *p->r, est_rows);
        if (bytes + need > s->share) break;
        bytes += need;
        idle->batch.push_back(p);
        s->ready.pop_front();
      }
      idle->busy = true;
      s->cv.notify_all();
      continue;
    }
    if (s->closing && s->ready.empty() && !any_busy) break;
    s->cv.wait(lk);
  }
  s->stop = true;
  s->cv.notify_all();
}

// Validation shared by the live server and the replay.
int check_config(const mdrq_dataset* ds, const mdrq_serve_config_t* cfg) {
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (!cfg) return fail(MDRQ_EINVAL, "NULL argument");
  if (cfg->max_batch == 0 || cfg->max_batch > MDRQ_MAX_BATCH)
    return fail(MDRQ_EINVAL, "max_batch must be in 1..MDRQ_MAX_BATCH");
  if (cfg->n_streams == 0 || cfg->n_streams > 8) return fail(MDRQ_EINVAL, "n_streams must be in 1..8");
  if (cfg->use_estimator > 3) return fail(MDRQ_EINVAL, "use_estimator must be 0..3");
  if (cfg->segments > 4096) return fail(MDRQ_EINVAL, "segments must be 0..4096");
  if (cfg->segments && (cfg->use_estimator & 2u))
    return fail(MDRQ_EINVAL, "the circular scan keeps full bitmap rows: use_estimator bit 1 does not apply");
  if (cfg->use_estimator && !ds->estimator)
    return fail(MDRQ_EINVAL, "use_estimator needs an attached estimator");
  return MDRQ_OK;
}

int check_request(const mdrq_server* s, const mdrq_query_t* q, const mdrq_result_t* r) {
  int rc = check_query(s->ds, q);
  if (rc) return rc;
  rc = check_result(r);
  if (rc) return rc;
  if (needs_row(*r) && r->mem != MDRQ_MEM_DEVICE)
    return fail(MDRQ_EINVAL, "serving writes results to device memory only (mem = MDRQ_MEM_DEVICE)");
  if (request_scratch_bytes(s->ds, *r, -1.0) > s->share)
    return fail(MDRQ_EBUSY, "a request's bitmap row does not fit in one stream's share of the result budget");
  return MDRQ_OK;
}

void destroy(mdrq_server* s) {
  for (Worker& w : s->workers) {
    free_batch(w.ws);
    circular_destroy(w.circ);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  for (Pending* p : s->ready) {
    if (p->ready) (void)hipEventDestroy(p->ready);
    delete p;
  }
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  delete s;
}

// Create the workers and the dispatcher.  `reserve_rows`: reserve the scratch up front.
int create(mdrq_dataset* ds, const mdrq_serve_config_t* cfg, bool reserve_rows, mdrq_server** out) {
  mdrq_server* s = new mdrq_server();
  s->ds = ds;
  s->cfg = *cfg;
  s->share = cfg->result_budget_bytes / cfg->n_streams;
  s->separate_when_idle = (ds->circular_mode & 2) != 0;
  (void)hipGetDevice(&s->dev);
  s->workers.resize(cfg->n_streams);
  for (Worker& w : s->workers) {
    hipError_t e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      destroy(s);
      return fail_hip(e, "serving stream");
    }
    int rc = MDRQ_OK;
    if (cfg->segments) {
      // Circular scan: as many query slots as the share holds, at most max_batch.
      // (An empty dataset's slots take no memory.)
      const uint64_t slot_bytes = circular_slot_bytes(ds);
      const uint64_t slots = slot_bytes ? std::min<uint64_t>(cfg->max_batch, s->share / slot_bytes) : cfg->max_batch;
      rc = slots ? circular_create(ds, static_cast<uint32_t>(slots), cfg->segments, &w.circ)
                 : fail(MDRQ_EBUSY, "one query slot of the circular scan does not fit in one stream's share of the result budget");
    } else {
      // At most max_batch bitmap rows are ever used by one batch.
      const uint64_t row = request_scratch_bytes(ds, mdrq_result_t{MDRQ_OUT_IDS, 0, nullptr, 0, 0, 0, 0, 0}, -1.0);
      const uint64_t bytes = std::min<uint64_t>(s->share, row * cfg->max_batch);
      rc = reserve_batch(ds, w.ws, cfg->max_batch, reserve_rows ? bytes : 0);
    }
    // Its own single-query scratch, so workers' single-query scans do not wait for
    // each other.
    if (rc == MDRQ_OK) rc = reserve_single(ds, w.ws.single);
    if (rc) {
      destroy(s);
      return rc;
    }
  }
  for (Worker& w : s->workers) w.th = std::thread(cfg->segments ? circular_worker_loop : worker_loop, s, &w);
  if (!cfg->segments) s->dispatcher = std::thread(dispatch_loop, s);
  *out = s;
  return MDRQ_OK;
}

// Queue one request (caller holds no lock).  arrival: the time its latency counts from.
// order: record an event on `stream` that the request's scan waits for.
int enqueue(mdrq_server* s, const mdrq_query_t* q, mdrq_result_t* r, Clock::time_point arrival,
            bool bounded, bool order, hipStream_t stream, uint64_t* ticket) {
  Pending* p = new Pending();
  p->q = *q;
  p->preds.assign(q->preds, q->preds + q->n_preds);
  p->q.preds = p->preds.data();
  if (s->cfg.use_estimator & 1u) p->q.flags |= MDRQ_Q_ORDER_ESTIMATED;
  if (s->cfg.use_estimator & 2u) p->q.flags |= MDRQ_Q_SIZE_ESTIMATED;
  p->r = r;
  p->res = *r;
  p->arrival = arrival;
  if (order) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (!s->free_events.empty()) {
        p->ready = s->free_events.back();
        s->free_events.pop_back();
      }
    }
    hipError_t e = p->ready ? hipSuccess : hipEventCreateWithFlags(&p->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(p->ready, stream);
    if (e != hipSuccess) {
      if (p->ready) (void)hipEventDestroy(p->ready);
      delete p;
      return fail_hip(e, "serving: event on the submitting stream");
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto reject = [&](int code, const std::string& msg) {
    if (p->ready) s->free_events.push_back(p->ready);
    delete p;
    return fail(code, msg);
  };
  if (s->closing) return reject(MDRQ_EINVAL, "server is closing");
  if (s->error != MDRQ_OK) return reject(s->error, "serving: " + s->error_msg);
  if (bounded && s->cfg.max_queue && s->ready.size() >= s->cfg.max_queue)
    return reject(MDRQ_EBUSY, "serving queue is full");
  if (s->next_ticket == 0 || arrival < s->first_arrival) s->first_arrival = arrival;
  p->ticket = s->next_ticket++;
  if (ticket) *ticket = p->ticket;
  s->ready.push_back(p);
  s->cv.notify_all();
  return MDRQ_OK;
}

// Drain and stop; summary statistics over every request answered.
int shutdown(mdrq_server* s, mdrq_serve_stats_t* stats) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->closing = true;
    s->cv.notify_all();
  }
  if (s->dispatcher.joinable()) s->dispatcher.join();
  for (Worker& w : s->workers) w.th.join();
  const int err = s->error;
  const std::string msg = s->error_msg;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    const uint64_t n = s->completed;
    std::vector<uint64_t> sorted(s->lat_ns.begin(), s->lat_ns.begin() + std::min<uint64_t>(n, s->lat_ns.size()));
    std::sort(sorted.begin(), sorted.end());
    auto pct = [&](double p) {
      const size_t k = static_cast<size_t>(std::min<double>(sorted.size() - 1, std::floor(p * (sorted.size() - 1) + 0.5)));
      return sorted[k] * 1e-3;
    };
    stats->completed = n;
    stats->scans = s->st.scans;
    if (!sorted.empty()) {
      double sum = 0.0;
      for (uint64_t v : sorted) sum += static_cast<double>(v);
      stats->wall_s = std::max(0.0, std::chrono::duration<double>(s->last_done - s->first_arrival).count());
      stats->qps = stats->wall_s > 0 ? n / stats->wall_s : 0.0;
      stats->p50_us = pct(0.50);
      stats->p99_us = pct(0.99);
      stats->mean_us = sum / sorted.size() * 1e-3;
      stats->max_us = sorted.back() * 1e-3;
    }
    stats->mean_batch = !s->batches ? 0.0
                        : s->cfg.segments ? static_cast<double>(s->active_sum) / s->batches
                                          : static_cast<double>(n) / s->batches;
    stats->hbm_gbps = stats->wall_s > 0 ? s->st.column_bytes / stats->wall_s * 1e-9 : 0.0;
    stats->overflow_reruns = s->st.reruns;
    stats->sized_by_estimate = s->st.sparse;
  }
  const bool overflow = s->overflow;
  {
    std::lock_guard<std::mutex> lk(s->ds->stat_mu);
    auto& v = s->ds->servers;
    v.erase(std::remove(v.begin(), v.end(), s), v.end());
  }
  destroy(s);
  if (err != MDRQ_OK) return fail(err, "serving: " + msg);
  return overflow ? MDRQ_EOVERFLOW : MDRQ_OK;
}

}  // namespace

namespace mdrq {
void close_servers(mdrq_dataset* ds) {
  for (;;) {
    mdrq_server* s = nullptr;
    {
      std::lock_guard<std::mutex> lk(ds->stat_mu);
      if (ds->servers.empty()) return;
      s = ds->servers.back();
    }
    (void)shutdown(s, nullptr);
  }
}
}  // namespace mdrq

extern "C" int mdrq_serve_open(mdrq_dataset* ds, const mdrq_serve_config_t* cfg, mdrq_server** out) {
  return guarded([&]() -> int {
    clear_error();
    if (!out) return fail(MDRQ_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = check_config(ds, cfg);
    if (rc) return rc;
    rc = create(ds, cfg, true, out);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ds->stat_mu);
    ds->servers.push_back(*out);
    return MDRQ_OK;
  });
}

extern "C" int mdrq_serve_submit(mdrq_server* s, const mdrq_query_t* q, mdrq_result_t* r,
                                 void* stream, uint64_t* ticket) {
  return guarded([&]() -> int {
    clear_error();
    if (!s || !q || !r) return fail(MDRQ_EINVAL, "NULL argument");
    int rc = check_request(s, q, r);
    if (rc) return rc;
    return enqueue(s, q, r, Clock::now(), true, true, static_cast<hipStream_t>(stream), ticket);
  });
}

extern "C" int mdrq_serve_poll(mdrq_server* s, uint64_t* tickets, uint32_t max_tickets,
                               uint32_t* n_out, uint64_t wait_ns) {
  clear_error();
  if (!s || !n_out || (max_tickets && !tickets)) return fail(MDRQ_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait_ns && s->done.empty() && s->error == MDRQ_OK)
    s->cv.wait_for(lk, std::chrono::nanoseconds(wait_ns),
                   [&] { return !s->done.empty() || s->error != MDRQ_OK; });
  const size_t n = std::min<size_t>(max_tickets, s->done.size());
  std::copy(s->done.begin(), s->done.begin() + n, tickets);
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *n_out = static_cast<uint32_t>(n);
  if (s->error != MDRQ_OK) return fail(s->error, "serving: " + s->error_msg);
  return MDRQ_OK;
}

extern "C" int mdrq_serve_close(mdrq_server* s, mdrq_serve_stats_t* stats) {
  clear_error();
  if (!s) return fail(MDRQ_EINVAL, "server is NULL");
  return shutdown(s, stats);
}

extern "C" int mdrq_serve(mdrq_dataset* ds, const mdrq_serve_config_t* cfg, const mdrq_request_t* reqs,
                          uint32_t n_reqs, mdrq_result_t* rs, uint64_t* latency_ns,
                          mdrq_serve_stats_t* stats) {
  return guarded([&]() -> int {
    clear_error();
    int rc = check_config(ds, cfg);
    if (rc) return rc;
    if (!reqs || !rs) return fail(MDRQ_EINVAL, "NULL argument");
    if (n_reqs == 0) return fail(MDRQ_EINVAL, "no requests");
    std::lock_guard<std::mutex> lock(ds->mu);
    // The result buffers may have been prepared by work still queued on any stream: the
    // replay starts once the device is idle (its requests then need no events).
    const hipError_t idle = hipDeviceSynchronize();
    if (idle != hipSuccess) return fail_hip(idle, "serving: device synchronisation");
    bool any_row = false;
    for (uint32_t i = 0; i < n_reqs; ++i) any_row |= needs_row(rs[i]);
    mdrq_server* s = nullptr;
    rc = create(ds, cfg, any_row, &s);
    if (rc) return rc;
    for (uint32_t i = 0; i < n_reqs; ++i) {
      rc = check_request(s, &reqs[i].query, &rs[i]);
      if (rc) {
        std::string msg = mdrq_last_error();
        (void)shutdown(s, nullptr);
        return fail(rc, msg);
      }
    }

    // Replay: each request is queued when the clock reaches its arrival stamp (arrival
    // order, stable for equal stamps); its latency counts from that stamp.
    std::vector<uint32_t> order(n_reqs);
    for (uint32_t i = 0; i < n_reqs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return reqs[a].arrival_ns < reqs[b].arrival_ns; });
    std::vector<uint32_t> index_of_ticket(n_reqs);
    const Clock::time_point t0 = Clock::now();
    for (uint32_t k = 0; k < n_reqs; ++k) {
      const uint32_t i = order[k];
      const Clock::time_point at = t0 + std::chrono::nanoseconds(reqs[i].arrival_ns);
      std::this_thread::sleep_until(at);
      uint64_t ticket = 0;
      rc = enqueue(s, &reqs[i].query, &rs[i], at, false, false, nullptr, &ticket);
      if (rc) break;
      index_of_ticket[ticket] = i;
    }
    if (latency_ns) {
      // Latencies are final once the server has drained; copy them before it is freed.
      {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv.wait(lk, [&] { return s->completed == s->next_ticket || s->error != MDRQ_OK; });
        for (uint64_t t = 0; t < s->next_ticket && t < s->lat_ns.size(); ++t)
          latency_ns[index_of_ticket[t]] = s->lat_ns[t];
      }
    }
    const int rc_close = shutdown(s, stats);
    if (rc) return rc;
    return rc_close;
  });
}
