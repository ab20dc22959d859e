// Host side of the learned selectivity estimator: histograms, features, training
// (forward, backward, Adam), prediction, exact labels from shared count scans, and
// the hook that orders a query's predicates by estimated selectivity.
//
// Ordering dimensions most-selective-first needs selectivity estimates (section 2.2.4)
// and learning them is future work in the paper (section 8); the non-learned baseline
// is the independence product of per-dimension selectivities (section 2.1).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "mdrq_internal.h"

using namespace mdrq;

namespace {

constexpr uint32_t kMaxTrainBatch = 65536;
constexpr uint32_t kPredictChunk = 65536;

#define EST_CHECK(call, what)                 \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return fail_hip(e_, what); \
  } while (0)

// Device buffer that only grows.
struct DevBuf {
  void* p = nullptr;
  uint64_t bytes = 0;
  int grow(uint64_t need) {
    if (need <= bytes) return MDRQ_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, need) != hipSuccess) return fail(MDRQ_ENOMEM, "estimator: device allocation failed");
    bytes = need;
    return MDRQ_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as(uint64_t byte_offset = 0) const {
    return reinterpret_cast<T*>(static_cast<char*>(p) + byte_offset);
  }
};

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator.
uint64_t splitmix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
double unit(uint64_t seed, uint64_t i) {
  return static_cast<double>(splitmix(seed ^ splitmix(i)) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

struct mdrq_estimator {
  mdrq_dataset* ds = nullptr;
  std::mutex mu;
  uint32_t d = 0, F = 0, H = 0, O = 0;
  uint64_t n_rows = 0;
  uint64_t n_params = 0;
  uint64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float* bounds = nullptr;  // device [d][kBins + 1]
  float* state = nullptr;   // device: params, grads, Adam m, Adam v (n_params each)
  uint16_t* wb = nullptr;   // device bfloat16 copies of W1, W2, W3 (same offsets as params)
  int step = 0;
  uint32_t work_rows = 0;   // rows the work buffers hold
  DevBuf work;              // per-batch activations and gradients
  DevBuf data;              // per-call query data (qd, features, targets, permutation)
  DevBuf losses;
  std::vector<float> h_qd;

  // One-query prediction (the per-query path of estimated ordering) as a captured HIP
  // graph on its own stream: query upload, features, the three layers, the estimates
  // and their download replay as one launch.  Its buffers never move.
  // The evaluation order of a plan's predicates (order_fused_kernel) is left in device
  // memory for the scan that follows on the same stream.
  hipStream_t stream = nullptr;
  DevBuf one_work;           // work buffers for one row
  DevBuf one_dev;            // qd (d x 3 floats), estimates (O floats), order[128]
  float* one_host = nullptr; // pinned: qd, estimates
  hipGraph_t one_graph = nullptr;
  hipGraphExec_t one_exec = nullptr;
  uint64_t qd_floats() const { return static_cast<uint64_t>(d) * 3; }
  float* dev_qd() const { return one_dev.as<float>(); }
  float* dev_sel() const { return dev_qd() + qd_floats(); }
  uint32_t* dev_order() const { return reinterpret_cast<uint32_t*>(dev_sel() + O); }
  float* host_sel() const { return one_host + qd_floats(); }

  float* params() const { return state; }
  float* grads() const { return state + n_params; }
  float* adam_m() const { return state + 2 * n_params; }
  float* adam_v() const { return state + 3 * n_params; }

  // Work buffer layout for `rows` rows (byte offsets, 256-aligned).
  struct Layout {
    uint64_t X, Bs, Z1, Z2, H1, H2, Y, T, M, dY, dYb, dH, dZ, dZb, end;
  };
  Layout layout(uint32_t rows) const {
    Layout l{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
      const uint64_t at = o;
      o = round_up(o + bytes, 256);
      return at;
    };
    const uint64_t r = rows;
    l.X = take(r * F * 2);
    l.Bs = take(r * O * 4);
    l.Z1 = take(r * H * 4);
    l.Z2 = take(r * H * 4);
    l.H1 = take(r * H * 2);
    l.H2 = take(r * H * 2);
    l.Y = take(r * O * 4);
    l.T = take(r * O * 4);
    l.M = take(r * O * 4);
    l.dY = take(r * O * 4);
    l.dYb = take(r * O * 2);
    l.dH = take(r * H * 4);
    l.dZ = take(r * H * 4);
    l.dZb = take(r * H * 2);
    l.end = o;
    return l;
  }
  int ensure_work(uint32_t rows) {
    if (rows <= work_rows) return MDRQ_OK;
    int rc = work.grow(layout(rows).end);
    if (rc) return rc;
    work_rows = rows;
    return MDRQ_OK;
  }
};

namespace {

bool restricts(const mdrq_pred& p) {
  const float inf = std::numeric_limits<float>::infinity();
  return !(p.lo == -inf && p.hi == inf);
}

int check_queries(const mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n) {
  if (!qs) return fail(MDRQ_EINVAL, "queries are NULL");
  if (n == 0 || n > MDRQ_EST_MAX_QUERIES) return fail(MDRQ_EINVAL, "query count out of range");
  for (uint32_t i = 0; i < n; ++i) {
    int rc = check_query(e->ds, &qs[i]);
    if (rc) return rc;
  }
  return MDRQ_OK;
}

// (lo, hi, restricted) per (query, dimension) into e->h_qd.
void build_qd(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n) {
  e->h_qd.assign(static_cast<size_t>(n) * e->d * 3, 0.0f);
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t k = 0; k < qs[i].n_preds; ++k) {
      const mdrq_pred& p = qs[i].preds[k];
      if (!restricts(p)) continue;
      float* t = &e->h_qd[(static_cast<size_t>(i) * e->d + p.dim) * 3];
      t[0] = p.lo;
      t[1] = p.hi;
      t[2] = 1.0f;
    }
}

// Features and base estimates of n queries into X and base (device) from qd (device).
int features(mdrq_estimator* e, const float* qd_dev, uint32_t n, uint16_t* X, float* base,
             hipStream_t stream = nullptr) {
  FeatureArgs f{};
  f.qd = qd_dev;
  f.bounds = e->bounds;
  f.x = X;
  f.base = base;
  f.n = n;
  f.d = e->d;
  const double rows = static_cast<double>(e->n_rows);
  f.inv_rows = static_cast<float>(1.0 / rows);
  f.inv_ln_rows = static_cast<float>(1.0 / std::log(rows));
  EST_CHECK(launch_features(f, stream), "estimator features");
  return MDRQ_OK;
}

GemmArgs gemm(const uint16_t* a, uint64_t a_m, uint64_t a_k, const uint16_t* b, uint64_t b_k,
              uint64_t b_n, uint32_t M, uint32_t N, uint32_t K) {
  GemmArgs g{};
  g.a = a;
  g.b = b;
  g.a_m = a_m;
  g.a_k = a_k;
  g.b_k = b_k;
  g.b_n = b_n;
  g.M = M;
  g.N = N;
  g.K = K;
  g.c_ld = N;
  return g;
}

// Forward pass of `rows` rows whose features and base estimates are in the work
// buffer's X and Bs: the network's output corrects the base estimate.  `work` (laid out
// for `cap` rows) defaults to the estimator's own work buffer.
int forward(mdrq_estimator* e, uint32_t rows, const DevBuf* work = nullptr, uint32_t cap = 0,
            hipStream_t stream = nullptr) {
  if (!work) {
    work = &e->work;
    cap = e->work_rows;
  }
  const auto L = e->layout(cap);
  const uint32_t F = e->F, H = e->H, O = e->O;
  uint16_t* X = work->as<uint16_t>(L.X);
  GemmArgs g = gemm(X, F, 1, e->wb + e->oW1, H, 1, rows, H, F);
  g.bias = e->params() + e->ob1;
  g.c = work->as<float>(L.Z1);
  g.act = work->as<uint16_t>(L.H1);
  g.gelu = 1;
  EST_CHECK(launch_gemm(g, stream), "estimator layer 1");
  g = gemm(work->as<uint16_t>(L.H1), H, 1, e->wb + e->oW2, H, 1, rows, H, H);
  g.bias = e->params() + e->ob2;
  g.c = work->as<float>(L.Z2);
  g.act = work->as<uint16_t>(L.H2);
  g.gelu = 1;
  EST_CHECK(launch_gemm(g, stream), "estimator layer 2");
  g = gemm(work->as<uint16_t>(L.H2), H, 1, e->wb + e->oW3, O, 1, rows, O, H);
  g.bias = e->params() + e->ob3;
  g.add = work->as<float>(L.Bs);
  g.c = work->as<float>(L.Y);
  EST_CHECK(launch_gemm(g, stream), "estimator layer 3");
  return MDRQ_OK;
}

// Loss gradient and backward pass of `rows` rows (targets in T and M); gradients land
// in e->grads(), the batch loss is added to *loss_dev.
int backward(mdrq_estimator* e, uint32_t rows, float inv_count, float* loss_dev) {
  const auto L = e->layout(e->work_rows);
  const uint32_t F = e->F, H = e->H, O = e->O;
  float* G = e->grads();
  LossArgs la{};
  la.y = e->work.as<float>(L.Y);
  la.t = e->work.as<float>(L.T);
  la.mask = e->work.as<float>(L.M);
  la.dy = e->work.as<float>(L.dY);
  la.dyb = e->work.as<uint16_t>(L.dYb);
  la.loss = loss_dev;
  la.rows = rows;
  la.cols = O;
  la.inv_count = inv_count;
  EST_CHECK(launch_loss_grad(la, nullptr), "estimator loss");
  const uint16_t* X = e->work.as<uint16_t>(L.X);
  const uint16_t* H1 = e->work.as<uint16_t>(L.H1);
  const uint16_t* H2 = e->work.as<uint16_t>(L.H2);
  const uint16_t* dYb = e->work.as<uint16_t>(L.dYb);
  float* dH = e->work.as<float>(L.dH);
  float* dZ = e->work.as<float>(L.dZ);
  uint16_t* dZb = e->work.as<uint16_t>(L.dZb);
  // Layer 3: dW3 = H2^T dY, db3 = colsum(dY), dH2 = dY W3^T.
  GemmArgs g = gemm(H2, 1, H, dYb, O, 1, H, O, rows);
  g.c = G + e->oW3;
  EST_CHECK(launch_gemm(g, nullptr), "estimator dW3");
  EST_CHECK(launch_colsum(la.dy, rows, O, G + e->ob3, nullptr), "estimator db3");
  g = gemm(dYb, O, 1, e->wb + e->oW3, 1, O, rows, H, O);
  g.c = dH;
  EST_CHECK(launch_gemm(g, nullptr), "estimator dH2");
  const uint64_t nh = static_cast<uint64_t>(rows) * H;
  EST_CHECK(launch_gelu_back(dH, e->work.as<float>(L.Z2), dZ, dZb, nh, nullptr), "estimator dZ2");
  // Layer 2: dW2 = H1^T dZ2, db2 = colsum(dZ2), dH1 = dZ2 W2^T.
  g = gemm(H1, 1, H, dZb, H, 1, H, H, rows);
  g.c = G + e->oW2;
  EST_CHECK(launch_gemm(g, nullptr), "estimator dW2");
  EST_CHECK(launch_colsum(dZ, rows, H, G + e->ob2, nullptr), "estimator db2");
  g = gemm(dZb, H, 1, e->wb + e->oW2, 1, H, rows, H, H);
  g.c = dH;
  EST_CHECK(launch_gemm(g, nullptr), "estimator dH1");
  EST_CHECK(launch_gelu_back(dH, e->work.as<float>(L.Z1), dZ, dZb, nh, nullptr), "estimator dZ1");
  // Layer 1: dW1 = X^T dZ1, db1 = colsum(dZ1).
  g = gemm(X, 1, F, dZb, H, 1, F, H, rows);
  g.c = G + e->oW1;
  EST_CHECK(launch_gemm(g, nullptr), "estimator dW1");
  EST_CHECK(launch_colsum(dZ, rows, H, G + e->ob1, nullptr), "estimator db1");
  return MDRQ_OK;
}

int refresh_bf16(mdrq_estimator* e) {
  const float* P = e->params();
  EST_CHECK(launch_to_bf16(P + e->oW1, static_cast<uint64_t>(e->F) * e->H, e->wb + e->oW1, nullptr),
            "estimator W1 copy");
  EST_CHECK(launch_to_bf16(P + e->oW2, static_cast<uint64_t>(e->H) * e->H, e->wb + e->oW2, nullptr),
            "estimator W2 copy");
  EST_CHECK(launch_to_bf16(P + e->oW3, static_cast<uint64_t>(e->H) * e->O, e->wb + e->oW3, nullptr),
            "estimator W3 copy");
  return MDRQ_OK;
}

int check_labels(const mdrq_estimator* e, const float* sel, uint32_t n, std::vector<uint32_t>& present) {
  if (!sel) return fail(MDRQ_EINVAL, "selectivities are NULL");
  present.assign(n, 0);
  for (uint32_t i = 0; i < n; ++i) {
    const float* row = sel + static_cast<size_t>(i) * e->O;
    for (uint32_t j = 0; j < e->O; ++j) {
      const float s = row[j];
      if (!(s <= 1.0f) || (j == e->d && !(s >= 0.0f)))
        return fail(MDRQ_EINVAL, "selectivity out of range (NaN, > 1, or joint < 0)");
      present[i] += s >= 0.0f ? 1u : 0u;
    }
  }
  return MDRQ_OK;
}

// Upload qd and sel of n queries, compute their features and targets into `data`.
// Layout: qd [n][d][3] f32, X [n][F] bf16, sel/T/M [n][O] f32.
struct DataLayout {
  uint64_t qd, X, base, sel, T, M, perm, end;
};
DataLayout data_layout(const mdrq_estimator* e, uint32_t n, bool with_targets) {
  DataLayout l{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  l.qd = take(static_cast<uint64_t>(n) * e->d * 12);
  l.X = take(static_cast<uint64_t>(n) * e->F * 2);
  l.base = take(static_cast<uint64_t>(n) * e->O * 4);
  l.sel = take(static_cast<uint64_t>(n) * e->O * 4);
  if (with_targets) {
    l.T = take(static_cast<uint64_t>(n) * e->O * 4);
    l.M = take(static_cast<uint64_t>(n) * e->O * 4);
    l.perm = take(static_cast<uint64_t>(n) * 4);
  }
  l.end = o;
  return l;
}

int upload_queries(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, const DataLayout& l) {
  build_qd(e, qs, n);
  EST_CHECK(hipMemcpy(e->data.as<float>(l.qd), e->h_qd.data(), e->h_qd.size() * 4, hipMemcpyHostToDevice),
            "estimator query upload");
  return features(e, e->data.as<float>(l.qd), n, e->data.as<uint16_t>(l.X), e->data.as<float>(l.base));
}

int upload_targets(mdrq_estimator* e, const float* sel, uint32_t n, const DataLayout& l) {
  EST_CHECK(hipMemcpy(e->data.as<float>(l.sel), sel, static_cast<uint64_t>(n) * e->O * 4,
                      hipMemcpyHostToDevice),
            "estimator label upload");
  EST_CHECK(launch_targets(e->data.as<float>(l.sel), n, e->O, e->n_rows, e->data.as<float>(l.T),
                           e->data.as<float>(l.M), nullptr),
            "estimator targets");
  return MDRQ_OK;
}

int predict_locked(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, float* sel) {
  for (uint32_t at = 0; at < n; at += kPredictChunk) {
    const uint32_t rows = std::min(kPredictChunk, n - at);
    const DataLayout dl = data_layout(e, rows, false);
    int rc = e->data.grow(dl.end);
    if (rc) return rc;
    rc = e->ensure_work(rows);
    if (rc) return rc;
    const auto L = e->layout(e->work_rows);
    build_qd(e, qs + at, rows);
    EST_CHECK(hipMemcpy(e->data.as<float>(dl.qd), e->h_qd.data(), e->h_qd.size() * 4,
                        hipMemcpyHostToDevice),
              "estimator query upload");
    rc = features(e, e->data.as<float>(dl.qd), rows, e->work.as<uint16_t>(L.X), e->work.as<float>(L.Bs));
    if (rc) return rc;
    rc = forward(e, rows);
    if (rc) return rc;
    EST_CHECK(launch_to_selectivity(e->work.as<float>(L.Y), e->data.as<float>(dl.qd), rows, e->d,
                                    e->n_rows, e->data.as<float>(dl.sel), nullptr),
              "estimator outputs");
    EST_CHECK(hipMemcpy(sel + static_cast<size_t>(at) * e->O, e->data.as<float>(dl.sel),
                        static_cast<uint64_t>(rows) * e->O * 4, hipMemcpyDeviceToHost),
              "estimator result download");
  }
  return MDRQ_OK;
}

// Buffers of the one-query graphs (allocated once, never moved).
int ensure_one(mdrq_estimator* e) {
  if (e->one_host) return MDRQ_OK;
  const uint64_t floats = e->qd_floats() + e->O;
  const uint64_t words = MDRQ_MAX_DIMS;
  int rc;
  if ((rc = e->one_work.grow(e->layout(1).end)) || (rc = e->one_dev.grow((floats + words) * 4))) return rc;
  if (hipHostMalloc(reinterpret_cast<void**>(&e->one_host), (floats + words) * 4, hipHostMallocDefault) !=
      hipSuccess)
    return fail(MDRQ_ENOMEM, "estimator: pinned allocation failed");
  if (!e->stream) EST_CHECK(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking), "estimator stream");
  return MDRQ_OK;
}

// Capture the one-query graph: upload the query, features, the three layers, the
// estimates and their download.
int capture_one(mdrq_estimator* e, hipGraphExec_t* exec_out, hipGraph_t* graph_out) {
  const auto L = e->layout(1);
  EST_CHECK(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal), "graph capture");
  hipError_t ce = hipMemcpyAsync(e->dev_qd(), e->one_host, e->qd_floats() * 4, hipMemcpyHostToDevice, e->stream);
  int rc = ce == hipSuccess ? features(e, e->dev_qd(), 1, e->one_work.as<uint16_t>(L.X),
                                       e->one_work.as<float>(L.Bs), e->stream)
                            : MDRQ_EDEVICE;
  if (rc == MDRQ_OK) rc = forward(e, 1, &e->one_work, 1, e->stream);
  if (rc == MDRQ_OK)
    ce = launch_to_selectivity(e->one_work.as<float>(L.Y), e->dev_qd(), 1, e->d, e->n_rows, e->dev_sel(),
                               e->stream);
  if (rc == MDRQ_OK && ce == hipSuccess)
    ce = hipMemcpyAsync(e->host_sel(), e->dev_sel(), e->O * 4, hipMemcpyDeviceToHost, e->stream);
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(e->stream, &graph);
  if (rc != MDRQ_OK || ce != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != MDRQ_OK ? rc : fail_hip(ce != hipSuccess ? ce : ee, "estimator graph capture");
  }
  *graph_out = graph;
  EST_CHECK(hipGraphInstantiate(exec_out, graph, nullptr, nullptr, 0), "estimator graph instantiate");
  return MDRQ_OK;
}

void fill_one(mdrq_estimator* e, const mdrq_query_t* q) {
  std::memset(e->one_host, 0, e->qd_floats() * 4);
  for (uint32_t k = 0; k < q->n_preds; ++k) {
    const mdrq_pred& p = q->preds[k];
    if (!restricts(p)) continue;
    float* t = e->one_host + static_cast<uint64_t>(p.dim) * 3;
    t[0] = p.lo;
    t[1] = p.hi;
    t[2] = 1.0f;
  }
}

// One query through the captured graph (captured on first use).
int predict_one(mdrq_estimator* e, const mdrq_query_t* q, float* sel) {
  int rc = ensure_one(e);
  if (rc) return rc;
  if (!e->one_exec && (rc = capture_one(e, &e->one_exec, &e->one_graph))) return rc;
  fill_one(e, q);
  EST_CHECK(hipGraphLaunch(e->one_exec, e->stream), "estimator graph launch");
  EST_CHECK(hipStreamSynchronize(e->stream), "estimator graph completion");
  std::memcpy(sel, e->host_sel(), e->O * 4);
  return MDRQ_OK;
}

}  // namespace

namespace mdrq {

int estimate_for_order(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, std::vector<float>& est) {
  est.clear();
  mdrq_estimator* e = ds->estimator;
  if (!e) return MDRQ_OK;
  bool any = false;
  for (uint32_t i = 0; i < n && !any; ++i)
    any = (qs[i].flags & (MDRQ_Q_ORDER_ESTIMATED | MDRQ_Q_SIZE_ESTIMATED)) != 0;
  if (!any) return MDRQ_OK;
  std::lock_guard<std::mutex> lock(e->mu);
  est.resize(static_cast<size_t>(n) * e->O);
  return n == 1 ? predict_one(e, qs, est.data()) : predict_locked(e, qs, n, est.data());
}

void order_plan(Plan& plan, const float* est_row) {
  const size_t k = plan.preds.size();
  std::vector<size_t> idx(k);
  for (size_t i = 0; i < k; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](size_t a, size_t b) { return est_row[plan.dims[a]] < est_row[plan.dims[b]]; });
  std::vector<DevPred> p(k);
  std::vector<uint32_t> d(k);
  for (size_t i = 0; i < k; ++i) {
    p[i] = plan.preds[idx[i]];
    d[i] = plan.dims[idx[i]];
  }
  plan.preds.swap(p);
  plan.dims.swap(d);
}

void detach_estimator(mdrq_dataset* ds) { ds->estimator = nullptr; }

int order_on_device(mdrq_dataset* ds, const mdrq_query_t* q, Plan& plan, hipStream_t stream,
                    std::unique_lock<std::mutex>& hold) {
  mdrq_estimator* e = ds->estimator;
  if (!e || plan.preds.size() < 2) return MDRQ_OK;
  hold = std::unique_lock<std::mutex>(e->mu);
  int rc = ensure_one(e);
  if (rc) return rc;
  OrderArgs a{};
  a.bounds = e->bounds;
  a.wb = e->wb;
  a.params = e->params();
  a.oW1 = e->oW1;
  a.ob1 = e->ob1;
  a.oW2 = e->oW2;
  a.ob2 = e->ob2;
  a.oW3 = e->oW3;
  a.ob3 = e->ob3;
  a.d = e->d;
  a.H = e->H;
  a.k = static_cast<uint32_t>(plan.dims.size());
  const double rows = static_cast<double>(e->n_rows);
  a.inv_rows = static_cast<float>(1.0 / rows);
  a.inv_ln_rows = static_cast<float>(1.0 / std::log(rows));
  a.ln_rows = static_cast<float>(std::log(rows));
  a.order = e->dev_order();
  for (uint32_t k = 0; k < q->n_preds; ++k) {
    const mdrq_pred& p = q->preds[k];
    if (!restricts(p)) continue;
    a.restricted[p.dim >> 5] |= 1u << (p.dim & 31);
    a.lo[p.dim] = p.lo;
    a.hi[p.dim] = p.hi;
  }
  for (size_t i = 0; i < plan.dims.size(); ++i) a.dims[i] = plan.dims[i];
  EST_CHECK(launch_order_fused(a, stream), "estimator order launch");
  plan.order = e->dev_order();
  return MDRQ_OK;
}

}  // namespace mdrq

extern "C" {

int mdrq_estimator_create(mdrq_dataset* ds, const mdrq_estimator_config_t* cfg, mdrq_estimator** out) {
  return guarded([&]() -> int {
    clear_error();
    if (!ds || !cfg || !out) return fail(MDRQ_EINVAL, "NULL argument");
    *out = nullptr;
    const uint32_t H = cfg->hidden ? cfg->hidden : 64;
    if (H < 16 || H > 256 || H % 16) return fail(MDRQ_EINVAL, "hidden width must be a multiple of 16 in 16..256");
    if (ds->n_rows < 2) return fail(MDRQ_EINVAL, "the estimator needs at least 2 rows");
    uint32_t m = cfg->sample_rows ? cfg->sample_rows
                                  : static_cast<uint32_t>(std::min<uint64_t>(kSampleMax, ds->n_rows));
    if (m < 2 || m > kSampleMax || m > ds->n_rows) return fail(MDRQ_EINVAL, "sample_rows out of range");

    auto* e = new mdrq_estimator();
    e->ds = ds;
    e->d = ds->n_dims;
    e->F = ds->n_dims * kFeatPerDim;
    e->H = H;
    e->O = ds->n_dims + 1;
    e->n_rows = ds->n_rows;
    uint64_t o = 0;
    e->oW1 = o; o += static_cast<uint64_t>(e->F) * H;
    e->ob1 = o; o += H;
    e->oW2 = o; o += static_cast<uint64_t>(H) * H;
    e->ob2 = o; o += H;
    e->oW3 = o; o += static_cast<uint64_t>(H) * e->O;
    e->ob3 = o; o += e->O;
    e->n_params = o;
    auto cleanup = [&](int rc) {
      mdrq_estimator_free(e);
      return rc;
    };
    if (hipMalloc(&e->bounds, static_cast<uint64_t>(e->d) * (kBins + 1) * 4) != hipSuccess ||
        hipMalloc(&e->state, 4 * e->n_params * 4) != hipSuccess ||
        hipMalloc(&e->wb, e->n_params * 2) != hipSuccess)
      return cleanup(fail(MDRQ_ENOMEM, "estimator: device allocation failed"));

    // Histograms: a strided sample of each column, sorted on the device.
    HistArgs ha{};
    ha.n_rows = ds->n_rows;
    ha.m = m;
    ha.m_pow2 = 1;
    while (ha.m_pow2 < m) ha.m_pow2 <<= 1;
    ha.bounds = e->bounds;
    for (uint32_t j = 0; j < e->d; ++j) ha.cols[j] = ds->cols[j];
    hipError_t he = launch_sample_sort(ha, e->d, nullptr);
    if (he != hipSuccess) return cleanup(fail_hip(he, "estimator histograms"));

    // Glorot-uniform hidden weights; zero output layer, so that an untrained network
    // returns the base (histogram independence) estimate; zero biases and moments.
    std::vector<float> p(e->n_params, 0.0f);
    auto fill = [&](uint64_t off, uint32_t fan_in, uint32_t fan_out, uint64_t stream) {
      const double a = std::sqrt(6.0 / (fan_in + fan_out));
      for (uint64_t i = 0; i < static_cast<uint64_t>(fan_in) * fan_out; ++i)
        p[off + i] = static_cast<float>((2.0 * unit(cfg->seed + stream, i) - 1.0) * a);
    };
    fill(e->oW1, e->F, H, 1);
    fill(e->oW2, H, H, 2);
    int rc = mdrq_estimator_set_params(e, p.data());
    if (rc) return cleanup(rc);
    *out = e;
    return MDRQ_OK;
  });
}

void mdrq_estimator_free(mdrq_estimator* e) {
  if (!e) return;
  if (e->ds) {
    std::lock_guard<std::mutex> lock(e->ds->mu);
    if (e->ds->estimator == e) detach_estimator(e->ds);
  }
  (void)hipDeviceSynchronize();
  if (e->bounds) (void)hipFree(e->bounds);
  if (e->state) (void)hipFree(e->state);
  if (e->wb) (void)hipFree(e->wb);
  e->work.release();
  e->data.release();
  e->losses.release();
  if (e->one_exec) (void)hipGraphExecDestroy(e->one_exec);
  if (e->one_graph) (void)hipGraphDestroy(e->one_graph);
  e->one_work.release();
  e->one_dev.release();
  if (e->one_host) (void)hipHostFree(e->one_host);
  if (e->stream) (void)hipStreamDestroy(e->stream);
  delete e;
}

int mdrq_estimator_histograms(const mdrq_estimator* e, float* bounds) {
  clear_error();
  if (!e || !bounds) return fail(MDRQ_EINVAL, "NULL argument");
  EST_CHECK(hipMemcpy(bounds, e->bounds, static_cast<uint64_t>(e->d) * (kBins + 1) * 4, hipMemcpyDeviceToHost),
            "estimator histogram download");
  return MDRQ_OK;
}

int mdrq_estimator_features(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, uint16_t* out) {
  return guarded([&]() -> int {
    clear_error();
    if (!e || !out) return fail(MDRQ_EINVAL, "NULL argument");
    int rc = check_queries(e, qs, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(e->mu);
    const DataLayout dl = data_layout(e, n, false);
    rc = e->data.grow(dl.end);
    if (rc) return rc;
    rc = upload_queries(e, qs, n, dl);
    if (rc) return rc;
    EST_CHECK(hipMemcpy(out, e->data.as<uint16_t>(dl.X), static_cast<uint64_t>(n) * e->F * 2, hipMemcpyDeviceToHost),
              "estimator feature download");
    return MDRQ_OK;
  });
}

int mdrq_estimator_param_count(const mdrq_estimator* e, uint64_t* count) {
  clear_error();
  if (!e || !count) return fail(MDRQ_EINVAL, "NULL argument");
  *count = e->n_params;
  return MDRQ_OK;
}

int mdrq_estimator_get_params(const mdrq_estimator* e, float* out) {
  clear_error();
  if (!e || !out) return fail(MDRQ_EINVAL, "NULL argument");
  EST_CHECK(hipMemcpy(out, e->params(), e->n_params * 4, hipMemcpyDeviceToHost), "estimator parameter download");
  return MDRQ_OK;
}

int mdrq_estimator_set_params(mdrq_estimator* e, const float* in) {
  clear_error();
  if (!e || !in) return fail(MDRQ_EINVAL, "NULL argument");
  for (uint64_t i = 0; i < e->n_params; ++i)
    if (!std::isfinite(in[i])) return fail(MDRQ_EINVAL, "parameters must be finite");
  std::lock_guard<std::mutex> lock(e->mu);
  EST_CHECK(hipMemcpy(e->params(), in, e->n_params * 4, hipMemcpyHostToDevice), "estimator parameter upload");
  EST_CHECK(hipMemset(e->grads(), 0, 3 * e->n_params * 4), "estimator state clear");
  e->step = 0;
  int rc = refresh_bf16(e);
  if (rc) return rc;
  EST_CHECK(hipDeviceSynchronize(), "estimator parameter upload");
  return MDRQ_OK;
}

int mdrq_label_selectivities(mdrq_dataset* ds, const mdrq_query_t* qs, uint32_t n, float* sel) {
  return guarded([&]() -> int {
    clear_error();
    if (!ds || !qs || !sel) return fail(MDRQ_EINVAL, "NULL argument");
    if (n == 0 || n > MDRQ_EST_MAX_QUERIES) return fail(MDRQ_EINVAL, "query count out of range");
    for (uint32_t i = 0; i < n; ++i) {
      int rc = check_query(ds, &qs[i]);
      if (rc) return rc;
    }
    const uint32_t O = ds->n_dims + 1;
    const double N = static_cast<double>(ds->n_rows);
    // Every restricting predicate alone: counted from sorted copies of the columns.
    std::vector<mdrq_pred> singles;
    std::vector<std::pair<uint32_t, uint32_t>> single_where;  // (query, dimension)
    for (uint32_t i = 0; i < n; ++i) {
      float* row = sel + static_cast<size_t>(i) * O;
      for (uint32_t j = 0; j < O; ++j) row[j] = -1.0f;
      for (uint32_t k = 0; k < qs[i].n_preds; ++k)
        if (restricts(qs[i].preds[k])) {
          singles.push_back(qs[i].preds[k]);
          single_where.emplace_back(i, qs[i].preds[k].dim);
        }
    }
    std::lock_guard<std::mutex> lock(ds->mu);
    std::vector<uint64_t> single_counts;
    int rc = count_single_predicates(ds, singles, single_counts);
    if (rc != MDRQ_OK) return rc;
    for (size_t k = 0; k < singles.size(); ++k)
      sel[static_cast<size_t>(single_where[k].first) * O + single_where[k].second] =
          static_cast<float>(static_cast<double>(single_counts[k]) / N);
    // The whole queries: shared count-only scans.
    std::vector<mdrq_query_t> ex(n);
    for (uint32_t i = 0; i < n; ++i) ex[i] = mdrq_query_t{qs[i].preds, qs[i].n_preds, 0};
    std::vector<mdrq_result_t> rs(MDRQ_MAX_BATCH);
    for (uint32_t at = 0; at < n; at += MDRQ_MAX_BATCH) {
      const uint32_t m = std::min<uint32_t>(MDRQ_MAX_BATCH, n - at);
      for (uint32_t i = 0; i < m; ++i) rs[i] = mdrq_result_t{MDRQ_OUT_COUNT, MDRQ_MEM_HOST, nullptr, 0, 0, 0, 0, 0};
      rc = run_batch(ds, ex.data() + at, m, rs.data(), nullptr);
      if (rc != MDRQ_OK) return rc;
      for (uint32_t i = 0; i < m; ++i)
        sel[static_cast<size_t>(at + i) * O + ds->n_dims] = static_cast<float>(static_cast<double>(rs[i].count) / N);
    }
    return MDRQ_OK;
  });
}

int mdrq_estimator_gradient(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, const float* sel,
                            float* loss, float* grad) {
  return guarded([&]() -> int {
    clear_error();
    if (!e || !loss || !grad) return fail(MDRQ_EINVAL, "NULL argument");
    if (n > kMaxTrainBatch) return fail(MDRQ_EINVAL, "at most 65536 queries per gradient");
    int rc = check_queries(e, qs, n);
    if (rc) return rc;
    std::vector<uint32_t> present;
    rc = check_labels(e, sel, n, present);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(e->mu);
    const DataLayout dl = data_layout(e, n, true);
    if ((rc = e->data.grow(dl.end)) || (rc = e->ensure_work(n)) || (rc = e->losses.grow(4))) return rc;
    rc = upload_queries(e, qs, n, dl);
    if (rc) return rc;
    rc = upload_targets(e, sel, n, dl);
    if (rc) return rc;
    const auto L = e->layout(e->work_rows);
    EST_CHECK(hipMemcpy(e->work.as<char>(L.X), e->data.as<char>(dl.X), static_cast<uint64_t>(n) * e->F * 2,
                        hipMemcpyDeviceToDevice), "estimator copy");
    EST_CHECK(hipMemcpy(e->work.as<char>(L.Bs), e->data.as<char>(dl.base), static_cast<uint64_t>(n) * e->O * 4,
                        hipMemcpyDeviceToDevice), "estimator copy");
    EST_CHECK(hipMemcpy(e->work.as<char>(L.T), e->data.as<char>(dl.T), static_cast<uint64_t>(n) * e->O * 4,
                        hipMemcpyDeviceToDevice), "estimator copy");
    EST_CHECK(hipMemcpy(e->work.as<char>(L.M), e->data.as<char>(dl.M), static_cast<uint64_t>(n) * e->O * 4,
                        hipMemcpyDeviceToDevice), "estimator copy");
    EST_CHECK(hipMemset(e->losses.p, 0, 4), "estimator loss clear");
    uint64_t cnt = 0;
    for (uint32_t c : present) cnt += c;
    rc = forward(e, n);
    if (rc) return rc;
    rc = backward(e, n, static_cast<float>(1.0 / static_cast<double>(cnt)), e->losses.as<float>());
    if (rc) return rc;
    EST_CHECK(hipMemcpy(grad, e->grads(), e->n_params * 4, hipMemcpyDeviceToHost), "estimator gradient download");
    EST_CHECK(hipMemcpy(loss, e->losses.p, 4, hipMemcpyDeviceToHost), "estimator loss download");
    return MDRQ_OK;
  });
}

int mdrq_estimator_train(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, const float* sel,
                         const mdrq_train_config_t* cfg, float* epoch_loss) {
  return guarded([&]() -> int {
    clear_error();
    if (!e || !cfg) return fail(MDRQ_EINVAL, "NULL argument");
    if (cfg->epochs == 0 || cfg->epochs > 100000) return fail(MDRQ_EINVAL, "epochs out of range");
    if (cfg->batch == 0 || cfg->batch > kMaxTrainBatch) return fail(MDRQ_EINVAL, "batch out of range");
    if (!(cfg->lr > 0.0f) || !std::isfinite(cfg->lr)) return fail(MDRQ_EINVAL, "learning rate must be positive");
    int rc = check_queries(e, qs, n);
    if (rc) return rc;
    std::vector<uint32_t> present;
    rc = check_labels(e, sel, n, present);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(e->mu);
    const uint32_t B = std::min(cfg->batch, n);
    const DataLayout dl = data_layout(e, n, true);
    if ((rc = e->data.grow(dl.end)) || (rc = e->ensure_work(B)) ||
        (rc = e->losses.grow(static_cast<uint64_t>(cfg->epochs) * 4)))
      return rc;
    rc = upload_queries(e, qs, n, dl);
    if (rc) return rc;
    rc = upload_targets(e, sel, n, dl);
    if (rc) return rc;
    EST_CHECK(hipMemset(e->losses.p, 0, static_cast<uint64_t>(cfg->epochs) * 4), "estimator loss clear");
    const auto L = e->layout(e->work_rows);
    std::vector<uint32_t> perm(n);
    const uint32_t steps = (n + B - 1) / B;
    for (uint32_t ep = 0; ep < cfg->epochs; ++ep) {
      // Fisher-Yates shuffle from the counter-based generator.
      for (uint32_t i = 0; i < n; ++i) perm[i] = i;
      for (uint32_t i = n; i > 1; --i) {
        const uint64_t r = splitmix(cfg->seed ^ splitmix((static_cast<uint64_t>(ep) << 32) | i));
        const uint32_t j = static_cast<uint32_t>(r % i);
        std::swap(perm[i - 1], perm[j]);
      }
      EST_CHECK(hipMemcpy(e->data.as<uint32_t>(dl.perm), perm.data(), static_cast<uint64_t>(n) * 4,
                          hipMemcpyHostToDevice), "estimator permutation upload");
      for (uint32_t s = 0; s < steps; ++s) {
        const uint32_t at = s * B;
        const uint32_t rows = std::min(B, n - at);
        const uint32_t* idx = e->data.as<uint32_t>(dl.perm) + at;
        uint64_t cnt = 0;
        for (uint32_t i = 0; i < rows; ++i) cnt += present[perm[at + i]];
        EST_CHECK(launch_gather_rows(e->data.as<void>(dl.X), idx, rows, e->F * 2, e->work.as<void>(L.X), nullptr),
                  "estimator gather");
        EST_CHECK(launch_gather_rows(e->data.as<void>(dl.base), idx, rows, e->O * 4, e->work.as<void>(L.Bs), nullptr),
                  "estimator gather");
        EST_CHECK(launch_gather_rows(e->data.as<void>(dl.T), idx, rows, e->O * 4, e->work.as<void>(L.T), nullptr),
                  "estimator gather");
        EST_CHECK(launch_gather_rows(e->data.as<void>(dl.M), idx, rows, e->O * 4, e->work.as<void>(L.M), nullptr),
                  "estimator gather");
        rc = forward(e, rows);
        if (rc) return rc;
        rc = backward(e, rows, static_cast<float>(1.0 / static_cast<double>(cnt)), e->losses.as<float>() + ep);
        if (rc) return rc;
        e->step += 1;
        EST_CHECK(launch_adam(e->params(), e->grads(), e->adam_m(), e->adam_v(), e->n_params, cfg->lr, e->step,
                              nullptr), "estimator Adam");
        rc = refresh_bf16(e);
        if (rc) return rc;
      }
    }
    std::vector<float> sums(cfg->epochs);
    EST_CHECK(hipMemcpy(sums.data(), e->losses.p, sums.size() * 4, hipMemcpyDeviceToHost), "estimator loss download");
    if (epoch_loss)
      for (uint32_t ep = 0; ep < cfg->epochs; ++ep) epoch_loss[ep] = sums[ep] / static_cast<float>(steps);
    return MDRQ_OK;
  });
}

int mdrq_estimator_predict(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, float* sel) {
  return guarded([&]() -> int {
    clear_error();
    if (!e || !sel) return fail(MDRQ_EINVAL, "NULL argument");
    int rc = check_queries(e, qs, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(e->mu);
    return n == 1 ? predict_one(e, qs, sel) : predict_locked(e, qs, n, sel);
  });
}

int mdrq_estimator_activations(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, uint16_t* h1,
                               uint16_t* h2, float* y) {
  return guarded([&]() -> int {
    clear_error();
    if (!e) return fail(MDRQ_EINVAL, "estimator is NULL");
    if (n > kPredictChunk) return fail(MDRQ_EINVAL, "at most 65536 queries per activation call");
    int rc = check_queries(e, qs, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(e->mu);
    const DataLayout dl = data_layout(e, n, false);
    if ((rc = e->data.grow(dl.end)) || (rc = e->ensure_work(n))) return rc;
    const auto L = e->layout(e->work_rows);
    build_qd(e, qs, n);
    EST_CHECK(hipMemcpy(e->data.as<float>(dl.qd), e->h_qd.data(), e->h_qd.size() * 4, hipMemcpyHostToDevice),
              "estimator query upload");
    rc = features(e, e->data.as<float>(dl.qd), n, e->work.as<uint16_t>(L.X), e->work.as<float>(L.Bs));
    if (rc) return rc;
    rc = forward(e, n);
    if (rc) return rc;
    const uint64_t nh = static_cast<uint64_t>(n) * e->H;
    if (h1) EST_CHECK(hipMemcpy(h1, e->work.as<uint16_t>(L.H1), nh * 2, hipMemcpyDeviceToHost), "activation download");
    if (h2) EST_CHECK(hipMemcpy(h2, e->work.as<uint16_t>(L.H2), nh * 2, hipMemcpyDeviceToHost), "activation download");
    if (y)
      EST_CHECK(hipMemcpy(y, e->work.as<float>(L.Y), static_cast<uint64_t>(n) * e->O * 4, hipMemcpyDeviceToHost),
                "output download");
    return MDRQ_OK;
  });
}

int mdrq_estimator_gate(mdrq_estimator* e, const mdrq_query_t* qs, uint32_t n, const float* sel, uint32_t* kept) {
  return guarded([&]() -> int {
    clear_error();
    if (!e) return fail(MDRQ_EINVAL, "estimator is NULL");
    int rc = check_queries(e, qs, n);
    if (rc) return rc;
    std::vector<uint32_t> present;
    rc = check_labels(e, sel, n, present);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(e->mu);
    const uint32_t O = e->O;
    const double ln_rows = std::log(static_cast<double>(e->n_rows));
    const double floor = 1.0 / static_cast<double>(e->n_rows);
    // Per output: squared and absolute errors on the log scale of the network's estimate
    // and of the base estimate alone, over the targets present.  The squared error is
    // dominated by the few queries with the largest errors, the absolute one (the log of
    // the geometric-mean q-error) by the typical query; a correction is kept only if it
    // lowers both.
    std::vector<double> err_net(O, 0.0), err_base(O, 0.0), abs_net(O, 0.0), abs_base(O, 0.0);
    std::vector<float> y, base;
    for (uint32_t at = 0; at < n; at += kPredictChunk) {
      const uint32_t rows = std::min(kPredictChunk, n - at);
      const DataLayout dl = data_layout(e, rows, false);
      if ((rc = e->data.grow(dl.end)) || (rc = e->ensure_work(rows))) return rc;
      const auto L = e->layout(e->work_rows);
      build_qd(e, qs + at, rows);
      EST_CHECK(hipMemcpy(e->data.as<float>(dl.qd), e->h_qd.data(), e->h_qd.size() * 4, hipMemcpyHostToDevice),
                "estimator query upload");
      rc = features(e, e->data.as<float>(dl.qd), rows, e->work.as<uint16_t>(L.X), e->work.as<float>(L.Bs));
      if (rc) return rc;
      rc = forward(e, rows);
      if (rc) return rc;
      y.resize(static_cast<size_t>(rows) * O);
      base.resize(static_cast<size_t>(rows) * O);
      EST_CHECK(hipMemcpy(y.data(), e->work.as<float>(L.Y), y.size() * 4, hipMemcpyDeviceToHost), "output download");
      EST_CHECK(hipMemcpy(base.data(), e->work.as<float>(L.Bs), base.size() * 4, hipMemcpyDeviceToHost),
                "base download");
      for (uint32_t i = 0; i < rows; ++i)
        for (uint32_t j = 0; j < O; ++j) {
          const double s = sel[static_cast<size_t>(at + i) * O + j];
          if (s < 0.0) continue;
          const double t = -std::log(std::max(s, floor)) / ln_rows;
          // Estimates are clamped to [0, 1] on the log scale, as predictions are.
          const double yn = std::min(1.0, std::max(0.0, static_cast<double>(y[static_cast<size_t>(i) * O + j])));
          const double yb = std::min(1.0, std::max(0.0, static_cast<double>(base[static_cast<size_t>(i) * O + j])));
          err_net[j] += (yn - t) * (yn - t);
          err_base[j] += (yb - t) * (yb - t);
          abs_net[j] += std::fabs(yn - t);
          abs_base[j] += std::fabs(yb - t);
        }
    }
    // Remove the correction of every output it does not improve: its column of W3 and
    // its entry of b3 become zero (and their Adam moments with them).
    std::vector<float> w3(static_cast<size_t>(e->H) * O), b3(O);
    EST_CHECK(hipMemcpy(w3.data(), e->params() + e->oW3, w3.size() * 4, hipMemcpyDeviceToHost), "parameter download");
    EST_CHECK(hipMemcpy(b3.data(), e->params() + e->ob3, b3.size() * 4, hipMemcpyDeviceToHost), "parameter download");
    std::vector<bool> keep_out(O);
    for (uint32_t j = 0; j < O; ++j) keep_out[j] = err_net[j] < err_base[j] && abs_net[j] < abs_base[j];
    for (uint32_t j = 0; j < O; ++j) {
      const bool keep = keep_out[j];
      if (kept) kept[j] = keep ? 1u : 0u;
      if (keep) continue;
      for (uint32_t h = 0; h < e->H; ++h) w3[static_cast<size_t>(h) * O + j] = 0.0f;
      b3[j] = 0.0f;
    }
    for (float* m : {e->adam_m(), e->adam_v()}) {
      std::vector<float> mw(w3.size()), mb(O);
      EST_CHECK(hipMemcpy(mw.data(), m + e->oW3, mw.size() * 4, hipMemcpyDeviceToHost), "moment download");
      EST_CHECK(hipMemcpy(mb.data(), m + e->ob3, mb.size() * 4, hipMemcpyDeviceToHost), "moment download");
      for (uint32_t j = 0; j < O; ++j) {
        if (keep_out[j]) continue;
        for (uint32_t h = 0; h < e->H; ++h) mw[static_cast<size_t>(h) * O + j] = 0.0f;
        mb[j] = 0.0f;
      }
      EST_CHECK(hipMemcpy(m + e->oW3, mw.data(), mw.size() * 4, hipMemcpyHostToDevice), "moment upload");
      EST_CHECK(hipMemcpy(m + e->ob3, mb.data(), mb.size() * 4, hipMemcpyHostToDevice), "moment upload");
    }
    EST_CHECK(hipMemcpy(e->params() + e->oW3, w3.data(), w3.size() * 4, hipMemcpyHostToDevice), "parameter upload");
    EST_CHECK(hipMemcpy(e->params() + e->ob3, b3.data(), b3.size() * 4, hipMemcpyHostToDevice), "parameter upload");
    rc = refresh_bf16(e);
    if (rc) return rc;
    EST_CHECK(hipDeviceSynchronize(), "estimator gate");
    return MDRQ_OK;
  });
}

int mdrq_attach_estimator(mdrq_dataset* ds, mdrq_estimator* e) {
  clear_error();
  if (!ds) return fail(MDRQ_EINVAL, "dataset is NULL");
  if (e && e->ds != ds) return fail(MDRQ_EINVAL, "the estimator was created on another dataset");
  std::lock_guard<std::mutex> lock(ds->mu);
  ds->estimator = e;
  return MDRQ_OK;
}

}  // extern "C"
