// Exact counts of single predicates for the estimator's training labels.
//
// A label of a query's dimension j is the selectivity of its predicate on j alone,
// |{i : lo <= C_j[i] <= hi}| / N (section 2.1, with one predicate).  Many such
// predicates on the same column are counted at once from a sorted copy of the
// column's order-preserving keys: the count is upper_bound(key(hi)) -
// lower_bound(key(lo)), exact because the key map is monotone on non-NaN floats and
// takes -0 and +0 to one key (they compare equal).  One radix sort per column (a
// library primitive) replaces a full scan per predicate.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "mdrq_internal.h"

namespace mdrq {
namespace {

__device__ __forceinline__ uint32_t order_key(float x) {
  uint32_t b = __float_as_uint(x);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ void __launch_bounds__(256) column_keys_kernel(const float* col, uint64_t n, uint32_t* keys) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
    keys[i] = order_key(col[i]);
}

// First position in sorted[0, n) whose key is >= k (or > k when `after`).
__device__ __forceinline__ uint64_t bound(const uint32_t* sorted, uint64_t n, uint32_t k, bool after) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    const uint32_t v = sorted[mid];
    if (after ? v <= k : v < k) {
      lo = mid + 1;
    } else {
      hi = mid;
    }
  }
  return lo;
}

__global__ void __launch_bounds__(256) range_count_kernel(const uint32_t* sorted, uint64_t n,
                                                          const float* lo, const float* hi,
                                                          uint32_t m, uint64_t* out) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  if (!(lo[i] <= hi[i])) {  // empty interval
    out[i] = 0;
    return;
  }
  const uint64_t a = bound(sorted, n, order_key(lo[i]), false);
  const uint64_t b = bound(sorted, n, order_key(hi[i]), true);
  out[i] = b > a ? b - a : 0;
}

}  // namespace

int count_single_predicates(const mdrq_dataset* ds, const std::vector<mdrq_pred>& preds,
                            std::vector<uint64_t>& counts) {
  counts.assign(preds.size(), 0);
  const uint64_t n = ds->n_rows;
  if (preds.empty() || n == 0) return MDRQ_OK;
  std::vector<std::vector<size_t>> by_dim(ds->n_dims);
  for (size_t k = 0; k < preds.size(); ++k) by_dim[preds[k].dim].push_back(k);
  size_t max_m = 0;
  for (const auto& v : by_dim) max_m = std::max(max_m, v.size());

  uint32_t *keys = nullptr, *sorted = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  float* d_bounds = nullptr;
  uint64_t* d_counts = nullptr;
  hipStream_t stream = nullptr;
  auto release = [&]() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (keys) (void)hipFree(keys);
    if (sorted) (void)hipFree(sorted);
    if (temp) (void)hipFree(temp);
    if (d_bounds) (void)hipFree(d_bounds);
    if (d_counts) (void)hipFree(d_counts);
    if (stream) (void)hipStreamDestroy(stream);
  };
  hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&keys, n * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&sorted, n * sizeof(uint32_t));
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortKeys(nullptr, temp_bytes, keys, sorted, n, 0, 32, stream);
  if (e == hipSuccess) e = hipMalloc(&temp, std::max<size_t>(temp_bytes, 1));
  if (e == hipSuccess) e = hipMalloc(&d_bounds, 2 * max_m * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&d_counts, max_m * sizeof(uint64_t));
  if (e != hipSuccess) {
    release();
    return e == hipErrorOutOfMemory ? fail(MDRQ_ENOMEM, "label sort buffers") : fail_hip(e, "label sort buffers");
  }
  std::vector<float> h_bounds(2 * max_m);
  std::vector<uint64_t> h_counts(max_m);
  for (uint32_t d = 0; d < ds->n_dims && e == hipSuccess; ++d) {
    const std::vector<size_t>& idx = by_dim[d];
    if (idx.empty()) continue;
    const uint32_t m = static_cast<uint32_t>(idx.size());
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>((n + 255) / 256, 65536));
    column_keys_kernel<<<blocks, 256, 0, stream>>>(ds->cols[d], n, keys);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, keys, sorted, n, 0, 32, stream);
    for (uint32_t i = 0; i < m; ++i) {
      h_bounds[i] = preds[idx[i]].lo;
      h_bounds[max_m + i] = preds[idx[i]].hi;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_bounds, h_bounds.data(), 2 * max_m * sizeof(float), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
      range_count_kernel<<<(m + 255) / 256, 256, 0, stream>>>(sorted, n, d_bounds, d_bounds + max_m, m,
                                                              d_counts);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_counts.data(), d_counts, m * sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    for (uint32_t i = 0; i < m && e == hipSuccess; ++i) counts[idx[i]] = h_counts[i];
  }
  release();
  if (e != hipSuccess) return fail_hip(e, "single-predicate counts");
  return MDRQ_OK;
}

}  // namespace mdrq
