// Learned selectivity estimator: kernels for gfx950.
//
// A small MLP (features -> 64 -> 64 -> d+1, GELU) corrects histogram estimates of the
// selectivity of each queried dimension and of the whole query.  The paper notes that
// evaluating the most selective dimension first needs selectivity estimates (section
// 2.2.4) and leaves it as future work (section 8); the estimator only orders a query's
// predicates, so results never depend on it.
//
// Kernels:
//  * sample_sort_kernel: per column, a strided sample of up to 16384 rows sorted by a
//    bitonic network in LDS; equi-depth boundaries are read off the sorted sample.
//  * features_kernel: per (query, dimension) the histogram CDF of both bounds, the
//    histogram estimate and the covered fraction of each bin, written as bfloat16 rows,
//    and the base estimate the network corrects.
//  * order_fused_kernel: one query's features, network and the ranking of its
//    predicates in one workgroup, ahead of the scan on the same stream.
//  * gemm_bf16_kernel: C = A * B with bfloat16 operands and float32 accumulation on the
//    matrix cores (v_mfma_f32_16x16x32_bf16); four waves per 16x16 tile of C split the
//    k steps, operands read through strides so that transposed products need no copies.
//  * small elementwise kernels: bias + GELU (and its derivative), the masked squared
//    loss and its gradient, column sums (bias gradients), Adam, float32 -> bfloat16.
#include <hip/hip_bfloat16.h>

#include <cmath>
#include <cstring>

#include "mdrq_internal.h"

namespace mdrq {
namespace {

typedef short short8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest, ties to even (inputs are finite).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  const float phi = 0.3989422804014327f * expf(-0.5f * z * z);
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * phi;
}

// ---------------------------------------------------------------- histograms

constexpr int kSortThreads = 1024;

__global__ void __launch_bounds__(kSortThreads) sample_sort_kernel(HistArgs a) {
  __shared__ float s[kSampleMax];
  const uint32_t j = blockIdx.x;
  const float* col = a.cols[j];
  const uint32_t m = a.m;          // sample size (<= kSampleMax)
  const uint32_t p2 = a.m_pow2;    // power of two >= m
  for (uint32_t i = threadIdx.x; i < p2; i += kSortThreads) {
    if (i < m) {
      const uint64_t row = static_cast<uint64_t>(i) * a.n_rows / m;
      s[i] = col[row];
    } else {
      s[i] = INFINITY;
    }
  }
  __syncthreads();
  for (uint32_t k = 2; k <= p2; k <<= 1) {
    for (uint32_t h = k >> 1; h > 0; h >>= 1) {
      for (uint32_t i = threadIdx.x; i < p2; i += kSortThreads) {
        const uint32_t o = i ^ h;
        if (o > i) {
          const bool up = (i & k) == 0;
          const float x = s[i], y = s[o];
          if ((x > y) == up) {
            s[i] = y;
            s[o] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x <= kBins) {
    const uint32_t b = threadIdx.x;
    const uint32_t idx = b < kBins ? (b * m) / kBins : m - 1;
    a.bounds[j * (kBins + 1) + b] = s[idx];
  }
}

// ---------------------------------------------------------------- features

__device__ float hist_cdf(const float* b, float x) {
  if (x < b[0]) return 0.0f;
  if (x >= b[kBins]) return 1.0f;
  for (int i = 0; i < kBins; ++i)
    if (b[i] <= x && x < b[i + 1]) return (static_cast<float>(i) + (x - b[i]) / (b[i + 1] - b[i])) / kBins;
  return 1.0f;
}

// Log scale of a selectivity: -ln(max(s, 1/N)) / ln N.
__device__ __forceinline__ float log_scale(float s, float inv_rows, float inv_ln_rows) {
  return -logf(s > inv_rows ? s : inv_rows) * inv_ln_rows;
}

// Features of one dimension of one query (kFeatPerDim bfloat16 values into row) and
// its histogram estimate on the log scale (returned; 0 if not restricted).
__device__ float dim_features(const float* b, float lo, float hi, bool restricted, uint16_t* row,
                              float inv_rows, float inv_ln_rows) {
  if (!restricted) {
    row[0] = to_bf16(-1.0f);
    row[1] = to_bf16(-1.0f);
    row[2] = 0;
    for (int i = 0; i < kBins; ++i) row[3 + i] = to_bf16(1.0f);
    return 0.0f;
  }
  row[0] = to_bf16(hist_cdf(b, lo));
  row[1] = to_bf16(hist_cdf(b, hi));
  float sum = 0.0f;
  for (int i = 0; i < kBins; ++i) {
    const float a0 = b[i], a1 = b[i + 1];
    float c;
    if (a1 > a0) {
      const float top = hi < a1 ? hi : a1;
      const float bot = lo > a0 ? lo : a0;
      c = top > bot ? (top - bot) / (a1 - a0) : 0.0f;
    } else {
      c = (lo <= a0 && a0 <= hi) ? 1.0f : 0.0f;
    }
    row[3 + i] = to_bf16(c);
    sum += c;
  }
  // Histogram estimate: the mean coverage (H(hi) - H(lo) without the cancellation).
  const float y = log_scale(sum * (1.0f / kBins), inv_rows, inv_ln_rows);
  row[2] = to_bf16(y);
  return y;
}

// One thread per (query, dimension); qd holds (lo, hi, restricted) per (query, dimension).
__global__ void features_kernel(FeatureArgs f) {
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<uint64_t>(f.n) * f.d) return;
  const float* qd = f.qd + t * 3;
  const uint32_t j = static_cast<uint32_t>(t % f.d);
  const uint64_t q = t / f.d;
  f.base[q * (f.d + 1) + j] = dim_features(f.bounds + j * (kBins + 1), qd[0], qd[1], qd[2] != 0.0f,
                                           f.x + t * kFeatPerDim, f.inv_rows, f.inv_ln_rows);
}

// Joint base estimate of each query: min(1, sum of its per-dimension estimates), the
// independence product on the log scale.
__global__ void base_joint_kernel(float* base, uint32_t n, uint32_t d) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float* row = base + static_cast<uint64_t>(q) * (d + 1);
  float s = 0.0f;
  for (uint32_t j = 0; j < d; ++j) s += row[j];
  row[d] = s < 1.0f ? s : 1.0f;
}

// ---------------------------------------------------------------- matrix products

// C[m][n] = sum_k A(m, k) * B(k, n) (+ bias[n]) (+ add[m][n]); A(m,k) = a[m*a_m + k*a_k] and
// B(k,n) = b[k*b_k + n*b_n] are bfloat16, out of range reads are zero.  A workgroup
// computes a 16x16 tile of C with 16x16x32 matrix-core steps (lane 16 j + r holds k
// values 8 j .. 8 j + 7 of the step for row r of A and column r of B: any k order
// shared by both operands gives the same sum); its kGemmWaves waves take
// every kGemmWaves-th step (wave w: steps w, w + kGemmWaves, ...), so the chains of
// dependent operand loads are that many times shorter, and wave 0 adds the waves'
// partial tiles in wave order.  (The products are small and the operands are read
// through strides: the loads' latency, not the matrix cores, sets the time.)
constexpr uint32_t kGemmWaves = 4;
__global__ void __launch_bounds__(64 * kGemmWaves) gemm_bf16_kernel(GemmArgs g) {
  __shared__ floatx4 part[kGemmWaves - 1][64];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t m0 = blockIdx.y * 16, n0 = blockIdx.x * 16;
  const uint32_t r = lane % 16;        // row of A / column of B and C held by this lane
  const uint32_t kq = (lane / 16) * 8; // first of the 8 k values held by this lane
  const uint32_t am = m0 + r, bn = n0 + r;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (uint32_t k0 = 32 * wave; k0 < g.K; k0 += 32 * kGemmWaves) {
    short8 av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t k = k0 + kq + i;
      av[i] = (am < g.M && k < g.K)
                  ? static_cast<short>(g.a[static_cast<uint64_t>(am) * g.a_m + static_cast<uint64_t>(k) * g.a_k])
                  : static_cast<short>(0);
      bv[i] = (bn < g.N && k < g.K)
                  ? static_cast<short>(g.b[static_cast<uint64_t>(k) * g.b_k + static_cast<uint64_t>(bn) * g.b_n])
                  : static_cast<short>(0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                  acc, 0, 0, 0);
  }
  if (wave > 0) part[wave - 1][lane] = acc;
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (uint32_t w = 0; w + 1 < kGemmWaves; ++w) {
    const floatx4 o = part[w][lane];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += o[i];
  }
  // acc[i] holds C[m0 + 4*(lane/16) + i][n0 + lane%16].
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t m = m0 + 4 * (lane / 16) + i, n = n0 + r;
    if (m < g.M && n < g.N) {
      const uint64_t o = static_cast<uint64_t>(m) * g.c_ld + n;
      float v = acc[i] + (g.bias ? g.bias[n] : 0.0f);
      if (g.add) v += g.add[o];
      if (g.c) g.c[o] = v;
      if (g.act) g.act[o] = to_bf16(g.gelu ? gelu(v) : v);
    }
  }
}

// ---------------------------------------------------------------- elementwise

// dY = 2 * mask * (Y - T) / count (float32, and bfloat16 for the products); the
// loss of the batch is accumulated into *loss.
__global__ void loss_grad_kernel(LossArgs l) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<uint64_t>(l.rows) * l.cols) return;
  const float d = (l.y[i] - l.t[i]) * l.mask[i];
  const float g = 2.0f * d * l.inv_count;
  if (d != 0.0f) atomicAdd(l.loss, d * d * l.inv_count);
  l.dy[i] = g;
  l.dyb[i] = to_bf16(g);
}

// dZ = dH * gelu'(Z) (float32, and bfloat16 for the products).
__global__ void gelu_back_kernel(const float* dh, const float* z, float* dz, uint16_t* dzb,
                                 uint64_t n) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = dh[i] * gelu_grad(z[i]);
  dz[i] = v;
  dzb[i] = to_bf16(v);
}

// out[c] = sum over rows r of in[r][c] (bias gradients).  A workgroup takes 64 columns
// with 16 waves: wave w sums rows w, w + 16, ... of its lane's column into four partial
// sums (four loads in flight), then wave 0 adds the 16 waves' sums.
constexpr uint32_t kColsumWaves = 16;
__global__ void __launch_bounds__(64 * kColsumWaves) colsum_kernel(const float* in, uint32_t rows, uint32_t cols,
                                                                   float* out) {
  __shared__ float part[kColsumWaves][64];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t c = blockIdx.x * 64 + lane;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  if (c < cols) {
    uint32_t r = wave;
    for (; r + 3 * kColsumWaves < rows; r += 4 * kColsumWaves) {
      s0 += in[static_cast<uint64_t>(r) * cols + c];
      s1 += in[static_cast<uint64_t>(r + kColsumWaves) * cols + c];
      s2 += in[static_cast<uint64_t>(r + 2 * kColsumWaves) * cols + c];
      s3 += in[static_cast<uint64_t>(r + 3 * kColsumWaves) * cols + c];
    }
    for (; r < rows; r += kColsumWaves) s0 += in[static_cast<uint64_t>(r) * cols + c];
  }
  part[wave][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (wave == 0 && c < cols) {
    float t = 0.0f;
#pragma unroll
    for (uint32_t w = 0; w < kColsumWaves; ++w) t += part[w][lane];
    out[c] = t;
  }
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, uint64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void to_bf16_kernel(const float* src, uint64_t n, uint16_t* dst) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = to_bf16(src[i]);
}

// Training targets: y = -ln(max(s, 1/N)) / ln N where a selectivity is given (s >= 0),
// mask 1 there and 0 elsewhere.
__global__ void targets_kernel(const float* sel, uint64_t n, float inv_rows, float inv_ln_rows,
                               float* t, float* mask) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = sel[i];
  const bool present = s >= 0.0f;
  t[i] = present ? -logf(s > inv_rows ? s : inv_rows) * inv_ln_rows : 0.0f;
  mask[i] = present ? 1.0f : 0.0f;
}

// Estimates from network outputs: s = N^-clamp(y, 0, 1); 1 for a dimension the query
// does not restrict.
__global__ void to_selectivity_kernel(const float* y, const float* qd, uint32_t n, uint32_t d,
                                      float ln_rows, float* sel) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint32_t o = d + 1;
  if (i >= static_cast<uint64_t>(n) * o) return;
  const uint64_t q = i / o;
  const uint32_t j = static_cast<uint32_t>(i % o);
  if (j < d && qd[(q * d + j) * 3 + 2] == 0.0f) {
    sel[i] = 1.0f;
    return;
  }
  const float v = fminf(fmaxf(y[i], 0.0f), 1.0f);
  sel[i] = expf(-v * ln_rows);
}

// Gather rows of training data: dst[i] = src[idx[i]] for row-major rows of `width`
// elements of `elem` bytes (elem 2 or 4).
__global__ void gather_rows_kernel(const uint8_t* src, const uint32_t* idx, uint32_t n,
                                   uint32_t row_bytes, uint8_t* dst) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t words = row_bytes / 4;
  if (i >= static_cast<uint64_t>(n) * words) return;
  const uint64_t r = i / words, w = i % words;
  reinterpret_cast<uint32_t*>(dst)[i] =
      reinterpret_cast<const uint32_t*>(src)[static_cast<uint64_t>(idx[r]) * words + w];
}

// One query's evaluation order in one workgroup: features, the three layers (dot
// products on the vector units -- a single row is no matrix product), the estimates,
// and the rank of each of the plan's predicates by ascending estimated selectivity
// (ties keep plan order): order[rank] = position in the plan.  The per-dimension
// arrays are read through the kernel-argument segment pointer (indexed per lane).
typedef __attribute__((address_space(4))) const OrderArgs korder;

__device__ __forceinline__ float bf16_val(uint16_t v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
__device__ __forceinline__ float in_val(float v) { return v; }
__device__ __forceinline__ float in_val(uint16_t v) { return bf16_val(v); }

// out[j] (for j < n_out, left in part[0][j]) = sum_i in[i] * W[i][j] over the 256
// threads of the workgroup: thread t takes column j = j0 + t % 64 and every fourth
// input row from t / 64; four independent partial sums keep several weight loads in
// flight; the four row partitions are added in LDS.
template <class T>
__device__ void gemv(const T* in, uint32_t n_in, const uint16_t* W, uint32_t n_out, float (*part)[256]) {
  const uint32_t t = threadIdx.x;
  const uint32_t c = t & 63, r0 = t >> 6;
  for (uint32_t j0 = 0; j0 < n_out; j0 += 64) {
    const uint32_t j = j0 + c;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (j < n_out) {
      uint32_t i = r0;
      for (; i + 12 < n_in; i += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[u] += in_val(in[i + 4 * u]) * bf16_val(W[static_cast<uint64_t>(i + 4 * u) * n_out + j]);
      }
      for (; i < n_in; i += 4) acc[0] += in_val(in[i]) * bf16_val(W[static_cast<uint64_t>(i) * n_out + j]);
    }
    part[r0][j0 + c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  __syncthreads();
  for (uint32_t j = t; j < n_out; j += 256) part[0][j] = (part[0][j] + part[1][j]) + (part[2][j] + part[3][j]);
  __syncthreads();
}

// One query's evaluation order in one workgroup: features, the three layers (dot
// products on the vector units -- a single row is no matrix product), the estimates,
// and the rank of each of the plan's predicates by ascending estimated selectivity
// (ties keep plan order): order[rank] = position in the plan.  The per-dimension
// arrays are read through the kernel-argument segment pointer (indexed per lane).
__global__ void __launch_bounds__(256) order_fused_kernel(OrderArgs a_) {
  korder& a = *(korder*)__builtin_amdgcn_kernarg_segment_ptr();
  __shared__ uint16_t s_x[MDRQ_MAX_DIMS * kFeatPerDim];
  __shared__ float s_base[MDRQ_MAX_DIMS + 1];
  __shared__ float s_h1[256];
  __shared__ float s_h2[256];
  __shared__ float s_part[4][256];
  __shared__ float s_sel[MDRQ_MAX_DIMS + 1];
  (void)a_;
  const uint32_t t = threadIdx.x;
  const uint32_t d = a.d, H = a.H, O = d + 1, F = d * kFeatPerDim;
  if (t < d) {
    const bool r = (a.restricted[t >> 5] >> (t & 31)) & 1u;
    s_base[t] = dim_features(a.bounds + t * (kBins + 1), a.lo[t], a.hi[t], r, s_x + t * kFeatPerDim,
                             a.inv_rows, a.inv_ln_rows);
  }
  __syncthreads();
  if (t == 0) {
    float sum = 0.0f;
    for (uint32_t j = 0; j < d; ++j) sum += s_base[j];
    s_base[d] = sum < 1.0f ? sum : 1.0f;
  }
  gemv(s_x, F, a.wb + a.oW1, H, s_part);
  if (t < H) s_h1[t] = bf16_val(to_bf16(gelu(s_part[0][t] + a.params[a.ob1 + t])));
  __syncthreads();
  gemv(s_h1, H, a.wb + a.oW2, H, s_part);
  if (t < H) s_h2[t] = bf16_val(to_bf16(gelu(s_part[0][t] + a.params[a.ob2 + t])));
  __syncthreads();
  gemv(s_h2, H, a.wb + a.oW3, O, s_part);
  for (uint32_t o = t; o < O; o += 256) {
    const float v = fminf(fmaxf(s_part[0][o] + a.params[a.ob3 + o] + s_base[o], 0.0f), 1.0f);
    s_sel[o] = expf(-v * a.ln_rows);
  }
  __syncthreads();
  if (t < a.k) {
    const float si = s_sel[a.dims[t]];
    uint32_t rank = 0;
    for (uint32_t j = 0; j < a.k; ++j) {
      const float sj = s_sel[a.dims[j]];
      rank += (sj < si || (sj == si && j < t)) ? 1u : 0u;
    }
    a.order[rank] = t;
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t t) { return static_cast<uint32_t>((n + t - 1) / t); }

}  // namespace

hipError_t launch_sample_sort(const HistArgs& a, uint32_t n_cols, hipStream_t s) {
  sample_sort_kernel<<<n_cols, kSortThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_features(const FeatureArgs& f, hipStream_t s) {
  const uint64_t n = static_cast<uint64_t>(f.n) * f.d;
  if (n == 0) return hipSuccess;
  features_kernel<<<blocks_for(n, 256), 256, 0, s>>>(f);
  base_joint_kernel<<<blocks_for(f.n, 256), 256, 0, s>>>(f.base, f.n, f.d);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  gemm_bf16_kernel<<<dim3((g.N + 15) / 16, (g.M + 15) / 16), 64 * kGemmWaves, 0, s>>>(g);
  return hipGetLastError();
}

hipError_t launch_loss_grad(const LossArgs& l, hipStream_t s) {
  loss_grad_kernel<<<blocks_for(static_cast<uint64_t>(l.rows) * l.cols, 256), 256, 0, s>>>(l);
  return hipGetLastError();
}

hipError_t launch_gelu_back(const float* dh, const float* z, float* dz, uint16_t* dzb, uint64_t n,
                            hipStream_t s) {
  gelu_back_kernel<<<blocks_for(n, 256), 256, 0, s>>>(dh, z, dz, dzb, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* in, uint32_t rows, uint32_t cols, float* out, hipStream_t s) {
  colsum_kernel<<<blocks_for(cols, 64), 64 * kColsumWaves, 0, s>>>(in, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint64_t n, float lr,
                       int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, static_cast<float>(step));
  const float c2 = 1.0f - powf(b2, static_cast<float>(step));
  adam_kernel<<<blocks_for(n, 256), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint64_t n, uint16_t* dst, hipStream_t s) {
  to_bf16_kernel<<<blocks_for(n, 256), 256, 0, s>>>(src, n, dst);
  return hipGetLastError();
}

hipError_t launch_targets(const float* sel, uint32_t n, uint32_t o, uint64_t n_rows, float* t,
                          float* mask, hipStream_t s) {
  const uint64_t total = static_cast<uint64_t>(n) * o;
  const double rows = static_cast<double>(n_rows);
  targets_kernel<<<blocks_for(total, 256), 256, 0, s>>>(
      sel, total, static_cast<float>(1.0 / rows), static_cast<float>(1.0 / std::log(rows)), t, mask);
  return hipGetLastError();
}

hipError_t launch_order_fused(const OrderArgs& a, hipStream_t s) {
  order_fused_kernel<<<1, 256, 0, s>>>(a);
  return hipGetLastError();
}


hipError_t launch_to_selectivity(const float* y, const float* qd, uint32_t n, uint32_t d,
                                 uint64_t n_rows, float* sel, hipStream_t s) {
  const uint64_t total = static_cast<uint64_t>(n) * (d + 1);
  to_selectivity_kernel<<<blocks_for(total, 256), 256, 0, s>>>(
      y, qd, n, d, static_cast<float>(std::log(static_cast<double>(n_rows))), sel);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const void* src, const uint32_t* idx, uint32_t n, uint32_t row_bytes,
                              void* dst, hipStream_t s) {
  const uint64_t words = static_cast<uint64_t>(n) * (row_bytes / 4);
  if (words == 0) return hipSuccess;
  gather_rows_kernel<<<blocks_for(words, 256), 256, 0, s>>>(
      static_cast<const uint8_t*>(src), idx, n, row_bytes, static_cast<uint8_t*>(dst));
  return hipGetLastError();
}

}  // namespace mdrq
