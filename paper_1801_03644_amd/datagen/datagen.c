/*
 * Seeded synthetic inputs for multidimensional range queries.
 *
 * This module only draws numbers: it holds none of the query arithmetic.  Both the
 * GPU path and the CPU oracle consume what it writes, and nothing else is shared
 * between them.
 *
 * Random numbers come from a counter-based use of SplitMix64 (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014): the value drawn
 * for (seed, column, draw stream, counter) is the SplitMix64 output function applied
 * to key + (counter + 1) * golden-gamma, so any row can be generated independently
 * and the output does not depend on the number of threads.
 *
 * Column kinds (the workloads are shaped after the paper's Table 2 data sets and the
 * synthetic configurations derived from them):
 *   UNIFORM24  x = u * 2^-24, u uniform on {0 .. 2^24-1}: exact float32 in [0, 1).
 *   GMM        equal-weight mixture of K Gaussians (means uniform in [0,1), common
 *              sigma), rounded to float32 and then clamped to [0, 1 - 2^-24].
 *   ZIPF       integer k in {1 .. n} with P(k) proportional to k^-s, stored as float32.
 *   CORR       x = clamp(float32(y + sigma * z)) where y is the UNIFORM24 value of a
 *              source column at the same row and z is standard normal.
 *   GRID       x = float32(k * 1e-6), k uniform on {0 .. L}: a uniform [0,1] domain
 *              with L + 1 distinct levels (the SYNT-UNI reading, paper section 7.2.1).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

enum { DG_UNIFORM24 = 0, DG_GMM = 1, DG_ZIPF = 2, DG_CORR = 3, DG_GRID = 4 };
enum { DRAW_MAIN = 1, DRAW_COMP = 2, DRAW_BM1 = 3, DRAW_BM2 = 4, DRAW_MEANS = 5 };

typedef struct {
  int32_t kind;
  int32_t iparam;  /* GMM: components; ZIPF: n; CORR: source column; GRID: levels L */
  double fparam;   /* GMM: sigma; ZIPF: exponent s; CORR: sigma */
} dg_spec;

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Key of one random stream: (seed, column, draw). */
uint64_t dg_key(uint64_t seed, uint64_t col, uint64_t draw) {
  uint64_t k = sm64_mix(seed + GOLDEN);
  k = sm64_mix(k ^ (col * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
  return sm64_mix(k ^ (draw * 0xABC98388FB8FAC03ULL + 0x8CB92BA72F3D8DD7ULL));
}

static inline uint64_t dg_rnd(uint64_t key, uint64_t ctr) { return sm64_mix(key + (ctr + 1) * GOLDEN); }

/* Uniform double in [0, 1) with 53 random bits. */
static inline double dg_u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

static const float kTop = 1.0f - 0x1.0p-24f; /* largest float32 below 1 on the 2^-24 grid */

static inline float clamp01(float x) {
  if (x < 0.0f) return 0.0f;
  if (x > kTop) return kTop;
  return x;
}

static inline double std_normal(uint64_t k1, uint64_t k2, uint64_t row) {
  /* Box-Muller (Box & Muller 1958), cosine branch; 1 - u keeps the log argument > 0. */
  double u1 = dg_u01(dg_rnd(k1, row));
  double u2 = dg_u01(dg_rnd(k2, row));
  return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925 * u2);
}

static inline float uniform24_at(uint64_t key, uint64_t row) {
  return (float)((double)(dg_rnd(key, row) >> 40) * 0x1.0p-24);
}

typedef struct {
  uint64_t seed;
  uint32_t col;
  dg_spec spec;
  const uint64_t* rows; /* NULL: consecutive rows starting at row0 */
  uint64_t row0;
  uint64_t begin, end;  /* output index range of this worker */
  float* out;
  const double* cdf;    /* ZIPF cumulative table (n entries) */
  const double* means;  /* GMM component means */
} dg_job;

static void* dg_worker(void* p) {
  dg_job* j = (dg_job*)p;
  const dg_spec* s = &j->spec;
  uint64_t kmain = dg_key(j->seed, j->col, DRAW_MAIN);
  uint64_t kcomp = dg_key(j->seed, j->col, DRAW_COMP);
  uint64_t kb1 = dg_key(j->seed, j->col, DRAW_BM1);
  uint64_t kb2 = dg_key(j->seed, j->col, DRAW_BM2);
  uint64_t ksrc = s->kind == DG_CORR ? dg_key(j->seed, (uint64_t)s->iparam, DRAW_MAIN) : 0;
  for (uint64_t i = j->begin; i < j->end; ++i) {
    uint64_t row = j->rows ? j->rows[i] : j->row0 + i;
    float x;
    switch (s->kind) {
      case DG_UNIFORM24:
        x = uniform24_at(kmain, row);
        break;
      case DG_GMM: {
        int K = s->iparam;
        int c = (int)(dg_u01(dg_rnd(kcomp, row)) * K);
        if (c >= K) c = K - 1;
        double z = std_normal(kb1, kb2, row);
        x = clamp01((float)(j->means[c] + s->fparam * z));
        break;
      }
      case DG_ZIPF: {
        double u = dg_u01(dg_rnd(kmain, row));
        int lo = 0, hi = s->iparam - 1; /* smallest index with cdf > u */
        while (lo < hi) {
          int mid = lo + (hi - lo) / 2;
          if (j->cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        x = (float)(lo + 1);
        break;
      }
      case DG_CORR: {
        float y = uniform24_at(ksrc, row);
        double z = std_normal(kb1, kb2, row);
        x = clamp01((float)((double)y + s->fparam * z));
        break;
      }
      case DG_GRID: {
        uint64_t L = (uint64_t)s->iparam;
        uint64_t k = (uint64_t)(((dg_rnd(kmain, row) >> 32) * (L + 1)) >> 32);
        x = (float)((double)k * 1e-6);
        break;
      }
      default:
        x = 0.0f;
    }
    j->out[i] = x;
  }
  return NULL;
}

static int dg_run(uint64_t seed, uint32_t col, const dg_spec* spec, const uint64_t* rows,
                  uint64_t row0, uint64_t n, float* out, int threads) {
  if (!spec || !out) return -1;
  if (spec->kind < DG_UNIFORM24 || spec->kind > DG_GRID) return -1;
  if ((spec->kind == DG_GMM || spec->kind == DG_ZIPF || spec->kind == DG_GRID) && spec->iparam <= 0)
    return -1;
  double* cdf = NULL;
  double* means = NULL;
  if (spec->kind == DG_ZIPF) {
    int n_vals = spec->iparam;
    cdf = (double*)malloc(sizeof(double) * (size_t)n_vals);
    if (!cdf) return -2;
    double acc = 0.0;
    for (int k = 1; k <= n_vals; ++k) { acc += pow((double)k, -spec->fparam); cdf[k - 1] = acc; }
    for (int k = 0; k < n_vals; ++k) cdf[k] /= acc;
    cdf[n_vals - 1] = 1.0;
  }
  if (spec->kind == DG_GMM) {
    means = (double*)malloc(sizeof(double) * (size_t)spec->iparam);
    if (!means) return -2;
    uint64_t km = dg_key(seed, col, DRAW_MEANS);
    for (int c = 0; c < spec->iparam; ++c) means[c] = dg_u01(dg_rnd(km, (uint64_t)c));
  }
  if (threads < 1) threads = 1;
  if ((uint64_t)threads > n / 65536 + 1) threads = (int)(n / 65536 + 1);
  if (threads > 256) threads = 256;
  pthread_t tid[256];
  int created[256];
  dg_job jobs[256];
  for (int t = 0; t < threads; ++t) {
    dg_job* j = &jobs[t];
    j->seed = seed; j->col = col; j->spec = *spec; j->rows = rows; j->row0 = row0;
    j->begin = n * (uint64_t)t / (uint64_t)threads;
    j->end = n * (uint64_t)(t + 1) / (uint64_t)threads;
    j->out = out; j->cdf = cdf; j->means = means;
    created[t] = t < threads - 1 && pthread_create(&tid[t], NULL, dg_worker, j) == 0;
    if (!created[t]) dg_worker(j);
  }
  for (int t = 0; t < threads; ++t)
    if (created[t]) pthread_join(tid[t], NULL);
  free(cdf);
  free(means);
  return 0;
}

/* Values of column `col` for rows row0 .. row0+n-1. */
int dg_column(uint64_t seed, uint32_t col, const dg_spec* spec, uint64_t row0, uint64_t n,
              float* out, int threads) {
  return dg_run(seed, col, spec, NULL, row0, n, out, threads);
}

/* Values of column `col` at the given row indices. */
int dg_column_at(uint64_t seed, uint32_t col, const dg_spec* spec, const uint64_t* rows,
                 uint64_t n, float* out, int threads) {
  if (!rows) return -1;
  return dg_run(seed, col, spec, rows, 0, n, out, threads);
}

/* n row indices uniform on [0, n_rows) (n_rows < 2^32), from stream (seed, stream). */
int dg_rows(uint64_t seed, uint64_t stream, uint64_t n_rows, uint64_t n, uint64_t* out) {
  if (!out || n_rows == 0 || n_rows > 0xFFFFFFFFULL) return -1;
  uint64_t k = dg_key(seed, 0xFFFFFFFFULL, stream);
  for (uint64_t i = 0; i < n; ++i) out[i] = ((dg_rnd(k, i) >> 32) * n_rows) >> 32;
  return 0;
}

/* Raw 64-bit draws of stream (seed, stream), counters ctr0 .. ctr0+n-1. */
int dg_raw(uint64_t seed, uint64_t stream, uint64_t ctr0, uint64_t n, uint64_t* out) {
  if (!out) return -1;
  uint64_t k = dg_key(seed, 0xFFFFFFFEULL, stream);
  for (uint64_t i = 0; i < n; ++i) out[i] = dg_rnd(k, ctr0 + i);
  return 0;
}
