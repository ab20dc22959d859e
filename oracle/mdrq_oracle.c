/*
 * CPU oracle for exact multidimensional range queries (MDRQ).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU baseline may load this file's library.  The product path never
 * links, calls or falls back to it, and it shares no code, header or table with the
 * GPU library.
 *
 * What it computes is the paper's problem definition (section 2.1): a data set of n
 * objects with m attributes; a query gives a closed interval [lb_j, ub_j] on some of
 * the dimensions (a dimension without a predicate behaves as [-inf, +inf]); an
 * object qualifies iff every predicate holds, and the answer is the set of the
 * identifiers of the qualifying objects.  The identifier of an object is its index
 * in the data arrays (section 2.2.4), counted from 0.
 *
 * The scan follows the paper's plain sequential scan (section 2.2.4) with its early
 * break, on the column layout of the vertically partitioned scan (section 5.5):
 * objects are visited in ascending index order, predicates in the order given, and
 * the first failing predicate rejects the object.  Identifiers are therefore emitted
 * in ascending order.
 *
 * Readings where the paper is silent or inconsistent:
 *  - both interval ends are inclusive (section 2.1);
 *  - NaN bounds are rejected as invalid input, and NaN data is rejected by
 *    oracle_validate_columns; the test !(lo <= x && x <= hi) rejects NaN anyway;
 *  - lo > hi is a valid, empty interval;
 *  - a dimension may carry at most one predicate per query (section 2.1 gives one
 *    predicate p_j per dimension): a repeated dimension is invalid input;
 *  - a query with no predicate selects every object;
 *  - when the caller's buffer holds fewer identifiers than qualify, the first
 *    `capacity` identifiers are written and the exact count is still returned.
 *
 * Build: plain C99, no fast-math, no intrinsics, no threads.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EOVERFLOW (-3)
#define ORC_MAX_DIMS 128

static int orc_check(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                     const uint32_t* dims, const float* lo, const float* hi, uint32_t k) {
  if (!cols || n_dims == 0 || n_dims > ORC_MAX_DIMS) return ORC_EINVAL;
  if (n_rows > 0xFFFFFFFFULL) return ORC_EINVAL;
  if (k > 0 && (!dims || !lo || !hi)) return ORC_EINVAL;
  if (k > n_dims) return ORC_EINVAL;
  for (uint32_t j = 0; j < n_dims; ++j)
    if (!cols[j] && n_rows > 0) return ORC_EINVAL;
  for (uint32_t p = 0; p < k; ++p) {
    if (dims[p] >= n_dims) return ORC_EINVAL;
    if (isnan(lo[p]) || isnan(hi[p])) return ORC_EINVAL;
    for (uint32_t q = 0; q < p; ++q)
      if (dims[q] == dims[p]) return ORC_EINVAL;
  }
  return ORC_OK;
}

/* Does object i satisfy every predicate?  Early break on the first failure. */
static int orc_match(const float* const* cols, uint64_t i, const uint32_t* dims,
                     const float* lo, const float* hi, uint32_t k) {
  for (uint32_t p = 0; p < k; ++p) {
    float x = cols[dims[p]][i];
    if (!(lo[p] <= x && x <= hi[p])) return 0;
  }
  return 1;
}

/* Ascending identifiers of the qualifying objects.  Writes min(count, capacity)
 * identifiers to out_ids (may be NULL when capacity is 0) and the exact count to
 * *count.  Returns ORC_OK, ORC_EOVERFLOW (count > capacity) or ORC_EINVAL. */
int oracle_query(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                 const uint32_t* dims, const float* lo, const float* hi, uint32_t k,
                 uint32_t* out_ids, uint64_t capacity, uint64_t* count) {
  if (!count || (capacity > 0 && !out_ids)) return ORC_EINVAL;
  int rc = orc_check(cols, n_dims, n_rows, dims, lo, hi, k);
  if (rc) return rc;
  uint64_t c = 0;
  for (uint64_t i = 0; i < n_rows; ++i) {
    if (orc_match(cols, i, dims, lo, hi, k)) {
      if (c < capacity) out_ids[c] = (uint32_t)i;
      ++c;
    }
  }
  *count = c;
  return c > capacity ? ORC_EOVERFLOW : ORC_OK;
}

/* The same answer as a bitmap: bit (i mod 64) of word i/64 is set iff object i
 * qualifies; bits of positions >= n_rows are zero.  `words` must hold
 * ceil(n_rows / 64) words. */
int oracle_bitmap(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                  const uint32_t* dims, const float* lo, const float* hi, uint32_t k,
                  uint64_t* words, uint64_t* count) {
  if (!count || (n_rows > 0 && !words)) return ORC_EINVAL;
  int rc = orc_check(cols, n_dims, n_rows, dims, lo, hi, k);
  if (rc) return rc;
  uint64_t n_words = (n_rows + 63) / 64;
  memset(words, 0, n_words * sizeof(uint64_t));
  uint64_t c = 0;
  for (uint64_t i = 0; i < n_rows; ++i) {
    if (orc_match(cols, i, dims, lo, hi, k)) {
      words[i / 64] |= (uint64_t)1 << (i % 64);
      ++c;
    }
  }
  *count = c;
  return ORC_OK;
}

/* Number of qualifying objects only. */
int oracle_count(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                 const uint32_t* dims, const float* lo, const float* hi, uint32_t k,
                 uint64_t* count) {
  return oracle_query(cols, n_dims, n_rows, dims, lo, hi, k, NULL, 0, count) == ORC_EINVAL
             ? ORC_EINVAL
             : ORC_OK;
}

/* Does object `row` qualify?  1 / 0, or ORC_EINVAL. */
int oracle_match_row(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                     const uint32_t* dims, const float* lo, const float* hi, uint32_t k,
                     uint64_t row) {
  int rc = orc_check(cols, n_dims, n_rows, dims, lo, hi, k);
  if (rc) return rc;
  if (row >= n_rows) return ORC_EINVAL;
  return orc_match(cols, row, dims, lo, hi, k);
}

/* Data validation of a load: ORC_EINVAL if any value is NaN, else ORC_OK, with
 * the per-column minimum and maximum (NULL to skip). */
int oracle_validate_columns(const float* const* cols, uint32_t n_dims, uint64_t n_rows,
                            float* col_min, float* col_max) {
  if (!cols || n_dims == 0 || n_dims > ORC_MAX_DIMS || n_rows > 0xFFFFFFFFULL) return ORC_EINVAL;
  for (uint32_t j = 0; j < n_dims; ++j) {
    if (!cols[j] && n_rows > 0) return ORC_EINVAL;
    float mn = INFINITY, mx = -INFINITY;
    for (uint64_t i = 0; i < n_rows; ++i) {
      float x = cols[j][i];
      if (isnan(x)) return ORC_EINVAL;
      if (x < mn) mn = x;
      if (x > mx) mx = x;
    }
    if (col_min) col_min[j] = mn;
    if (col_max) col_max[j] = mx;
  }
  return ORC_OK;
}
