/*
 * Plain C oracle for DBSCAN (float64, brute force) -- TEST INFRASTRUCTURE ONLY.
 *
 * The GPU library is checked against this file and the numpy oracle next to
 * it; the benchmark also times it as the CPU baseline.  The product path never
 * links or calls it.  It shares no code, header or constant with the GPU
 * sources.
 *
 * What it computes (the paper's Section II definitions and serial steps):
 *   step 1  squared distance of every pair in float64, compared with eps^2
 *           (Section IV-A: compare against eps^2, no square root; Section
 *           IV-B: distance <= eps^2 means "in the neighbourhood");
 *   step 2  neighbour counts (the point itself included) and core flags,
 *           core = count >= MinPts (Section II, definition 2);
 *   step 3  clusters = connected components of the core-core eps-graph,
 *           found by breadth-first search started from each unvisited core
 *           point in ascending index order, so the cluster id is the lowest
 *           core index of the component; a non-core point takes the cluster
 *           of its lowest-index core neighbour, else it is noise (-1).
 *
 * Arithmetic: coordinates are widened exactly from float32; for each pair
 * s = 0; for k in 0..d-1 { t = x_ik - x_jk; s = s + t*t; } with every
 * operation rounded separately.  Build with -ffp-contract=off so that no
 * multiply is fused into the following add.  eps^2 is eps*eps rounded once.
 *
 * OpenMP only splits independent rows across threads; no result depends on
 * the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double pair_sq(const float *a, const float *b, int32_t d) {
  double s = 0.0;
  for (int32_t k = 0; k < d; ++k) {
    double t = (double)a[k] - (double)b[k];
    double tt = t * t;
    s = s + tt;
  }
  return s;
}

static int set_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  return omp_get_max_threads();
#else
  (void)threads;
  return 1;
#endif
}

int oracle_max_threads(int threads) { return set_threads(threads); }

/* counts[i] = |{ j : s(i,j) <= eps^2 }| for rows i = rows[0..m-1] (or every
 * row when rows == NULL, m == n). */
int oracle_row_counts(const float *x, int64_t n, int32_t d, double eps, const int64_t *rows,
                      int64_t m, int32_t *out, int threads) {
  if (!x || !out || n < 1 || d < 1 || m < 0) return -1;
  const double eps2 = eps * eps;
  set_threads(threads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < m; ++r) {
    const int64_t i = rows ? rows[r] : r;
    const float *xi = x + i * d;
    int32_t c = 0;
    for (int64_t j = 0; j < n; ++j)
      if (pair_sq(xi, x + j * d, d) <= eps2) ++c;
    out[r] = c;
  }
  return 0;
}

/* flags[j] = (s(i,j) <= eps^2) for one row i. */
int oracle_row_neighbours(const float *x, int64_t n, int32_t d, double eps, int64_t i,
                          uint8_t *flags) {
  if (!x || !flags || i < 0 || i >= n) return -1;
  const double eps2 = eps * eps;
  const float *xi = x + i * d;
  for (int64_t j = 0; j < n; ++j) flags[j] = pair_sq(xi, x + j * d, d) <= eps2;
  return 0;
}

/* Full DBSCAN.  labels: -1 noise, else lowest core index of the cluster. */
int oracle_dbscan(const float *x, int64_t n, int32_t d, double eps, int32_t minpts,
                  int32_t *labels, uint8_t *core, int32_t *counts, int threads) {
  if (!x || !labels || !core || !counts || n < 1 || d < 1 || minpts < 1) return -1;
  const double eps2 = eps * eps;
  int rc = oracle_row_counts(x, n, d, eps, NULL, n, counts, threads);
  if (rc) return rc;
  for (int64_t i = 0; i < n; ++i) core[i] = counts[i] >= minpts;
  for (int64_t i = 0; i < n; ++i) labels[i] = -1;

  int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!queue) return -2;
  /* step 3: breadth-first search over core points, seeds in ascending order.
   * Every core point reached from seed s gets label s, whatever the order in
   * which a level is queued: each q belongs to one iteration of the parallel
   * loop, which labels it and takes the next queue slot atomically. */
  for (int64_t s = 0; s < n; ++s) {
    if (!core[s] || labels[s] != -1) continue;
    int64_t head = 0, tail = 0;
    labels[s] = (int32_t)s;
    queue[tail++] = s;
    while (head < tail) {
      const int64_t p = queue[head++];
      const float *xp = x + p * d;
      int64_t next = tail;
#pragma omp parallel for schedule(static)
      for (int64_t q = 0; q < n; ++q) {
        if (core[q] && labels[q] == -1 && pair_sq(xp, x + q * d, d) <= eps2) {
          int64_t slot;
          labels[q] = (int32_t)s;
#pragma omp atomic capture
          slot = next++;
          queue[slot] = q;
        }
      }
      tail = next;
    }
  }
  /* border points: cluster of the lowest-index core neighbour */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    if (core[i]) continue;
    const float *xi = x + i * d;
    for (int64_t j = 0; j < n; ++j) {
      if (core[j] && pair_sq(xi, x + j * d, d) <= eps2) {
        labels[i] = labels[j];
        break;
      }
    }
  }
  free(queue);
  return 0;
}

/* Label of one point given the full core flags: lowest-index core neighbour's
 * label is looked up by the caller; this returns that neighbour's index, or -1. */
int64_t oracle_first_core_neighbour(const float *x, int64_t n, int32_t d, double eps,
                                    const uint8_t *core, int64_t i) {
  if (!x || !core || i < 0 || i >= n) return -2;
  const double eps2 = eps * eps;
  const float *xi = x + i * d;
  for (int64_t j = 0; j < n; ++j)
    if (core[j] && pair_sq(xi, x + j * d, d) <= eps2) return j;
  return -1;
}
