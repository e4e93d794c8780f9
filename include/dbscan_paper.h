/*
 * libdbscan -- the paper's own kernel designs, kept beside the main path as
 * measured ablations (Wang et al., "Design and optimization of DBSCAN
 * Algorithm based on CUDA", Sections IV-A to IV-C and VI; Tables III-IV).
 *
 * The main path (dbscan.h) never stores an n x n matrix.  These entry points
 * reproduce the paper's three-step design on the GPU instead, so that its
 * steps can be timed and checked on the same data:
 *   step 1  the float distance matrix (Section IV-A), by four kernels of
 *           Table III: one thread per row with row-major points and row
 *           writes; transposed points point[d][n] with column writes
 *           (coalesced); tiles of points in LDS with the goal point in
 *           registers; and that with the inner loop unrolled 32 times;
 *   step 2  the byte cluster matrix and the valid vector (Section IV-B), from
 *           the distance matrix, fused with the distance (Section IV-B.1), or
 *           fused with the hoisted form T + P[n] - (X p_x + Y p_y + Z p_z)
 *           (Section IV-B.2);
 *   step 3  the merge of Section IV-C (every valid cluster sharing a core
 *           point with a target is merged into it, targets in ascending
 *           order, repeated until nothing merges) or the Warshall transitive
 *           closure that Section VI abandoned (one launch per point).
 * The distance matrix holds float32 squared distances computed in coordinate
 * order with every operation rounded alone.  Every decision of the cluster
 * matrix equals the float64 definition of dbscan.h: float32 values inside a
 * rigorous band around eps^2 are re-evaluated in float64, so counts, valid
 * flags (= core flags) and labels equal those of dbscan_fit.
 *
 * Conventions are those of dbscan.h (DEVICE / HOST pointers, stream as void*,
 * return codes).  Inputs must be finite.  1 <= d <= 4 and
 * 1 <= n <= DBSCAN_PAPER_MAX_N: the matrices need 4 n^2 and n^2 bytes.
 */
#ifndef DBSCAN_PAPER_MI355X_H
#define DBSCAN_PAPER_MI355X_H

#include <stdint.h>

#include "dbscan.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DBSCAN_PAPER_MAX_N 131072LL

/* Kernels of Section IV-A (Table III). */
#define DBSCAN_PAPER_DIST_BASELINE 1   /* thread per row, points n x d, writes row i */
#define DBSCAN_PAPER_DIST_COALESCED 2  /* points as point[d][n], writes column i */
#define DBSCAN_PAPER_DIST_SHARED 3     /* + 64-point tiles in LDS, goal point in registers */
#define DBSCAN_PAPER_DIST_UNROLLED 4   /* + inner loop unrolled 32 times */
/* Kernels of Section IV-B (Table IV). */
#define DBSCAN_PAPER_CLUSTER_FROM_DIST 5  /* reads the distance matrix */
#define DBSCAN_PAPER_CLUSTER_FUSED 6      /* distance and cluster matrix in one pass */
#define DBSCAN_PAPER_CLUSTER_HOISTED 7    /* fused, with the hoisted form */
/* Merges of Section IV-C and Section VI. */
#define DBSCAN_PAPER_MERGE_TARGETS 8
#define DBSCAN_PAPER_MERGE_WARSHALL 9

/*
 * dbscan_paper_distance -- step 1 as a float distance matrix (Section IV-A).
 *   points  DEVICE const float[n*d], row-major.
 *   kernel  DBSCAN_PAPER_DIST_* (1-4).
 *   dist    DEVICE float[n*n] out: dist[i*n + j] = the float32 squared
 *           distance of points i and j (coordinate order, unfused); the
 *           matrix is symmetric bit for bit.
 * Asynchronous on `stream`.  DBSCAN_E_INVAL for bad arguments.
 */
int dbscan_paper_distance(const float *points, int64_t n, int32_t d, int32_t kernel, float *dist,
                          void *stream);

/*
 * dbscan_paper_cluster -- step 2 (Section IV-B): the byte cluster matrix,
 * valid vector and neighbour counts.
 *   points     DEVICE const float[n*d], row-major.
 *   dist       DEVICE const float[n*n] from dbscan_paper_distance (kernel 5
 *              only; NULL otherwise).
 *   kernel     DBSCAN_PAPER_CLUSTER_* (5-7).
 *   cluster    DEVICE uint8[n*n] out: cluster[i*n + j] = 1 iff point j is in
 *              the eps-neighbourhood of point i (the primitive cluster of i),
 *              else 0; symmetric.
 *   valid      DEVICE uint8[n] out: 1 iff count >= minpts (a core point, whose
 *              primitive cluster is valid).
 *   counts     DEVICE int32[n] out: neighbourhood sizes, the point included.
 *   rechecked  HOST uint64*, nullable: when given, the call waits for the
 *              stream and stores the number of pairs re-evaluated in float64.
 */
int dbscan_paper_cluster(const float *points, const float *dist, int64_t n, int32_t d,
                         double eps, int32_t minpts, int32_t kernel, uint8_t *cluster,
                         uint8_t *valid, int32_t *counts, uint64_t *rechecked, void *stream);

/*
 * dbscan_paper_merge -- step 3: canonical labels from the cluster matrix.
 *   cluster  DEVICE uint8[n*n] from dbscan_paper_cluster.  Targets (kernel 8)
 *            merge in place: afterwards the row of each surviving target is
 *            the union of its cluster's primitive rows; the rows of non-core
 *            points are unchanged.  Warshall (kernel 9) leaves it unchanged.
 *   valid    DEVICE const uint8[n] from dbscan_paper_cluster.
 *   kernel   DBSCAN_PAPER_MERGE_TARGETS or DBSCAN_PAPER_MERGE_WARSHALL.
 *   labels   DEVICE int32[n] out: as in dbscan_fit (-1 noise, else the lowest
 *            core index of the cluster; a border point takes the label of its
 *            lowest-index core neighbour).
 *   alive    DEVICE uint8[n] out, nullable: targets only, 1 for the clusters
 *            that survive the merge.
 *   launches HOST int64*, nullable: kernel launches the merge made.
 * Synchronous: the host reads flags between launches (the merge iterates).
 */
int dbscan_paper_merge(uint8_t *cluster, const uint8_t *valid, int64_t n, int32_t kernel,
                       int32_t *labels, uint8_t *alive, int64_t *launches, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DBSCAN_PAPER_MI355X_H */
