// Host-side launch interface between the C ABI (dbscan_api.hip) and the
// kernel files.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dbscan_device.h"

namespace dbk {

// Device buffers of one call (all DEVICE pointers).
struct Buffers {
  const float *soa;    // [d_pad][n_pad] staged coordinates (NaN-padded columns)
  int *counts;         // [n]
  const uint32_t *corebits;  // [n_pad/32]
  int *parent;         // [n_pad] union-find forest
  int *jstar;          // [n_pad] lowest-index core neighbour of non-core points
  const int *list;     // [n_pad] compacted non-core rows
  void *adjT;          // triangular uint32 bitmask adjacency (bitmask form only, adj_index)
  uint8_t *tflag;      // [n_pad/64][n_pad/32] non-empty flags of its 32 x 64 tiles
  int2 *pairs;         // [edge_cap] neighbour pairs (i, j), j < i (on-the-fly form)
  int2 *band;          // [band_cap] pairs the matrix-core filter leaves undecided
  DevState *st;
  const int *okey;     // [n] caller's index of each staged row (spatial order), or null
};

// Spatial order of one call (all null when the rows keep the caller's order).
struct Order {
  const int *perm;  // [n] staged row -> caller's index
  int *inv;         // [n] caller's index -> staged row
  int *rootmin;     // [n] lowest caller index of the core points under each root
};

// Bits per coordinate of the spatial-order key for d <= 4 (at most 32 in all;
// larger d use a pivot index, one radix pass).
__host__ __device__ inline int order_bits_per_coord(int d) {
  return d == 1 ? 24 : (d == 2 ? 12 : (d == 3 ? 10 : 8));
}

// Scalars of one sweep (passed by value; SGPRs in the kernels).
struct SweepScalars {
  int n, n_pad, d, d_pad;
  int nchunks, chunk;  // column split: chunk = columns (multiple of 64) or 32-bit words
  float lo, hi;        // float32 band: s <= lo in, s > hi out, else float64
  double eps2;
  long long edge_cap;  // capacity of the pair list (entries)
  int flags;           // kOnlyOnOverflow / kOnlyOnFilterFail
  int rgroup;          // rows per block of the triangular sweeps (multiple of 64)
  float *box;          // tile pruning: boxes of the 64-point blocks, [2k][n_pad/64] lo / hi,
                       // then the same for row groups and for column chunks
};

// The bit matrix keeps, for each 32-row block q, the words of the columns j
// from its 64-column diagonal block on (j >= 64 floor(q/2)): block q starts
// after sum over q' < q of (n_pad - 64 floor(q'/2)) words, which is
// q n_pad - 64 S(q) with S(2m) = m (m - 1) and S(2m + 1) = m^2.  About half
// of the n_pad^2 / 32 words of the full square.
__host__ __device__ inline long long adj_block_base(int q, int n_pad) {
  const long long m = q >> 1;
  const long long S = (q & 1) ? m * m : m * (m - 1);
  return (long long)q * n_pad - 64 * S - 64 * m;  // word index of column 0 of block q
}
__host__ __device__ inline size_t adj_index(int q, int j, int n_pad) {
  return (size_t)(adj_block_base(q, n_pad) + j);
}
__host__ inline unsigned long long adj_words(int n_pad) {
  const long long nq = n_pad / 32, m = nq / 2;  // nq is even
  return (unsigned long long)(nq * (long long)n_pad - 64 * m * (m - 1));
}

// Tile pruning: launch helpers of the persistent sweeps.
hipError_t run_coarse_boxes(const SweepScalars &sc, hipStream_t s);
unsigned pruned_grid(unsigned full_grid);

constexpr int kOnlyOnOverflow = 1;    // run only if the pair list overflowed
constexpr int kOnlyOnFilterFail = 2;  // run only if the matrix-core filter gave up

// Scalars of the matrix-core sweep.
struct MfmaScalars {
  int n, n_pad, d;
  int nchunks, chunk;  // row split: chunk = 32-row tiles per chunk
  long long pair_cap, band_cap;
};

// Work items of the triangular matrix-core sweep: (column group g of 256
// columns, row chunk c of 8k row tiles of 32) with c >= g / k (integer
// division).  Their number, counted column group by column group (items
// before group g):
__host__ __device__ inline long long mfma_items_before(int g, int nchunks, int k) {
  const long long q = g / k, r = g - q * k;
  return (long long)g * nchunks - (k * q * (q - 1) / 2 + q * r);
}
// Row tiles of 32 per matrix-core work item, at most: an item's row counts
// sit in LDS, and at K <= 64 (ks <= 4) 256 tiles still leave room for four
// work-groups per CU.
__host__ __device__ constexpr int mfma_chunk_tiles(int ks) { return ks <= 4 ? 256 : 128; }
// Row tiles per work item for `tiles` row tiles (a multiple of 8): `most`
// for large inputs; small ones take fewer (a multiple of 8, at least 8) so
// that the triangle still splits into about 2,048 items, eight per CU,
// rather than a few long ones (n = 2,048 had 8 items of 64 tiles each).
__host__ inline int mfma_chunk_for(int tiles, int most) {
  long long c = ((long long)tiles * tiles / (16LL * 2048) + 7) / 8 * 8;
  if (c < 8) c = 8;
  if (c > most) c = most;
  if (c > tiles) c = tiles;
  return (int)c;
}
// They are listed row chunk by row chunk: chunk c holds the groups
// 0 .. min(G, (c+1) k) - 1, so that items running at the same time share
// their rows (one chunk's a-tiles serve many column groups from L2).  Items
// before chunk c:
__host__ __device__ inline long long mfma_items_before_chunk(int c, int G, int k) {
  const long long c1 = G / k;  // chunks below c1 hold (c+1) k <= G groups
  if (c <= c1) return (long long)k * c * (c + 1) / 2;
  return (long long)k * c1 * (c1 + 1) / 2 + (long long)(c - c1) * G;
}

int rows_per_wave(int d);
int coord_chunk(int d);

hipError_t run_reset(DevState *st, long long pair_cap, hipStream_t s);
long long order_hist_entries(long long n);
int order_max_d();
hipError_t run_spatial_order(const float *pts, int n, int d, unsigned *keys[2], int *vals[2],
                             int *hist, DevState *st, int **perm, hipStream_t s);
hipError_t run_stage(const float *pts, int n, int d, int n_pad, int d_pad, float *soa, int *counts,
                     int *parent, int *jstar, DevState *st, const Order &ord, hipStream_t s);
hipError_t run_count(const Buffers &b, const SweepScalars &sc, bool emit_pairs, hipStream_t s);
hipError_t run_block_boxes(const float *soa, int n_pad, int d, float *box, hipStream_t s);
hipError_t run_union(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_border(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_core(const int *counts, int n, int n_pad, int minpts, uint8_t *core,
                    uint32_t *corebits, DevState *st, const Order &ord, int *counts_out,
                    bool count, hipStream_t s);
hipError_t run_compact_noncore(const uint32_t *corebits, int n, int *list, DevState *st,
                               bool only_on_overflow, hipStream_t s);
hipError_t run_merge_list(const Buffers &b, long long cap, hipStream_t s);
hipError_t run_filter_fallback(const float *pts, const int *perm, int n, int d, int n_pad,
                               int d_pad, float *soa, int *counts, DevState *st, hipStream_t s);

int mfma_k(int d);
// Bytes of the a-rows of the matrix-core filter: n_pad rows of K 16-bit
// values, then the n_pad FP32 norms.
inline uint64_t mfma_a_bytes(int64_t n_pad, int K) {
  return (uint64_t)n_pad * K * 2 + (uint64_t)n_pad * 4;
}
hipError_t run_mfma_prep(const float *pts, const int *perm, int n, int d, int n_pad, int prec,
                         void *a_aug, void *b_aug, DevState *st, hipStream_t s);
hipError_t run_mfma_thresholds(DevState *st, double eps2, int d, int prec, double band_rel,
                               hipStream_t s);
hipError_t run_mfma_count(const void *a_aug, const void *b_aug, const Buffers &b,
                          const MfmaScalars &sc, int prec, hipStream_t s);
hipError_t run_recheck_band(const float *pts, int d, const Buffers &b, double eps2,
                            long long band_cap, long long pair_cap, hipStream_t s);
hipError_t run_merge_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_labels(int n, const uint32_t *corebits, const int *jstar, int *parent, int *labels,
                      const DevState *st, const Order &ord, hipStream_t s);

}  // namespace dbk
