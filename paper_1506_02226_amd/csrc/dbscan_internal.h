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
  const float *hoist;  // rows of the hoisted test (hoist_view), or null: direct form
};

// Rows of the hoisted float32 test of the d <= 4 on-the-fly sweep (Section
// IV-B.2's T + P[n] - 2 t.p, taken about a local origin): each 16-row block
// of the staged order has an origin c (the centre of its box), and row i
// keeps a = -2 fl(x_i - c) and its float32 thresholds (hoist_prep_body).
// Layout (floats): a [k][n_pad], lo [n_pad], hi [n_pad], the blocks' boxes
// [2k][n_pad/16] (lo, hi), their origins [k][n_pad/16], per 8-row group
// the largest hi [n_pad/8], and per 16-row block its gate [n_pad/16]
// (hoist_gate).
// The float32 value next to finite x, upwards (dir = 1) or downwards (-1).
__host__ __device__ inline float f32_step(float x, int dir) {
  if (x == 0.0f) return dir > 0 ? 1.40129846e-45f : -1.40129846e-45f;
  const unsigned b = __builtin_bit_cast(unsigned, x);
  return __builtin_bit_cast(float, ((x > 0.0f) == (dir > 0)) ? b + 1u : b - 1u);
}

// Float32 thresholds of the hoisted test for one row.  With c the origin of
// the row's block, a = fl(x - c) the row (T = |a|^2), b = fl(y - c) a
// column and q the float32 value of |b|^2 - 2 a.b (2d roundings, any order,
// fused or not), let t = |x - y| (exact) and r >= |x - c|.  Rounding the
// shifted points moves |a - b| from t by at most u (2r + t), and
// |q + T - |a - b|^2| <= g (r + t)(3r + t) + e, with g = gamma_2d (1 + u)^2
// and e = 4d 2^-149 for gradual underflow.  Hence q <= G(t) and q >= F(t):
//   G(t) = ((1 + u) t + 2ur)^2 + g (r + t)(3r + t) + e - T,
//   F(t) = ((1 - u) t - 2ur)^2 - g (r + t)(3r + t) - e - T  ((1 - u) t >= 2ur).
// G grows with t, and F from its vertex t_v on.  t_in and t_out bound the
// exact distances at which the float64 value of the definition is surely
// <= eps2 or surely > eps2 (the factors of band_fp32), so hi >= G(t_out)
// makes q > hi "out" and lo <= F(t_in) makes q <= lo "in" (lo = -inf when
// t_in is below t_v or 2ur / (1 - u)).  The double arithmetic is widened by
// 2^-48 of the magnitudes and the results rounded outward.
__host__ __device__ inline void hoist_band(double T, int d, double eps2, float *lo, float *hi) {
  if (__builtin_isinf(eps2)) {
    *lo = __builtin_inff();
    *hi = __builtin_inff();
    return;
  }
  const double u = 0x1p-24, u64 = 0x1p-53;
  const double g = (2.0 * d * u / (1.0 - 2.0 * d * u)) * (1.0 + u) * (1.0 + u) * (1.0 + 0x1p-40);
  const double e = 4.0 * d * 0x1p-149;
  const double g64 = (d + 2) * u64 / (1.0 - (d + 2) * u64);
  const double t_in = __builtin_sqrt(eps2 * (1.0 - 4 * u64) / (1.0 + g64)) * (1.0 - 0x1p-50);
  const double t_out = __builtin_sqrt(eps2 * (1.0 + 4 * u64) / (1.0 - g64)) * (1.0 + 0x1p-50);
  const double T_lo = T * (1.0 - 0x1p-50), T_hi = T * (1.0 + 0x1p-50);
  const double r = __builtin_sqrt(T_hi) * (1.0 + 0x1p-50) / (1.0 - u);
  const double wo = (1.0 + u) * t_out + 2.0 * u * r;
  const double eo = g * (r + t_out) * (3.0 * r + t_out) + e;
  double h = wo * wo + eo - T_lo;
  h += 0x1p-48 * (wo * wo + eo + T_lo);
  float hf = (float)h;
  if ((double)hf < h) hf = __builtin_isinf(hf) ? -3.40282347e38f : f32_step(hf, 1);
  *hi = hf;
  const double A = (1.0 - u) * (1.0 - u) - g;
  const double tv = (4.0 * u * (1.0 - u) * r + 4.0 * g * r) / (2.0 * A) * (1.0 + 0x1p-40);
  const double wi = (1.0 - u) * t_in - 2.0 * u * r;
  if (!(wi >= 0.0 && t_in >= tv)) {  // also for a NaN row (padding)
    *lo = -__builtin_inff();
    return;
  }
  const double ei = g * (r + t_in) * (3.0 * r + t_in) + e;
  double l = wi * wi - ei - T_hi;
  l -= 0x1p-48 * (wi * wi + ei + T_hi);
  float lf = (float)l;
  if ((double)lf > l) lf = __builtin_isinf(lf) ? 3.40282347e38f : f32_step(lf, -1);
  *lo = lf;
}

// Gate of a 16-row block of the hoisted test.  Per column the sweep forms,
// for each row r of the block, s_r = fl(a'_r . b) with a'_r = -2 fl(x_r - c)
// (a product, then d - 1 fused multiply-adds), and compares fl(min_r s_r + P)
// once with the block's gate (P = the column's float32 |b|^2); only when that
// passes does it form the rows' values q_r = fl(P + a'_r . b) (d fused
// multiply-adds from P) and test them against their thresholds.  The gate
// must pass every column with q_r <= hi_r for some row.  With g = gamma_d,
// E_r = P + a'_r . b exact, S_r = sum_k |a'_rk b_k| <= 2 rho |b| (rho >= every
// |fl(x_r - c)| of the block) and e an allowance for gradual underflow:
//   |q_r - E_r| <= g (P + S_r) + e,  |s_r - a'_r . b| <= g S_r + e,
//   |P - |b|^2| <= g |b|^2 + e.
// If q_r <= hi_r <= H (H the block's largest hi), then
// (1 - g) |b|^2 - 2 rho |b| - e <= E_r <= H + g (P + 2 rho |b|) + e bounds |b|
// by B, the positive root of (1 - 2g - g^2) z^2 - 2 rho (1 + g) z - H+ = 0
// (H+ = max(H, 0) plus the underflow terms), and
//   min_r s_r + P <= s_r + P <= H + g ((1 + g) B^2 + 4 rho B) + 3e.
// Rounding is monotone, so fl(min_r s_r + P) is at most that bound rounded
// up, which is the gate.  A NaN H (every row padding) gives a NaN gate, which
// no column passes; H = +inf (eps = inf) gives +inf.
__host__ __device__ inline float hoist_gate(float H, double rho2, int d) {
  if (!(H == H) || __builtin_isinf(H)) return H;
  const double u = 0x1p-24;
  const double g = (d * u / (1.0 - d * u)) * (1.0 + 0x1p-40);
  const double e = 8.0 * d * 0x1p-149;
  const double rho = __builtin_sqrt(rho2) * (1.0 + 0x1p-48);
  const double Hp = ((double)H > 0.0 ? (double)H : 0.0) + 4.0 * e;
  const double al = 1.0 - 2.0 * g - g * g;
  const double be = rho * (1.0 + g);
  const double B = (be + __builtin_sqrt(be * be + al * Hp)) / al * (1.0 + 0x1p-48);
  const double S = g * ((1.0 + g) * B * B + 4.0 * rho * B) + 3.0 * e;
  double G = (double)H + S;
  G += 0x1p-48 * (__builtin_fabs((double)H) + S);
  float gf = (float)G;
  if ((double)gf < G) gf = f32_step(gf, 1);
  return gf;
}

template <typename F>
struct HoistView {
  F *a, *lo, *hi, *box, *cen, *hg, *g16;
};
__host__ __device__ inline unsigned long long hoist_floats(int n_pad, int d) {
  return (unsigned long long)(d + 2) * n_pad + (3ull * d + 1) * (n_pad / 16) + n_pad / 8;
}
template <typename F>
__host__ __device__ inline HoistView<F> hoist_view(F *base, int n_pad, int d) {
  HoistView<F> v;
  v.a = base;
  v.lo = v.a + (size_t)d * n_pad;
  v.hi = v.lo + n_pad;
  v.box = v.hi + n_pad;
  v.cen = v.box + (size_t)2 * d * (n_pad / 16);
  v.hg = v.cen + (size_t)d * (n_pad / 16);
  v.g16 = v.hg + n_pad / 8;
  return v;
}

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
// With `hoist` (d <= 4, float32 sweep) the staging also writes the rows of
// the hoisted test for eps2.
hipError_t run_stage(const float *pts, int n, int d, int n_pad, int d_pad, float *soa, int *counts,
                     int *parent, int *jstar, DevState *st, const Order &ord, hipStream_t s,
                     float *hoist = nullptr, double eps2 = 0.0);
hipError_t run_count(const Buffers &b, const SweepScalars &sc, bool emit_pairs, hipStream_t s);
hipError_t run_block_boxes(const float *soa, int n_pad, int d, float *box, hipStream_t s);
hipError_t run_union(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_border(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_core(const int *counts, int n, int n_pad, int minpts, uint8_t *core,
                    uint32_t *corebits, DevState *st, const Order &ord, int *counts_out,
                    bool count, hipStream_t s, bool degree = false);
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
// Inputs of at most this many (padded) rows in the caller's order run the
// bitmask merge's hook and compress passes, gated by the core points' degree
// (run_merge_bitmask).
constexpr int kHookCallerOrderMax = 16384;
hipError_t run_merge_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s);
hipError_t run_labels(int n, const uint32_t *corebits, const int *jstar, int *parent, int *labels,
                      const DevState *st, const Order &ord, hipStream_t s);

}  // namespace dbk
