// Block-level bodies of the matrix-core filter (preparation, thresholds, tile
// sweep, float64 band pass), shared by the standalone kernels and the
// persistent serving loop.  The method and the bounds are described in
// mfma_kernels.hip.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

template <typename T> struct LowPrec;
template <> struct LowPrec<__bf16> {
  using vec8 = bf16x8;
  static constexpr double u = 0x1p-8;        // unit roundoff (8-bit significand)
  static constexpr double tiny = 0x1p-126;   // smallest normal
  static constexpr float big = 0x1p100f;     // padding norm: any padded pair is far
  // |x| bound of the filter: the FP32 norms and accumulators stay finite
  // (4 K maxval^2 < FLT_MAX for K <= 128); larger inputs fall back to float32
  static constexpr float maxval = 1.0e17f;
  __device__ static vec8 zero() { return vec8{}; }
  __device__ static f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct LowPrec<_Float16> {
  using vec8 = f16x8;
  static constexpr double u = 0x1p-11;
  static constexpr double tiny = 0x1p-14;
  static constexpr float big = 60000.0f;
  static constexpr float maxval = 30000.0f;  // |x| and the norm parts must stay in range
  __device__ static vec8 zero() { return vec8{}; }
  __device__ static f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// ---------------------------------------------------------------- prepare
// A block prepares 256 (padded) points, each wave 64 of them one after the
// other with the lanes over the coordinates (coalesced loads and stores): the
// rounded coordinates x~ (row of a_aug, zero-padded to K), -2 x~ (row of
// b_aug), the FP32 norm of the rounded point (a wave sum; +inf for padded
// rows, so that no padded pair can reach the band) in the float array that
// follows the n_pad rows of a_aug, and the float64 norm of the original point
// for the bounds (max via an atomic on its bit pattern).  K <= 128.  With a
// spatial order, row i of the copies is input row perm[i].
template <typename T>
__device__ __forceinline__ const float *mfma_norms(const T *a_aug, int n_pad, int K) {
  return reinterpret_cast<const float *>(a_aug + (size_t)n_pad * K);
}

template <typename T>
__device__ __forceinline__ void mfma_prep_body(const float *__restrict__ pts, int n, int d,
                                               int n_pad, int K, T *__restrict__ a_aug,
                                               T *__restrict__ b_aug, DevState *st, int bid,
                                               const int *__restrict__ perm = nullptr) {
  const int lane = lane_id();
  const int w = (int)(threadIdx.x >> 6);
  float *norms = const_cast<float *>(mfma_norms<T>(a_aug, n_pad, K));
  bool bad = false, nonfinite = false;
  double mx = 0.0;
  for (int t = 0; t < 64; ++t) {
    const int i = bid * 256 + w * 64 + t;  // wave-uniform
    if (i >= n_pad) break;
    T *a = a_aug + (size_t)i * K;
    T *b = b_aug + (size_t)i * K;
    if (i < n) {
      const size_t src = perm ? (size_t)perm[i] : (size_t)i;
      float part = 0.0f;
      double part64 = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        if (k < d) {
          const float x = pts[src * d + k];
          nonfinite |= !__builtin_isfinite(x);
          bad |= nonfinite || __builtin_fabsf(x) > LowPrec<T>::maxval;
          const T xr = (T)x;
          const float xf = (float)xr;
          part = __builtin_fmaf(xf, xf, part);
          part64 += (double)x * (double)x;
          a[k] = xr;
          b[k] = (T)(-2.0f * xf);
        } else if (k < K) {
          a[k] = (T)0.0f;
          b[k] = (T)0.0f;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        part += __shfl_xor(part, off);
        part64 += __shfl_xor(part64, off);
      }
      if (lane == 0) norms[i] = part;  // same value in every lane
      mx = part64 > mx ? part64 : mx;
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        if (k < K) {
          a[k] = (T)0.0f;
          b[k] = (T)0.0f;
        }
      }
      if (lane == 0) norms[i] = __builtin_inff();
    }
  }
  if (lane == 0 && mx > 0.0)
    atomicMax(&st->max_norm, (unsigned long long)__double_as_longlong(__builtin_sqrt(mx)));
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(&st->status, kStatusRange);
  if (__ballot(nonfinite) != 0ull && lane == 0) atomicOr(&st->status, kStatusNonFinite);
}

// ------------------------------------------------------------- thresholds

// Bounds (all in float64, then rounded outward to float32):
//   |x - x~| <= u |x| + sqrt(d) tiny per point, so |D - D~| <= Delta with
//   Delta = 2 (u M + sqrt(d) tiny), M = max |x_i| (D = |x_i - x_j| exact,
//   D~ the same for the rounded points);
//   |s~ - D~^2| <= E = c (|x~_i|^2 + |x~_j|^2) with c covering the FP32 norms
//   (gamma_d) and the FP32 sum of the K exact products (-2 x~_ik x~_jk) and
//   the two norms: the contraction accumulates onto n_i in the matrix core
//   (whose internal order is not specified) and n_j is added last, K+2 terms
//   whose absolute sum is at most 2 (n_i + n_j), bounded here with
//   gamma_{2K+2} counted twice; the 4u^2 + 2u32 term is further slack;
//   |x~|^2 <= (M(1+u) + sqrt(d) tiny)^2;
//   the float64 definition decides in when S <= eps2 (1 - 2 g64) and out when
//   S >= eps2 (1 + 2 g64), g64 = (d+2) 2^-53.
// In: s~ <= (eps_in - Delta)^2 - E.  Out: s~ > (eps_out + Delta)^2 + E.  The
// band is then widened to at least |s - eps2| <= band_rel * eps2.
template <typename T>
__device__ __forceinline__ void mfma_thresholds_body(DevState *st, double eps2, int d, int K,
                                                     double band_rel) {
  const double u = LowPrec<T>::u, tiny = LowPrec<T>::tiny;
  const double M = __longlong_as_double((long long)st->max_norm) * (1.0 + 1e-12);
  const double sd = __builtin_sqrt((double)d) * (1.0 + 1e-12);
  const double delta = 2.0 * (u * M + sd * tiny);
  const double mt = M * (1.0 + u) + sd * tiny;
  const double u32 = 0x1p-24;
  const double g_norm = (d + 1) * u32 / (1.0 - (d + 1) * u32);
  const double g_acc = (2.0 * K + 2) * u32 / (1.0 - (2.0 * K + 2) * u32);
  const double split = 4.0 * u * u + 2.0 * u32;
  const double c = g_norm + split + 2.01 * g_acc + 1e-12;
  const double E = c * 2.0 * mt * mt + 4.0 * K * 0x1p-126;
  const double g64 = (d + 2) * 0x1p-53;
  const double eps_in = __builtin_sqrt(eps2 * (1.0 - 2.0 * g64)) * (1.0 - 1e-12);
  const double eps_out = __builtin_sqrt(eps2 * (1.0 + 2.0 * g64)) * (1.0 + 1e-12);
  double t_lo = (eps_in > delta) ? (eps_in - delta) * (eps_in - delta) - E : -1.0;
  double t_hi = (eps_out + delta) * (eps_out + delta) + E;
  t_lo = t_lo > 0.0 ? t_lo * (1.0 - 1e-12) : -1.0;
  t_hi *= (1.0 + 1e-12);
  const double s_lo = (1.0 - band_rel) * eps2, s_hi = (1.0 + band_rel) * eps2;
  if (s_lo < t_lo) t_lo = s_lo;
  if (s_hi > t_hi) t_hi = s_hi;
  float lo = (float)t_lo, hi = (float)t_hi;
  if (!__builtin_isfinite(lo)) lo = 0x1.fffffep127f;  // t_lo beyond FLT_MAX: round down
  if ((double)lo > t_lo) lo = next_down(lo);
  if (__builtin_isfinite(hi) && (double)hi < t_hi) hi = next_up(hi);
  if (t_lo < 0.0) lo = -__builtin_inff();
  st->thr[0] = lo;
  st->thr[1] = hi;
}

// ------------------------------------------------------------ tile sweep
constexpr int kMfmaColsPerWave = 64;                   // two 32-column tiles
constexpr unsigned kBandBoth = 0x80000000u;            // band entry flag (row index bit 31)
constexpr int kMfmaColsPerGroup = 4 * kMfmaColsPerWave;  // 256

// LDS for one block of the tile sweep: two a-tiles and the pair/band queues.
// An a-tile is 32 rows of 2KS 16-byte chunks, row-major with a pitch of
// 2KS+1 chunks: the pitch is odd, so the 16 rows that one pass of a 16-byte
// read touches fall in 16 distinct bank groups (no conflicts), and the
// writes, which follow the global row-major order, stay nearly conflict-free.
constexpr int kBandQueue = 128;       // band queue (pairs); appended 64 at a time

template <int KS>
struct MfmaLds {
  static constexpr int kPitch = 2 * KS + 1;
  uint4 atile[2][32 * kPitch];
  float anorm[2][32];  // FP32 norms of the a-tile's rows
  int2 qpair[4][kListQueue];
  int2 qband[4][kBandQueue];
  // row-side counts of the item's rows, two 16-bit counts per word (a row
  // meets at most 256 columns in one item)
  unsigned rowcnt[mfma_chunk_tiles(KS) * 32 / 2];
  unsigned long long xfer[5];
};


template <typename T, int KS>
__device__ __forceinline__ void mfma_count_body(const T *__restrict__ a_aug,
                                                const T *__restrict__ b_aug,
                                                int *__restrict__ counts,
                                                int2 *__restrict__ pairs,
                                                int2 *__restrict__ band,
                                                DevState *__restrict__ st,
                                                const MfmaScalars &sc, int bid,
                                                MfmaLds<KS> &lds) {
  using V = typename LowPrec<T>::vec8;
  constexpr int K = KS * 16;
  constexpr int kPitch = MfmaLds<KS>::kPitch;
  V (*atile)[32 * kPitch] = reinterpret_cast<V (*)[32 * kPitch]>(lds.atile);
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int w = wave_uniform(tid >> 6);
  // item -> (chunk, column group); sc.chunk is a multiple of 8 row tiles
  const int G = sc.n_pad / kMfmaColsPerGroup, kpc = sc.chunk / 8;
  int lo = 0, hi = sc.nchunks - 1;
  while (lo < hi) {  // last chunk whose first item is <= bid
    const int mid = (lo + hi + 1) >> 1;
    if (mfma_items_before_chunk(mid, G, kpc) <= bid) lo = mid;
    else hi = mid - 1;
  }
  const int chunk = lo;
  const int cgroup = bid - (int)mfma_items_before_chunk(lo, G, kpc);
  const int col0 = cgroup * kMfmaColsPerGroup + w * kMfmaColsPerWave;
  // Lower triangle only: row tiles from the group's own columns onwards.  The
  // 8 row tiles that overlap the group's 256 columns (the diagonal zone) are
  // computed in both orders and counted on the column side only; below them
  // every pair (i > j) is tested once and counted on both sides.
  const int diag_rt = cgroup * (kMfmaColsPerGroup / 32);
  const int diag_end = diag_rt + kMfmaColsPerGroup / 32;
  const int rt0 = max(chunk * sc.chunk, diag_rt);                  // first row tile
  const int rt1 = min(chunk * sc.chunk + sc.chunk, sc.n_pad / 32);  // end row tile
  const float t_lo = st->thr[0];
  const float t_hi = st->thr[1];
  const bool range_bad =
      __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStatusRange;
  if (range_bad || rt0 >= rt1) return;  // uniform over the work-group

  // stationary b-fragments: lane l holds b[8*(l/32) + 16 s .. +7] of column
  // l%32, and that column's norm
  const float *norms = mfma_norms<T>(a_aug, sc.n_pad, K);
  V bfr[2][KS];
  float cn[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int j = col0 + c * 32 + (lane & 31);
    const V *src = (const V *)(b_aug + (size_t)j * K);
#pragma unroll
    for (int s = 0; s < KS; ++s) bfr[c][s] = src[2 * s + (lane >> 5)];
    cn[c] = norms[j];
  }
  // wait for them here: inside the loop only the next a-tile's loads are in
  // flight, so the matrix-core work never waits on global memory
  __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
  int cnt[2] = {0, 0};
  WaveQueue qp{lds.qpair[w], 0, kListDrain};
  WaveQueue qb{lds.qband[w], 0, kBandQueue - 64};
  const int row_first = chunk * sc.chunk * 32;  // rowcnt[k] covers rows row_first + 2k, +1
  for (int k = tid; k < sc.chunk * 16; k += 256) lds.rowcnt[k] = 0u;  // before the first barrier

  // cooperative a-tile load: 32 rows x 2KS 16-byte chunks (coalesced).
  // Two LDS buffers: at the top of iteration t, tile t+1 (fetched into
  // registers one iteration earlier) is written to buffer (t+1)%2 and tile t+2
  // is fetched, then tile t is computed from buffer t%2; one barrier per
  // iteration.  Buffer (t+1)%2 last held tile t-1, which every wave finished
  // before the barrier that ended iteration t-1.  A global load has a whole
  // iteration to land before its registers are written out, and no wait sits
  // between the matrix-core work and the epilogue.
  constexpr int kChunks = 32 * 2 * KS;
  constexpr int kPer = (kChunks + 255) / 256;  // chunks per thread (1 or 2)
  float pre_n = 0.0f;  // threads 0..31: the norm of row tid of the fetched tile
  // scalar bases at the item's first row tile and 32-bit byte offsets (an
  // item spans at most 256 row tiles: 1 MB of a-rows at K = 64), so that the
  // loads take a scalar base and one 32-bit vector offset
  const char *a_base = reinterpret_cast<const char *>(a_aug) + (size_t)rt0 * 32 * K * sizeof(T);
  const char *n_base = reinterpret_cast<const char *>(norms) + (size_t)rt0 * 32 * sizeof(float);
  auto fetch = [&](V(&pre)[kPer], int rt) {
    const unsigned trel = (unsigned)(rt - rt0);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const unsigned off =
          (trel * 32u * K + (unsigned)(e < kChunks ? e : kChunks - 1) * 8u) * (unsigned)sizeof(T);
      pre[u] = *reinterpret_cast<const V *>(a_base + off);  // unconditional: no branch
    }
    pre_n = *reinterpret_cast<const float *>(n_base + (trel * 32u + (unsigned)(tid & 31)) * 4u);
  };
  auto stash = [&](const V(&pre)[kPer], int buf) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      if (e < kChunks) {
        const int row = e / (2 * KS), ch = e - row * (2 * KS);
        atile[buf][row * kPitch + ch] = pre[u];
      }
    }
    if (tid < 32) lds.anorm[buf][tid] = pre_n;
  };
  auto tile = [&](int rt, int buf) {
    V afr[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) afr[s] = atile[buf][(lane & 31) * kPitch + 2 * s + (lane >> 5)];
    // the accumulators start at |x~_i|^2 (the matrix core reads the row
    // norms as its addend; accumulator r of this lane is row
    // 4 (lane / 32) + 8 (r / 4) + r % 4, column lane % 32) and |x~_j|^2 is
    // added after the contraction, so s~ = (n_i - 2 x~_i.x~_j) + n_j
    f32x16 rn;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = *reinterpret_cast<const float4 *>(&lds.anorm[buf][4 * (lane >> 5) + 8 * q]);
      rn[4 * q] = v.x;
      rn[4 * q + 1] = v.y;
      rn[4 * q + 2] = v.z;
      rn[4 * q + 3] = v.w;
    }
    // two independent accumulation chains, interleaved
    f32x16 acc0 = LowPrec<T>::mfma(afr[0], bfr[0][0], rn);
    f32x16 acc1 = LowPrec<T>::mfma(afr[0], bfr[1][0], rn);
#pragma unroll
    for (int s = 1; s < KS; ++s) {
      acc0 = LowPrec<T>::mfma(afr[s], bfr[0][s], acc0);
      acc1 = LowPrec<T>::mfma(afr[s], bfr[1][s], acc1);
    }
    const int row_base = rt * 32 + 4 * (lane >> 5);
    const bool sym = rt >= diag_end;  // every row of the tile above every column
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const f32x16 acc = c ? acc1 : acc0;
      // one test per tile: does any pair of this lane reach the band?  The
      // FP32 addition of n_j is monotone, so (min_r a_r) + n_j is the
      // smallest of the lane's 16 values a_r + n_j
      float mn = acc[0];
#pragma unroll
      for (int r = 1; r < 16; ++r) mn = __builtin_fminf(mn, acc[r]);
      if (__ballot(mn + cn[c] <= t_hi) == 0ull) continue;
      const int j = col0 + c * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float v = acc[r] + cn[c];
        if (__ballot(v <= t_hi) != 0ull) {
          const int i = row_base + 8 * (r >> 2) + (r & 3);
          const bool valid = i < sc.n && j < sc.n;
          const bool in = valid && v <= t_lo;
          const bool amb = valid && !(v <= t_lo) && v <= t_hi;
          cnt[c] += in ? 1 : 0;
          if (sym) {
            // row side: lanes 0-31 share one row, lanes 32-63 another
            const uint64_t bm = __ballot(in);
            const uint32_t half = (uint32_t)(bm >> (lane & 32));
            if ((lane & 31) == 0 && half != 0u) {
              const int k = i - row_first;
              atomicAdd(&lds.rowcnt[k >> 1], (unsigned)__popc(half) << ((k & 1) * 16));
            }
          }
          wq_push(qp, in && i > j, i, j);
          wq_drain_list(qp, pairs, sc.pair_cap, st, false);
          // band entries of the once-tested zone carry bit 31: both sides count
          wq_push(qb, amb, sym ? (int)((unsigned)i | kBandBoth) : i, j);
          wq_drain_band(qb, band, sc.band_cap, st, false);
        }
      }
    }
  };
  V pre[kPer];
  fetch(pre, rt0);
  stash(pre, 0);
  if (rt0 + 1 < rt1) fetch(pre, rt0 + 1);
  __syncthreads();
  int bcur = 0;
  for (int rt = rt0; rt < rt1; ++rt) {
    const int bnext = bcur ^ 1;
    if (rt + 1 < rt1) stash(pre, bnext);
    if (rt + 2 < rt1) fetch(pre, rt + 2);
    tile(rt, bcur);
    __syncthreads();
    bcur = bnext;
  }
  wq_flush_pairs(qp, pairs, sc.pair_cap, st, lds.xfer);
  wq_flush_block(qb, band, sc.band_cap, &st->band_list, &st->status, kStatusBandOverflow, lds.xfer);
  // row-side counts (wq_flush_block ends with a barrier)
  for (int k = tid; k < sc.chunk * 16; k += 256) {
    const unsigned v = lds.rowcnt[k];
    if (v == 0u) continue;
    const int i = row_first + 2 * k;
    if ((v & 0xffffu) && i < sc.n) atomicAdd(counts + i, (int)(v & 0xffffu));
    if ((v >> 16) && i + 1 < sc.n) atomicAdd(counts + i + 1, (int)(v >> 16));
  }
  // lanes l and l+32 hold the same column
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int tot = cnt[c] + __shfl_xor(cnt[c], 32);
    const int j = col0 + c * 32 + lane;
    if (lane < 32 && j < sc.n) atomicAdd(counts + j, tot);
  }
}

// ------------------------------------------------------- float64 band pass
// Each queued pair (i, j) is decided with the definition's arithmetic on the
// FP32 inputs; "in" adds to the count of column j, and also of row i when the
// entry carries kBandBoth (a pair the sweep tested in one order only), and
// i > j pairs go to the pair list.  This block handles band entries
// [e_begin, e_end); `qbuf` is [4][128] pairs of LDS.  With a spatial order
// (perm: staged index -> input row) the rows are read through it.
__device__ __forceinline__ void recheck_band_range(const float *__restrict__ pts, int d,
                                                   const int2 *__restrict__ band,
                                                   int *__restrict__ counts,
                                                   int2 *__restrict__ pairs,
                                                   DevState *__restrict__ st, double eps2,
                                                   long long pair_cap,
                                                   unsigned long long e_begin,
                                                   unsigned long long e_end,
                                                   int2 (*qbuf)[128],
                                                   const int *__restrict__ perm = nullptr) {
  const int w = wave_uniform(threadIdx.x >> 6);
  WaveQueue qp{qbuf[w], 0, 64};
  for (unsigned long long e0 = e_begin + 64ull * w; e0 < e_end; e0 += 256) {
    const unsigned long long e = e0 + (unsigned long long)lane_id();
    bool in = false;
    int2 pr = make_int2(0, 0);
    if (e < e_end) {
      pr = band[e];
      const bool both = ((unsigned)pr.x & kBandBoth) != 0u;
      pr.x = (int)((unsigned)pr.x & ~kBandBoth);
      const size_t ra = perm ? (size_t)perm[pr.x] : (size_t)pr.x;
      const size_t rb = perm ? (size_t)perm[pr.y] : (size_t)pr.y;
      in = exact_within_rows(pts + ra * d, pts + rb * d, d, eps2);
      if (in) {
        atomicAdd(counts + pr.y, 1);
        if (both) atomicAdd(counts + pr.x, 1);
      }
    }
    wq_push(qp, in && pr.x > pr.y, pr.x, pr.y);
    wq_drain_list(qp, pairs, pair_cap, st, false);
  }
  wq_drain_list(qp, pairs, pair_cap, st, true);
}

}  // namespace dbk
