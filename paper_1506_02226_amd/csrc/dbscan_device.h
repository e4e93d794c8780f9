// Device-side building blocks shared by the DBSCAN kernels (gfx950, wave64).
//
//  * the float64 re-evaluation of a pair that the float32 filter could not
//    decide, written exactly as the definition states it: coordinates widened
//    from float32, per coordinate t = x_ik - x_jk and s = s + t*t, every
//    operation rounded on its own (no fused multiply-add), compared as
//    s <= eps^2 (Sections IV-A and IV-B compare squared distances with eps^2);
//  * the float32 direct form of the squared distance (Section IV-B.2, the
//    expression dist(t, p[n]) before hoisting), used only as a filter;
//  * a lock-free union-find over core points for the merge of Section IV-C:
//    a root is only ever hooked under a smaller root, so every tree's root is
//    the smallest index of its component whatever the order of the hooks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbk {

constexpr unsigned kStatusNonFinite = 1u;      // an input coordinate is NaN or inf
constexpr unsigned kStatusEdgeOverflow = 2u;   // the neighbour-pair list ran out of room
constexpr unsigned kStatusBandOverflow = 4u;   // the matrix-core band list ran out of room
constexpr unsigned kStatusRange = 8u;          // inputs outside the low-precision range
constexpr unsigned kStatusNoHoist = 16u;       // a coordinate beyond the hoisted form's range

constexpr int kPrecBf16 = 2;  // values of dbscan_opts.precision
constexpr int kPrecFp16 = 3;

// Per-call device state (first section of the workspace).
struct DevState {
  unsigned int status;             // kStatus* bits
  unsigned int noncore;            // compaction cursor for non-core rows
  unsigned long long band_pairs;   // pairs re-evaluated in float64 (all passes)
  unsigned long long core_points;
  unsigned long long edges;        // pairs (i, j), j < i, appended to the pair list
  unsigned long long band_list;    // pairs appended to the matrix-core band list
  unsigned long long max_norm;     // bit pattern of max |x_i| (float64, >= 0)
  float thr[2];                    // matrix-core filter thresholds (in, out)
  unsigned long long core_degree;   // sum of the core points' counts (when asked for)
  unsigned long long reserved1;
  unsigned int box_lo[4], box_hi[4];  // bounding box of the input (order-preserving bits)
  unsigned long long tests;           // pair tests made by a pruned sweep
  // Pair list in segments (0 or 1: one list at `edges`): segment s holds
  // entries [s * cap / pair_segs, ...) and counts its appends in
  // edge_seg[s][0], so the appends of many blocks spread over several
  // counters, each on a 128-byte line of its own.
  unsigned int pair_segs;
  unsigned int pad0;
  unsigned long long edge_seg[32][16];
};

constexpr int kPairSegments = 32;  // segments of the standalone pair list

constexpr int kNoNeighbour = 0x7fffffff;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A wave-uniform float in a scalar register.  Its load is waited for here: a
// value loaded before a loop and first read inside it makes the compiler wait
// at that read on every iteration, for every memory operation in flight
// (stores included).
__device__ __forceinline__ float wave_uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Neighbouring float32 values (finite x).
__device__ __forceinline__ float next_down(float x) {
  if (x == 0.0f) return -__uint_as_float(1u);
  const unsigned b = __float_as_uint(x);
  return __uint_as_float(x > 0.0f ? b - 1u : b + 1u);
}
__device__ __forceinline__ float next_up(float x) { return -next_down(-x); }

// Number of set bits of m below this lane.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Bits of the 64 columns cb..cb+63 that lie below row i (j < i).
__device__ __forceinline__ uint64_t below_mask(int i, int cb) {
  const int lim = i - cb;
  if (lim <= 0) return 0ull;
  if (lim >= 64) return ~0ull;
  return (1ull << lim) - 1ull;
}

// Exact float64 test of one pair: the definition's own arithmetic.
template <int D>
__device__ __forceinline__ bool exact_within(const float (&a)[D], const float (&b)[D], double eps2) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double t = (double)a[k] - (double)b[k];
    const double tt = t * t;
    s = s + tt;
  }
  return s <= eps2;
}

// Same, for coordinates read from memory (generic d).
__device__ __forceinline__ bool exact_within_mem(const float *a, int sa, const float *b, int sb,
                                                 int d, double eps2) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int k = 0; k < d; ++k) {
    const double t = (double)a[k * sa] - (double)b[k * sb];
    const double tt = t * t;
    s = s + tt;
  }
  return s <= eps2;
}

// Same, for two row-major rows of d floats: 16-byte loads when both rows are
// 16-byte aligned and d is a multiple of 4 (same order of operations).
__device__ __forceinline__ bool exact_within_rows(const float *a, const float *b, int d,
                                                  double eps2) {
#pragma clang fp contract(off)
  if ((d & 3) == 0 && ((((uintptr_t)a) | ((uintptr_t)b)) & 15) == 0) {
    const float4 *a4 = (const float4 *)a, *b4 = (const float4 *)b;
    double s = 0.0;
    for (int k = 0; k < (d >> 2); ++k) {
      const float4 x = a4[k], y = b4[k];
      double t = (double)x.x - (double)y.x;
      double tt = t * t;
      s = s + tt;
      t = (double)x.y - (double)y.y;
      tt = t * t;
      s = s + tt;
      t = (double)x.z - (double)y.z;
      tt = t * t;
      s = s + tt;
      t = (double)x.w - (double)y.w;
      tt = t * t;
      s = s + tt;
    }
    return s <= eps2;
  }
  return exact_within_mem(a, 1, b, 1, d, eps2);
}

// float32 direct form; any evaluation order is covered by the band.
template <int D>
__device__ __forceinline__ float sq_dist32(const float (&a)[D], const float (&b)[D]) {
  float t = a[0] - b[0];
  float s = t * t;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    t = a[k] - b[k];
    s = __builtin_fmaf(t, t, s);
  }
  return s;
}

// Smallest of G values (G = 4 or 8) as a tree of three-operand minima
// (v_min3_f32): one compare of the minimum then tells whether any of G
// squared distances reaches the band, where G compares would cost G
// instructions at the compare issue rate.  A NaN operand (padded column) is
// skipped as fminf skips it, and compares false like the value itself.
template <int G>
__device__ __forceinline__ float min_of(const float (&v)[G]) {
  static_assert(G == 4 || G == 8 || G == 16, "group size");
  if constexpr (G == 4) {
    return __builtin_fminf(__builtin_fminf(__builtin_fminf(v[0], v[1]), v[2]), v[3]);
  } else if constexpr (G == 16) {  // eight three-operand minima
    const float a = __builtin_fminf(__builtin_fminf(v[0], v[1]), v[2]);
    const float b = __builtin_fminf(__builtin_fminf(v[3], v[4]), v[5]);
    const float c = __builtin_fminf(__builtin_fminf(v[6], v[7]), v[8]);
    const float e = __builtin_fminf(__builtin_fminf(v[9], v[10]), v[11]);
    const float f = __builtin_fminf(__builtin_fminf(v[12], v[13]), v[14]);
    const float g = __builtin_fminf(__builtin_fminf(a, b), c);
    const float h = __builtin_fminf(__builtin_fminf(e, f), v[15]);
    return __builtin_fminf(g, h);
  } else {
    const float a = __builtin_fminf(__builtin_fminf(v[0], v[1]), v[2]);
    const float b = __builtin_fminf(__builtin_fminf(v[3], v[4]), v[5]);
    const float c = __builtin_fminf(__builtin_fminf(v[6], v[7]), a);
    return __builtin_fminf(b, c);
  }
}

// ------------------------------------------------------------ tile pruning
// Squared gap between two boxes (per-coordinate lo / hi) evaluated like a
// pair's squared distance: the corners are float32 coordinates of the input,
// so the band's guarantee holds for them -- gap2 > hi means the float64
// value of the corners' squared distance exceeds eps^2 -- and every real pair
// from the two boxes has per-coordinate differences at least the gaps, whose
// rounded squares and sums are then no smaller (rounding is monotone): no
// pair of the two boxes is a neighbour.  An empty box (lo = +inf, hi = -inf)
// gives an infinite gap.
template <int D>
__device__ __forceinline__ float box_gap2(const float (&alo)[D], const float (&ahi)[D],
                                          const float (&blo)[D], const float (&bhi)[D]) {
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float g = __builtin_fmaxf(__builtin_fmaxf(blo[k] - ahi[k], alo[k] - bhi[k]), 0.0f);
    s = __builtin_fmaf(g, g, s);
  }
  return s;
}

// Lane l takes the box of 64-point block b0 + l from the per-block boxes
// `box` ([2k][nb] lo, [2k+1][nb] hi); lanes past b1 take an empty box.
template <int D>
__device__ __forceinline__ void lane_box(const float *__restrict__ box, int nb, int b0, int b1,
                                         float (&lo)[D], float (&hi)[D]) {
  const int b = b0 + lane_id();
#pragma unroll
  for (int k = 0; k < D; ++k) {
    lo[k] = b < b1 ? box[(size_t)(2 * k) * nb + b] : __builtin_inff();
    hi[k] = b < b1 ? box[(size_t)(2 * k + 1) * nb + b] : -__builtin_inff();
  }
}

// Union of the lanes' boxes (the same value in every lane).
template <int D>
__device__ __forceinline__ void wave_box(const float (&lo)[D], const float (&hi)[D],
                                         float (&ulo)[D], float (&uhi)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    float l = lo[k], h = hi[k];
    for (int off = 32; off > 0; off >>= 1) {
      l = __builtin_fminf(l, __shfl_xor(l, off));
      h = __builtin_fmaxf(h, __shfl_xor(h, off));
    }
    ulo[k] = l;
    uhi[k] = h;
  }
}

// Box of the 64-point blocks [b0, b1) (b1 - b0 <= 64), in every lane.
template <int D>
__device__ __forceinline__ void span_box(const float *__restrict__ box, int nb, int b0, int b1,
                                         float (&lo)[D], float (&hi)[D]) {
  float l[D], h[D];
  lane_box<D>(box, nb, b0, b1, l, h);
  wave_box<D>(l, h, lo, hi);
}

// Re-decide the lanes in `band` in float64; returns the exact in-mask.
template <int D>
__device__ __forceinline__ uint64_t recheck_band(uint64_t band, uint64_t in, const float (&a)[D],
                                                 const float (&b)[D], double eps2,
                                                 DevState *st) {
  const int lane = lane_id();
  bool ex = false;
  if ((band >> lane) & 1ull) ex = exact_within<D>(a, b, eps2);
  const uint64_t exm = __ballot(ex);
  if (lane == 0) atomicAdd(&st->band_pairs, (unsigned long long)__popcll(band));
  return in | exm;
}

// Same, with the float64 operands read back from the transposed coordinates
// (soa[k * n_pad + i]) of row `row` and this lane's column `col`, so that the
// sweep keeps no float64 copies of its rows in registers.
__device__ __forceinline__ uint64_t recheck_band_soa(uint64_t band, uint64_t in,
                                                     const float *__restrict__ soa, int n_pad,
                                                     int d, int row, int col, double eps2,
                                                     DevState *st) {
  const int lane = lane_id();
  bool ex = false;
  if ((band >> lane) & 1ull) {
    // opaque to the optimizer: the sweep's own loads of these rows are not
    // reused (they would be widened and kept live across the whole loop)
    asm volatile("" : "+v"(row));
    ex = exact_within_mem(soa + row, n_pad, soa + col, n_pad, d, eps2);
  }
  const uint64_t exm = __ballot(ex);
  if (lane == 0) atomicAdd(&st->band_pairs, (unsigned long long)__popcll(band));
  return in | exm;
}

// A wave-uniform value moved into a vector register: VALU operations whose
// operands are all vector registers issue at twice the rate of those that
// read a scalar register on gfx950.
__device__ __forceinline__ float to_vgpr(float x) {
  float v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

// ---------------------------------------------------------------- union-find
// Reads and path-halving writes are relaxed atomics at work-group scope: they
// may be served by this XCD's caches and return an older value.  An older
// value of parent[v] is still an ancestor of v (links are never undone), so
// every walk stays correct and ends.  Only the hook itself -- a
// compare-and-swap at device scope on a node that must still be a root --
// needs the current value, and a failed swap returns it.
__device__ __forceinline__ int uf_load(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void uf_store(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving.  parent[v] <= v always holds, so the walk
// ends at a node whose parent is itself.
__device__ __forceinline__ int uf_find(int *parent, int x) {
  int cur = uf_load(parent + x);
  if (cur != x) {
    int prev = x;
    int next;
    while (cur > (next = uf_load(parent + cur))) {
      uf_store(parent + prev, next);
      prev = cur;
      cur = next;
    }
  }
  return cur;
}

// Join the trees whose (possibly outdated) roots are ra and rb: hook the
// larger root under the smaller one.  Returns a common ancestor.
__device__ __forceinline__ int uf_link(int *parent, int ra, int rb) {
  while (ra != rb) {
    if (ra < rb) {
      const int t = ra;
      ra = rb;
      rb = t;
    }
    int expected = ra;
    if (__hip_atomic_compare_exchange_strong(parent + ra, &expected, rb, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return rb;
    ra = uf_find(parent, expected);
  }
  return ra;
}

__device__ __forceinline__ void uf_union(int *parent, int a, int b) {
  uf_link(parent, uf_find(parent, a), uf_find(parent, b));
}

// ------------------------------------------------------- wave pair queue
// A wave-private queue of (a, b) pairs in LDS.  Ballots fill it from
// whichever lanes found a pair.  Union queues (128 entries) are drained 64
// pairs at a time so that every lane of the wave works on one pair (union-find
// walks are latency bound, so a full wave of independent walks hides the
// latency).  List queues are appended to a global list once `limit` pairs are
// queued (the buffer holds limit + 64), with one atomic on the list cursor for
// the whole batch: the cursor is shared by the whole grid.
constexpr int kListQueue = 320;  // list-queue buffer (pairs)
constexpr int kListDrain = 256;  // ... appended to the global list at this fill

struct WaveQueue {
  int2 *buf;
  int count;  // wave-uniform
  int limit;  // list queues: append once this many are queued
};

__device__ __forceinline__ void wq_push(WaveQueue &q, bool has, int a, int b) {
  const uint64_t m = __ballot(has);
  if (m == 0ull) return;
  if (has) q.buf[q.count + lanes_below(m)] = make_int2(a, b);
  q.count += __popcll(m);
}

__device__ __forceinline__ void wq_pop(WaveQueue &q, int take) {
  const int lane = lane_id();
  const int rest = q.count - take;
  int2 v = make_int2(0, 0);
  if (lane < rest) v = q.buf[take + lane];
  if (lane < rest) q.buf[lane] = v;
  q.count = rest;
}

// Join the queued pairs (all of them when `all`, else 64 at a time while
// at least 64 are queued).
__device__ __forceinline__ void wq_drain_union(WaveQueue &q, int *parent, bool all) {
  while (q.count >= 64 || (all && q.count > 0)) {
    const int take = q.count < 64 ? q.count : 64;
    if (lane_id() < take) {
      const int2 e = q.buf[lane_id()];
      uf_union(parent, e.x, e.y);
    }
    wq_pop(q, take);
  }
}

// Append the queued pairs to a global list at *cursor (when at least q.limit
// are queued, or any when `all`); past `cap` entries the pairs are dropped
// and `flag` is raised in the status word.
__device__ __forceinline__ void wq_drain_to(WaveQueue &q, int2 *list, long long cap,
                                            unsigned long long *cursor, unsigned *status,
                                            unsigned flag, bool all) {
  if (q.count < q.limit && !(all && q.count > 0)) return;
  const int lane = lane_id();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(cursor, (unsigned long long)q.count);
  base = __shfl(base, 0);
  for (int k = lane; k < q.count; k += 64) {
    const unsigned long long idx = base + (unsigned long long)k;
    if (idx < (unsigned long long)cap) list[idx] = q.buf[k];
  }
  if (lane == 0 && base + (unsigned long long)q.count > (unsigned long long)cap)
    atomicOr(status, flag);
  q.count = 0;
}

// End of a block: the leftovers of the 4 waves' queues go to the list with
// one atomic for the block.  Every thread of the block calls it; `xfer` is 5
// words of LDS.
__device__ __forceinline__ void wq_flush_block(WaveQueue &q, int2 *list, long long cap,
                                               unsigned long long *cursor, unsigned *status,
                                               unsigned flag, unsigned long long *xfer) {
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  if (lane == 0) xfer[w] = (unsigned long long)q.count;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tot = xfer[0] + xfer[1] + xfer[2] + xfer[3];
    const unsigned long long base = tot ? atomicAdd(cursor, tot) : 0ull;
    if (tot && base + tot > (unsigned long long)cap) atomicOr(status, flag);
    xfer[4] = base;
  }
  __syncthreads();
  unsigned long long off = xfer[4];
  for (int k = 0; k < w; ++k) off += xfer[k];
  for (int k = lane; k < q.count; k += 64) {
    const unsigned long long idx = off + (unsigned long long)k;
    if (idx < (unsigned long long)cap) list[idx] = q.buf[k];
  }
  q.count = 0;
  __syncthreads();  // xfer is reused by the next flush
}

// The pair-list segment of this work-group: its first entry, capacity and
// append counter.
struct PairSegment {
  int2 *list;
  long long cap;
  unsigned long long *cursor;
};

__device__ __forceinline__ PairSegment pair_segment(int2 *list, long long cap, DevState *st) {
  const unsigned S = st->pair_segs;
  if (S <= 1u) return PairSegment{list, cap, &st->edges};
  const unsigned sgm = blockIdx.x % S;
  const long long seg_cap = cap / S;
  return PairSegment{list + sgm * seg_cap, seg_cap, &st->edge_seg[sgm][0]};
}

// Neighbour pairs (i, j), j < i, for the merge.
__device__ __forceinline__ void wq_drain_list(WaveQueue &q, int2 *list, long long cap,
                                              DevState *st, bool all) {
  if (q.count < q.limit && !(all && q.count > 0)) return;
  const PairSegment g = pair_segment(list, cap, st);
  wq_drain_to(q, g.list, g.cap, g.cursor, &st->status, kStatusEdgeOverflow, all);
}

// End of a block for a pair-list queue (wq_flush_block on this block's segment).
__device__ __forceinline__ void wq_flush_pairs(WaveQueue &q, int2 *list, long long cap,
                                               DevState *st, unsigned long long *xfer) {
  const PairSegment g = pair_segment(list, cap, st);
  wq_flush_block(q, g.list, g.cap, g.cursor, &st->status, kStatusEdgeOverflow, xfer);
}

// Pairs the matrix-core filter could not decide.
__device__ __forceinline__ void wq_drain_band(WaveQueue &q, int2 *list, long long cap,
                                              DevState *st, bool all) {
  wq_drain_to(q, list, cap, &st->band_list, &st->status, kStatusBandOverflow, all);
}

}  // namespace dbk
