// Block-level bodies of the kernels shared by both forms (staging, core flags,
// merge from the pair list, labels).  Each body does the work of one
// 256-thread block given its block index, so the standalone kernels and the
// persistent serving loop run the same code.
#pragma once

#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// soa[k][i] = points[p][k] for k < d, 0 for d <= k < d_pad, NaN for i >= n,
// where p = perm[i] (the spatial order) or i without one; flags non-finite
// input.
__device__ __forceinline__ void stage_soa_body(const float *__restrict__ pts, int n, int d,
                                               int n_pad, int d_pad, float *__restrict__ soa,
                                               DevState *st, int bid,
                                               const int *__restrict__ perm = nullptr) {
  const int i = bid * 256 + (int)threadIdx.x;
  if (i >= n_pad) return;
  bool bad = false;
  const float qnan = __builtin_nanf("");
  const size_t src = (perm && i < n) ? (size_t)perm[i] : (size_t)i;
  for (int k = 0; k < d_pad; ++k) {
    float v;
    if (i < n) {
      v = (k < d) ? pts[src * d + k] : 0.0f;
      bad |= !__builtin_isfinite(v);
    } else {
      v = qnan;
    }
    soa[(size_t)k * n_pad + i] = v;
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&st->status, kStatusNonFinite);
}

// Rows of the hoisted test (HoistView) for the staged coordinates: thread i
// of the grid (n_pad threads) takes row i.  The 16 rows of a block are 16
// lanes of one wave, so their box comes from lane shuffles (NaN padding
// skipped).  A coordinate beyond 2^60 in magnitude (where |b|^2 and the
// products could overflow) sets kStatusNoHoist: the sweep then takes the
// direct form.
__device__ __forceinline__ void hoist_prep_body(const float *__restrict__ soa, int n, int d,
                                                int n_pad, double eps2, float *__restrict__ hoist,
                                                DevState *st, int bid) {
  const int i = bid * 256 + (int)threadIdx.x;  // every lane of the wave is a row
  const HoistView<float> v = hoist_view(hoist, n_pad, d);
  const int blk = i >> 4;
  bool far = false;
  double T = 0.0;
  for (int k = 0; k < d; ++k) {
    const float x = soa[(size_t)k * n_pad + i];
    far |= i < n && !(__builtin_fabsf(x) <= 0x1p60f);
    float lo = x, hi = x;
    for (int off = 1; off < 16; off <<= 1) {
      lo = __builtin_fminf(lo, __shfl_xor(lo, off));
      hi = __builtin_fmaxf(hi, __shfl_xor(hi, off));
    }
    const float c = 0.5f * lo + 0.5f * hi;
    if ((i & 15) == 0) {
      v.box[(size_t)(2 * k) * (n_pad / 16) + blk] = lo;
      v.box[(size_t)(2 * k + 1) * (n_pad / 16) + blk] = hi;
      v.cen[(size_t)k * (n_pad / 16) + blk] = c;
    }
    const float a = x - c;
    v.a[(size_t)k * n_pad + i] = -2.0f * a;
    T += (double)a * (double)a;
  }
  float lo, hi;
  hoist_band(T, d, eps2, &lo, &hi);
  v.lo[i] = lo;
  v.hi[i] = hi;
  float h = hi;
  for (int off = 1; off < 8; off <<= 1) h = __builtin_fmaxf(h, __shfl_xor(h, off));
  if ((i & 7) == 0) v.hg[i >> 3] = h;
  // the 16-row block's gate: its largest hi and largest |fl(x - c)|^2
  // (padding rows are NaN and drop out of both maxima)
  h = __builtin_fmaxf(h, __shfl_xor(h, 8));
  double t2 = T;
  for (int off = 1; off < 16; off <<= 1) t2 = __builtin_fmax(t2, __shfl_xor(t2, off));
  if ((i & 15) == 0) v.g16[blk] = hoist_gate(h, t2, d);
  if (__ballot(far) != 0ull && lane_id() == 0) atomicOr(&st->status, kStatusNoHoist);
}

// Clears counts, parent = identity, jstar = none; with `soa`, also stages the
// coordinates (stage_soa_body).  With a spatial order `perm` (staged index ->
// caller's index) it also fills its inverse and clears the per-root lowest
// caller index used by the labels.
__device__ __forceinline__ void stage_body(const float *__restrict__ pts, int n, int d, int n_pad,
                                           int d_pad, float *__restrict__ soa,
                                           int *__restrict__ counts, int *__restrict__ parent,
                                           int *__restrict__ jstar, DevState *st, int bid,
                                           const int *__restrict__ perm = nullptr,
                                           int *__restrict__ inv = nullptr,
                                           int *__restrict__ rootmin = nullptr) {
  if (soa) stage_soa_body(pts, n, d, n_pad, d_pad, soa, st, bid, perm);
  const int i = bid * 256 + (int)threadIdx.x;
  if (i < n) {
    counts[i] = 0;
    parent[i] = i;
    jstar[i] = kNoNeighbour;
    if (perm) {
      inv[perm[i]] = i;
      rootmin[i] = kNoNeighbour;
    }
  }
}

// ------------------------------------------------------------- core flags
// corebits in the staged order; core[] (and, with a spatial order, the
// counts) written in the caller's order.  With `count` the number of core
// points goes to st->core_points, and with `degree` the sum of the core
// points' counts to st->core_degree (one atomic per block each).  Every
// thread of the block must call it (it synchronises the block).
__device__ __forceinline__ void core_body(const int *__restrict__ counts, int n, int n_pad,
                                          int minpts, uint8_t *__restrict__ core,
                                          uint32_t *__restrict__ corebits, DevState *st, int bid,
                                          const int *__restrict__ perm = nullptr,
                                          int *__restrict__ counts_out = nullptr,
                                          bool count = false, bool degree = false) {
  __shared__ unsigned block_cores;
  __shared__ unsigned long long block_degree;
  const int i = bid * 256 + (int)threadIdx.x;
  const bool c = i < n && counts[i] >= minpts;
  if (i < n) {
    if (perm) {
      const int o = perm[i];
      core[o] = c ? 1 : 0;
      counts_out[o] = counts[i];
    } else {
      core[i] = c ? 1 : 0;
    }
  }
  const uint64_t m = __ballot(c);
  const int lane = lane_id();
  if (lane == 0 && i < n_pad) {  // n_pad is a multiple of 64: whole waves
    corebits[i >> 5] = (uint32_t)m;
    corebits[(i >> 5) + 1] = (uint32_t)(m >> 32);
  }
  if (!count && !degree) return;  // uniform over the launch
  if (threadIdx.x == 0) {
    block_cores = 0u;
    block_degree = 0ull;
  }
  __syncthreads();
  if (count && lane == 0 && m) atomicAdd(&block_cores, (unsigned)__popcll(m));
  if (degree) {
    unsigned long long v = c ? (unsigned long long)counts[i] : 0ull;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0 && v) atomicAdd(&block_degree, v);
  }
  __syncthreads();
  if (threadIdx.x == 0 && block_cores) atomicAdd(&st->core_points, (unsigned long long)block_cores);
  if (threadIdx.x == 0 && block_degree) atomicAdd(&st->core_degree, block_degree);
}

// --------------------------------------------- merge + border from the list
// Every neighbour pair (a, b), b < a, found by step 1: core-core pairs are
// joined in the union-find; a non-core end takes the smaller caller index
// (okey[], or the index itself without a spatial order) of its core
// neighbours (atomicMin), which after all pairs is its lowest-index core
// neighbour.  This block handles pairs [e_begin, e_end).
__device__ __forceinline__ void merge_pairs_range(const int2 *__restrict__ pairs,
                                                  const uint32_t *__restrict__ corebits,
                                                  int *__restrict__ parent,
                                                  int *__restrict__ jstar,
                                                  unsigned long long e_begin,
                                                  unsigned long long e_end,
                                                  const int *__restrict__ okey = nullptr) {
  for (unsigned long long e = e_begin + threadIdx.x; e < e_end; e += 256) {
    const int2 pr = pairs[e];
    const bool ca = (corebits[pr.x >> 5] >> (pr.x & 31)) & 1u;
    const bool cb = (corebits[pr.y >> 5] >> (pr.y & 31)) & 1u;
    if (ca && cb)
      uf_union(parent, pr.x, pr.y);
    else if (ca)
      atomicMin(jstar + pr.y, okey ? okey[pr.x] : pr.x);
    else if (cb)
      atomicMin(jstar + pr.x, okey ? okey[pr.y] : pr.y);
  }
}

// ------------------------------------------------------------------ labels
// Without a spatial order a tree's root is the lowest index of its component
// (the union-find hooks larger roots under smaller ones), so it is the label.
// With one (perm: staged index -> caller's index), the label of a component
// is the lowest caller index of its core points, gathered per root first by
// rootmin_body; jstar then holds caller indices and inv maps them back.
__device__ __forceinline__ void rootmin_body(int n, const uint32_t *__restrict__ corebits,
                                             int *__restrict__ parent,
                                             const int *__restrict__ perm,
                                             int *__restrict__ rootmin, int bid) {
  const int i = bid * 256 + (int)threadIdx.x;
  const bool is_core = i < n && ((corebits[i >> 5] >> (i & 31)) & 1u);
  const int root = is_core ? uf_find(parent, i) : 0;
  const int key = is_core ? perm[i] : kNoNeighbour;
  // the lanes of a wave mostly share a root: one atomic per distinct root
  bool pending = is_core;
  uint64_t left = __ballot(pending);
  while (left != 0ull) {
    const int leader = __builtin_ctzll(left);
    const int r = __shfl(root, leader);
    const bool mine = pending && root == r;
    int v = mine ? key : kNoNeighbour;
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    if (lane_id() == leader) atomicMin(rootmin + r, v);
    pending = pending && !mine;
    left = __ballot(pending);
  }
}

__device__ __forceinline__ void labels_body(int n, const uint32_t *__restrict__ corebits,
                                            const int *__restrict__ jstar, int *__restrict__ parent,
                                            int *__restrict__ labels, const DevState *st, int bid,
                                            const int *__restrict__ perm = nullptr,
                                            const int *__restrict__ inv = nullptr,
                                            const int *__restrict__ rootmin = nullptr) {
  const int i = bid * 256 + (int)threadIdx.x;
  if (i >= n) return;
  const int o = perm ? perm[i] : i;
  if (st->status & kStatusNonFinite) {
    labels[o] = -2;
    return;
  }
  int root;
  if ((corebits[i >> 5] >> (i & 31)) & 1u) {
    root = uf_find(parent, i);
  } else {
    const int j = jstar[i];
    if (j == kNoNeighbour) {
      labels[o] = -1;
      return;
    }
    root = uf_find(parent, perm ? inv[j] : j);
  }
  labels[o] = perm ? rootmin[root] : root;
}

}  // namespace dbk
