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

constexpr unsigned kStatusNonFinite = 1u;

// Per-call device state (first 256 bytes of the workspace).
struct DevState {
  unsigned int status;           // kStatusNonFinite when an input is NaN/inf
  unsigned int noncore;          // compaction cursor for non-core rows
  unsigned long long band_pairs; // step-1 pairs re-evaluated in float64
  unsigned long long core_points;
  unsigned long long reserved[5];
};

constexpr int kNoNeighbour = 0x7fffffff;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// ---------------------------------------------------------------- union-find
__device__ __forceinline__ int uf_load(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void uf_store(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.  parent[v] <= v always holds, so the walk
// ends; a stale read only returns an older ancestor, which is still valid.
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

// Join the trees of a and b: hook the larger root under the smaller one.
__device__ __forceinline__ void uf_union(int *parent, int a, int b) {
  int ra = uf_find(parent, a);
  int rb = uf_find(parent, b);
  while (ra != rb) {
    if (ra < rb) {
      const int t = ra;
      ra = rb;
      rb = t;
    }
    int expected = ra;
    if (__hip_atomic_compare_exchange_strong(parent + ra, &expected, rb, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
    ra = uf_find(parent, expected);
  }
}

}  // namespace dbk
