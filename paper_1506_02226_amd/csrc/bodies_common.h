// Block-level bodies of the kernels shared by both forms (staging, core flags,
// merge from the pair list, labels).  Each body does the work of one
// 256-thread block given its block index, so the standalone kernels and the
// persistent serving loop run the same code.
#pragma once

#include "dbscan_device.h"

namespace dbk {

// soa[k][i] = points[i][k] for k < d, 0 for d <= k < d_pad, NaN for i >= n;
// flags non-finite input.
__device__ __forceinline__ void stage_soa_body(const float *__restrict__ pts, int n, int d,
                                               int n_pad, int d_pad, float *__restrict__ soa,
                                               DevState *st, int bid) {
  const int i = bid * 256 + (int)threadIdx.x;
  if (i >= n_pad) return;
  bool bad = false;
  const float qnan = __builtin_nanf("");
  for (int k = 0; k < d_pad; ++k) {
    float v;
    if (i < n) {
      v = (k < d) ? pts[(size_t)i * d + k] : 0.0f;
      bad |= !__builtin_isfinite(v);
    } else {
      v = qnan;
    }
    soa[(size_t)k * n_pad + i] = v;
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&st->status, kStatusNonFinite);
}

// Clears counts, parent = identity, jstar = none; with `soa`, also stages the
// coordinates (stage_soa_body).
__device__ __forceinline__ void stage_body(const float *__restrict__ pts, int n, int d, int n_pad,
                                           int d_pad, float *__restrict__ soa,
                                           int *__restrict__ counts, int *__restrict__ parent,
                                           int *__restrict__ jstar, DevState *st, int bid) {
  if (soa) stage_soa_body(pts, n, d, n_pad, d_pad, soa, st, bid);
  const int i = bid * 256 + (int)threadIdx.x;
  if (i < n) {
    counts[i] = 0;
    parent[i] = i;
    jstar[i] = kNoNeighbour;
  }
}

// ------------------------------------------------------------- core flags
__device__ __forceinline__ void core_body(const int *__restrict__ counts, int n, int n_pad,
                                          int minpts, uint8_t *__restrict__ core,
                                          uint32_t *__restrict__ corebits, DevState *st, int bid) {
  const int i = bid * 256 + (int)threadIdx.x;
  if (i >= n_pad) return;  // n_pad is a multiple of 64: whole waves
  const bool c = i < n && counts[i] >= minpts;
  if (i < n) core[i] = c ? 1 : 0;
  const uint64_t m = __ballot(c);
  const int lane = lane_id();
  if (lane == 0) {
    corebits[i >> 5] = (uint32_t)m;
    corebits[(i >> 5) + 1] = (uint32_t)(m >> 32);
    if (m) atomicAdd(&st->core_points, (unsigned long long)__popcll(m));
  }
}

// --------------------------------------------- merge + border from the list
// Every neighbour pair (a, b), b < a, found by step 1: core-core pairs are
// joined in the union-find; a non-core end takes the smaller index of its
// core neighbours (atomicMin), which after all pairs is its lowest-index core
// neighbour.  This block handles pairs [e_begin, e_end).
__device__ __forceinline__ void merge_pairs_range(const int2 *__restrict__ pairs,
                                                  const uint32_t *__restrict__ corebits,
                                                  int *__restrict__ parent,
                                                  int *__restrict__ jstar,
                                                  unsigned long long e_begin,
                                                  unsigned long long e_end) {
  for (unsigned long long e = e_begin + threadIdx.x; e < e_end; e += 256) {
    const int2 pr = pairs[e];
    const bool ca = (corebits[pr.x >> 5] >> (pr.x & 31)) & 1u;
    const bool cb = (corebits[pr.y >> 5] >> (pr.y & 31)) & 1u;
    if (ca && cb)
      uf_union(parent, pr.x, pr.y);
    else if (ca)
      atomicMin(jstar + pr.y, pr.x);
    else if (cb)
      atomicMin(jstar + pr.x, pr.y);
  }
}

// ------------------------------------------------------------------ labels
__device__ __forceinline__ void labels_body(int n, const uint8_t *__restrict__ core,
                                            const int *__restrict__ jstar, int *__restrict__ parent,
                                            int *__restrict__ labels, const DevState *st, int bid) {
  const int i = bid * 256 + (int)threadIdx.x;
  if (i >= n) return;
  if (st->status & kStatusNonFinite) {
    labels[i] = -2;
    return;
  }
  if (core[i]) {
    labels[i] = uf_find(parent, i);
  } else {
    const int j = jstar[i];
    labels[i] = (j == kNoNeighbour) ? -1 : uf_find(parent, j);
  }
}

}  // namespace dbk
