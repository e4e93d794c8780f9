// Block-level body of the float32 step-1 sweep for d <= 4 (rows in scalar
// registers, columns in lanes), shared by the standalone kernel and the
// persistent serving loop.
#pragma once

#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// Lanes of the band (m & ~in) re-decided in float64; returns the exact mask.
template <int D>
__device__ __forceinline__ uint64_t settle_band(uint64_t m, uint64_t in, const float (&a)[D],
                                                const float (&b)[D], double eps2, DevState *st) {
  if (in == m) return in;
  return recheck_band<D>(m & ~in, in, a, b, eps2, st);
}

// ------------------------------------------------- step 1 + counts, d <= 4
// One block = 4 waves x R rows over one column chunk; `qbuf` is the
// block's LDS queue space ([4][128] pairs).
template <int D, int R, bool EMIT>
__device__ __forceinline__ void count_small_body(const float *__restrict__ soa,
                                                 int *__restrict__ counts,
                                                 int2 *__restrict__ pairs,
                                                 DevState *__restrict__ st,
                                                 const SweepScalars &sc, int bid,
                                                 int2 (*qbuf)[128]) {
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = bid % sc.nchunks;
  const int row0 = ((bid / sc.nchunks) * 4 + w) * R;
  if (row0 >= sc.n) return;
  const int c0 = chunk * sc.chunk;
  const int c1 = min(c0 + sc.chunk, sc.n_pad);
  float xr[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < D; ++k) xr[r][k] = soa[(size_t)k * sc.n_pad + row0 + r];
  int cnt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) cnt[r] = 0;
  WaveQueue qu{qbuf[w], 0};
  float xn[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xn[k] = soa[(size_t)k * sc.n_pad + c0 + lane];
  for (int cb = c0; cb < c1; cb += 64) {
    float xc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xc[k] = xn[k];
    if (cb + 64 < c1) {
#pragma unroll
      for (int k = 0; k < D; ++k) xn[k] = soa[(size_t)k * sc.n_pad + cb + 64 + lane];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float s = sq_dist32<D>(xr[r], xc);
      const uint64_t m = __ballot(s <= sc.hi);
      if (m != 0ull) {
        const uint64_t in = settle_band<D>(m, __ballot(s <= sc.lo), xr[r], xc, sc.eps2, st);
        cnt[r] += __popcll(in);
        if (EMIT) {
          const uint64_t e = in & below_mask(row0 + r, cb);
          if (e != 0ull) {
            wq_push(qu, (e >> lane) & 1ull, row0 + r, cb + lane);
            wq_drain_list(qu, pairs, sc.edge_cap, st, false);
          }
        }
      }
    }
  }
  if (EMIT) wq_drain_list(qu, pairs, sc.edge_cap, st, true);
  int mine = 0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane == r) mine = cnt[r];
  const int row = row0 + lane;
  if (lane < R && row < sc.n) {
    if (sc.nchunks == 1)
      counts[row] = mine;
    else
      atomicAdd(counts + row, mine);
  }
}

}  // namespace dbk
