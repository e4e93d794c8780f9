// Row-uniform sweeps of the on-the-fly form (Section IV-B.1: the distance is
// fused with the neighbourhood test and never stored).  One wave owns R rows
// -- the "goal points" of Section IV-A.3, kept in vector registers (the same
// value in every lane) for d <= 4 or read from LDS as broadcasts otherwise --
// and the 64 lanes hold 64 columns, so one compare yields one 64-bit ballot
// word of the primitive cluster of a row.
//
//  * k_count_tri: step 1 + counts, each unordered pair tested once; also
//    appends every neighbour pair (i, j), j < i, to a pair list (the input of
//    the merge) while it fits.
//  * k_union_small / k_border_small: the merge and the border pass repeated
//    on the fly; they run only when the pair list overflowed (or always, for
//    the border pass of the bitmask form).
//  * k_rows_lds: the three sweeps for d > 4 (no pair list).
#include "dbscan_device.h"
#include "dbscan_internal.h"
#include "bodies_sweep.h"

namespace dbk {

// A fallback sweep runs only when the status word says its primary path
// gave up (pair list overflow, or matrix-core filter out of range / band
// list overflow).
__device__ __forceinline__ bool skip_sweep(const SweepScalars &sc, const DevState *st) {
  if (!sc.flags) return false;
  const unsigned status =
      __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((sc.flags & kOnlyOnOverflow) && (status & kStatusEdgeOverflow)) return false;
  if ((sc.flags & kOnlyOnFilterFail) && (status & (kStatusRange | kStatusBandOverflow)))
    return false;
  return true;
}

// ------------------------------------------------- step 1 + counts, d <= 4
// Triangular form (each unordered pair tested once); LDS column tallies.
constexpr int kTriMaxChunk = 4096;

template <int D, int R, bool EMIT, bool PRUNE>
__global__ __launch_bounds__(256) void k_count_tri(const float *__restrict__ soa,
                                                   int *__restrict__ counts,
                                                   int2 *__restrict__ pairs,
                                                   DevState *__restrict__ st, SweepScalars sc) {
  __shared__ int2 qbuf[4][kListQueue];
  __shared__ int colcnt[kTriMaxChunk];
  __shared__ unsigned long long xfer[5];
  if (skip_sweep(sc, st)) return;
  if (use_hoist(sc, st))
    count_tri_body<D, R, EMIT, PRUNE, kListQueue, true>(soa, counts, pairs, st, sc, blockIdx.x,
                                                        qbuf, colcnt, xfer);
  else
    count_tri_body<D, R, EMIT, PRUNE>(soa, counts, pairs, st, sc, blockIdx.x, qbuf, colcnt, xfer);
}

// Pruned form: a persistent grid over the blocks within reach.  Its tiles
// are mostly ones with neighbours, so the pairs come fast: the wave queues
// are four times longer, so that appends to the list are rarer.
constexpr int kPrunedQueue = 4 * kListDrain + 64;

template <int D, int R, bool EMIT>
__global__ __launch_bounds__(256) void k_count_tri_pruned(const float *__restrict__ soa,
                                                          int *__restrict__ counts,
                                                          int2 *__restrict__ pairs,
                                                          DevState *__restrict__ st,
                                                          SweepScalars sc) {
  __shared__ int2 qbuf[4][kPrunedQueue];
  __shared__ int colcnt[kTriMaxChunk];
  __shared__ unsigned long long xfer[5];
  if (skip_sweep(sc, st)) return;
  if (use_hoist(sc, st))
    for_near_blocks<D>(sc, sc.n, [&](int bid) {
      count_tri_body<D, R, EMIT, true, kPrunedQueue, true>(soa, counts, pairs, st, sc, bid, qbuf,
                                                           colcnt, xfer);
    });
  else
    for_near_blocks<D>(sc, sc.n, [&](int bid) {
      count_tri_body<D, R, EMIT, true, kPrunedQueue>(soa, counts, pairs, st, sc, bid, qbuf,
                                                     colcnt, xfer);
    });
}

// Boxes of the row groups and of the column chunks of a pruned sweep, each
// the union of its 64-point block boxes (one wave per box; at most 64
// blocks each).
__global__ __launch_bounds__(256) void k_coarse_boxes(float *__restrict__ box, int n_pad, int d,
                                                      int rgroup, int groups, int chunk,
                                                      int nchunks) {
  const int nb = n_pad / 64;
  const int wv = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (wv >= groups + nchunks) return;
  const bool is_group = wv < groups;
  const int idx = is_group ? wv : wv - groups;
  const int span = is_group ? rgroup : chunk;
  const int b0 = idx * span / 64, b1 = min((idx + 1) * span, n_pad) / 64;
  float *out = box + (is_group ? 2 : 4) * d * nb;
  const int b = b0 + lane_id();
  for (int k = 0; k < d; ++k) {
    float l = b < b1 ? box[(size_t)(2 * k) * nb + b] : __builtin_inff();
    float h = b < b1 ? box[(size_t)(2 * k + 1) * nb + b] : -__builtin_inff();
    for (int off = 32; off > 0; off >>= 1) {
      l = __builtin_fminf(l, __shfl_xor(l, off));
      h = __builtin_fmaxf(h, __shfl_xor(h, off));
    }
    if (lane_id() == 0) {
      out[(size_t)(2 * k) * nb + idx] = l;
      out[(size_t)(2 * k + 1) * nb + idx] = h;
    }
  }
}

hipError_t run_coarse_boxes(const SweepScalars &sc, hipStream_t s) {
  const int nb = sc.n_pad / 64;
  const int groups = (sc.n_pad + sc.rgroup - 1) / sc.rgroup;
  if (sc.rgroup > 64 * 64 || sc.chunk > 64 * 64 || groups > nb || sc.nchunks > nb)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse_boxes, dim3((groups + sc.nchunks + 3) / 4), dim3(256), 0, s, sc.box,
                     sc.n_pad, sc.d, sc.rgroup, groups, sc.chunk, sc.nchunks);
  return hipGetLastError();
}

unsigned pruned_grid(unsigned full_grid) { return full_grid < 4096 ? full_grid : 4096; }

// --------------------------------------- merge repeated on the fly, d <= 4
// Core rows i queue their core neighbours j < i; the queue is drained into
// the union-find 64 pairs at a time.
template <int D, int R>
__global__ __launch_bounds__(256) void k_union_small(const float *__restrict__ soa,
                                                     const uint32_t *__restrict__ corebits,
                                                     int *__restrict__ parent,
                                                     DevState *__restrict__ st, SweepScalars sc) {
  __shared__ int2 qbuf[4][128];
  if (skip_sweep(sc, st)) return;
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int total = (sc.n + R - 1) / R;
  const int rb = total - 1 - (int)(blockIdx.x * 4 + w);  // longest rows first
  if (rb < 0) return;
  const int row0 = rb * R;
  uint32_t active = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = row0 + r;
    if (i < sc.n && ((corebits[i >> 5] >> (i & 31)) & 1u)) active |= 1u << r;
  }
  if (active == 0u) return;
  const int last = row0 + 31 - __builtin_clz(active);
  const int c1 = ((last + 63) >> 6) << 6;  // columns j < last
  float xr[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < D; ++k) xr[r][k] = soa[(size_t)k * sc.n_pad + row0 + r];
  WaveQueue qu{qbuf[w], 0, 64};
  for (int cb = 0; cb < c1; cb += 64) {
    const uint64_t cw = (uint64_t)corebits[cb >> 5] | ((uint64_t)corebits[(cb >> 5) + 1] << 32);
    if (cw == 0ull) continue;
    float xc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xc[k] = soa[(size_t)k * sc.n_pad + cb + lane];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!((active >> r) & 1u)) continue;
      const uint64_t cm = cw & below_mask(row0 + r, cb);
      if (cm == 0ull) continue;
      const float s = sq_dist32<D>(xr[r], xc);
      const uint64_t m = __ballot(s <= sc.hi) & cm;
      if (m != 0ull) {
        const uint64_t in =
            settle_band<D>(m, __ballot(s <= sc.lo) & cm, xr[r], xc, sc.eps2, st);
        wq_push(qu, (in >> lane) & 1ull, row0 + r, cb + lane);
        wq_drain_union(qu, parent, false);
      }
    }
  }
  wq_drain_union(qu, parent, true);
}

// ----------------------------------- border points repeated on the fly, d <= 4
// Work item = (group of R listed non-core rows, column chunk); a persistent
// grid strides over the items.  Each item records the first core neighbour
// in its chunk with atomicMin, so the lowest-index one survives.  With a
// spatial order (okey: caller's index of each staged row) the item takes the
// smallest okey over all the core neighbours in its chunk instead.
template <int D, int R>
__global__ __launch_bounds__(256) void k_border_small(const float *__restrict__ soa,
                                                      const uint32_t *__restrict__ corebits,
                                                      const int *__restrict__ list,
                                                      int *__restrict__ jstar,
                                                      const int *__restrict__ okey,
                                                      DevState *__restrict__ st, SweepScalars sc) {
  if (skip_sweep(sc, st)) return;
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int listed = wave_uniform((int)__hip_atomic_load(&st->noncore, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
  const int groups = (listed + R - 1) / R;
  const int items = groups * sc.nchunks;
  const int nwaves = gridDim.x * 4;
  for (int item = blockIdx.x * 4 + w; item < items; item += nwaves) {
    const int chunk = item % sc.nchunks;
    const int e0 = (item / sc.nchunks) * R;
    int rows[R];
    uint32_t active = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rows[r] = 0;
      if (e0 + r < listed) {
        rows[r] = wave_uniform(list[e0 + r]);
        active |= 1u << r;
      }
    }
    float xr[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < D; ++k) xr[r][k] = soa[(size_t)k * sc.n_pad + rows[r]];
    int found[R];
#pragma unroll
    for (int r = 0; r < R; ++r) found[r] = kNoNeighbour;
    const int c0 = chunk * sc.chunk;
    const int c1 = min(c0 + sc.chunk, sc.n_pad);
    float xn[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xn[k] = soa[(size_t)k * sc.n_pad + c0 + lane];
    for (int cb = c0; cb < c1 && active != 0u; cb += 64) {
      float xc[D];
#pragma unroll
      for (int k = 0; k < D; ++k) xc[k] = xn[k];
      if (cb + 64 < c1) {  // next block's columns in flight during this one
#pragma unroll
        for (int k = 0; k < D; ++k) xn[k] = soa[(size_t)k * sc.n_pad + cb + 64 + lane];
      }
      const uint64_t cw = (uint64_t)corebits[cb >> 5] | ((uint64_t)corebits[(cb >> 5) + 1] << 32);
      if (cw == 0ull) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!((active >> r) & 1u)) continue;
        const float s = sq_dist32<D>(xr[r], xc);
        const uint64_t m = __ballot(s <= sc.hi) & cw;
        if (m != 0ull) {
          const uint64_t in =
              settle_band<D>(m, __ballot(s <= sc.lo) & cw, xr[r], xc, sc.eps2, st);
          if (in != 0ull) {
            if (okey) {
              for (uint64_t m2 = in; m2 != 0ull; m2 &= m2 - 1ull)
                found[r] = min(found[r], okey[cb + __builtin_ctzll(m2)]);
            } else {
              found[r] = cb + __builtin_ctzll(in);
              active &= ~(1u << r);
            }
          }
        }
      }
    }
    int mine = kNoNeighbour, myrow = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane == r) {
        mine = found[r];
        myrow = rows[r];
      }
    if (lane < R && mine != kNoNeighbour) atomicMin(jstar + myrow, mine);
  }
}

// ------------------------------------- step 1 + counts, d > 4, triangular
// The tiling of count_tri_body (blocks of sc.rgroup rows x sc.chunk columns,
// R-row blocks from their own diagonal 64-column block on, row counts from
// ballots, column counts from per-lane tallies summed in LDS, pair list
// through wave queues), with the R rows of a wave staged in LDS (d_pad
// floats each, read as broadcasts), NB column blocks at a time and the
// coordinates taken KC at a time (d_pad is a multiple of DC >= 8).
template <int DC, int R, bool EMIT>
__global__ __launch_bounds__(256) void k_count_tri_lds(const float *__restrict__ soa,
                                                       int *__restrict__ counts,
                                                       int2 *__restrict__ pairs,
                                                       DevState *__restrict__ st,
                                                       SweepScalars sc) {
  constexpr int NB = 4, KC = 8;
  static_assert(DC % KC == 0, "coordinate chunk");
  extern __shared__ float lds_rows[];  // [4][R][d_pad]
  __shared__ int2 qbuf[4][kListQueue];
  __shared__ int colcnt[kTriMaxChunk];
  __shared__ unsigned long long xfer[5];
  if (skip_sweep(sc, st)) return;
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % sc.nchunks;
  const int g0 = (blockIdx.x / sc.nchunks) * sc.rgroup;
  const int c0 = chunk * sc.chunk;
  const int c1 = min(c0 + sc.chunk, sc.n_pad);
  if (g0 >= sc.n || c1 <= g0) return;  // block-uniform
  for (int t = threadIdx.x; t < sc.chunk; t += 256) colcnt[t] = 0;
  __syncthreads();
  const int g1 = min(g0 + sc.rgroup, sc.n);
  const int dp = sc.d_pad;
  float *my_rows = lds_rows + (size_t)w * R * dp;
  WaveQueue qu{qbuf[w], 0, kListDrain};
  for (int row0 = g0 + w * R; row0 < g1; row0 += 4 * R) {
    const int diag = row0 & ~63;
    const int cs = max(c0, diag);
    if (cs >= c1) continue;  // wave-uniform
    // this wave's rows (only this wave reads them; LDS is in order per wave)
    for (int e = lane; e < R * dp; e += 64) {
      const int r = e / dp, k = e - r * dp;
      my_rows[e] = soa[(size_t)k * sc.n_pad + row0 + r];  // padded rows are NaN
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    int cnt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) cnt[r] = 0;
    // NB column blocks (NB x 64 columns) at a time: each row coordinate read
    // from LDS (a broadcast) serves NB tests per lane
    for (int cg = cs; cg < c1; cg += NB * 64) {
      float s[NB][R];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) s[b][r] = 0.0f;
      for (int kc = 0; kc < dp; kc += KC) {
        float xc[NB][KC];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int jl = min(cg + b * 64 + lane, sc.n_pad - 1);  // blocks past c1 are not used
#pragma unroll
          for (int k = 0; k < KC; ++k) xc[b][k] = soa[(size_t)(kc + k) * sc.n_pad + jl];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float xr[KC];
#pragma unroll
          for (int k = 0; k < KC; ++k) xr[k] = my_rows[r * dp + kc + k];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            float a = s[b][r];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
              const float t = xr[k] - xc[b][k];
              a = __builtin_fmaf(t, t, a);
            }
            s[b][r] = a;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int cb = cg + b * 64;
        if (cb >= c1) break;  // wave-uniform
        const int j = cb + lane;
        const bool off = cb != diag;
        uint32_t tally = 0;
        uint64_t mg[R], any = 0ull;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          mg[r] = __ballot(s[b][r] <= sc.hi);
          any |= mg[r];
        }
        if (any == 0ull) continue;  // one branch per block of R rows in the common case
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint64_t m = mg[r];
          if (m != 0ull) {  // rare: the column tally and the row's count only then
            const uint64_t lo_m = __ballot(s[b][r] <= sc.lo);
            uint64_t in = m;
            if (lo_m != m) {
              const uint64_t band = m & ~lo_m;
              bool ex = false;
              if ((band >> lane) & 1ull)
                ex = exact_within_mem(my_rows + r * dp, 1, soa + j, sc.n_pad, sc.d, sc.eps2);
              in = lo_m | __ballot(ex);
              if (lane == 0) atomicAdd(&st->band_pairs, (unsigned long long)__popcll(band));
            }
            tally += ((in >> lane) & 1ull) ? 1u : 0u;
            cnt[r] += __popcll(in);
            if (EMIT) {
              if (off) {
                wq_push(qu, (in >> lane) & 1ull, j, row0 + r);
              } else {
                const uint64_t e = in & below_mask(row0 + r, cb);
                if (e != 0ull) wq_push(qu, (e >> lane) & 1ull, row0 + r, j);
              }
              wq_drain_list(qu, pairs, sc.edge_cap, st, false);
            }
          }
        }
        if (off && tally != 0u) atomicAdd(&colcnt[cb - c0 + lane], (int)tally);
      }
    }
    int mine = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane == r) mine = cnt[r];
    const int row = row0 + lane;
    if (lane < R && row < sc.n && mine != 0) atomicAdd(counts + row, mine);
  }
  if (EMIT) wq_flush_pairs(qu, pairs, sc.edge_cap, st, xfer);
  __syncthreads();
  for (int t = threadIdx.x; t < c1 - c0; t += 256) {
    const int v = colcnt[t];
    if (v != 0 && c0 + t < sc.n) atomicAdd(counts + c0 + t, v);
  }
}

// ---------------------------------------------- row-uniform sweeps, any d
// Rows staged in LDS ([4 waves][R][d_pad], read as broadcasts), columns in
// lanes, coordinates processed DC at a time.  Same three modes as above.
enum { MODE_COUNT = 0, MODE_UNION = 1, MODE_BORDER = 2 };

// One block's work (`bid` = its index in the full grid).
// With a spatial order (okey: caller's index of each staged row), the border
// mode takes the smallest okey over all the core neighbours instead of the
// first one in staged order.
template <int DC, int R, int MODE>
__device__ __forceinline__ void rows_lds_block(const float *__restrict__ soa,
                                               int *__restrict__ counts,
                                               const uint32_t *__restrict__ corebits,
                                               int *__restrict__ parent,
                                               const int *__restrict__ list,
                                               int *__restrict__ jstar,
                                               const int *__restrict__ okey,
                                               DevState *__restrict__ st, const SweepScalars &sc,
                                               float *lds_rows, int bid) {
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int n = sc.n;
  int rows[R];
  uint32_t active = 0;
  int cb_begin = 0, cb_end = sc.n_pad;
  if (MODE == MODE_COUNT) {
    const int chunk = bid % sc.nchunks;
    const int rb = (bid / sc.nchunks) * 4 + w;
    cb_begin = chunk * sc.chunk;
    cb_end = min(cb_begin + sc.chunk, sc.n_pad);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rows[r] = rb * R + r;
      if (rows[r] < n) active |= 1u << r;
    }
  } else if (MODE == MODE_UNION) {
    const int total = (n + R - 1) / R;
    const int rb = total - 1 - (int)(bid * 4 + w);
    int last = -1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rows[r] = rb * R + r;
      if (rb >= 0 && rows[r] < n && ((corebits[rows[r] >> 5] >> (rows[r] & 31)) & 1u)) {
        active |= 1u << r;
        last = rows[r];
      }
    }
    cb_end = min(((last + 63) / 64) * 64, sc.n_pad);
  } else {
    const int listed = wave_uniform((int)__hip_atomic_load(&st->noncore, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
    const int e0 = (bid * 4 + w) * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rows[r] = 0;
      if (e0 + r < listed) {
        rows[r] = wave_uniform(list[e0 + r]);
        active |= 1u << r;
      }
    }
  }
  float *my_rows = lds_rows + (size_t)w * R * sc.d_pad;
  for (int e = lane; e < R * sc.d_pad; e += 64) {
    const int r = e / sc.d_pad, k = e - r * sc.d_pad;
    float v = 0.0f;
    if ((active >> r) & 1u) v = soa[(size_t)k * sc.n_pad + rows[r]];
    my_rows[e] = v;
  }
  __syncthreads();

  int acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = (MODE == MODE_BORDER) ? kNoNeighbour : 0;

  for (int cb = cb_begin; cb < cb_end; cb += 64) {
    if (MODE != MODE_COUNT && active == 0u) break;
    uint64_t colmask = ~0ull;
    if (MODE != MODE_COUNT) {
      colmask = (uint64_t)corebits[cb >> 5] | ((uint64_t)corebits[(cb >> 5) + 1] << 32);
      if (colmask == 0ull) continue;
    }
    const int j = cb + lane;
    float s[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = 0.0f;
    for (int kc = 0; kc < sc.d_pad; kc += DC) {
      float xc[DC];
#pragma unroll
      for (int k = 0; k < DC; ++k) xc[k] = soa[(size_t)(kc + k) * sc.n_pad + j];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float *xrow = my_rows + r * sc.d_pad + kc;
        float a = s[r];
#pragma unroll
        for (int k = 0; k < DC; ++k) {
          const float t = xrow[k] - xc[k];
          a = __builtin_fmaf(t, t, a);
        }
        s[r] = a;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!((active >> r) & 1u)) continue;
      uint64_t cm = colmask;
      if (MODE == MODE_UNION) {
        const int lim = rows[r] - cb;
        if (lim <= 0) continue;
        if (lim < 64) cm &= (1ull << lim) - 1ull;
      }
      const uint64_t m = __ballot(s[r] <= sc.hi) & cm;
      if (m == 0ull) continue;
      uint64_t in = __ballot(s[r] <= sc.lo) & cm;
      if (in != m) {
        const uint64_t band = m & ~in;
        bool ex = false;
        if ((band >> lane) & 1ull)
          ex = exact_within_mem(my_rows + r * sc.d_pad, 1, soa + j, sc.n_pad, sc.d, sc.eps2);
        in |= __ballot(ex);
        if (lane == 0) atomicAdd(&st->band_pairs, (unsigned long long)__popcll(band));
      }
      if (MODE == MODE_COUNT) {
        acc[r] += __popcll(in);
      } else if (MODE == MODE_UNION) {
        if ((in >> lane) & 1ull) uf_union(parent, rows[r], j);
      } else if (in != 0ull) {
        if (okey) {
          for (uint64_t m2 = in; m2 != 0ull; m2 &= m2 - 1ull)
            acc[r] = min(acc[r], okey[cb + __builtin_ctzll(m2)]);
        } else {
          acc[r] = cb + __builtin_ctzll(in);
          active &= ~(1u << r);
        }
      }
    }
  }
  if (MODE == MODE_UNION) return;
  int mine = 0, myrow = 0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane == r) {
      mine = acc[r];
      myrow = rows[r];
    }
  if (MODE == MODE_COUNT) {
    if (lane < R && myrow < n) {
      if (sc.nchunks == 1)
        counts[myrow] = mine;
      else
        atomicAdd(counts + myrow, mine);
    }
  } else if (lane < R && mine != kNoNeighbour) {
    atomicMin(jstar + myrow, mine);
  }
}

// The sweep kernel.  A fallback launch (sc.flags set) usually has nothing to
// do, so it runs on a small grid that strides over the `nblocks` blocks of
// the full launch instead of launching them all.
template <int DC, int R, int MODE>
__global__ __launch_bounds__(256) void k_rows_lds(const float *__restrict__ soa,
                                                  int *__restrict__ counts,
                                                  const uint32_t *__restrict__ corebits,
                                                  int *__restrict__ parent,
                                                  const int *__restrict__ list,
                                                  int *__restrict__ jstar,
                                                  const int *__restrict__ okey,
                                                  DevState *__restrict__ st, SweepScalars sc,
                                                  int nblocks) {
  extern __shared__ float lds_rows[];
  if (skip_sweep(sc, st)) return;
  for (int bid = blockIdx.x; bid < nblocks; bid += gridDim.x) {
    rows_lds_block<DC, R, MODE>(soa, counts, corebits, parent, list, jstar, okey, st, sc,
                                lds_rows, bid);
    __syncthreads();
  }
}

// ------------------------------------------------------------ host launchers
constexpr int kRowsSmall = 16;  // rows per wave, d <= 4 (vector registers)
constexpr int kRowsLds = 8;    // rows per wave, d > 4 (LDS)

int rows_per_wave(int d) { return d <= 4 ? kRowsSmall : kRowsLds; }

int coord_chunk(int d) {
  if (d <= 4) return d;
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  return 64;
}

template <int MODE>
static hipError_t launch_lds(const Buffers &b, const SweepScalars &sc, int blocks, hipStream_t s) {
  const size_t lds = (size_t)4 * kRowsLds * sc.d_pad * sizeof(float);
  const int grid = (sc.flags && blocks > 2048) ? 2048 : blocks;
  if (blocks <= 0) return hipSuccess;
  switch (coord_chunk(sc.d)) {
#define DBK_LDS_CASE(DC)                                                                      \
  case DC:                                                                                    \
    hipLaunchKernelGGL((k_rows_lds<DC, kRowsLds, MODE>), dim3(grid), dim3(256), lds, s,      \
                       b.soa, b.counts, b.corebits, b.parent, b.list, b.jstar, b.okey, b.st,  \
                       sc, blocks);                                                           \
    break;
    DBK_LDS_CASE(8)
    DBK_LDS_CASE(16)
    DBK_LDS_CASE(32)
    DBK_LDS_CASE(64)
#undef DBK_LDS_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_count(const Buffers &b, const SweepScalars &sc, bool emit_pairs, hipStream_t s) {
  const dim3 block(256);
  // the triangular sweeps; sc.chunk / sc.rgroup give their tiles
  if (sc.chunk % 64 != 0 || sc.chunk > kTriMaxChunk || sc.rgroup % 64 != 0 || sc.rgroup <= 0)
    return hipErrorInvalidValue;
  const dim3 tgrid(((sc.n + sc.rgroup - 1) / sc.rgroup) * sc.nchunks);
  const dim3 pgrid(pruned_grid(tgrid.x));
  if (sc.box && sc.d <= 4) {
    hipError_t e = run_coarse_boxes(sc, s);
    if (e != hipSuccess) return e;
  }
  if (sc.d > 4) {
    const size_t lds = (size_t)4 * kRowsLds * sc.d_pad * sizeof(float);
    switch (coord_chunk(sc.d)) {
#define DBK_TRI_LDS(DC)                                                                       \
  case DC:                                                                                    \
    if (emit_pairs)                                                                           \
      hipLaunchKernelGGL((k_count_tri_lds<DC, kRowsLds, true>), tgrid, block, lds, s, b.soa,  \
                         b.counts, b.pairs, b.st, sc);                                        \
    else                                                                                      \
      hipLaunchKernelGGL((k_count_tri_lds<DC, kRowsLds, false>), tgrid, block, lds, s, b.soa, \
                         b.counts, b.pairs, b.st, sc);                                        \
    break;
      DBK_TRI_LDS(8)
      DBK_TRI_LDS(16)
      DBK_TRI_LDS(32)
      DBK_TRI_LDS(64)
#undef DBK_TRI_LDS
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
#define DBK_COUNT(D)                                                                          \
  if (sc.box) {                                                                               \
    if (emit_pairs)                                                                           \
      hipLaunchKernelGGL((k_count_tri_pruned<D, kRowsSmall, true>), pgrid, block, 0, s,       \
                         b.soa, b.counts, b.pairs, b.st, sc);                                 \
    else                                                                                      \
      hipLaunchKernelGGL((k_count_tri_pruned<D, kRowsSmall, false>), pgrid, block, 0, s,      \
                         b.soa, b.counts, b.pairs, b.st, sc);                                 \
  } else if (emit_pairs) {                                                                    \
    hipLaunchKernelGGL((k_count_tri<D, kRowsSmall, true, false>), tgrid, block, 0, s, b.soa,  \
                       b.counts, b.pairs, b.st, sc);                                          \
  } else {                                                                                    \
    hipLaunchKernelGGL((k_count_tri<D, kRowsSmall, false, false>), tgrid, block, 0, s, b.soa, \
                       b.counts, b.pairs, b.st, sc);                                          \
  }                                                                                           \
  break;
  switch (sc.d) {
    case 1: DBK_COUNT(1)
    case 2: DBK_COUNT(2)
    case 3: DBK_COUNT(3)
    case 4: DBK_COUNT(4)
    default: return hipErrorInvalidValue;
  }
#undef DBK_COUNT
  return hipGetLastError();
}

hipError_t run_union(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int R = rows_per_wave(sc.d);
  const dim3 grid(((sc.n + R - 1) / R + 3) / 4), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL((k_union_small<1, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.parent, b.st, sc); break;
    case 2: hipLaunchKernelGGL((k_union_small<2, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.parent, b.st, sc); break;
    case 3: hipLaunchKernelGGL((k_union_small<3, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.parent, b.st, sc); break;
    case 4: hipLaunchKernelGGL((k_union_small<4, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.parent, b.st, sc); break;
    default: return launch_lds<MODE_UNION>(b, sc, (int)grid.x, s);
  }
  return hipGetLastError();
}

hipError_t run_border(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int R = rows_per_wave(sc.d);
  if (sc.d > 4) {
    const int blocks = ((sc.n + R - 1) / R + 3) / 4;
    return launch_lds<MODE_BORDER>(b, sc, blocks, s);
  }
  const dim3 grid(4096), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL((k_border_small<1, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.okey, b.st, sc); break;
    case 2: hipLaunchKernelGGL((k_border_small<2, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.okey, b.st, sc); break;
    case 3: hipLaunchKernelGGL((k_border_small<3, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.okey, b.st, sc); break;
    case 4: hipLaunchKernelGGL((k_border_small<4, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.okey, b.st, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dbk
