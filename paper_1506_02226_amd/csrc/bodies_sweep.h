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

// The hoisted test when its rows were prepared and the input is in its
// range (hoist_prep_body), else the direct form.
__device__ __forceinline__ bool use_hoist(const SweepScalars &sc, const DevState *st) {
  if (!sc.hoist) return false;
  return !(__hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
           kStatusNoHoist);
}

// ------------------------------------------------------ pruned launches
// Persistent form of the triangular sweeps with tile pruning: work-group b
// of the grid takes the (row group, column chunk) blocks b, b + G, b + 2G,
// ... (G = grid size), 64 at a time -- each lane tests one block's row-group
// box against its chunk's box (coarse boxes at sc.box + 2 d nb and + 4 d nb)
// -- and runs body(bid) for the blocks within reach only, one after another.
// Every wave computes the same mask, so the loop is block-uniform and the
// body may synchronise the block.
template <int D, typename F>
__device__ __forceinline__ void for_near_blocks(const SweepScalars &sc, int rows_end, F &&body) {
  const int nb = sc.n_pad / 64;
  const float *gbox = sc.box + 2 * D * nb;  // [2k][row group]
  const float *kbox = sc.box + 4 * D * nb;  // [2k][chunk]
  const long long groups = (rows_end + sc.rgroup - 1) / sc.rgroup;
  const long long total = groups * sc.nchunks;
  const long long G = gridDim.x;
  for (long long it = 0; (long long)blockIdx.x + it * 64 * G < total; ++it) {
    const long long id = (long long)blockIdx.x + (it * 64 + lane_id()) * G;
    bool near = false;
    if (id < total) {
      const int rg = (int)(id / sc.nchunks), ch = (int)(id - (long long)rg * sc.nchunks);
      const int g0 = rg * sc.rgroup;
      const int c1 = min(ch * sc.chunk + sc.chunk, sc.n_pad);
      if (c1 > g0) {  // the triangle: some column at or after the block's rows
        float alo[D], ahi[D], blo[D], bhi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          alo[k] = gbox[(size_t)(2 * k) * nb + rg];
          ahi[k] = gbox[(size_t)(2 * k + 1) * nb + rg];
          blo[k] = kbox[(size_t)(2 * k) * nb + ch];
          bhi[k] = kbox[(size_t)(2 * k + 1) * nb + ch];
        }
        near = box_gap2<D>(alo, ahi, blo, bhi) <= sc.hi;
      }
    }
    uint64_t m = __ballot(near);
    while (m != 0ull) {
      const int b = __builtin_ctzll(m);
      m &= m - 1ull;
      body((int)((long long)blockIdx.x + (it * 64 + b) * G));
      __syncthreads();  // the body's LDS is reused by the next block
    }
  }
}

// ------------------------------- step 1 + counts, d <= 4, one test per pair
// A block owns sc.rgroup rows and
// the sc.chunk columns of one chunk, and an R-row block of a wave only visits
// the 64-column blocks from the one holding its own rows onwards, so each
// unordered pair is tested once.  Counts come from both sides of a test: the
// row side as ballot popcounts (scalar registers), the column side as LDS
// additions (made only when a row's ballot is not empty) into `colcnt`
// (sc.chunk entries), added to counts[] at the end.  In the
// diagonal 64x64 block every row visits all 64 columns itself, so there the
// column tally is not taken, and only pairs below the diagonal are listed.
//
// PRUNE (rows in spatial order; not the paper's all-pairs sweep, so reported
// apart): a block whose rows and columns have boxes farther apart than eps
// (box_gap2 > hi over the 64-point block boxes sc.box) returns at once, and a
// wave visits only the 64-column blocks whose box is within reach of its R
// rows' box (all 64 blocks of the chunk tested at once, one per lane).
// Skipped pairs are provably not neighbours; the tests actually made go to
// st->tests.
//
// HOIST (sc.hoist, rows prepared by hoist_prep_body): the hoisted form of
// Section IV-B.2 about the origin c of the wave's 16 rows.  Per 64-column
// tile the wave forms b = fl(y - c) and P = |b|^2 once; per pair it forms
// s = -2a.b (a product and d - 1 fused multiply-adds, no term from the
// column, so the product issues at the two-operand rate), and the tile is
// skipped when fl(min s + P) exceeds the block's gate (hoist_gate: sound for
// every pair the thresholds could let in).  Otherwise each row's
// q = fl(P - 2a.b) (d fused multiply-adds from P) is compared with the row's
// thresholds: q <= lo in, q > hi out, else float64 -- the same decisions as
// the direct form at about half its instructions.  An 8-row group is
// skipped when its smallest q exceeds the group's largest hi.
template <int D, int R, bool EMIT, bool PRUNE = false, int QN = kListQueue, bool HOIST = false>
__device__ __forceinline__ void count_tri_body(const float *__restrict__ soa,
                                               int *__restrict__ counts,
                                               int2 *__restrict__ pairs,
                                               DevState *__restrict__ st,
                                               const SweepScalars &sc, int bid,
                                               int2 (*qbuf)[QN], int *colcnt,
                                               unsigned long long *xfer) {
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = bid % sc.nchunks;
  const int g0 = (bid / sc.nchunks) * sc.rgroup;
  const int c0 = chunk * sc.chunk;
  const int c1 = min(c0 + sc.chunk, sc.n_pad);
  if (g0 >= sc.n || c1 <= g0) return;  // block-uniform
  const int g1 = min(g0 + sc.rgroup, sc.n);
  const int nb = sc.n_pad / 64;
  // PRUNE: lane l holds the box of column block c0 / 64 + l (a chunk has at
  // most 64 of them), read back with a lane read when the wave reaches it
  float lbl[D], lbh[D];
  if (PRUNE) {
    // every wave derives the same boxes, so the exit is block-uniform
    float rlo[D], rhi[D], clo[D], chi[D];
    span_box<D>(sc.box, nb, g0 / 64, (g1 + 63) / 64, rlo, rhi);
    lane_box<D>(sc.box, nb, c0 / 64, c1 / 64, lbl, lbh);
    wave_box<D>(lbl, lbh, clo, chi);
    if (box_gap2<D>(rlo, rhi, clo, chi) > sc.hi) return;
  }
  static_assert(R == 16, "16 rows per wave: two 8-row groups, one 16-row block of the hoisted rows");
  HoistView<const float> hv{};
  if (HOIST) hv = hoist_view(sc.hoist, sc.n_pad, D);
  for (int t = threadIdx.x; t < sc.chunk; t += 256) colcnt[t] = 0;
  __syncthreads();
  WaveQueue qu{qbuf[w], 0, QN - 64};  // appended once QN - 64 pairs are queued
  unsigned long long tested = 0;  // PRUNE: pair tests made by this wave
  constexpr int GR = R > 8 ? 8 : R;  // rows per group of the minimum test
  for (int row0 = g0 + w * R; row0 < g1; row0 += 4 * R) {
    const int diag = row0 & ~63;
    const int cs = max(c0, diag);
    if (cs >= c1) continue;  // wave-uniform
    // the rows: coordinates (direct form) or -2 fl(x - c) (HOIST)
    float xr[R][D];
    const float *rows = HOIST ? hv.a : soa;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < D; ++k) xr[r][k] = to_vgpr(rows[(size_t)k * sc.n_pad + row0 + r]);
    float cen[D];         // HOIST: the rows' origin
    float gate[R / GR];   // largest "out" threshold of each group
    float gate16 = sc.hi; // the 16 rows' gate (HOIST: hoist_gate, on min s + P)
#pragma unroll
    for (int g = 0; g < R / GR; ++g) gate[g] = sc.hi;
    if (HOIST) {
#pragma unroll
      for (int k = 0; k < D; ++k) cen[k] = to_vgpr(hv.cen[(size_t)k * (sc.n_pad / 16) + row0 / 16]);
#pragma unroll
      for (int g = 0; g < R / GR; ++g) gate[g] = to_vgpr(hv.hg[row0 / GR + g]);
      gate16 = to_vgpr(hv.g16[row0 / 16]);
    } else {
      gate16 = __builtin_fmaxf(gate[0], gate[1]);
    }
    int cnt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) cnt[r] = 0;
    float rlo[D], rhi[D];  // PRUNE: box of the R rows (padded rows are NaN, skipped)
    if (PRUNE && HOIST) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        rlo[k] = hv.box[(size_t)(2 * k) * (sc.n_pad / 16) + row0 / 16];
        rhi[k] = hv.box[(size_t)(2 * k + 1) * (sc.n_pad / 16) + row0 / 16];
      }
    } else if (PRUNE) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        rlo[k] = xr[0][k];
        rhi[k] = xr[0][k];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          rlo[k] = __builtin_fminf(rlo[k], xr[r][k]);
          rhi[k] = __builtin_fmaxf(rhi[k], xr[r][k]);
        }
      }
    }
    // the tests of the R rows against the 64 columns cb .. cb + 63 (coordinates xc)
    auto tile = [&](int cb, const float (&xc)[D]) {
      const bool off = cb != diag;
      // HOIST: the column about the rows' origin, and its squared norm
      float bq[D], pn = 0.0f;
      if (HOIST) {
#pragma unroll
        for (int k = 0; k < D; ++k) bq[k] = xc[k] - cen[k];
        pn = bq[0] * bq[0];
#pragma unroll
        for (int k = 1; k < D; ++k) pn = __builtin_fmaf(bq[k], bq[k], pn);
      }
      // every row's value, then one compare of their minimum against the
      // largest threshold and one branch per tile in the common case (with
      // 16 rows); the groups' own minima and the rows' ballots only in the
      // rare case
      float sv[R];
      if (HOIST) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float s = xr[r][0] * bq[0];
#pragma unroll
          for (int kk = 1; kk < D; ++kk) s = __builtin_fmaf(xr[r][kk], bq[kk], s);
          sv[r] = s;
        }
        if (__ballot(min_of<R>(sv) + pn <= gate16) == 0ull) return;
        // the rows' values as the thresholds were derived for
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float q = pn;
#pragma unroll
          for (int kk = 0; kk < D; ++kk) q = __builtin_fmaf(xr[r][kk], bq[kk], q);
          sv[r] = q;
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) sv[r] = sq_dist32<D>(xr[r], xc);
        if (__ballot(min_of<R>(sv) <= gate16) == 0ull) return;
      }
#pragma unroll
      for (int g = 0; g < R / GR; ++g) {
        float sg[GR];
#pragma unroll
        for (int k = 0; k < GR; ++k) sg[k] = sv[g * GR + k];
        if (__ballot(min_of<GR>(sg) <= gate[g]) == 0ull) continue;
#pragma unroll
        for (int k = 0; k < GR; ++k) {
          const int r = g * GR + k;
          const float hi_r = HOIST ? hv.hi[row0 + r] : sc.hi;
          const float lo_r = HOIST ? hv.lo[row0 + r] : sc.lo;
          const uint64_t m = __ballot(sg[k] <= hi_r);
          if (m == 0ull) continue;
          const uint64_t lo_m = __ballot(sg[k] <= lo_r);
          uint64_t in = m;
          if (lo_m != m)
            in = recheck_band_soa(m & ~lo_m, lo_m, soa, sc.n_pad, D, row0 + r, cb + lane,
                                  sc.eps2, st);
          // the column side, into the block's tally (only on this rare path)
          if (off && ((in >> lane) & 1ull)) atomicAdd(&colcnt[cb - c0 + lane], 1);
          cnt[r] += __popcll(in);
          if (EMIT) {
            if (off) {
              wq_push(qu, (in >> lane) & 1ull, cb + lane, row0 + r);
            } else {
              const uint64_t e = in & below_mask(row0 + r, cb);
              if (e != 0ull) wq_push(qu, (e >> lane) & 1ull, row0 + r, cb + lane);
            }
            wq_drain_list(qu, pairs, sc.edge_cap, st, false);
          }
        }
      }
    };
    float xn[D];
    if (PRUNE) {
      // the column blocks within reach of the rows' box: one test per lane
      // (lane l against column block c0 / 64 + l), then only those blocks
      const int cbl = c0 + 64 * lane;
      uint64_t cand = __ballot(cbl >= cs && cbl < c1 && box_gap2<D>(rlo, rhi, lbl, lbh) <= sc.hi);
      tested += (unsigned long long)__popcll(cand) * R * 64;
      if (cand != 0ull) {
#pragma unroll
        for (int k = 0; k < D; ++k)
          xn[k] = soa[(size_t)k * sc.n_pad + c0 + 64 * __builtin_ctzll(cand) + lane];
      }
      while (cand != 0ull) {
        const int cb = c0 + 64 * __builtin_ctzll(cand);
        cand &= cand - 1ull;
        float xc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xc[k] = xn[k];
        if (cand != 0ull) {
#pragma unroll
          for (int k = 0; k < D; ++k)
            xn[k] = soa[(size_t)k * sc.n_pad + c0 + 64 * __builtin_ctzll(cand) + lane];
        }
        tile(cb, xc);
      }
    } else {
      // two tiles per iteration in alternating registers: the next tile's
      // columns load into the other set while one is tested (no copies).
      // The loads are unconditional (past the chunk's last tile they read
      // that tile again), so the compiler knows how many are in flight and
      // waits only for the ones a tile uses.
      const int clast = c1 - 64;  // c1 - cs is a multiple of 64
      // a wave-uniform base per tile and the lane as the only per-lane offset
      // scalar bases (coordinate k from column cs) and one 32-bit index
      const float *base[D];
#pragma unroll
      for (int k = 0; k < D; ++k) base[k] = soa + ((size_t)k * sc.n_pad + (size_t)cs);
      auto load = [&](float (&x)[D], int cb) {
        // a 32-bit byte offset (a chunk spans at most 4,096 columns)
        const unsigned off = ((unsigned)(cb - cs) + (unsigned)lane) * 4u;
#pragma unroll
        for (int k = 0; k < D; ++k)
          x[k] = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base[k]) + off);
      };
      float xa[D], xb[D];
      load(xa, cs);
      for (int cb = cs; cb < c1; cb += 128) {
        load(xb, min(cb + 64, clast));
        tile(cb, xa);
        if (cb + 64 >= c1) break;
        load(xa, min(cb + 128, clast));
        tile(cb + 64, xb);
      }
    }
    int mine = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane == r) mine = cnt[r];
    const int row = row0 + lane;
    if (lane < R && row < sc.n && mine != 0) atomicAdd(counts + row, mine);
  }
  if (PRUNE && lane == 0 && tested) atomicAdd(&st->tests, tested);
  if (EMIT) wq_flush_pairs(qu, pairs, sc.edge_cap, st, xfer);
  __syncthreads();
  for (int t = threadIdx.x; t < c1 - c0; t += 256) {
    const int v = colcnt[t];
    if (v != 0 && c0 + t < sc.n) atomicAdd(counts + c0 + t, v);
  }
}

}  // namespace dbk
