// Bitmask form of steps 1 and 3 (d <= 4): the neighbour relation kept as one
// bit per ordered pair -- the paper's `cluster` matrix of Section IV-B, at one
// bit instead of one byte per entry, in 32-bit words -- and the merge of
// Section IV-C read from it.
#include "dbscan_device.h"
#include "dbscan_internal.h"
#include "bodies_sweep.h"

namespace dbk {

// ----------------------------------------------------- bitmask pass (d <= 4)
// One wave takes 32 rows at a time (the "goal points" of Section IV-A.3,
// wave-uniform values held in vector registers so that the subtractions issue
// at the full rate) and the 64 lanes hold 64 columns.  Per group of 8 rows
// one compare of the distances' minimum tells whether any row has a
// neighbour among the columns; only then -- rare at these densities -- does
// each row's ballot give its popcount to the row's count (scalar unit) and
// the lane set bit r of its 32-bit word.  (64 rows per wave at d = 2 take 188
// vector registers and ran a third slower.)  After the 32 rows, lane j holds
// the pairs (rows row0..row0+31, column j); by symmetry that is row j's word
// for the columns row0..row0+31, stored at adj[row0/32][j] -- a coalesced
// 256-byte store per wave.  Bit b of adj[q][i] is the pair (i, 32q+b).  Padded rows and columns
// (index >= n) are NaN, so their bits are zero.  Each 32 x 64 tile also gets
// a flag byte, tflag[j/64][row0/32], telling whether any of its bits is set
// (the merge reads only flagged tiles); the flags are gathered in LDS and
// written once per block.  The words themselves are stored unconditionally:
// a store that only some iterations make leaves the compiler unable to count
// the memory operations in flight, and the next column block's prefetched
// coordinates would then wait for the store to complete.
//
// The relation is symmetric, so each unordered pair is tested once: a 16-row
// block only visits the 64-column blocks from the one holding its own rows
// onwards.  That stores adj[q][i] for every i >= 32q (all the lower triangle
// the merge reads), and the counts come from both sides of each test: the
// row side as ballot popcounts in scalar registers, the column side as the
// popcount of the lane's word, summed per block in LDS and added to counts[]
// once per block.  In the diagonal 64x64 block every row visits all 64
// columns itself, so column sums are taken only off that block.
//
// A block owns sc.rgroup rows (4 waves, 32-row blocks dealt round-robin) and
// the sc.chunk columns of one chunk; the grid is row groups x chunks, and a
// block whose columns all lie before its rows has nothing to do.
constexpr int kBitmaskMaxChunk = 4096;
// The all-pairs launch stages its chunk's columns in LDS (LDSCOL): at most
// this many per block, so that the waves read them there instead of from L2.
constexpr int kBitmaskLdsChunk = 2048;
constexpr int kBitmaskMaxRows = 512;  // rows per block (sc.rgroup) at most

// PRUNE (rows in spatial order; not the paper's all-pairs sweep, so reported
// apart): blocks and 32 x 64 tiles whose row and column boxes are farther
// apart than eps (box_gap2 > hi) are skipped and left flagged empty (a wave
// tests the 64 column boxes of its chunk at once, one per lane, and visits
// only the blocks within reach); the tests actually made go to st->tests.
//
// HOIST (sc.hoist): the hoisted test of count_tri_body, each 16-row half of
// the wave's rows about its own origin (two column preparations per tile).
// The group thresholds stay in scalar registers (read with readfirstlane, so
// their loads are waited for before the tile loop, not at the loop's first
// compare on every iteration, where the wait would also cover the previous
// tile's word store).
//
// LDSCOL (sc.chunk <= kBitmaskLdsChunk): the block first copies its chunk's
// column coordinates to `lcol` ([k][kBitmaskLdsChunk], LDS) and the waves
// read the columns there.  With the hoisted test the sweep issues a third
// fewer instructions and the latency of column loads from L2 (fetched one
// tile ahead) showed.
template <int D, bool PRUNE, bool HOIST = false, bool LDSCOL = false>
__device__ __forceinline__ void bitmask_body(const float *__restrict__ soa,
                                             uint32_t *__restrict__ adj,
                                             uint8_t *__restrict__ tflag,
                                             int *__restrict__ counts, DevState *__restrict__ st,
                                             const SweepScalars &sc, int bid, int *colcnt,
                                             uint8_t (*tiles)[kBitmaskMaxChunk / 64],
                                             float *lcol = nullptr) {
  constexpr int R = 32, G = 8;
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = bid % sc.nchunks;
  const int g0 = (bid / sc.nchunks) * sc.rgroup;
  const int c0 = chunk * sc.chunk;
  const int c1 = min(c0 + sc.chunk, sc.n_pad);
  if (g0 >= sc.n_pad || c1 <= g0) return;  // block-uniform
  const int g1 = min(g0 + sc.rgroup, sc.n_pad);
  const int nq = sc.n_pad / 32, nb = sc.n_pad / 64;
  // PRUNE: lane l holds the box of column block c0 / 64 + l (a chunk has at
  // most 64 of them), read back with a lane read when the wave reaches it
  float lbl[D], lbh[D];
  if (PRUNE) {
    // every wave derives the same boxes, so the exit is block-uniform (the
    // flags were cleared beforehand, so a skipped block leaves its tiles empty)
    float rlo[D], rhi[D], clo[D], chi[D];
    span_box<D>(sc.box, nb, g0 / 64, g1 / 64, rlo, rhi);
    lane_box<D>(sc.box, nb, c0 / 64, c1 / 64, lbl, lbh);
    wave_box<D>(lbl, lbh, clo, chi);
    if (box_gap2<D>(rlo, rhi, clo, chi) > sc.hi) return;
  }
  HoistView<const float> hv{};
  if (HOIST) hv = hoist_view(sc.hoist, sc.n_pad, D);
  for (int t = threadIdx.x; t < sc.chunk; t += 256) colcnt[t] = 0;
  if (LDSCOL)
    for (int t = threadIdx.x; t < c1 - c0; t += 256)
#pragma unroll
      for (int k = 0; k < D; ++k) lcol[k * kBitmaskLdsChunk + t] = soa[(size_t)k * sc.n_pad + c0 + t];
  // column coordinate k of column j (j in the chunk)
  auto col = [&](int k, int j) -> float {
    return LDSCOL ? lcol[k * kBitmaskLdsChunk + (j - c0)] : soa[(size_t)k * sc.n_pad + j];
  };
  if (PRUNE)  // tiles a wave does not visit stay empty
    for (int t = threadIdx.x; t < (kBitmaskMaxRows / 32) * (kBitmaskMaxChunk / 64); t += 256)
      tiles[t / (kBitmaskMaxChunk / 64)][t % (kBitmaskMaxChunk / 64)] = 0;
  __syncthreads();
  unsigned long long tested = 0;  // PRUNE: pair tests made by this wave
  for (int row0 = g0 + w * R; row0 < g1; row0 += 4 * R) {
    const int diag = row0 & ~63;
    const int cs = max(c0, diag);
    if (cs >= c1) continue;  // wave-uniform
    // the rows: coordinates (direct form) or -2 fl(x - c) (HOIST).  One
    // coalesced load per coordinate (lane l holds row row0 + l % 32), then
    // each row's value broadcast from its lane: loaded one by one, the
    // values went through the same few registers, one round trip each
    float xr[R][D];
    const float *rows = HOIST ? hv.a : soa;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int v = __builtin_bit_cast(int, rows[(size_t)k * sc.n_pad + row0 + (lane & (R - 1))]);
#pragma unroll
      for (int r = 0; r < R; ++r)
        xr[r][k] = to_vgpr(__builtin_bit_cast(float, __builtin_amdgcn_readlane(v, r)));
    }
    float cen[2][D];     // HOIST: the origins of the two 16-row halves
    float gate[R / G];   // largest "out" threshold of each group
#pragma unroll
    for (int g = 0; g < R / G; ++g) gate[g] = sc.hi;
    if (HOIST) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < D; ++k) cen[h][k] = hv.cen[(size_t)k * (sc.n_pad / 16) + row0 / 16 + h];
#pragma unroll
      for (int g = 0; g < R / G; ++g) gate[g] = wave_uniform_f(hv.hg[row0 / G + g]);
    }
    float gate16[R / 16];  // the larger threshold of each half's two groups
#pragma unroll
    for (int h = 0; h < R / 16; ++h)
      gate16[h] = wave_uniform_f(__builtin_fmaxf(gate[2 * h], gate[2 * h + 1]));
    // two rows' counts per scalar register (a chunk has at most 4096 columns)
    uint32_t cnt2[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) cnt2[r] = 0;
    uint32_t *out = adj + adj_block_base(row0 / R, sc.n_pad);  // indexed by column, from diag
    uint8_t *flag = tiles[(row0 - g0) / R];  // [column block - c0 / 64]
    uint64_t filled = 0;  // bit t: the tile of column block c0 / 64 + t holds a bit
    float rlo[D], rhi[D];  // PRUNE: box of the R rows (padded rows are NaN, skipped)
    if (PRUNE && HOIST) {
      const size_t nb16 = sc.n_pad / 16;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        rlo[k] = __builtin_fminf(hv.box[(2 * k) * nb16 + row0 / 16],
                                 hv.box[(2 * k) * nb16 + row0 / 16 + 1]);
        rhi[k] = __builtin_fmaxf(hv.box[(2 * k + 1) * nb16 + row0 / 16],
                                 hv.box[(2 * k + 1) * nb16 + row0 / 16 + 1]);
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
      uint32_t word = 0;
      // rows in 16-row halves (HOIST: each about its own origin, so the
      // column and its squared norm are formed per half): the common case
      // (no neighbour among the 64 columns for any of the 16 rows) costs one
      // compare of their minimum with the larger of the halves' two group
      // thresholds and one branch; the groups' own minima, the rows'
      // ballots, the lane's bits and the row counts only in the rare case
#pragma unroll
      for (int h = 0; h < R / 16; ++h) {
        float bq[D], pn = 0.0f;
        if (HOIST) {
#pragma unroll
          for (int k = 0; k < D; ++k) bq[k] = xc[k] - cen[h][k];
          pn = bq[0] * bq[0];
#pragma unroll
          for (int k = 1; k < D; ++k) pn = __builtin_fmaf(bq[k], bq[k], pn);
        }
        float sv[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (HOIST) {
            float q = pn;
#pragma unroll
            for (int kk = 0; kk < D; ++kk) q = __builtin_fmaf(xr[h * 16 + k][kk], bq[kk], q);
            sv[k] = q;
          } else {
            sv[k] = sq_dist32<D>(xr[h * 16 + k], xc);
          }
        }
        if (__ballot(min_of<16>(sv) <= gate16[h]) == 0ull) continue;
#pragma unroll
        for (int gg = 0; gg < 16 / G; ++gg) {
          const int g = h * (16 / G) + gg;
          float sg[G];
#pragma unroll
          for (int k = 0; k < G; ++k) sg[k] = sv[gg * G + k];
          if (__ballot(min_of<G>(sg) <= gate[g]) == 0ull) continue;
#pragma unroll
          for (int k = 0; k < G; ++k) {
            const int r = g * G + k;
            const float hi_r = HOIST ? hv.hi[row0 + r] : sc.hi;
            const float lo_r = HOIST ? hv.lo[row0 + r] : sc.lo;
            const uint64_t mk = __ballot(sg[k] <= hi_r);
            if (mk == 0ull) continue;
            const uint64_t lo_m = __ballot(sg[k] <= lo_r);
            uint64_t in = mk;
            if (lo_m != in)
              in = recheck_band_soa(in & ~lo_m, lo_m, soa, sc.n_pad, D, row0 + r, cb + lane,
                                    sc.eps2, st);
            word |= ((in >> lane) & 1ull) ? (1u << r) : 0u;
            cnt2[r >> 1] += (uint32_t)__popcll(in) << ((r & 1) * 16);
          }
        }
      }
      // a 32-bit byte offset from the row block's base (a bit matrix that
      // fits in memory has n_pad well below 2^30)
      *reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(out) + (unsigned)(cb + lane) * 4u) =
          word;
      // the tile's flag and column tallies only when it holds a bit (a
      // wave-uniform branch: no LDS operation in the common case, so the
      // next tile's wait for its prefetched columns waits for nothing else)
      if (__ballot(word != 0u) != 0ull) {
        filled |= 1ull << ((cb - c0) >> 6);
        if (cb != diag && word != 0u) atomicAdd(&colcnt[cb - c0 + lane], __popc(word));
      }
    };
    float xn[D];
    if (PRUNE) {
      // the column blocks within reach of the rows' box: one test per lane
      // (lane l against column block c0 / 64 + l), then only those blocks;
      // the others keep the empty flag set when the block started
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
      // two tiles per iteration in alternating registers (no copies); the
      // loads are unconditional, past the chunk's last tile they read it again
      const int clast = c1 - 64;  // c1 - cs is a multiple of 64
      float xa[D], xb[D];
#pragma unroll
      for (int k = 0; k < D; ++k) xa[k] = col(k, cs + lane);
      for (int cb = cs; cb < c1; cb += 128) {
        const int nb = min(cb + 64, clast);
#pragma unroll
        for (int k = 0; k < D; ++k) xb[k] = col(k, nb + lane);
        tile(cb, xa);
        if (cb + 64 >= c1) break;
        const int na = min(cb + 128, clast);
#pragma unroll
        for (int k = 0; k < D; ++k) xa[k] = col(k, na + lane);
        tile(cb + 64, xb);
      }
    }
    // the flags of the tiles from cs on, one per lane (a chunk has at most
    // 64 column blocks); pruned-away tiles hold no bit
    {
      const int cbl = c0 + 64 * lane;
      if (cbl >= cs && cbl < c1) flag[lane] = (uint8_t)((filled >> lane) & 1ull);
    }
    int mine = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane == r) mine = (int)((cnt2[r >> 1] >> ((r & 1) * 16)) & 0xffffu);
    const int row = row0 + lane;
    if (lane < R && row < sc.n && mine != 0) atomicAdd(counts + row, mine);
  }
  if (PRUNE && lane == 0 && tested) atomicAdd(&st->tests, tested);
  __syncthreads();
  for (int t = threadIdx.x; t < c1 - c0; t += 256) {
    const int v = colcnt[t];
    if (v != 0 && c0 + t < sc.n) atomicAdd(counts + c0 + t, v);
  }
  // flags of the tiles this block computed: 32-row block q, column block
  // cb >= the diagonal block of q's rows
  const int nr = (g1 - g0) / 32, nc = (c1 - c0) / 64;
  for (int t = threadIdx.x; t < nr * nc; t += 256) {
    const int rr = t % nr, cc = t / nr;
    const int q = g0 / 32 + rr, cb = c0 + 64 * cc;
    if (cb >= ((32 * q) & ~63)) tflag[(size_t)(cb >> 6) * nq + q] = tiles[rr][cc];
  }
}

// Launch bounds: the hoisted body needs a few more registers than the direct
// one; bounded like this the kernel keeps four waves per SIMD at d <= 2 and
// three at d = 3 (the compiler would otherwise lose one wave per SIMD).
template <int D>
__global__ __launch_bounds__(256, D <= 2 ? 4 : (D == 3 ? 3 : 2)) void k_bitmask(const float *__restrict__ soa,
                                                 uint32_t *__restrict__ adj,
                                                 uint8_t *__restrict__ tflag,
                                                 int *__restrict__ counts,
                                                 DevState *__restrict__ st, SweepScalars sc) {
  __shared__ int colcnt[kBitmaskLdsChunk];
  __shared__ uint8_t tiles[kBitmaskMaxRows / 32][kBitmaskMaxChunk / 64];  // non-empty flags
  __shared__ float lcol[D * kBitmaskLdsChunk];
  if (use_hoist(sc, st))
    bitmask_body<D, false, true, true>(soa, adj, tflag, counts, st, sc, blockIdx.x, colcnt, tiles,
                                       lcol);
  else
    bitmask_body<D, false, false, true>(soa, adj, tflag, counts, st, sc, blockIdx.x, colcnt,
                                        tiles, lcol);
}

// Pruned form: a persistent grid over the blocks that survive the coarse
// box test (for_near_blocks), the flags cleared beforehand.
template <int D>
__global__ __launch_bounds__(256) void k_bitmask_pruned(const float *__restrict__ soa,
                                                        uint32_t *__restrict__ adj,
                                                        uint8_t *__restrict__ tflag,
                                                        int *__restrict__ counts,
                                                        DevState *__restrict__ st,
                                                        SweepScalars sc) {
  __shared__ int colcnt[kBitmaskMaxChunk];
  __shared__ uint8_t tiles[kBitmaskMaxRows / 32][kBitmaskMaxChunk / 64];
  if (use_hoist(sc, st))
    for_near_blocks<D>(sc, sc.n_pad, [&](int bid) {
      bitmask_body<D, true, true>(soa, adj, tflag, counts, st, sc, bid, colcnt, tiles);
    });
  else
    for_near_blocks<D>(sc, sc.n_pad, [&](int bid) {
      bitmask_body<D, true>(soa, adj, tflag, counts, st, sc, bid, colcnt, tiles);
    });
}

// --------------------------------------------------- merge from the bitmask
// Step 3 and the border points, from the lower triangle of the bitmask.  The
// passes read only the 32 x 64 tiles flagged non-empty (64 flags at a time),
// and one wave owns 64 rows i (lanes).  With rows in spatial order, and in
// the caller's order for at most 16,384 rows (HOOKED), first:
//
//  1. k_merge_hook: every core row i hooks under its lowest-index core
//     neighbour j < i among the 2048 columns below its 64-row block (the
//     first core bit in ascending column order).  Only row i writes
//     parent[i], and j < i, so this is a plain store and the forest keeps
//     parent[v] <= v.  It only speeds up the last pass (which sees every
//     pair): most of each cluster is joined here.
//  2. k_merge_compress: parent[v] = root of v.
//
// Then, in either order:
//
//  3. k_merge_bitmask: every neighbour pair (i, j), j < i, once:
//     * core i, core j: joined in the union-find (queued, drained 64 pairs
//       at a time).  When hooked, the word's 32 column parents are loaded
//       too (one per lane): when all its core columns hang under one parent
//       P -- the common case in spatial order -- the word needs no union if
//       P is i's root and one union otherwise; in the caller's order, where
//       a word's columns mix clusters, each pair is skipped when its column's
//       parent is i's root.  (Without the hook, in the caller's order, the
//       parents of a word's columns rarely agree and the loads would only
//       add latency.)
//     * core i, non-core j: i is a core neighbour of j (atomicMin on
//       jstar[j]);
//     * non-core i: its first core j in ascending order is its lowest core
//       neighbour below it (atomicMin on jstar[i], then the row stops
//       looking).
// A non-core point's core neighbours above it are found by those rows, so
// after the pass jstar[v] is the lowest-index core neighbour of every
// non-core v.  With a spatial order (ORDERED) the index that counts is the
// caller's, okey[j]: jstar takes okey values, and a non-core row takes the
// smallest okey over all its core neighbours below it instead of stopping
// at the first.
//
// Skipping a pair is safe whatever the timing: parent values only ever move
// to ancestors, so equal values mean a common ancestor, i.e. one tree.

// Rows of the wave that owns 64-row block rb, the words of the chunk and
// their flags: the common prologue of the passes.
struct MergeRows {
  int i, qi, q0, q1;
  bool valid, is_core;
  const uint8_t *flags;
};

__device__ __forceinline__ MergeRows merge_rows(const uint8_t *__restrict__ tflag,
                                                const uint32_t *__restrict__ corebits, int rb,
                                                int chunk, const SweepScalars &p) {
  MergeRows m;
  m.i = rb * 64 + lane_id();
  m.valid = m.i < p.n;
  m.is_core = m.valid && ((corebits[m.i >> 5] >> (m.i & 31)) & 1u);
  m.qi = m.i >> 5;
  m.q0 = chunk * p.chunk;
  m.q1 = min(m.q0 + p.chunk, (rb * 64 + 63) / 32 + 1);  // lower triangle
  m.flags = tflag + (size_t)rb * (p.n_pad / 32);
  return m;
}

// The word of row m.i for columns 32q..32q+31, limited to columns j < i.
__device__ __forceinline__ uint32_t lower_word(const MergeRows &m, int q, uint32_t word) {
  if (!m.valid || q > m.qi || q >= m.q1) return 0u;
  if (q == m.qi) return word & ((1u << (m.i & 31)) - 1u);
  return word;
}

constexpr int kMergeLoads = 8;  // words in flight per lane

// Calls f(q, word) for the flagged words q of the chunk, ascending, kU at a
// time loaded before any is used (the loop is bound by load latency
// otherwise), while `more` (a wave-uniform predicate) holds.
template <typename F, typename M>
__device__ __forceinline__ void for_flagged_words(const uint32_t *__restrict__ adj,
                                                  const MergeRows &m, int n_pad, F &&f,
                                                  M &&more) {
  const int lane = lane_id();
  for (int qf = m.q0; qf < m.q1 && more(); qf += 64) {
    uint64_t pend = __ballot(qf + lane < m.q1 && m.flags[qf + lane] != 0);
    while (pend != 0ull && more()) {
      int qs[kMergeLoads];
      uint32_t wv[kMergeLoads];
#pragma unroll
      for (int u = 0; u < kMergeLoads; ++u) {
        qs[u] = m.q1;  // none
        if (pend != 0ull) {
          qs[u] = qf + __builtin_ctzll(pend);
          pend &= pend - 1ull;
        }
        wv[u] = (qs[u] < m.q1) ? adj[adj_index(qs[u], m.i, n_pad)] : 0u;
      }
#pragma unroll
      for (int u = 0; u < kMergeLoads; ++u) f(qs[u], lower_word(m, qs[u], wv[u]));
    }
  }
}

// gate (caller's order): the passes run only when the core points' counts
// sum to at least kHookDegree per point (st->core_degree, from the core
// pass); below it the pair pass alone is cheaper.
constexpr unsigned long long kHookDegree = 4;

__device__ __forceinline__ bool hook_off(const DevState *gate, int n) {
  return gate && __hip_atomic_load(&gate->core_degree, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) < kHookDegree * (unsigned long long)n;
}

__global__ __launch_bounds__(256) void k_merge_hook(const uint32_t *__restrict__ adj,
                                                    const uint8_t *__restrict__ tflag,
                                                    const uint32_t *__restrict__ corebits,
                                                    int *__restrict__ parent, SweepScalars p,
                                                    const DevState *gate) {
  const int rb = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (rb * 64 >= p.n || hook_off(gate, p.n)) return;
  MergeRows m = merge_rows(tflag, corebits, rb, 0, p);
  m.q0 = max(0, m.q1 - 64);  // one batch of flags: the window below the diagonal
  bool seek = m.is_core;
  for_flagged_words(
      adj, m, p.n_pad,
      [&](int q, uint32_t word) {
        if (!seek || word == 0u) return;
        const uint32_t hit = word & corebits[q < m.q1 ? q : 0];
        if (hit != 0u) {
          parent[m.i] = q * 32 + __builtin_ctz(hit);
          seek = false;
        }
      },
      [&]() { return __ballot(seek) != 0ull; });
}

__global__ void k_merge_compress(int *__restrict__ parent, int n, const DevState *gate) {
  const int i = blockIdx.x * 256 + (int)threadIdx.x;
  if (i < n && !hook_off(gate, n)) {
    const int r = uf_find(parent, i);
    if (r != i) uf_store(parent + i, r);
  }
}

template <bool ORDERED, bool HOOKED>
__global__ __launch_bounds__(256) void k_merge_bitmask(const uint32_t *__restrict__ adj,
                                                       const uint8_t *__restrict__ tflag,
                                                       const uint32_t *__restrict__ corebits,
                                                       int *__restrict__ parent,
                                                       int *__restrict__ jstar,
                                                       const int *__restrict__ okey,
                                                       SweepScalars p, const DevState *gate) {
  __shared__ int2 qbuf[4][128];
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % p.nchunks;
  const int rb = (blockIdx.x / p.nchunks) * 4 + w;
  if (rb * 64 >= p.n) return;
  const MergeRows m = merge_rows(tflag, corebits, rb, chunk, p);
  if (m.q0 >= m.q1) return;
  // whether the hook and compress passes ran (their gate, read the same way)
  const bool hooked = HOOKED && !hook_off(gate, p.n);
  const int i = m.i;
  bool seek = m.valid && !m.is_core;
  int best = kNoNeighbour;                                 // ORDERED, non-core rows
  const int my_key = (ORDERED && m.valid) ? okey[i] : i;  // key of row i in jstar
  const int root_i = (hooked && m.is_core) ? parent[i] : -1;  // after the compress pass
  WaveQueue qu{qbuf[w], 0, 64};
  for_flagged_words(
      adj, m, p.n_pad,
      [&](int q, uint32_t word) {
        // every lane takes part in the cross-lane steps: no per-lane return
        if (__ballot(word != 0u) == 0ull) return;
        const uint32_t cw = corebits[q];  // core flags of the columns 32q..32q+31
        if (!m.is_core) {
          uint32_t hit = word & cw;
          if (ORDERED) {
            // the smallest caller index among the core neighbours
            for (; hit != 0u; hit &= hit - 1u)
              best = min(best, okey[q * 32 + __builtin_ctz(hit)]);
          } else if (seek && hit != 0u) {
            // the first core neighbour of a non-core row, in ascending order
            atomicMin(jstar + i, q * 32 + __builtin_ctz(hit));
            seek = false;
          }
        } else {
          // core row: its non-core columns take i as a core neighbour
          for (uint32_t nc = word & ~cw; nc != 0u; nc &= nc - 1u)
            atomicMin(jstar + q * 32 + __builtin_ctz(nc), my_key);
        }
        // core-core pairs
        uint32_t cc = m.is_core ? (word & cw) : 0u;
        if (__ballot(cc != 0u) == 0ull) return;
        if (hooked) {
          const int pc = parent[q * 32 + (lane & 31)];  // lanes l and l + 32: column l
          const int P = __builtin_amdgcn_readlane(pc, __builtin_ctz(cw));
          if (__ballot(((cw >> (lane & 31)) & 1u) && pc != P) == 0ull) {
            // every core column hangs under P: at most one union for the word
            wq_push(qu, cc != 0u && root_i != P, i, q * 32 + (cc ? __builtin_ctz(cc) : 0));
            wq_drain_union(qu, parent, false);
            return;
          }
        }
        while (__ballot(cc != 0u) != 0ull) {
          const bool has = cc != 0u;
          const int b = has ? __builtin_ctz(cc) : 0;
          cc &= cc - 1u;
          // hooked, in the caller's order: a column whose parent is i's
          // root is in i's tree already (its parent is a common ancestor)
          const bool join = (hooked && !ORDERED && has) ? parent[q * 32 + b] != root_i : has;
          wq_push(qu, join, i, q * 32 + b);
          wq_drain_union(qu, parent, false);
        }
      },
      []() { return true; });
  if (ORDERED && best != kNoNeighbour) atomicMin(jstar + i, best);
  wq_drain_union(qu, parent, true);
}

// Tile flags cleared before a pruned sweep (16-byte stores).
__global__ __launch_bounds__(256) void k_clear_flags(uint4 *__restrict__ p, long long n16) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n16;
       i += (long long)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ------------------------------------------------------------ host launchers
hipError_t run_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  // the all-pairs launch keeps its chunk's columns in LDS
  const int max_chunk = sc.box ? kBitmaskMaxChunk : kBitmaskLdsChunk;
  if (sc.chunk % 64 != 0 || sc.chunk > max_chunk || sc.rgroup % 64 != 0 || sc.rgroup <= 0 ||
      sc.rgroup > kBitmaskMaxRows)
    return hipErrorInvalidValue;
  const int groups = (sc.n_pad + sc.rgroup - 1) / sc.rgroup;
  const dim3 grid(groups * sc.nchunks), block(256);
  if (sc.box) {
    hipError_t e = run_coarse_boxes(sc, s);
    if (e != hipSuccess) return e;
    // n_pad is a multiple of 256, so the flags are whole 16-byte pieces
    const long long n16 = (long long)(sc.n_pad / 64) * (sc.n_pad / 32) / 16;
    hipLaunchKernelGGL(k_clear_flags, dim3(n16 < 4096 * 256 ? (unsigned)((n16 + 255) / 256) : 4096),
                       dim3(256), 0, s, (uint4 *)b.tflag, n16);
  }
#define DBK_BITMASK(D)                                                                        \
  case D:                                                                                     \
    if (sc.box)                                                                               \
      hipLaunchKernelGGL((k_bitmask_pruned<D>), dim3(pruned_grid(grid.x)), block, 0, s, b.soa, \
                         (uint32_t *)b.adjT, b.tflag, b.counts, b.st, sc);                    \
    else                                                                                      \
      hipLaunchKernelGGL((k_bitmask<D>), grid, block, 0, s, b.soa, (uint32_t *)b.adjT,        \
                         b.tflag, b.counts, b.st, sc);                                        \
    break;
  switch (sc.d) {
    DBK_BITMASK(1)
    DBK_BITMASK(2)
    DBK_BITMASK(3)
    DBK_BITMASK(4)
    default: return hipErrorInvalidValue;
  }
#undef DBK_BITMASK
  return hipGetLastError();
}

// The hook and compress passes run in spatial order, and in the caller's
// order up to 16,384 rows, where the hook's window (the 2,048 columns below a
// row's 64-row block) is at least an eighth of each row's lower triangle.
// Without them every core-core pair there was a union, and the unions of a
// cluster all contended for its few roots.  Measured per call (whole step):
// blobs2d_small 0.096 -> 0.074 ms, the same recipe at n = 8,000 0.76 -> 0.43
// ms, the blobs2d_200k recipe at n = 16,000 0.30 -> 0.18 ms.  On sparse
// inputs they cost more than they save (two launches and a scan: 6 to 11 us
// more for step 3 where the core points' counts sum to at most 3 per point),
// so in the caller's order they return at once below kHookDegree per point;
// the pair pass is correct with or without them.  (kHookCallerOrderMax:
// dbscan_internal.h.)

hipError_t run_merge_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 64 + 3) / 4;
  const bool hooked = b.okey || sc.n_pad <= kHookCallerOrderMax;
  if (hooked) {
    SweepScalars whole = sc;  // the hook pass scans each row's words in one piece
    whole.nchunks = 1;
    whole.chunk = sc.n_pad / 32;
    // in the caller's order the passes check the core points' degree first
    const DevState *gate = b.okey ? nullptr : b.st;
    hipLaunchKernelGGL(k_merge_hook, dim3(groups), dim3(256), 0, s, (const uint32_t *)b.adjT,
                       b.tflag, b.corebits, b.parent, whole, gate);
    hipLaunchKernelGGL(k_merge_compress, dim3((sc.n + 255) / 256), dim3(256), 0, s, b.parent,
                       sc.n, gate);
  }
  if (b.okey)
    hipLaunchKernelGGL((k_merge_bitmask<true, true>), dim3(groups * sc.nchunks), dim3(256), 0, s,
                       (const uint32_t *)b.adjT, b.tflag, b.corebits, b.parent, b.jstar, b.okey,
                       sc, nullptr);
  else if (hooked)
    hipLaunchKernelGGL((k_merge_bitmask<false, true>), dim3(groups * sc.nchunks), dim3(256), 0,
                       s, (const uint32_t *)b.adjT, b.tflag, b.corebits, b.parent, b.jstar,
                       b.okey, sc, b.st);
  else
    hipLaunchKernelGGL((k_merge_bitmask<false, false>), dim3(groups * sc.nchunks), dim3(256), 0,
                       s, (const uint32_t *)b.adjT, b.tflag, b.corebits, b.parent, b.jstar,
                       b.okey, sc, nullptr);
  return hipGetLastError();
}

}  // namespace dbk
