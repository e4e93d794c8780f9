// Bitmask form of steps 1 and 3 (d <= 4): the neighbour relation kept as one
// bit per ordered pair -- the paper's `cluster` matrix of Section IV-B, at one
// bit instead of one byte per entry, in 32-bit words -- and the merge of
// Section IV-C read from it.
#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// ----------------------------------------------------- bitmask pass (d <= 4)
// One wave takes 32 rows at a time (the "goal points" of Section IV-A.3,
// wave-uniform values held in vector registers so that the subtractions issue
// at the full rate) and the 64 lanes hold 64 columns.  Per row, one compare
// gives the 64-bit ballot of the row's neighbours among the columns; only
// when a ballot is not empty -- rare at these densities, and tested once per
// group of 4 rows -- does its popcount go to the row's count (scalar unit)
// and the lane set bit r of its 32-bit word.  After the 32 rows, lane j holds
// the pairs (rows
// row0..row0+31, column j); by symmetry that is row j's word for the columns
// row0..row0+31, stored at adj[row0/32][j] -- a coalesced 256-byte store per
// wave.  Bit b of adj[q][i] is the pair (i, 32q+b).  Padded rows and columns
// (index >= n) are NaN, so their bits are zero.
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

template <int D>
__global__ __launch_bounds__(256) void k_bitmask(const float *__restrict__ soa,
                                                 uint32_t *__restrict__ adj,
                                                 int *__restrict__ counts,
                                                 DevState *__restrict__ st, SweepScalars sc) {
  constexpr int R = 32, G = 4;
  __shared__ int colcnt[kBitmaskMaxChunk];
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % sc.nchunks;
  const int g0 = (blockIdx.x / sc.nchunks) * sc.rgroup;
  const int c0 = chunk * sc.chunk;
  const int c1 = min(c0 + sc.chunk, sc.n_pad);
  if (g0 >= sc.n_pad || c1 <= g0) return;  // block-uniform
  for (int t = threadIdx.x; t < sc.chunk; t += 256) colcnt[t] = 0;
  __syncthreads();
  const int g1 = min(g0 + sc.rgroup, sc.n_pad);
  for (int row0 = g0 + w * R; row0 < g1; row0 += 4 * R) {
    const int diag = row0 & ~63;
    const int cs = max(c0, diag);
    if (cs >= c1) continue;  // wave-uniform
    float xr[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < D; ++k) xr[r][k] = to_vgpr(soa[(size_t)k * sc.n_pad + row0 + r]);
    // two rows' counts per scalar register (a chunk has at most 4096 columns)
    uint32_t cnt2[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) cnt2[r] = 0;
    uint32_t *out = adj + (size_t)(row0 / R) * sc.n_pad;
    float xn[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xn[k] = soa[(size_t)k * sc.n_pad + cs + lane];
    for (int cb = cs; cb < c1; cb += 64) {
      float xc[D];
#pragma unroll
      for (int k = 0; k < D; ++k) xc[k] = xn[k];
      if (cb + 64 < c1) {
#pragma unroll
        for (int k = 0; k < D; ++k) xn[k] = soa[(size_t)k * sc.n_pad + cb + 64 + lane];
      }
      uint32_t word = 0;
      // rows in groups of G: the common case (no neighbour among the 64
      // columns for any of the G rows) costs one compare per row and one
      // branch per group; the lane's bits and the row counts are set only
      // in the rare case
#pragma unroll
      for (int g = 0; g < R / G; ++g) {
        float sg[G];
        uint64_t mg[G], any = 0ull;
#pragma unroll
        for (int k = 0; k < G; ++k) {
          sg[k] = sq_dist32<D>(xr[g * G + k], xc);
          mg[k] = __ballot(sg[k] <= sc.hi);
          any |= mg[k];
        }
        if (any == 0ull) continue;
#pragma unroll
        for (int k = 0; k < G; ++k) {
          const int r = g * G + k;
          if (mg[k] == 0ull) continue;
          const uint64_t lo_m = __ballot(sg[k] <= sc.lo);
          uint64_t in = mg[k];
          if (lo_m != in)
            in = recheck_band_soa(in & ~lo_m, lo_m, soa, sc.n_pad, D, row0 + r, cb + lane,
                                  sc.eps2, st);
          word |= ((in >> lane) & 1ull) ? (1u << r) : 0u;
          cnt2[r >> 1] += (uint32_t)__popcll(in) << ((r & 1) * 16);
        }
      }
      out[cb + lane] = word;
      if (cb != diag && word != 0u) atomicAdd(&colcnt[cb - c0 + lane], __popc(word));
    }
    int mine = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane == r) mine = (int)((cnt2[r >> 1] >> ((r & 1) * 16)) & 0xffffu);
    const int row = row0 + lane;
    if (lane < R && row < sc.n && mine != 0) atomicAdd(counts + row, mine);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < c1 - c0; t += 256) {
    const int v = colcnt[t];
    if (v != 0 && c0 + t < sc.n) atomicAdd(counts + c0 + t, v);
  }
}

// --------------------------------------------------- merge from the bitmask
// Step 3 and the border points in one read of the lower triangle.  One wave
// owns 64 rows i (lanes) and walks the 32-column words q of a chunk up to the
// diagonal, so it sees every neighbour pair (i, j), j < i, once, and takes
// the set bits of its word one per lane per round:
//  * core i, core j: queued, and the queue is drained into the union-find 64
//    pairs at a time;
//  * core i, non-core j: i is a core neighbour of j (atomicMin on jstar[j]);
//  * non-core i: its first core j in ascending order is its lowest core
//    neighbour below it (atomicMin on jstar[i], then the row stops looking).
// A non-core point's core neighbours above it are found by those rows, so
// after the pass jstar[v] is the lowest-index core neighbour of every
// non-core v.  With a spatial order (ORDERED) the index that counts is the
// caller's, okey[j]: jstar takes okey values, and a non-core row takes the
// smallest okey over all its core neighbours below it instead of stopping
// at the first.
template <bool ORDERED>
__global__ __launch_bounds__(256) void k_merge_bitmask(const uint32_t *__restrict__ adj,
                                                       const uint32_t *__restrict__ corebits,
                                                       int *__restrict__ parent,
                                                       int *__restrict__ jstar,
                                                       const int *__restrict__ okey,
                                                       SweepScalars p) {
  __shared__ int2 qbuf[4][128];
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % p.nchunks;
  const int rb = (blockIdx.x / p.nchunks) * 4 + w;
  if (rb * 64 >= p.n) return;
  const int i = rb * 64 + lane;
  const bool valid = i < p.n;
  const bool is_core = valid && ((corebits[i >> 5] >> (i & 31)) & 1u);
  bool seek = valid && !is_core;
  int best = kNoNeighbour;                               // ORDERED, non-core rows
  const int my_key = (ORDERED && valid) ? okey[i] : i;  // key of row i in jstar
  const int qi = i >> 5;
  const int q0 = chunk * p.chunk;
  const int q1 = min(q0 + p.chunk, (rb * 64 + 63) / 32 + 1);  // lower triangle
  if (q0 >= q1) return;
  WaveQueue qu{qbuf[w], 0, 64};
  // kU words per lane are loaded before any is used, so that kU loads per
  // wave are in flight (the loop is bound by load latency otherwise)
  constexpr int kU = 8;
  for (int qb = q0; qb < q1; qb += kU) {
    uint32_t wv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = qb + u;
      wv[u] = (q < q1) ? adj[(size_t)q * p.n_pad + i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = qb + u;
      uint32_t word = wv[u];
      if (!valid || q > qi || q >= q1) word = 0u;
      else if (q == qi) word &= (1u << (i & 31)) - 1u;
      if (__ballot(word != 0u) == 0ull) continue;
      const uint32_t cw = corebits[q];  // core flags of the columns 32q..32q+31
      if (!is_core) {
        uint32_t hit = word & cw;
        if (ORDERED) {
          // the smallest caller index among the core neighbours
          for (; hit != 0u; hit &= hit - 1u) best = min(best, okey[q * 32 + __builtin_ctz(hit)]);
        } else if (seek && hit != 0u) {
          // the first core neighbour of a non-core row, in ascending order
          atomicMin(jstar + i, q * 32 + __builtin_ctz(hit));
          seek = false;
        }
        word = 0u;
      }
      while (__ballot(word != 0u) != 0ull) {
        const bool has = word != 0u;
        const int b = has ? __builtin_ctz(word) : 0;
        word &= word - 1u;
        const int j = q * 32 + b;
        const bool cj = (cw >> b) & 1u;
        if (has && is_core && !cj) atomicMin(jstar + j, my_key);
        wq_push(qu, has && is_core && cj, i, j);
        wq_drain_union(qu, parent, false);
      }
    }
  }
  if (ORDERED && best != kNoNeighbour) atomicMin(jstar + i, best);
  wq_drain_union(qu, parent, true);
}

// ------------------------------------------------------------ host launchers
hipError_t run_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  if (sc.chunk % 64 != 0 || sc.chunk > kBitmaskMaxChunk || sc.rgroup % 64 != 0 || sc.rgroup <= 0)
    return hipErrorInvalidValue;
  const int groups = (sc.n_pad + sc.rgroup - 1) / sc.rgroup;
  const dim3 grid(groups * sc.nchunks), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL(k_bitmask<1>, grid, block, 0, s, b.soa, (uint32_t *)b.adjT, b.counts, b.st, sc); break;
    case 2: hipLaunchKernelGGL(k_bitmask<2>, grid, block, 0, s, b.soa, (uint32_t *)b.adjT, b.counts, b.st, sc); break;
    case 3: hipLaunchKernelGGL(k_bitmask<3>, grid, block, 0, s, b.soa, (uint32_t *)b.adjT, b.counts, b.st, sc); break;
    case 4: hipLaunchKernelGGL(k_bitmask<4>, grid, block, 0, s, b.soa, (uint32_t *)b.adjT, b.counts, b.st, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_merge_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 64 + 3) / 4;
  if (b.okey)
    hipLaunchKernelGGL(k_merge_bitmask<true>, dim3(groups * sc.nchunks), dim3(256), 0, s,
                       (const uint32_t *)b.adjT, b.corebits, b.parent, b.jstar, b.okey, sc);
  else
    hipLaunchKernelGGL(k_merge_bitmask<false>, dim3(groups * sc.nchunks), dim3(256), 0, s,
                       (const uint32_t *)b.adjT, b.corebits, b.parent, b.jstar, b.okey, sc);
  return hipGetLastError();
}

}  // namespace dbk
