// Bitmask form of steps 1 and 3 (d <= 4): the neighbour relation kept as one
// bit per ordered pair -- the paper's `cluster` matrix of Section IV-B, at one
// bit instead of one byte per entry, in 16-bit words -- and the merge of
// Section IV-C read from it.
#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// ----------------------------------------------------- bitmask pass (d <= 4)
// One wave owns 16 rows (the "goal points" of Section IV-A.3, in scalar
// registers) and the 64 lanes hold 64 columns.  Per row, one compare gives
// the 64-bit ballot of the row's neighbours among the columns (its popcount
// is the row's count, on the scalar unit), and the same compare's result is
// shifted into a per-lane 16-bit word with an add-with-carry (w = 2w + bit).
// After the 16 rows, lane j holds the pairs (rows row0..row0+15, column j);
// by symmetry that is row j's word for the columns row0..row0+15, stored at
// adj[row0/16][j] -- a coalesced 128-byte store per wave.  Bit b of
// adj[q][i] is the pair (i, 16q+b).  Padded rows (i >= n) are NaN, so their
// words are written as zeros.
template <int D>
__global__ __launch_bounds__(256) void k_bitmask(const float *__restrict__ soa,
                                                 uint16_t *__restrict__ adj,
                                                 int *__restrict__ counts,
                                                 DevState *__restrict__ st, SweepScalars sc) {
  constexpr int R = 16;
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % sc.nchunks;
  const int row0 = ((blockIdx.x / sc.nchunks) * 4 + w) * R;
  if (row0 >= sc.n_pad) return;
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
  uint16_t *out = adj + (size_t)(row0 / R) * sc.n_pad;
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
    uint32_t word = 0;
#pragma unroll
    for (int r = R - 1; r >= 0; --r) {
      const float s = sq_dist32<D>(xr[r], xc);
      uint64_t m, carry;
      // m = ballot(s <= hi); word = 2*word + (this lane's bit of m)
      asm("v_cmp_ge_f32_e64 %1, %3, %4\n\t"
          "v_addc_co_u32_e64 %0, %2, %0, %0, %1"
          : "+v"(word), "=&s"(m), "=&s"(carry)
          : "s"(sc.hi), "v"(s));
      if (m != 0ull) {
        const uint64_t lo_m = __ballot(s <= sc.lo);
        uint64_t in = m;
        if (lo_m != m) {
          in = recheck_band<D>(m & ~lo_m, lo_m, xr[r], xc, sc.eps2, st);
          word = (word & ~1u) | (uint32_t)((in >> lane) & 1ull);
        }
        cnt[r] += __popcll(in);
      }
    }
    out[cb + lane] = (uint16_t)word;
  }
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

// --------------------------------------------------- merge from the bitmask
// One wave owns 64 rows; it walks the 16-column words q of a chunk up to the
// diagonal.  Core rows queue their core neighbours j < i; the queue is
// drained into the union-find 64 pairs at a time.
__global__ __launch_bounds__(256) void k_union_bitmask(const uint16_t *__restrict__ adj,
                                                       const uint32_t *__restrict__ corebits,
                                                       int *__restrict__ parent,
                                                       SweepScalars p) {
  __shared__ int2 qbuf[4][128];
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % p.nchunks;
  const int rb = (blockIdx.x / p.nchunks) * 4 + w;
  if (rb * 64 >= p.n) return;
  const int i = rb * 64 + lane;
  const bool is_core = i < p.n && ((corebits[i >> 5] >> (i & 31)) & 1u);
  const int qi = i >> 4;
  const int q0 = chunk * p.chunk;
  const int q1 = min(q0 + p.chunk, (rb * 64 + 63) / 16 + 1);  // lower triangle
  if (q0 >= q1 || __ballot(is_core) == 0ull) return;
  WaveQueue qu{qbuf[w], 0};
  for (int q = q0; q < q1; ++q) {
    const uint32_t cw = (corebits[q >> 1] >> ((q & 1) * 16)) & 0xffffu;
    uint32_t word = (uint32_t)adj[(size_t)q * p.n_pad + i] & cw;
    if (!is_core || q > qi) word = 0u;
    else if (q == qi) word &= (1u << (i & 15)) - 1u;
    while (__ballot(word != 0u) != 0ull) {
      const bool has = word != 0u;
      const int j = q * 16 + (has ? __builtin_ctz(word) : 0);
      word &= word - 1u;
      wq_push(qu, has, i, j);
      wq_drain_union(qu, parent, false);
    }
  }
  wq_drain_union(qu, parent, true);
}

// ------------------------------------------------------------ host launchers
hipError_t run_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 16 + 3) / 4;
  const dim3 grid(groups * sc.nchunks), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL(k_bitmask<1>, grid, block, 0, s, b.soa, (uint16_t *)b.adjT, b.counts, b.st, sc); break;
    case 2: hipLaunchKernelGGL(k_bitmask<2>, grid, block, 0, s, b.soa, (uint16_t *)b.adjT, b.counts, b.st, sc); break;
    case 3: hipLaunchKernelGGL(k_bitmask<3>, grid, block, 0, s, b.soa, (uint16_t *)b.adjT, b.counts, b.st, sc); break;
    case 4: hipLaunchKernelGGL(k_bitmask<4>, grid, block, 0, s, b.soa, (uint16_t *)b.adjT, b.counts, b.st, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_union_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 64 + 3) / 4;
  hipLaunchKernelGGL(k_union_bitmask, dim3(groups * sc.nchunks), dim3(256), 0, s,
                     (const uint16_t *)b.adjT, b.corebits, b.parent, sc);
  return hipGetLastError();
}

}  // namespace dbk
