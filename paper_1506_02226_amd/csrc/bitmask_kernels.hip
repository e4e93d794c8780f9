// Bitmask form of steps 1 and 3 (d <= 4): the neighbour relation kept as one
// bit per ordered pair -- the paper's `cluster` matrix of Section IV-B, at one
// bit instead of one byte per entry -- and the merge of Section IV-C read
// from it.
#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// ----------------------------------------------------- bitmask pass (d <= 4)
// One wave owns 64 consecutive rows (one per lane); columns are wave-uniform
// and arrive G at a time through scalar loads.  For each 32-column word q the
// lane shifts in the 32 neighbour bits of its row (compare + add-with-carry:
// w = 2w + bit, the highest column first) and stores the word at adjT[q][i],
// a coalesced 256-byte store per wave.  Bit b of adjT[q][i] is the pair
// (i, 32q+b).  Band pairs are looked for once per group of G columns.
template <int D>
__global__ __launch_bounds__(256) void k_bitmask(const float *__restrict__ soa,
                                                 uint32_t *__restrict__ adjT,
                                                 int *__restrict__ counts,
                                                 DevState *__restrict__ st, SweepScalars sc) {
  constexpr int G = (D <= 2) ? 16 : 8;  // columns per scalar batch
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % sc.nchunks;
  const int rb = (blockIdx.x / sc.nchunks) * 4 + w;
  if (rb * 64 >= sc.n_pad) return;
  const int i = rb * 64 + lane;
  float xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = soa[(size_t)k * sc.n_pad + i];
  const int nwords = sc.n_pad >> 5;
  const int q0 = chunk * sc.chunk;
  const int q1 = min(q0 + sc.chunk, nwords);
  int cnt = 0;
  for (int q = q0; q < q1; ++q) {
    uint32_t word = 0;
#pragma unroll
    for (int g = 32 / G - 1; g >= 0; --g) {
      const int jb = q * 32 + g * G;
      float xj[G][D];
#pragma unroll
      for (int c = 0; c < G; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) xj[c][k] = soa[(size_t)k * sc.n_pad + jb + c];
      float sv[G];
      uint64_t any = 0;
#pragma unroll
      for (int c = G - 1; c >= 0; --c) {
        sv[c] = sq_dist32<D>(xi, xj[c]);
        uint64_t m, carry;
        // m = ballot(s <= hi); word = 2*word + (this lane's bit of m)
        asm("v_cmp_ge_f32_e64 %1, %3, %4\n\t"
            "v_addc_co_u32_e64 %0, %2, %0, %0, %1"
            : "+v"(word), "=&s"(m), "=&s"(carry)
            : "s"(sc.hi), "v"(sv[c]));
        any |= m;
      }
      if (any != 0ull) {
        // column jb+c sits at bit c of the word now
#pragma unroll
        for (int c = 0; c < G; ++c) {
          const uint64_t m = __ballot(sv[c] <= sc.hi);
          const uint64_t lo_m = __ballot(sv[c] <= sc.lo);
          if (m != lo_m) {
            const uint64_t ex = recheck_band<D>(m & ~lo_m, lo_m, xi, xj[c], sc.eps2, st);
            const uint32_t bit = (uint32_t)((ex >> lane) & 1ull);
            word = (word & ~(1u << c)) | (bit << c);
          }
        }
      }
    }
    adjT[(size_t)q * sc.n_pad + i] = word;
    cnt += __popc(word);
  }
  if (i < sc.n) {
    if (sc.nchunks == 1)
      counts[i] = cnt;
    else
      atomicAdd(counts + i, cnt);
  }
}

// --------------------------------------------------- merge from the bitmask
// One wave owns 64 rows; it walks the words q of a chunk up to the diagonal.
// Core rows queue their core neighbours j < i; the queue is drained into the
// union-find 64 pairs at a time.
__global__ __launch_bounds__(256) void k_union_bitmask(const uint32_t *__restrict__ adjT,
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
  const int qi = i >> 5;
  const int q0 = chunk * p.chunk;
  const int q1 = min(q0 + p.chunk, (rb * 64 + 63) / 32 + 1);  // lower triangle
  if (q0 >= q1 || __ballot(is_core) == 0ull) return;
  WaveQueue qu{qbuf[w], 0};
  for (int q = q0; q < q1; ++q) {
    const uint32_t cw = corebits[q];
    uint32_t word = adjT[(size_t)q * p.n_pad + i] & cw;
    if (!is_core || q > qi) word = 0u;
    else if (q == qi) word &= (1u << (i & 31)) - 1u;
    while (__ballot(word != 0u) != 0ull) {
      const bool has = word != 0u;
      const int j = q * 32 + (has ? __builtin_ctz(word) : 0);
      word &= word - 1u;
      wq_push(qu, has, i, j);
      wq_drain_union(qu, parent, false);
    }
  }
  wq_drain_union(qu, parent, true);
}

// ------------------------------------------------------------ host launchers
hipError_t run_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 64 + 3) / 4;
  const dim3 grid(groups * sc.nchunks), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL(k_bitmask<1>, grid, block, 0, s, b.soa, b.adjT, b.counts, b.st, sc); break;
    case 2: hipLaunchKernelGGL(k_bitmask<2>, grid, block, 0, s, b.soa, b.adjT, b.counts, b.st, sc); break;
    case 3: hipLaunchKernelGGL(k_bitmask<3>, grid, block, 0, s, b.soa, b.adjT, b.counts, b.st, sc); break;
    case 4: hipLaunchKernelGGL(k_bitmask<4>, grid, block, 0, s, b.soa, b.adjT, b.counts, b.st, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_union_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 64 + 3) / 4;
  hipLaunchKernelGGL(k_union_bitmask, dim3(groups * sc.nchunks), dim3(256), 0, s, b.adjT,
                     b.corebits, b.parent, sc);
  return hipGetLastError();
}

}  // namespace dbk
