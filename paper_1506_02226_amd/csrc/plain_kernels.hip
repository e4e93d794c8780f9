// Plain-form DBSCAN kernels for gfx950 (wave64): float32 direct-form filter,
// float64 re-check of band pairs, counts, core flags, union-find merge,
// border assignment and canonical labels.
//
// Paper mapping:
//  * Section IV-A: every ordered pair is tested; the test is on squared
//    distances against eps^2.  Section IV-A.2 stores the coordinates
//    transposed (one array per coordinate) for coalesced reads -- here the
//    staging kernel writes that layout, padded with NaN so that padded
//    columns fail every comparison.  Section IV-A.3 keeps the goal point in
//    registers while a tile of other points streams by -- here the "goal"
//    rows are wave-uniform (scalar registers or LDS broadcast) and 64
//    columns ride in the lanes, so one compare yields one 64-bit ballot word.
//  * Section IV-B / IV-B.1: the neighbourhood test is fused with the
//    distance; no distance is stored.  Counts come from popcounts of the
//    ballot words; the primitive clusters are kept either as a bit matrix
//    (one bit per ordered pair) or not at all (recomputed on the fly).
//  * Section IV-C: the merge.  Instead of one launch per target cluster, a
//    lock-free union-find joins the primitive clusters of every pair of
//    neighbouring core points in one pass.
#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// ------------------------------------------------------------------ staging
__global__ void k_reset_state(DevState *st) {
  if (threadIdx.x == 0) {
    st->status = 0;
    st->noncore = 0;
    st->band_pairs = 0;
    st->core_points = 0;
  }
}

// soa[k][i] = points[i][k] for k < d, 0 for d <= k < d_pad, NaN for i >= n.
// Also clears counts, parent = identity, jstar = none; flags non-finite input.
__global__ void k_stage(const float *__restrict__ pts, int n, int d, int n_pad, int d_pad,
                        float *__restrict__ soa, int *__restrict__ counts,
                        int *__restrict__ parent, int *__restrict__ jstar, DevState *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
  if (i < n) {
    counts[i] = 0;
    parent[i] = i;
    jstar[i] = kNoNeighbour;
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&st->status, kStatusNonFinite);
}

// ------------------------------------------------ row-uniform sweeps, d <= 4
// One wave owns R rows ("goal points", kept in scalar registers); the 64
// lanes hold 64 columns, so one compare yields one 64-bit ballot word.  A
// pair is "in" when s32 <= lo, "out" when s32 > hi; the rare pairs between
// are decided in float64 from the same register coordinates.

// Lanes of `band` re-decided in float64; returns the exact in-mask.
template <int D>
__device__ __forceinline__ uint64_t settle_band(uint64_t m, uint64_t in, const float (&a)[D],
                                                const float (&b)[D], double eps2, DevState *st) {
  if (in == m) return in;
  return recheck_band<D>(m & ~in, in, a, b, eps2, st);
}

// step 1 + counts: all rows, a chunk of columns.
template <int D, int R>
__global__ __launch_bounds__(256) void k_count_small(const float *__restrict__ soa,
                                                     int *__restrict__ counts,
                                                     DevState *__restrict__ st, SweepScalars sc) {
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % sc.nchunks;
  const int row0 = ((blockIdx.x / sc.nchunks) * 4 + w) * R;
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
      }
    }
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

// step 3, merge: core rows i union with their core neighbours j < i.
template <int D, int R>
__global__ __launch_bounds__(256) void k_union_small(const float *__restrict__ soa,
                                                     const uint32_t *__restrict__ corebits,
                                                     int *__restrict__ parent,
                                                     DevState *__restrict__ st, SweepScalars sc) {
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
  for (int cb = 0; cb < c1; cb += 64) {
    const uint64_t cw = (uint64_t)corebits[cb >> 5] | ((uint64_t)corebits[(cb >> 5) + 1] << 32);
    if (cw == 0ull) continue;
    float xc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xc[k] = soa[(size_t)k * sc.n_pad + cb + lane];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!((active >> r) & 1u)) continue;
      const int lim = row0 + r - cb;
      if (lim <= 0) continue;
      const uint64_t cm = (lim < 64) ? (cw & ((1ull << lim) - 1ull)) : cw;
      const float s = sq_dist32<D>(xr[r], xc);
      const uint64_t m = __ballot(s <= sc.hi) & cm;
      if (m != 0ull) {
        const uint64_t in =
            settle_band<D>(m, __ballot(s <= sc.lo) & cm, xr[r], xc, sc.eps2, st);
        if ((in >> lane) & 1ull) uf_union(parent, row0 + r, cb + lane);
      }
    }
  }
}

// step 3, border: listed non-core rows find their lowest-index core neighbour.
template <int D, int R>
__global__ __launch_bounds__(256) void k_border_small(const float *__restrict__ soa,
                                                      const uint32_t *__restrict__ corebits,
                                                      const int *__restrict__ list,
                                                      int *__restrict__ jstar,
                                                      DevState *__restrict__ st, SweepScalars sc) {
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int listed = wave_uniform((int)__hip_atomic_load(&st->noncore, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
  const int e0 = (blockIdx.x * 4 + w) * R;
  if (e0 >= listed) return;
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
  for (int cb = 0; cb < sc.n_pad && active != 0u; cb += 64) {
    const uint64_t cw = (uint64_t)corebits[cb >> 5] | ((uint64_t)corebits[(cb >> 5) + 1] << 32);
    if (cw == 0ull) continue;
    float xc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xc[k] = soa[(size_t)k * sc.n_pad + cb + lane];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!((active >> r) & 1u)) continue;
      const float s = sq_dist32<D>(xr[r], xc);
      const uint64_t m = __ballot(s <= sc.hi) & cw;
      if (m != 0ull) {
        const uint64_t in =
            settle_band<D>(m, __ballot(s <= sc.lo) & cw, xr[r], xc, sc.eps2, st);
        if (in != 0ull) {
          found[r] = cb + __builtin_ctzll(in);
          active &= ~(1u << r);
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
  if (lane < R && mine != kNoNeighbour) jstar[myrow] = mine;
}

// ---------------------------------------------- row-uniform sweeps, any d
// Rows staged in LDS ([4 waves][R][d_pad], read as broadcasts), columns in
// lanes, coordinates processed DC at a time.  Same three modes as above.
enum { MODE_COUNT = 0, MODE_UNION = 1, MODE_BORDER = 2 };

template <int DC, int R, int MODE>
__global__ __launch_bounds__(256) void k_rows_lds(const float *__restrict__ soa,
                                                  int *__restrict__ counts,
                                                  const uint32_t *__restrict__ corebits,
                                                  int *__restrict__ parent,
                                                  const int *__restrict__ list,
                                                  int *__restrict__ jstar,
                                                  DevState *__restrict__ st, SweepScalars sc) {
  extern __shared__ float lds_rows[];
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int n = sc.n;
  int rows[R];
  uint32_t active = 0;
  int cb_begin = 0, cb_end = sc.n_pad;
  if (MODE == MODE_COUNT) {
    const int chunk = blockIdx.x % sc.nchunks;
    const int rb = (blockIdx.x / sc.nchunks) * 4 + w;
    cb_begin = chunk * sc.chunk;
    cb_end = min(cb_begin + sc.chunk, sc.n_pad);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rows[r] = rb * R + r;
      if (rows[r] < n) active |= 1u << r;
    }
  } else if (MODE == MODE_UNION) {
    const int total = (n + R - 1) / R;
    const int rb = total - 1 - (int)(blockIdx.x * 4 + w);
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
    const int e0 = (blockIdx.x * 4 + w) * R;
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
        acc[r] = cb + __builtin_ctzll(in);
        active &= ~(1u << r);
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
    jstar[myrow] = mine;
  }
}

// ----------------------------------------------------- bitmask pass (d <= 4)
// One wave owns 64 consecutive rows (one per lane); columns are wave-uniform
// (scalar loads).  For each 32-column word q the lane shifts in the 32
// neighbour bits of its row (compare + add-with-carry: w = 2w + bit) and
// stores the word at adjT[q][i], a coalesced 256-byte store per wave.
// Bit b of adjT[q][i] is the pair (i, 32q+b).
template <int D>
__global__ __launch_bounds__(256) void k_bitmask(const float *__restrict__ soa,
                                                 uint32_t *__restrict__ adjT,
                                                 int *__restrict__ counts,
                                                 DevState *__restrict__ st, SweepScalars sc) {
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
    for (int b = 31; b >= 0; --b) {
      const int j = q * 32 + b;
      float xj[D];
#pragma unroll
      for (int k = 0; k < D; ++k) xj[k] = soa[(size_t)k * sc.n_pad + j];
      const float s = sq_dist32<D>(xi, xj);
      uint64_t m, carry;
      // m = ballot(s <= hi); word = 2*word + (this lane's bit of m)
      asm("v_cmp_ge_f32_e64 %1, %3, %4\n\t"
          "v_addc_co_u32_e64 %0, %2, %0, %0, %1"
          : "+v"(word), "=&s"(m), "=&s"(carry)
          : "s"(sc.hi), "v"(s));
      if (m != 0ull) {
        const uint64_t lo_m = __ballot(s <= sc.lo);
        if (lo_m != m) {
          const uint64_t ex = recheck_band<D>(m & ~lo_m, lo_m, xi, xj, sc.eps2, st);
          word = (word & ~1u) | (uint32_t)((ex >> lane) & 1ull);
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

// ------------------------------------------------------------- core flags
__global__ void k_core(const int *__restrict__ counts, int n, int n_pad, int minpts,
                       uint8_t *__restrict__ core, uint32_t *__restrict__ corebits,
                       DevState *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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

// Non-core rows into a list (any order) for the on-the-fly border pass.
__global__ void k_compact_noncore(const uint8_t *__restrict__ core, int n, int *__restrict__ list,
                                  DevState *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool nc = i < n && core[i] == 0;
  const uint64_t m = __ballot(nc);
  if (m == 0ull) return;
  const int lane = lane_id();
  int base = 0;
  if (lane == 0) base = (int)atomicAdd(&st->noncore, (unsigned)__popcll(m));
  base = __shfl(base, 0);
  if (nc) list[base + __popcll(m & ((1ull << lane) - 1ull))] = i;
}

// -------------------------------------------- merge + border from the bitmask
// One wave owns 64 rows; it walks the words q of a chunk.  Core rows union
// with their core neighbours j < i; non-core rows record their first core
// neighbour in the chunk (atomicMin across chunks).
__global__ __launch_bounds__(256) void k_sweep_bitmask(const uint32_t *__restrict__ adjT,
                                                       const uint32_t *__restrict__ corebits,
                                                       int *__restrict__ parent,
                                                       int *__restrict__ jstar, SweepScalars p) {
  const int lane = lane_id();
  const int w = wave_uniform(threadIdx.x >> 6);
  const int chunk = blockIdx.x % p.nchunks;
  const int rb = (blockIdx.x / p.nchunks) * 4 + w;
  if (rb * 64 >= p.n_pad) return;
  const int i = rb * 64 + lane;
  const bool valid = i < p.n;
  const bool is_core = valid && ((corebits[i >> 5] >> (i & 31)) & 1u);
  bool need_border = valid && !is_core;
  const int qi = i >> 5;
  const int nwords = p.n_pad >> 5;
  const int q0 = chunk * p.chunk;
  const int q1 = min(q0 + p.chunk, nwords);
  for (int q = q0; q < q1; ++q) {
    const bool u_active = is_core && q <= qi;
    if (__ballot(u_active || need_border) == 0ull) break;
    const uint32_t cw = corebits[q];
    const uint32_t word = adjT[(size_t)q * p.n_pad + i] & cw;
    if (u_active) {
      uint32_t m = (q < qi) ? word : (word & ((1u << (i & 31)) - 1u));
      while (m) {
        const int b = __builtin_ctz(m);
        m &= m - 1u;
        uf_union(parent, i, q * 32 + b);
      }
    }
    if (need_border && word) {
      atomicMin(jstar + i, q * 32 + __builtin_ctz(word));
      need_border = false;
    }
  }
}

// ------------------------------------------------------------------ labels
__global__ void k_labels(int n, const uint8_t *__restrict__ core, const int *__restrict__ jstar,
                         int *__restrict__ parent, int *__restrict__ labels, const DevState *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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

// ------------------------------------------------------------ host launchers
constexpr int kRowsSmall = 8;   // rows per wave, d <= 4 (scalar registers)
constexpr int kRowsLds = 8;     // rows per wave, d > 4 (LDS)

int rows_per_wave(int d) { return d <= 4 ? kRowsSmall : kRowsLds; }

int coord_chunk(int d) {
  if (d <= 4) return d;
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  return 64;
}

hipError_t run_reset(DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t run_stage(const float *pts, int n, int d, int n_pad, int d_pad, float *soa, int *counts,
                     int *parent, int *jstar, DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_stage, dim3((n_pad + 255) / 256), dim3(256), 0, s, pts, n, d, n_pad, d_pad,
                     soa, counts, parent, jstar, st);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_lds(const Buffers &b, const SweepScalars &sc, int blocks, hipStream_t s) {
  const size_t lds = (size_t)4 * kRowsLds * sc.d_pad * sizeof(float);
  switch (coord_chunk(sc.d)) {
#define DBK_LDS_CASE(DC)                                                                      \
  case DC:                                                                                    \
    hipLaunchKernelGGL((k_rows_lds<DC, kRowsLds, MODE>), dim3(blocks), dim3(256), lds, s,    \
                       b.soa, b.counts, b.corebits, b.parent, b.list, b.jstar, b.st, sc);     \
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

hipError_t run_count(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int R = rows_per_wave(sc.d);
  const int groups = ((sc.n + R - 1) / R + 3) / 4;
  const dim3 grid(groups * sc.nchunks), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL((k_count_small<1, kRowsSmall>), grid, block, 0, s, b.soa, b.counts, b.st, sc); break;
    case 2: hipLaunchKernelGGL((k_count_small<2, kRowsSmall>), grid, block, 0, s, b.soa, b.counts, b.st, sc); break;
    case 3: hipLaunchKernelGGL((k_count_small<3, kRowsSmall>), grid, block, 0, s, b.soa, b.counts, b.st, sc); break;
    case 4: hipLaunchKernelGGL((k_count_small<4, kRowsSmall>), grid, block, 0, s, b.soa, b.counts, b.st, sc); break;
    default: return launch_lds<MODE_COUNT>(b, sc, groups * sc.nchunks, s);
  }
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
  const dim3 grid(((sc.n + R - 1) / R + 3) / 4), block(256);
  switch (sc.d) {
    case 1: hipLaunchKernelGGL((k_border_small<1, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.st, sc); break;
    case 2: hipLaunchKernelGGL((k_border_small<2, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.st, sc); break;
    case 3: hipLaunchKernelGGL((k_border_small<3, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.st, sc); break;
    case 4: hipLaunchKernelGGL((k_border_small<4, kRowsSmall>), grid, block, 0, s, b.soa, b.corebits, b.list, b.jstar, b.st, sc); break;
    default: return launch_lds<MODE_BORDER>(b, sc, (int)grid.x, s);
  }
  return hipGetLastError();
}

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

hipError_t run_core(const int *counts, int n, int n_pad, int minpts, uint8_t *core,
                    uint32_t *corebits, DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_core, dim3((n_pad + 255) / 256), dim3(256), 0, s, counts, n, n_pad, minpts,
                     core, corebits, st);
  return hipGetLastError();
}

hipError_t run_compact_noncore(const uint8_t *core, int n, int *list, DevState *st,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_compact_noncore, dim3((n + 255) / 256), dim3(256), 0, s, core, n, list, st);
  return hipGetLastError();
}

hipError_t run_sweep_bitmask(const Buffers &b, const SweepScalars &sc, hipStream_t s) {
  const int groups = (sc.n_pad / 64 + 3) / 4;
  hipLaunchKernelGGL(k_sweep_bitmask, dim3(groups * sc.nchunks), dim3(256), 0, s, b.adjT,
                     b.corebits, b.parent, b.jstar, sc);
  return hipGetLastError();
}

hipError_t run_labels(int n, const uint8_t *core, const int *jstar, int *parent, int *labels,
                      const DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_labels, dim3((n + 255) / 256), dim3(256), 0, s, n, core, jstar, parent,
                     labels, st);
  return hipGetLastError();
}

}  // namespace dbk
