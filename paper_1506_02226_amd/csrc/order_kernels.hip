// Spatial order of the points: a permutation that puts points close in
// space at close indices, applied when the coordinates are staged.  The
// epsilon tests are unchanged -- every pair is still tested (Section IV-A),
// with the same filter and float64 re-evaluation -- but the rare neighbour
// pairs gather into few tiles, so the sweeps take their rare branch (and the
// matrix-core filter settles its accumulators) far less often and the
// bitmask's non-zero words sit near its diagonal.  The outputs are returned
// in the caller's order and labels stay canonical in the caller's indices
// (the label passes map through the permutation).
//
// d <= 4: the key of a point is its coordinates quantised over the bounding
// box of the input (order_bits_per_coord(d) bits each) and interleaved bit by
// bit (Morton order).  5 <= d <= 128: the key is the index of the nearest of
// 256 (128 beyond d = 64) pivot rows taken at a fixed stride through the
// input, found on the matrix cores (a point and its neighbours mostly share
// the nearest pivot: a Morton key of a few coordinates would mix the
// clusters of high-dimensional data).  Either way
// the permutation is the stable LSD radix sort of the keys, 8 bits per pass;
// ties keep input order, so the permutation is deterministic.
#include <hip/hip_bf16.h>

#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

namespace {

constexpr int kSortItems = 8;                 // keys per thread per tile
constexpr int kPivotMaxD = 128;               // d > 4 up to this (pivots in 64 KiB of LDS)
constexpr int kPivotBlocks = 512;             // grid of the pivot kernel, at most
constexpr int kSortTile = 256 * kSortItems;   // keys per block

// float -> unsigned with the same order (for atomic min / max)
__device__ __forceinline__ unsigned ordered_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(unsigned o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// Bounding box of the finite coordinates: per-thread extremes over a
// grid-strided range, reduced across the wave and then the block, and one
// atomic per block and coordinate into st->box_lo / box_hi (reset to empty).
// The grid is small (at most kBoxBlocks), so the atomics do not queue up.
constexpr int kBoxBlocks = 256;

__global__ __launch_bounds__(256) void k_order_box(const float *__restrict__ pts, int n, int d,
                                                   DevState *st) {
  __shared__ unsigned red[2][4][4];  // [lo / hi][wave][coordinate]
  unsigned lo[4] = {~0u, ~0u, ~0u, ~0u}, hi[4] = {0u, 0u, 0u, 0u};
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    for (int k = 0; k < d; ++k) {
      const float v = pts[i * d + k];
      if (!__builtin_isfinite(v)) continue;
      const unsigned o = ordered_bits(v);
      lo[k] = min(lo[k], o);
      hi[k] = max(hi[k], o);
    }
  }
  const int w = threadIdx.x >> 6;
  for (int k = 0; k < 4; ++k) {
    unsigned a = lo[k], b = hi[k];
    for (int off = 32; off > 0; off >>= 1) {
      a = min(a, (unsigned)__shfl_xor((int)a, off));
      b = max(b, (unsigned)__shfl_xor((int)b, off));
    }
    if (lane_id() == 0) {
      red[0][w][k] = a;
      red[1][w][k] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < d) {
    const int k = threadIdx.x;
    const unsigned a = min(min(red[0][0][k], red[0][1][k]), min(red[0][2][k], red[0][3][k]));
    const unsigned b = max(max(red[1][0][k], red[1][1][k]), max(red[1][2][k], red[1][3][k]));
    if (a != ~0u) atomicMin(&st->box_lo[k], a);
    if (b != 0u) atomicMax(&st->box_hi[k], b);
  }
}

__global__ __launch_bounds__(256) void k_order_keys(const float *__restrict__ pts, int n, int d,
                                                    const DevState *__restrict__ st,
                                                    unsigned *__restrict__ keys,
                                                    int *__restrict__ vals) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int bits = order_bits_per_coord(d);
  const unsigned qmax = (1u << bits) - 1u;
  unsigned code = 0;
  for (int k = 0; k < d; ++k) {
    const float lo = from_ordered(st->box_lo[k]);
    const float span = from_ordered(st->box_hi[k]) - lo;
    float t = 0.0f;
    if (span > 0.0f && __builtin_isfinite(span)) t = (pts[i * d + k] - lo) / span;
    const float qf = t * (float)qmax;
    // NaN (a non-finite coordinate) compares false and takes cell 0
    const unsigned q = (qf > 0.0f) ? (qf < (float)qmax ? (unsigned)qf : qmax) : 0u;
    for (int b = 0; b < bits; ++b) code |= ((q >> b) & 1u) << (b * d + k);
  }
  keys[i] = code;
  vals[i] = (int)i;
}

// Digit histogram of each tile: hist[tile * 256 + digit].
__global__ __launch_bounds__(256) void k_sort_hist(const unsigned *__restrict__ keys, int n,
                                                   int shift, int *__restrict__ hist, int ntiles) {
  __shared__ int h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const long long idx = base + it * 256 + tid;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(long long)blockIdx.x * 256 + tid] = h[tid];
}

// Turns the tile histograms into each tile's first output index per digit:
// hist[t][g] = (keys with a digit below g) + (keys with digit g in tiles
// before t).  One block; thread (segment s, digit g) owns digit g over a
// quarter of the tiles, so every load of the block is 1 KiB contiguous.
__global__ __launch_bounds__(1024) void k_sort_scan(int *__restrict__ hist, int ntiles) {
  __shared__ int seg[4][256];
  __shared__ int base[256];
  const int g = threadIdx.x & 255, sgm = threadIdx.x >> 8;
  const int per = (ntiles + 3) / 4;
  const int t0 = sgm * per, t1 = min(t0 + per, ntiles);
  int sum = 0;
#pragma unroll 8
  for (int t = t0; t < t1; ++t) sum += hist[(long long)t * 256 + g];
  seg[sgm][g] = sum;
  __syncthreads();
  if (sgm == 0) base[g] = seg[0][g] + seg[1][g] + seg[2][g] + seg[3][g];
  __syncthreads();
  // exclusive scan of the 256 digit totals (threads of segment 0)
  for (int off = 1; off < 256; off <<= 1) {
    const int v = (sgm == 0 && g >= off) ? base[g - off] : 0;
    __syncthreads();
    if (sgm == 0) base[g] += v;
    __syncthreads();
  }
  int run = (g ? base[g - 1] : 0);
  for (int k = 0; k < sgm; ++k) run += seg[k][g];
  // eight loads in flight at a time (the loop is bound by load latency)
  for (int t = t0; t < t1; t += 8) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = t + u < t1 ? hist[(long long)(t + u) * 256 + g] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (t + u < t1) hist[(long long)(t + u) * 256 + g] = run;
      run += v[u];
    }
  }
}

// Stable scatter of one pass.  A tile's keys are taken 256 at a time in
// index order; within a wave, the lanes with equal digits are found with 8
// ballots (one per digit bit), and a key's place is: the tile's global base
// for its digit + the keys of that digit in earlier rounds + those in earlier
// waves of this round + those in lower lanes of its wave.
__global__ __launch_bounds__(256) void k_sort_scatter(const unsigned *__restrict__ kin,
                                                      const int *__restrict__ vin,
                                                      unsigned *__restrict__ kout,
                                                      int *__restrict__ vout, int n, int shift,
                                                      const int *__restrict__ hist, int ntiles) {
  __shared__ int run[256];
  __shared__ int wcnt[4][256];
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  run[tid] = hist[(long long)blockIdx.x * 256 + tid];
#pragma unroll
  for (int k = 0; k < 4; ++k) wcnt[k][tid] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const long long idx = base + it * 256 + tid;
    const bool valid = idx < n;
    const unsigned key = valid ? kin[idx] : 0u;
    const int val = valid ? vin[idx] : 0;
    const unsigned dg = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = lanes_below(peers);
    if (valid && rank == 0) wcnt[w][dg] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[dg] + rank;
      for (int k = 0; k < w; ++k) pos += wcnt[k][dg];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
#pragma unroll
    for (int k = 0; k < 4; ++k) wcnt[k][tid] = 0;
    __syncthreads();
  }
}

// Nearest pivot of each point.  The ranking score of pivot p for point x is
// |p - c|^2 - 2 (x - c).(p - c) = |x - p|^2 - |x - c|^2, c = the first row
// (centring keeps BF16 products meaningful for data far from the origin);
// the dot products of 32 points with all NP pivots are 32 x 32 BF16
// matrix-core tiles (K = KS x 16 coordinates, zero-padded), pivot fragments
// staged in LDS.  Each lane keeps the best pivot of its 16 accumulator rows,
// and the 32 lanes that share a row reduce to the smallest score (lowest
// pivot on ties).  The pivots are rows p * n / NP of the input; the more
// pivots, the fewer clusters of the data go without one of their own (their
// points would scatter over other clusters' cells).  Only the order depends
// on this arithmetic, never a decision; a non-finite coordinate gives NaN
// scores and leaves the point in cell 0.
template <int KS>
constexpr int pivots_for() { return KS <= 4 ? 256 : 128; }

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 pbf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float pf32x16;

template <int KS>
__global__ __launch_bounds__(256) void k_order_pivots(const float *__restrict__ pts, int n, int d,
                                                      unsigned *__restrict__ keys,
                                                      int *__restrict__ vals) {
  constexpr int K = KS * 16, NP = pivots_for<KS>(), NT = NP / 32;
  // B fragments: [pivot tile][k step][lane] = coordinates 16 s + 8 (lane / 32)
  // .. + 7 of pivot 32 t + lane % 32
  __shared__ pbf16x8 frag[NT][KS][64];
  __shared__ float pnorm[NP];
  __shared__ float cref[K];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = tid; k < K; k += 256) cref[k] = k < d ? pts[k] : 0.0f;
  __syncthreads();
  // rows of d floats split in whole 16-byte pieces when d is a multiple of 8
  const bool vec = (d & 7) == 0 && (((uintptr_t)pts) & 15) == 0;
  auto chunk8 = [&](long long row, int k0) {  // coordinates k0 .. k0 + 7 of a row, centred
    float v[8];
    if (vec && k0 < d) {
      const float4 *src = (const float4 *)(pts + row * d + k0);
      const float4 x0 = src[0], x1 = src[1];
      v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
      v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k0 + u < d ? pts[row * d + k0 + u] : 0.0f;
    }
    pbf16x8 r;
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = (__bf16)(k0 + u < d ? v[u] - cref[k0 + u] : 0.0f);
    return r;
  };
  for (int e = tid; e < NP * K / 8; e += 256) {
    const int p = e / (K / 8), c8 = e - p * (K / 8);  // 8 coordinates 8 c8 .. + 7
    frag[p / 32][c8 / 2][(c8 & 1) * 32 + p % 32] = chunk8((long long)p * n / NP, 8 * c8);
  }
  __syncthreads();
  for (int p = tid; p < NP; p += 256) {
    float s2 = 0.0f;
    for (int c8 = 0; c8 < K / 8; ++c8) {
      const pbf16x8 v = frag[p / 32][c8 / 2][(c8 & 1) * 32 + p % 32];
#pragma unroll
      for (int u = 0; u < 8; ++u) s2 = __builtin_fmaf((float)v[u], (float)v[u], s2);
    }
    pnorm[p] = s2;
  }
  __syncthreads();
  // the grid strides over groups of 128 points (one per wave of 32), so the
  // pivot staging above is paid once per block
  for (long long grp = blockIdx.x; grp * 128 < n; grp += gridDim.x) {
    // this wave's 32 points: A fragments (row lane % 32, coordinates as above)
    const long long base = (grp * 4 + w) * 32;
    const long long myrow = base + (lane & 31);
    pbf16x8 a[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st)
      a[st] = myrow < n ? chunk8(myrow, 16 * st + 8 * (lane >> 5)) : pbf16x8{};
    float best[16];
    int arg[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      best[r] = __builtin_inff();
      arg[r] = 0;
    }
    for (int t = 0; t < NT; ++t) {
      pf32x16 acc = pf32x16{};
#pragma unroll
      for (int st = 0; st < KS; ++st)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[st], frag[t][st][lane], acc, 0, 0, 0);
      const int p = t * 32 + (lane & 31);
      const float pn = pnorm[p];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float sc = __builtin_fmaf(-2.0f, acc[r], pn);
        if (sc < best[r]) {
          best[r] = sc;
          arg[r] = p;
        }
      }
    }
    // accumulator r of lane l is point 8 (r / 4) + 4 (l / 32) + r % 4 of the
    // wave's 32, against pivot column l % 32: reduce over the 32 lanes of each
    // half-wave
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float b = best[r];
      int g = arg[r];
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) {
        const float ob = __shfl_xor(b, off);
        const int og = __shfl_xor(g, off);
        if (ob < b || (ob == b && og < g) || (b != b && ob == ob)) {
          b = ob;
          g = og;
        }
      }
      const long long i = base + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if ((lane & 31) == 0 && i < n) {
        keys[i] = (unsigned)g;
        vals[i] = (int)i;
      }
    }
  }
}

}  // namespace

int order_max_d() { return kPivotMaxD; }

long long order_hist_entries(long long n) { return 256 * ((n + kSortTile - 1) / kSortTile); }

hipError_t run_spatial_order(const float *pts, int n, int d, unsigned *keys[2], int *vals[2],
                             int *hist, DevState *st, int **perm, hipStream_t s) {
  if (d < 1 || d > kPivotMaxD || n < 1) return hipErrorInvalidValue;
  const int blocks = (n + 255) / 256;
  int passes = 1;
  if (d <= 4) {
    hipLaunchKernelGGL(k_order_box, dim3(blocks < kBoxBlocks ? blocks : kBoxBlocks), dim3(256), 0,
                       s, pts, n, d, st);
    hipLaunchKernelGGL(k_order_keys, dim3(blocks), dim3(256), 0, s, pts, n, d, st, keys[0],
                       vals[0]);
    passes = (order_bits_per_coord(d) * d + 7) / 8;
  } else {
    static_assert(pivots_for<1>() <= 256, "pivot index in one radix digit");
    const int groups = (n + 127) / 128;  // 32 points per wave
    const int pblocks = groups < kPivotBlocks ? groups : kPivotBlocks;
#define DBK_PIVOTS(KS)                                                                         \
  case KS:                                                                                     \
    hipLaunchKernelGGL(k_order_pivots<KS>, dim3(pblocks), dim3(256), 0, s, pts, n, d, keys[0], \
                       vals[0]);                                                               \
    break;
    switch ((d + 15) / 16) {
      DBK_PIVOTS(1)
      DBK_PIVOTS(2)
      DBK_PIVOTS(3)
      DBK_PIVOTS(4)
      DBK_PIVOTS(5)
      DBK_PIVOTS(6)
      DBK_PIVOTS(7)
      DBK_PIVOTS(8)
      default: return hipErrorInvalidValue;
    }
#undef DBK_PIVOTS
  }
  const int ntiles = (n + kSortTile - 1) / kSortTile;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(256), 0, s, keys[cur], n, shift, hist,
                       ntiles);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, hist, ntiles);
    hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(256), 0, s, keys[cur], vals[cur],
                       keys[cur ^ 1], vals[cur ^ 1], n, shift, hist, ntiles);
    cur ^= 1;
  }
  *perm = vals[cur];
  return hipGetLastError();
}

}  // namespace dbk

