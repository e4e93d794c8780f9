// Spatial order of the points (d <= 4): a permutation that puts points close
// in space at close indices, applied when the coordinates are staged.  The
// epsilon tests are unchanged -- every pair is still tested (Section IV-A),
// with the same float32 filter and float64 re-evaluation -- but the rare
// neighbour pairs gather into few tiles, so the sweeps take their rare branch
// far less often and the bitmask's non-zero words sit near its diagonal.  The
// outputs are returned in the caller's order and labels stay canonical in the
// caller's indices (the label passes map through the permutation).
//
// Key of a point: its coordinates quantised over the bounding box of the
// input (bits_per_coord(d) bits each) and interleaved bit by bit (Morton
// order).  The permutation is the stable LSD radix sort of the keys, 8 bits
// per pass; ties keep input order, so the permutation is deterministic.
#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

namespace {

constexpr int kSortItems = 8;                 // keys per thread per tile
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
  for (int t = t0; t < t1; ++t) {
    const long long e = (long long)t * 256 + g;
    const int v = hist[e];
    hist[e] = run;
    run += v;
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

}  // namespace

long long order_hist_entries(long long n) { return 256 * ((n + kSortTile - 1) / kSortTile); }

hipError_t run_spatial_order(const float *pts, int n, int d, unsigned *keys[2], int *vals[2],
                             int *hist, DevState *st, int **perm, hipStream_t s) {
  if (d < 1 || d > 4 || n < 1) return hipErrorInvalidValue;
  const int blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_order_box, dim3(blocks < kBoxBlocks ? blocks : kBoxBlocks), dim3(256), 0, s,
                     pts, n, d, st);
  hipLaunchKernelGGL(k_order_keys, dim3(blocks), dim3(256), 0, s, pts, n, d, st, keys[0], vals[0]);
  const int ntiles = (n + kSortTile - 1) / kSortTile;
  const int passes = (order_bits_per_coord(d) * d + 7) / 8;
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
