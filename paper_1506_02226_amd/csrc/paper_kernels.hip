// The paper's own three-step design (Sections IV-A to IV-C, VI), kept beside
// the main path as measured ablations (include/dbscan_paper.h).
//
// Step 1 writes the n x n float distance matrix with the four kernels of
// Table III; step 2 writes the byte cluster matrix and the valid vector from
// it, or fused with the distance, or fused with the hoisted form of Section
// IV-B.2; step 3 merges primitive clusters by targets (Section IV-C) or by
// the Warshall closure of Section VI.  One wave per block (64 threads, and
// 64-point LDS tiles): at the paper's sizes (n = 5,061 to 60,032) a thread
// per row then still gives n / 64 = 80 to 938 work-groups for 256 CUs.
//
// The cluster matrix decides every pair as the float64 definition does:
// float32 values inside a rigorous band around eps^2 are re-evaluated in
// float64 from the input coordinates (dbscan_device.h), as on the main path.
#include <math.h>
#include <string.h>

#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/dbscan.h"
#include "../../include/dbscan_paper.h"
#include "dbscan_device.h"

namespace dbk {
namespace paper {

constexpr int kTpb = 64;  // threads per block = points per LDS tile

// float32 squared distance, coordinate order, each operation rounded alone
// (the matrix the distance kernels write).
template <int D>
__device__ __forceinline__ float dist_direct(const float (&a)[D], const float (&b)[D]) {
#pragma clang fp contract(off)
  float t = a[0] - b[0];
  float s = t * t;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    t = a[k] - b[k];
    const float tt = t * t;
    s = s + tt;
  }
  return s;
}

// ------------------------------------------------------------- preparation
// point[d][n] (Section IV-A.2's transposed point matrix) and, for the
// hoisted form, P[j] = |p_j|^2 in float32 and its maximum (bit pattern of a
// non-negative float, so unsigned order is float order).
template <int D>
__global__ __launch_bounds__(256) void k_prep(const float *__restrict__ pts, int n,
                                              float *__restrict__ soa, float *__restrict__ P,
                                              unsigned *__restrict__ pmax) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  float p = 0.0f;
  if (j < n) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const float x = pts[(size_t)j * D + k];
      soa[(size_t)k * n + j] = x;
      s = __builtin_fmaf(x, x, s);
    }
    P[j] = s;
    p = s;
  }
  for (int off = 32; off > 0; off >>= 1) p = __builtin_fmaxf(p, __shfl_xor(p, off));
  if ((threadIdx.x & 63) == 0) atomicMax(pmax, __float_as_uint(p));
}

// ----------------------------------------------------------- step 1 kernels
// Baseline: thread i fills row i, reading every point from the row-major
// point matrix; lanes write addresses n floats apart.
template <int D>
__global__ __launch_bounds__(kTpb) void k_dist_baseline(const float *__restrict__ pts, int n,
                                                        float *__restrict__ dist) {
  const int i = blockIdx.x * kTpb + threadIdx.x;
  if (i >= n) return;
  float a[D];
#pragma unroll
  for (int k = 0; k < D; ++k) a[k] = pts[(size_t)i * D + k];
  float *row = dist + (size_t)i * n;
#pragma unroll 1
  for (int j = 0; j < n; ++j) {
    float b[D];
#pragma unroll
    for (int k = 0; k < D; ++k) b[k] = pts[(size_t)j * D + k];
    row[j] = dist_direct<D>(a, b);
  }
}

// Coalesced: transposed points, thread i fills column i (the matrix is
// symmetric), so the lanes of a wave write consecutive addresses.
template <int D>
__global__ __launch_bounds__(kTpb) void k_dist_coalesced(const float *__restrict__ soa, int n,
                                                         float *__restrict__ dist) {
  const int i = blockIdx.x * kTpb + threadIdx.x;
  if (i >= n) return;
  float a[D];
#pragma unroll
  for (int k = 0; k < D; ++k) a[k] = soa[(size_t)k * n + i];
#pragma unroll 1
  for (int j = 0; j < n; ++j) {
    float b[D];
#pragma unroll
    for (int k = 0; k < D; ++k) b[k] = soa[(size_t)k * n + j];
    dist[(size_t)j * n + i] = dist_direct<D>(a, b);
  }
}

// Shared memory: the block stages 64 points at a time in LDS and each thread
// keeps its goal point in registers; UNROLL unrolls the inner loop 32 times.
template <int D, bool UNROLL>
__global__ __launch_bounds__(kTpb) void k_dist_shared(const float *__restrict__ soa, int n,
                                                      float *__restrict__ dist) {
  __shared__ float tile[D][kTpb];
  const int i = blockIdx.x * kTpb + threadIdx.x;
  const bool live = i < n;
  float a[D];
#pragma unroll
  for (int k = 0; k < D; ++k) a[k] = live ? soa[(size_t)k * n + i] : 0.0f;
  for (int j0 = 0; j0 < n; j0 += kTpb) {
    const int j = j0 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < D; ++k) tile[k][threadIdx.x] = j < n ? soa[(size_t)k * n + j] : 0.0f;
    __syncthreads();
    const int m = n - j0 < kTpb ? n - j0 : kTpb;
    if (live) {
      float *col = dist + (size_t)j0 * n + i;
      if constexpr (UNROLL) {
        if (m == kTpb) {
#pragma unroll 32
          for (int q = 0; q < kTpb; ++q) {
            float b[D];
#pragma unroll
            for (int k = 0; k < D; ++k) b[k] = tile[k][q];
            col[(size_t)q * n] = dist_direct<D>(a, b);
          }
        } else {
#pragma unroll 1
          for (int q = 0; q < m; ++q) {
            float b[D];
#pragma unroll
            for (int k = 0; k < D; ++k) b[k] = tile[k][q];
            col[(size_t)q * n] = dist_direct<D>(a, b);
          }
        }
      } else {
#pragma unroll 1
        for (int q = 0; q < m; ++q) {
          float b[D];
#pragma unroll
          for (int k = 0; k < D; ++k) b[k] = tile[k][q];
          col[(size_t)q * n] = dist_direct<D>(a, b);
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------- step 2 kernels
// Float32 neighbours of a positive finite double: the largest float <= v and
// the smallest float >= v (stepping the bit pattern once when the
// conversion rounded the wrong way).
__device__ __forceinline__ float round_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = __uint_as_float(__float_as_uint(f) - 1u);
  return f;
}
__device__ __forceinline__ float round_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}

// One pair's decision: float32 value v against the band [lo, hi], float64
// re-evaluation inside it.
template <int D>
__device__ __forceinline__ bool decide(float v, float lo, float hi, const float (&a)[D],
                                       const float (&b)[D], double eps2, unsigned &rech) {
  if (v <= lo) return true;
  if (!(v <= hi)) return false;
  ++rech;
  return exact_within<D>(a, b, eps2);
}

// From the distance matrix: thread t fills column t of the cluster matrix
// (coalesced reads and byte writes across the wave) and counts it.
template <int D>
__global__ __launch_bounds__(kTpb) void k_cluster_from_dist(
    const float *__restrict__ dist, const float *__restrict__ soa, int n, float lo, float hi,
    double eps2, int minpts, uint8_t *__restrict__ cluster, uint8_t *__restrict__ valid,
    int *__restrict__ counts, unsigned long long *__restrict__ rechecked) {
  const int t = blockIdx.x * kTpb + threadIdx.x;
  if (t >= n) return;
  float a[D];
#pragma unroll
  for (int k = 0; k < D; ++k) a[k] = soa[(size_t)k * n + t];
  int cnt = 0;
  unsigned rech = 0;
  for (int j = 0; j < n; ++j) {
    const float v = dist[(size_t)j * n + t];
    bool in = v <= lo;
    if (!in && v <= hi) {
      float b[D];
#pragma unroll
      for (int k = 0; k < D; ++k) b[k] = soa[(size_t)k * n + j];
      ++rech;
      in = exact_within<D>(a, b, eps2);
    }
    cluster[(size_t)j * n + t] = in ? 1 : 0;
    cnt += in ? 1 : 0;
  }
  counts[t] = cnt;
  valid[t] = cnt >= minpts ? 1 : 0;
  if (rech) atomicAdd(rechecked, (unsigned long long)rech);
}

// Fused (Section IV-B.1): the unrolled LDS-tiled distance kernel writes the
// cluster matrix instead of the distance.  HOISTED: the distance is
// T + P[n] - (X p_x + Y p_y + Z p_z) (Section IV-B.2) with T and X = 2 t
// taken once per thread and P[n] once per staged point, decided against
// per-row thresholds lo_i / hi_i that bound that form's rounding error.
template <int D, bool HOISTED>
__global__ __launch_bounds__(kTpb) void k_cluster_fused(
    const float *__restrict__ soa, const float *__restrict__ P,
    const unsigned *__restrict__ pmax_bits, int n, float lo, float hi, double eps2, int minpts,
    uint8_t *__restrict__ cluster, uint8_t *__restrict__ valid, int *__restrict__ counts,
    unsigned long long *__restrict__ rechecked) {
  __shared__ float tile[D + 1][kTpb];
  const int i = blockIdx.x * kTpb + threadIdx.x;
  const bool live = i < n;
  float a[D], X[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    a[k] = live ? soa[(size_t)k * n + i] : 0.0f;
    X[k] = 2.0f * a[k];  // exact
  }
  float T = 0.0f;
  if constexpr (HOISTED) {
#pragma unroll
    for (int k = 0; k < D; ++k) T = __builtin_fmaf(a[k], a[k], T);
    // |s~ - S| <= c (T* + P*) + tiny with T*, P* the exact squared norms:
    // the float32 norms and the dot product of X and p (X exact) each err by
    // at most gamma_D (T* + P*) (2 |t.p| <= T* + P*), the sum T + P and the
    // final subtraction by u times at most 2 (T* + P*) each, so
    // c = (2 gamma_D + 4u) plus slack; T* + P* <= (T + Pmax) / (1 - gamma_D).
    // The float64 definition decides "in" when S <= eps2 (1 - 2 g64) and
    // "out" when S > eps2 (1 + 2 g64), g64 = (D + 2) 2^-53.
    const double u = 0x1p-24, gD = D * u / (1.0 - D * u);
    const double c = (2.0 * gD + 8.0 * u) * (1.0 + 1e-6);
    const double pm = (double)__uint_as_float(*pmax_bits);
    const double E = c * ((double)T + pm) / (1.0 - gD) + (8.0 * D + 8.0) * 0x1p-149;
    const double g64 = (D + 2) * 0x1p-53;
    const double l = eps2 * (1.0 - 2.0 * g64) - E, h = eps2 * (1.0 + 2.0 * g64) + E;
    lo = l > 0.0 ? round_down(l) : -__builtin_inff();
    hi = round_up(h);
  }
  int cnt = 0;
  unsigned rech = 0;
  for (int j0 = 0; j0 < n; j0 += kTpb) {
    const int j = j0 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < D; ++k) tile[k][threadIdx.x] = j < n ? soa[(size_t)k * n + j] : 0.0f;
    if constexpr (HOISTED) tile[D][threadIdx.x] = j < n ? P[j] : 0.0f;
    __syncthreads();
    const int m = n - j0 < kTpb ? n - j0 : kTpb;
    if (live) {
      uint8_t *col = cluster + (size_t)j0 * n + i;
      auto one = [&](int q) {
        float b[D];
#pragma unroll
        for (int k = 0; k < D; ++k) b[k] = tile[k][q];
        float v;
        if constexpr (HOISTED) {
          float dot = X[0] * b[0];
#pragma unroll
          for (int k = 1; k < D; ++k) dot = __builtin_fmaf(X[k], b[k], dot);
          v = (T + tile[D][q]) - dot;
        } else {
          v = dist_direct<D>(a, b);
        }
        const bool in = decide<D>(v, lo, hi, a, b, eps2, rech);
        col[(size_t)q * n] = in ? 1 : 0;
        cnt += in ? 1 : 0;
      };
      if (m == kTpb) {
#pragma unroll 32
        for (int q = 0; q < kTpb; ++q) one(q);
      } else {
#pragma unroll 1
        for (int q = 0; q < m; ++q) one(q);
      }
    }
    __syncthreads();
  }
  if (live) {
    counts[i] = cnt;
    valid[i] = cnt >= minpts ? 1 : 0;
  }
  if (rech) atomicAdd(rechecked, (unsigned long long)rech);
}

// ----------------------------------------------------------- step 3 kernels
// Target merge (Section IV-C): block c tries to merge valid cluster c into
// target t.  They merge when their rows share a core point; the merge sets
// to 1 every element of row t where row c holds a 1 (elements only ever go
// from 0 to 1, so blocks merging into the same target at once need neither
// atomics nor ordering) and invalidates c.
__global__ __launch_bounds__(256) void k_merge_target(uint8_t *__restrict__ cluster,
                                                      const uint8_t *__restrict__ core,
                                                      uint8_t *__restrict__ alive, int n, int t,
                                                      int *__restrict__ changed) {
  const int c = blockIdx.x;
  if (c == t || !alive[c]) return;
  const uint8_t *rc = cluster + (size_t)c * n;
  uint8_t *rt = cluster + (size_t)t * n;
  // row t is read and set here by several blocks at once: relaxed byte
  // atomics (plain byte loads and stores on the device) make that defined
  bool hit = false;
  for (int k = threadIdx.x; k < n; k += 256) {
    const uint8_t v = __hip_atomic_load(rt + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hit |= (rc[k] & core[k] & v) != 0;
  }
  if (!__syncthreads_or(hit)) return;
  for (int k = threadIdx.x; k < n; k += 256)
    if (rc[k]) __hip_atomic_store(rt + k, (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) {
    alive[c] = 0;
    *changed = 1;
  }
}

// Core points take the surviving target whose row holds them.
__global__ __launch_bounds__(256) void k_labels_targets(const uint8_t *__restrict__ cluster,
                                                        const uint8_t *__restrict__ core,
                                                        const uint8_t *__restrict__ alive, int n,
                                                        int *__restrict__ labels) {
  const int t = blockIdx.x;
  if (!alive[t]) return;
  const uint8_t *rt = cluster + (size_t)t * n;
  for (int k = threadIdx.x; k < n; k += 256)
    if (rt[k] && core[k]) labels[k] = t;
}

__global__ __launch_bounds__(256) void k_labels_fill(int n, int *__restrict__ labels) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n) labels[j] = -1;
}

// A non-core point takes the label of its lowest-index core neighbour, found
// in its own (never merged) row of the cluster matrix.
__global__ __launch_bounds__(256) void k_labels_border(const uint8_t *__restrict__ cluster,
                                                       const uint8_t *__restrict__ core, int n,
                                                       int *__restrict__ labels) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n || core[j]) return;
  const uint8_t *rj = cluster + (size_t)j * n;
  int lab = -1;
  for (int k = 0; k < n; ++k)
    if (rj[k] && core[k]) {
      lab = labels[k];
      break;
    }
  labels[j] = lab;
}

// Warshall (Section VI): R = core-core relation as rows of 32-bit words;
// step k sets R[i] |= R[k] for every row i that holds bit k.  Row k itself
// is skipped (R[k] |= R[k] changes nothing), so a launch reads row k while
// it writes only other rows.
__global__ __launch_bounds__(256) void k_warshall_init(const uint8_t *__restrict__ cluster,
                                                       const uint8_t *__restrict__ core, int n,
                                                       int words, uint32_t *__restrict__ R) {
  const int w = blockIdx.y * 256 + threadIdx.x;
  const int i = blockIdx.x;
  if (w >= words) return;
  uint32_t v = 0;
  if (core[i]) {
    const uint8_t *ri = cluster + (size_t)i * n;
    for (int b = 0; b < 32; ++b) {
      const int j = 32 * w + b;
      if (j < n && ri[j] && core[j]) v |= 1u << b;
    }
  }
  R[(size_t)i * words + w] = v;
}

__global__ __launch_bounds__(64) void k_warshall_step(uint32_t *__restrict__ R, int n, int words,
                                                      int k) {
  const int i = blockIdx.x;
  if (i == k) return;
  uint32_t *ri = R + (size_t)i * words;
  if (!((ri[k >> 5] >> (k & 31)) & 1u)) return;
  const uint32_t *rk = R + (size_t)k * words;
  for (int w = threadIdx.x; w < words; w += 64) ri[w] |= rk[w];
}

// Core point i: the lowest set bit of its closed row (the row holds i).
__global__ __launch_bounds__(256) void k_labels_warshall(const uint32_t *__restrict__ R,
                                                         const uint8_t *__restrict__ core, int n,
                                                         int words, int *__restrict__ labels) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (!core[i]) {
    labels[i] = -1;
    return;
  }
  const uint32_t *ri = R + (size_t)i * words;
  int lab = i;
  for (int w = 0; w < words; ++w)
    if (ri[w]) {
      lab = 32 * w + __builtin_ctz(ri[w]);
      break;
    }
  labels[i] = lab;
}

// ------------------------------------------------------------------ host
struct Prep {
  float *soa = nullptr, *P = nullptr;
  unsigned *pmax = nullptr;
  unsigned long long *rech = nullptr;
  char *base = nullptr;
};

hipError_t prep(const float *pts, int n, int d, Prep &p, hipStream_t s) {
  const size_t soa_b = ((size_t)d * n * 4 + 255) / 256 * 256;
  const size_t P_b = ((size_t)n * 4 + 255) / 256 * 256;
  hipError_t e = hipMallocAsync((void **)&p.base, soa_b + P_b + 256, s);
  if (e != hipSuccess) return e;
  p.soa = (float *)p.base;
  p.P = (float *)(p.base + soa_b);
  p.pmax = (unsigned *)(p.base + soa_b + P_b);
  p.rech = (unsigned long long *)(p.base + soa_b + P_b + 64);
  e = hipMemsetAsync(p.pmax, 0, 128, s);
  if (e != hipSuccess) return e;
  const dim3 g((n + 255) / 256);
  switch (d) {
    case 1: hipLaunchKernelGGL(k_prep<1>, g, dim3(256), 0, s, pts, n, p.soa, p.P, p.pmax); break;
    case 2: hipLaunchKernelGGL(k_prep<2>, g, dim3(256), 0, s, pts, n, p.soa, p.P, p.pmax); break;
    case 3: hipLaunchKernelGGL(k_prep<3>, g, dim3(256), 0, s, pts, n, p.soa, p.P, p.pmax); break;
    default: hipLaunchKernelGGL(k_prep<4>, g, dim3(256), 0, s, pts, n, p.soa, p.P, p.pmax);
  }
  return hipGetLastError();
}

template <int D>
void launch_distance(int kernel, const float *pts, const float *soa, int n, float *dist,
                     hipStream_t s) {
  const dim3 g((n + kTpb - 1) / kTpb), b(kTpb);
  switch (kernel) {
    case DBSCAN_PAPER_DIST_BASELINE: hipLaunchKernelGGL(k_dist_baseline<D>, g, b, 0, s, pts, n, dist); break;
    case DBSCAN_PAPER_DIST_COALESCED: hipLaunchKernelGGL(k_dist_coalesced<D>, g, b, 0, s, soa, n, dist); break;
    case DBSCAN_PAPER_DIST_SHARED: hipLaunchKernelGGL((k_dist_shared<D, false>), g, b, 0, s, soa, n, dist); break;
    default: hipLaunchKernelGGL((k_dist_shared<D, true>), g, b, 0, s, soa, n, dist);
  }
}

template <int D>
void launch_cluster(int kernel, const float *dist, const Prep &p, int n, float lo, float hi,
                    double eps2, int minpts, uint8_t *cluster, uint8_t *valid, int *counts,
                    hipStream_t s) {
  const dim3 g((n + kTpb - 1) / kTpb), b(kTpb);
  switch (kernel) {
    case DBSCAN_PAPER_CLUSTER_FROM_DIST:
      hipLaunchKernelGGL(k_cluster_from_dist<D>, g, b, 0, s, dist, p.soa, n, lo, hi, eps2, minpts,
                         cluster, valid, counts, p.rech);
      break;
    case DBSCAN_PAPER_CLUSTER_FUSED:
      hipLaunchKernelGGL((k_cluster_fused<D, false>), g, b, 0, s, p.soa, p.P, p.pmax, n, lo, hi,
                         eps2, minpts, cluster, valid, counts, p.rech);
      break;
    default:
      hipLaunchKernelGGL((k_cluster_fused<D, true>), g, b, 0, s, p.soa, p.P, p.pmax, n, lo, hi,
                         eps2, minpts, cluster, valid, counts, p.rech);
  }
}

int fail(hipError_t e) {
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? DBSCAN_E_NOMEM : DBSCAN_E_DEVICE;
}

}  // namespace paper
}  // namespace dbk

using namespace dbk::paper;

extern "C" {

int dbscan_paper_distance(const float *points, int64_t n, int32_t d, int32_t kernel, float *dist,
                          void *stream) {
  if (!points || !dist || n < 1 || n > DBSCAN_PAPER_MAX_N || d < 1 || d > 4) return DBSCAN_E_INVAL;
  if (kernel < DBSCAN_PAPER_DIST_BASELINE || kernel > DBSCAN_PAPER_DIST_UNROLLED)
    return DBSCAN_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int ni = (int)n;
  Prep p;
  hipError_t e = hipSuccess;
  if (kernel != DBSCAN_PAPER_DIST_BASELINE) {
    e = prep(points, ni, d, p, s);
    if (e != hipSuccess) return fail(e);
  }
  switch (d) {
    case 1: launch_distance<1>(kernel, points, p.soa, ni, dist, s); break;
    case 2: launch_distance<2>(kernel, points, p.soa, ni, dist, s); break;
    case 3: launch_distance<3>(kernel, points, p.soa, ni, dist, s); break;
    default: launch_distance<4>(kernel, points, p.soa, ni, dist, s);
  }
  e = hipGetLastError();
  if (p.base) {
    const hipError_t f = hipFreeAsync(p.base, s);
    if (e == hipSuccess) e = f;
  }
  return e == hipSuccess ? DBSCAN_OK : fail(e);
}

int dbscan_paper_cluster(const float *points, const float *dist, int64_t n, int32_t d,
                         double eps, int32_t minpts, int32_t kernel, uint8_t *cluster,
                         uint8_t *valid, int32_t *counts, uint64_t *rechecked, void *stream) {
  if (!points || !cluster || !valid || !counts || n < 1 || n > DBSCAN_PAPER_MAX_N || d < 1 ||
      d > 4 || minpts < 1 || !(eps >= 0.0) || !isfinite(eps))
    return DBSCAN_E_INVAL;
  if (kernel < DBSCAN_PAPER_CLUSTER_FROM_DIST || kernel > DBSCAN_PAPER_CLUSTER_HOISTED)
    return DBSCAN_E_INVAL;
  if ((kernel == DBSCAN_PAPER_CLUSTER_FROM_DIST) != (dist != nullptr)) return DBSCAN_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int ni = (int)n;
  const double eps2 = eps * eps;
  float lo = 0.0f, hi = 0.0f;
  dbscan_fp32_band(eps2, d, &lo, &hi);
  Prep p;
  hipError_t e = prep(points, ni, d, p, s);
  if (e != hipSuccess) return fail(e);
  switch (d) {
    case 1: launch_cluster<1>(kernel, dist, p, ni, lo, hi, eps2, minpts, cluster, valid, counts, s); break;
    case 2: launch_cluster<2>(kernel, dist, p, ni, lo, hi, eps2, minpts, cluster, valid, counts, s); break;
    case 3: launch_cluster<3>(kernel, dist, p, ni, lo, hi, eps2, minpts, cluster, valid, counts, s); break;
    default: launch_cluster<4>(kernel, dist, p, ni, lo, hi, eps2, minpts, cluster, valid, counts, s);
  }
  e = hipGetLastError();
  unsigned long long rech = 0;
  if (e == hipSuccess && rechecked)
    e = hipMemcpyAsync(&rech, p.rech, sizeof(rech), hipMemcpyDeviceToHost, s);
  const hipError_t f = hipFreeAsync(p.base, s);
  if (e == hipSuccess) e = f;
  if (e == hipSuccess && rechecked) {
    e = hipStreamSynchronize(s);
    *rechecked = rech;
  }
  return e == hipSuccess ? DBSCAN_OK : fail(e);
}

int dbscan_paper_merge(uint8_t *cluster, const uint8_t *valid, int64_t n, int32_t kernel,
                       int32_t *labels, uint8_t *alive_out, int64_t *launches, void *stream) {
  if (!cluster || !valid || !labels || n < 1 || n > DBSCAN_PAPER_MAX_N) return DBSCAN_E_INVAL;
  if (kernel != DBSCAN_PAPER_MERGE_TARGETS && kernel != DBSCAN_PAPER_MERGE_WARSHALL)
    return DBSCAN_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int ni = (int)n;
  int64_t nl = 0;
  hipError_t e = hipSuccess;
  const dim3 g256((ni + 255) / 256);
  if (kernel == DBSCAN_PAPER_MERGE_TARGETS) {
    char *base = nullptr;
    const size_t alive_b = ((size_t)ni + 255) / 256 * 256;
    e = hipMallocAsync((void **)&base, alive_b + 256, s);
    if (e != hipSuccess) return fail(e);
    uint8_t *alive = (uint8_t *)base;
    int *changed = (int *)(base + alive_b);
    std::vector<uint8_t> h_alive((size_t)ni);
    // every valid primitive cluster starts alive
    e = hipMemcpyAsync(alive, valid, (size_t)ni, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_alive.data(), alive, (size_t)ni, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int t = 0; t < ni && e == hipSuccess; ++t) {
      if (!h_alive[t]) continue;
      int h_changed = 1;
      while (h_changed && e == hipSuccess) {
        e = hipMemsetAsync(changed, 0, sizeof(int), s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_merge_target, dim3(ni), dim3(256), 0, s, cluster, valid, alive, ni,
                           t, changed);
        ++nl;
        e = hipGetLastError();
        if (e == hipSuccess)
          e = hipMemcpyAsync(&h_changed, changed, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(h_alive.data(), alive, (size_t)ni, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_labels_fill, g256, dim3(256), 0, s, ni, labels);
      hipLaunchKernelGGL(k_labels_targets, dim3(ni), dim3(256), 0, s, cluster, valid, alive, ni,
                         labels);
      hipLaunchKernelGGL(k_labels_border, g256, dim3(256), 0, s, cluster, valid, ni, labels);
      nl += 3;
      e = hipGetLastError();
    }
    if (e == hipSuccess && alive_out)
      e = hipMemcpyAsync(alive_out, alive, (size_t)ni, hipMemcpyDeviceToDevice, s);
    const hipError_t f = hipFreeAsync(base, s);
    if (e == hipSuccess) e = f;
  } else {
    const int words = (ni + 31) / 32;
    uint32_t *R = nullptr;
    e = hipMallocAsync((void **)&R, (size_t)ni * words * 4, s);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(k_warshall_init, dim3(ni, (words + 255) / 256), dim3(256), 0, s, cluster,
                       valid, ni, words, R);
    ++nl;
    for (int k = 0; k < ni; ++k) {
      hipLaunchKernelGGL(k_warshall_step, dim3(ni), dim3(64), 0, s, R, ni, words, k);
      ++nl;
    }
    hipLaunchKernelGGL(k_labels_warshall, g256, dim3(256), 0, s, R, valid, ni, words, labels);
    hipLaunchKernelGGL(k_labels_border, g256, dim3(256), 0, s, cluster, valid, ni, labels);
    nl += 2;
    e = hipGetLastError();
    const hipError_t f = hipFreeAsync(R, s);
    if (e == hipSuccess) e = f;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (launches) *launches = nl;
  return e == hipSuccess ? DBSCAN_OK : fail(e);
}

}  // extern "C"
