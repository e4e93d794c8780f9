// Kernels shared by both forms: staging (the transposed coordinate layout of
// Section IV-A.2), core flags (Section II, definition 2; the `valid` vector of
// Section IV-B), compaction of non-core rows, the merge and border pass over
// the neighbour-pair list, and canonical labels.
#include "dbscan_device.h"
#include "dbscan_internal.h"
#include "bodies_common.h"

namespace dbk {

// ------------------------------------------------------------------ staging
__global__ void k_reset_state(DevState *st, unsigned pair_segs) {
  if (threadIdx.x < kPairSegments) st->edge_seg[threadIdx.x][0] = 0;
  if (threadIdx.x == 0) {
    st->pair_segs = pair_segs;
    st->status = 0;
    st->noncore = 0;
    st->band_pairs = 0;
    st->core_points = 0;
    st->core_degree = 0;
    st->edges = 0;
    st->band_list = 0;
    st->max_norm = 0;
    st->thr[0] = 0.0f;
    st->thr[1] = 0.0f;
    for (int k = 0; k < 4; ++k) {
      st->box_lo[k] = ~0u;
      st->box_hi[k] = 0u;
    }
    st->tests = 0;
  }
}

__global__ void k_stage(const float *__restrict__ pts, int n, int d, int n_pad, int d_pad,
                        float *__restrict__ soa, int *__restrict__ counts,
                        int *__restrict__ parent, int *__restrict__ jstar, DevState *st,
                        const int *__restrict__ perm, int *__restrict__ inv,
                        int *__restrict__ rootmin, float *__restrict__ hoist, double eps2) {
  stage_body(pts, n, d, n_pad, d_pad, soa, counts, parent, jstar, st, blockIdx.x, perm, inv,
             rootmin);
  // each thread reads back only the coordinates it wrote itself
  if (hoist) hoist_prep_body(soa, n, d, n_pad, eps2, hoist, st, blockIdx.x);
}

// ------------------------------------------------------------- core flags
__global__ void k_core(const int *__restrict__ counts, int n, int n_pad, int minpts,
                       uint8_t *__restrict__ core, uint32_t *__restrict__ corebits,
                       DevState *st, const int *__restrict__ perm, int *__restrict__ counts_out,
                       int count, int degree) {
  core_body(counts, n, n_pad, minpts, core, corebits, st, blockIdx.x, perm, counts_out,
            count != 0, degree != 0);
}

// Non-core rows into a list (any order) for the border pass that repeats the
// epsilon tests.  With `only_on_overflow` it runs only when the pair list
// overflowed (otherwise the pair list serves the border points).
__global__ void k_compact_noncore(const uint32_t *__restrict__ corebits, int n,
                                  int *__restrict__ list, DevState *st, int only_on_overflow) {
  if (only_on_overflow && !(__hip_atomic_load(&st->status, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) & kStatusEdgeOverflow))
    return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool nc = i < n && !((corebits[i >> 5] >> (i & 31)) & 1u);
  const uint64_t m = __ballot(nc);
  if (m == 0ull) return;
  const int lane = lane_id();
  int base = 0;
  if (lane == 0) base = (int)atomicAdd(&st->noncore, (unsigned)__popcll(m));
  base = __shfl(base, 0);
  if (nc) list[base + __popcll(m & ((1ull << lane) - 1ull))] = i;
}

// --------------------------------------------- merge + border from the list
// Skipped when the list overflowed (the repeated sweeps take over).
__global__ __launch_bounds__(256) void k_merge_list(const int2 *__restrict__ pairs,
                                                    const uint32_t *__restrict__ corebits,
                                                    int *__restrict__ parent,
                                                    int *__restrict__ jstar, DevState *st,
                                                    long long cap, const int *__restrict__ okey) {
  const unsigned status = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (status & kStatusEdgeOverflow) return;
  // segment of this block (the list is one segment when pair_segs <= 1)
  const unsigned S = st->pair_segs > 1u ? st->pair_segs : 1u;
  const unsigned sgm = blockIdx.x % S, part = blockIdx.x / S, parts = gridDim.x / S;
  if (part >= parts) return;
  const unsigned long long seg_cap = (unsigned long long)cap / S;
  unsigned long long total = __hip_atomic_load(S > 1u ? &st->edge_seg[sgm][0] : &st->edges,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (total > seg_cap) total = seg_cap;
  const unsigned long long per = (total + parts - 1) / parts;
  const unsigned long long b = (unsigned long long)part * per;
  const unsigned long long e = b + per < total ? b + per : total;
  merge_pairs_range(pairs + sgm * seg_cap, corebits, parent, jstar, b, e, okey);
}

// ------------------------------------------------------------------ labels
__global__ void k_rootmin(int n, const uint32_t *__restrict__ corebits, int *__restrict__ parent,
                          const int *__restrict__ perm, int *__restrict__ rootmin) {
  rootmin_body(n, corebits, parent, perm, rootmin, blockIdx.x);
}

__global__ void k_labels(int n, const uint32_t *__restrict__ corebits,
                         const int *__restrict__ jstar, int *__restrict__ parent,
                         int *__restrict__ labels, const DevState *st, const int *__restrict__ perm,
                         const int *__restrict__ inv, const int *__restrict__ rootmin) {
  labels_body(n, corebits, jstar, parent, labels, st, blockIdx.x, perm, inv, rootmin);
}

// ----------------------------------------------------- filter fallback
// The matrix-core path stages no float32 coordinates of its own.  When its
// filter gave up (inputs out of its range, or too many undecided pairs): clear
// the counts, stage the coordinates for the float32 sweep that redoes step 1,
// and mark the pair list incomplete so that step 3 repeats the tests.  When
// only the pair list ran out of room: stage the coordinates for the sweeps of
// step 3 that repeat the tests.
__global__ void k_filter_fallback(const float *__restrict__ pts, const int *__restrict__ perm,
                                  int n, int d, int n_pad, int d_pad, float *__restrict__ soa,
                                  int *__restrict__ counts, DevState *st) {
  const unsigned status =
      __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const bool filter_failed = (status & (kStatusRange | kStatusBandOverflow)) != 0u;
  if (!filter_failed && !(status & kStatusEdgeOverflow)) return;
  stage_soa_body(pts, n, d, n_pad, d_pad, soa, st, blockIdx.x, perm);
  if (!filter_failed) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counts[i] = 0;
  if (i == 0) atomicOr(&st->status, kStatusEdgeOverflow);
}

// --------------------------------------------------------- block boxes
// Box of each 64-point block of the staged coordinates (d <= 4): one wave per
// block, NaN padding ignored; an empty block gets lo = +inf, hi = -inf.
__global__ __launch_bounds__(256) void k_block_boxes(const float *__restrict__ soa, int n_pad,
                                                     int d, float *__restrict__ box) {
  const int nb = n_pad / 64;
  const int b = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (b >= nb) return;
  for (int k = 0; k < d; ++k) {
    const float v = soa[(size_t)k * n_pad + b * 64 + lane_id()];
    float l = v, h = v;
    for (int off = 32; off > 0; off >>= 1) {
      l = __builtin_fminf(l, __shfl_xor(l, off));
      h = __builtin_fmaxf(h, __shfl_xor(h, off));
    }
    if (lane_id() == 0) {
      box[(size_t)(2 * k) * nb + b] = (l == l) ? l : __builtin_inff();
      box[(size_t)(2 * k + 1) * nb + b] = (h == h) ? h : -__builtin_inff();
    }
  }
}

// ------------------------------------------------------------ host launchers
hipError_t run_block_boxes(const float *soa, int n_pad, int d, float *box, hipStream_t s) {
  const int nb = n_pad / 64;
  hipLaunchKernelGGL(k_block_boxes, dim3((nb + 3) / 4), dim3(256), 0, s, soa, n_pad, d, box);
  return hipGetLastError();
}

hipError_t run_reset(DevState *st, long long pair_cap, hipStream_t s) {
  // segments of at least 2^18 entries, so a small list is not split into
  // pieces that one block could fill
  long long segs = pair_cap >> 18;
  segs = segs < 1 ? 1 : (segs > kPairSegments ? kPairSegments : segs);
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, st, (unsigned)segs);
  return hipGetLastError();
}

hipError_t run_stage(const float *pts, int n, int d, int n_pad, int d_pad, float *soa, int *counts,
                     int *parent, int *jstar, DevState *st, const Order &ord, hipStream_t s,
                     float *hoist, double eps2) {
  if (hoist && (!soa || d > 4 || n_pad % 256 != 0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stage, dim3((n_pad + 255) / 256), dim3(256), 0, s, pts, n, d, n_pad, d_pad,
                     soa, counts, parent, jstar, st, ord.perm, ord.inv, ord.rootmin, hoist, eps2);
  return hipGetLastError();
}

hipError_t run_core(const int *counts, int n, int n_pad, int minpts, uint8_t *core,
                    uint32_t *corebits, DevState *st, const Order &ord, int *counts_out,
                    bool count, hipStream_t s, bool degree) {
  hipLaunchKernelGGL(k_core, dim3((n_pad + 255) / 256), dim3(256), 0, s, counts, n, n_pad, minpts,
                     core, corebits, st, ord.perm, counts_out, count ? 1 : 0, degree ? 1 : 0);
  return hipGetLastError();
}

hipError_t run_compact_noncore(const uint32_t *corebits, int n, int *list, DevState *st,
                               bool only_on_overflow, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_noncore, dim3((n + 255) / 256), dim3(256), 0, s, corebits, n, list,
                     st, only_on_overflow ? 1 : 0);
  return hipGetLastError();
}

hipError_t run_merge_list(const Buffers &b, long long cap, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_list, dim3(2048), dim3(256), 0, s, b.pairs, b.corebits, b.parent,
                     b.jstar, b.st, cap, b.okey);
  return hipGetLastError();
}

hipError_t run_filter_fallback(const float *pts, const int *perm, int n, int d, int n_pad,
                               int d_pad, float *soa, int *counts, DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_filter_fallback, dim3((n_pad + 255) / 256), dim3(256), 0, s, pts, perm, n,
                     d, n_pad, d_pad, soa, counts, st);
  return hipGetLastError();
}

hipError_t run_labels(int n, const uint32_t *corebits, const int *jstar, int *parent, int *labels,
                      const DevState *st, const Order &ord, hipStream_t s) {
  if (ord.perm)
    hipLaunchKernelGGL(k_rootmin, dim3((n + 255) / 256), dim3(256), 0, s, n, corebits, parent,
                       ord.perm, ord.rootmin);
  hipLaunchKernelGGL(k_labels, dim3((n + 255) / 256), dim3(256), 0, s, n, corebits, jstar, parent,
                     labels, st, ord.perm, ord.inv, ord.rootmin);
  return hipGetLastError();
}

}  // namespace dbk
