// Matrix-core filter for d >= 16 (gfx950 MFMA, BF16 or FP16 inputs, FP32
// accumulation).
//
// Section IV-B.2 hoists the terms that depend on one point only out of the
// inner loop: dist(t, p) = T + P[n] - (X p_x + Y p_y + Z p_z) with T = |t|^2,
// P[n] = |p|^2 and (X, Y, Z) = 2t.  Here the same expansion,
// |x_i|^2 + |x_j|^2 - 2 x_i.x_j, is evaluated for 32x32 tiles of pairs on the
// matrix cores: each accumulator starts at n_i (the FP32 squared norm of the
// rounded row point, the hoisted T), the contraction of
//   a_i = [x~_i, 0...],  b_j = [-2 x~_j, 0...]  (K = d rounded up to 16)
// is added onto it, and the column's n_j (P[n]) is added to the result, so
// that s~ = n_i - 2 x~_i.x~_j + n_j (x~ = x rounded to BF16/FP16).  The result is only a filter: with the rigorous bounds of
// k_mfma_thresholds a pair is "in" when s~ <= T_lo, "out" when s~ > T_hi, and
// every pair in between is queued and re-decided in float64 from the FP32
// inputs with the definition's own arithmetic (k_recheck_band).  Decisions,
// and so counts, core flags and labels, equal the float64 definition.
//
// Tile loop: a work-group of 4 waves owns 256 stationary columns (64 per wave:
// two 32-column MFMA tiles whose b-fragments stay in registers) and sweeps a
// chunk of 32-row tiles whose a-fragments are staged in LDS (double buffered,
// shared by the 4 waves).  Per tile pair a wave issues 2 x K/16 MFMAs
// (v_mfma_f32_32x32x16_{bf16,f16}) and one min-reduction per accumulator;
// the rare accumulators holding "in" or band pairs take a branch that counts
// (per lane: lane l holds column l%32), queues neighbour pairs i > j for the
// merge and queues band pairs for the float64 pass.  The relation is
// symmetric, so a group sweeps only the row tiles from its own columns on:
// below the 256x256 diagonal zone each pair is tested once and counted for
// both ends (the row side from a ballot per accumulator register).
#include "dbscan_device.h"
#include "dbscan_internal.h"
#include "bodies_mfma.h"

namespace dbk {

// ---------------------------------------------------------------- prepare
template <typename T>
__global__ void k_mfma_prep(const float *__restrict__ pts, int n, int d, int n_pad, int K,
                            T *__restrict__ a_aug, T *__restrict__ b_aug, DevState *st,
                            const int *__restrict__ perm) {
  mfma_prep_body<T>(pts, n, d, n_pad, K, a_aug, b_aug, st, blockIdx.x, perm);
}

// ------------------------------------------------------------- thresholds
template <typename T>
__global__ void k_mfma_thresholds(DevState *st, double eps2, int d, int K, double band_rel) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  mfma_thresholds_body<T>(st, eps2, d, K, band_rel);
}

// ------------------------------------------------------------ tile sweep
template <typename T, int KS>
__global__ __launch_bounds__(256) void k_mfma_count(const T *__restrict__ a_aug,
                                                    const T *__restrict__ b_aug,
                                                    int *__restrict__ counts,
                                                    int2 *__restrict__ pairs,
                                                    int2 *__restrict__ band,
                                                    DevState *__restrict__ st, MfmaScalars sc) {
  __shared__ MfmaLds<KS> lds;
  // consecutive work-groups are dealt round-robin to the 8 XCDs: renumber
  // them so that each XCD runs one contiguous range of items (rows shared in
  // its L2)
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned per = nb / 8, rem = nb % 8, x = b % 8, q = b / 8;
  const unsigned item = x < rem ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
  mfma_count_body<T, KS>(a_aug, b_aug, counts, pairs, band, st, sc, (int)item, lds);
}

// ------------------------------------------------------- float64 band pass
__global__ __launch_bounds__(256) void k_recheck_band(const float *__restrict__ pts, int d,
                                                      const int2 *__restrict__ band,
                                                      int *__restrict__ counts,
                                                      int2 *__restrict__ pairs,
                                                      DevState *__restrict__ st, double eps2,
                                                      long long band_cap, long long pair_cap,
                                                      const int *__restrict__ perm) {
  __shared__ int2 qbuf[4][128];
  const unsigned status =
      __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (status & (kStatusRange | kStatusBandOverflow)) return;
  unsigned long long total =
      __hip_atomic_load(&st->band_list, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (total > (unsigned long long)band_cap) total = (unsigned long long)band_cap;
  const unsigned long long per = (total + gridDim.x - 1) / gridDim.x;
  const unsigned long long b = (unsigned long long)blockIdx.x * per;
  const unsigned long long e = b + per < total ? b + per : total;
  recheck_band_range(pts, d, band, counts, pairs, st, eps2, pair_cap, b, e, qbuf, perm);
  if (threadIdx.x == 0 && blockIdx.x == 0) atomicAdd(&st->band_pairs, total);
}

// ------------------------------------------------------------ host launchers
int mfma_k(int d) { return (d + 15) / 16 * 16; }

hipError_t run_mfma_prep(const float *pts, const int *perm, int n, int d, int n_pad, int prec,
                         void *a_aug, void *b_aug, DevState *st, hipStream_t s) {
  const int K = mfma_k(d);
  const dim3 grid((n_pad + 255) / 256), block(256);
  if (prec == kPrecBf16)
    hipLaunchKernelGGL(k_mfma_prep<__bf16>, grid, block, 0, s, pts, n, d, n_pad, K,
                       (__bf16 *)a_aug, (__bf16 *)b_aug, st, perm);
  else
    hipLaunchKernelGGL(k_mfma_prep<_Float16>, grid, block, 0, s, pts, n, d, n_pad, K,
                       (_Float16 *)a_aug, (_Float16 *)b_aug, st, perm);
  return hipGetLastError();
}

hipError_t run_mfma_thresholds(DevState *st, double eps2, int d, int prec, double band_rel,
                               hipStream_t s) {
  const int K = mfma_k(d);
  if (prec == kPrecBf16)
    hipLaunchKernelGGL(k_mfma_thresholds<__bf16>, dim3(1), dim3(64), 0, s, st, eps2, d, K,
                       band_rel);
  else
    hipLaunchKernelGGL(k_mfma_thresholds<_Float16>, dim3(1), dim3(64), 0, s, st, eps2, d, K,
                       band_rel);
  return hipGetLastError();
}

hipError_t run_mfma_count(const void *a_aug, const void *b_aug, const Buffers &b,
                          const MfmaScalars &sc, int prec, hipStream_t s) {
  const int groups = sc.n_pad / kMfmaColsPerGroup;
  const int ks = mfma_k(sc.d) / 16;
  if (sc.chunk % 8 != 0 || sc.chunk <= 0 || sc.chunk > mfma_chunk_tiles(ks) ||
      (long long)sc.nchunks * sc.chunk < sc.n_pad / 32)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)mfma_items_before(groups, sc.nchunks, sc.chunk / 8)), block(256);
#define DBK_MFMA_CASE(KS)                                                                     \
  case KS:                                                                                    \
    if (prec == kPrecBf16)                                                                    \
      hipLaunchKernelGGL((k_mfma_count<__bf16, KS>), grid, block, 0, s, (const __bf16 *)a_aug, \
                         (const __bf16 *)b_aug, b.counts, b.pairs, b.band, b.st, sc);          \
    else                                                                                      \
      hipLaunchKernelGGL((k_mfma_count<_Float16, KS>), grid, block, 0, s,                     \
                         (const _Float16 *)a_aug, (const _Float16 *)b_aug, b.counts, b.pairs,  \
                         b.band, b.st, sc);                                                   \
    break;
  switch (ks) {
    DBK_MFMA_CASE(1)
    DBK_MFMA_CASE(2)
    DBK_MFMA_CASE(3)
    DBK_MFMA_CASE(4)
    DBK_MFMA_CASE(5)
    default: return hipErrorInvalidValue;
  }
#undef DBK_MFMA_CASE
  return hipGetLastError();
}

hipError_t run_recheck_band(const float *pts, int d, const Buffers &b, double eps2,
                            long long band_cap, long long pair_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_recheck_band, dim3(1024), dim3(256), 0, s, pts, d, b.band, b.counts,
                     b.pairs, b.st, eps2, band_cap, pair_cap, b.okey);
  return hipGetLastError();
}

}  // namespace dbk
