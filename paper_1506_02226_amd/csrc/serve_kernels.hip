// Served form: one persistent "epoch" kernel runs the block-sized tasks of
// every admitted job, taken from a device job table.
//
// Each job is a sequence of phases (serve_internal.h); a phase is a set of
// independent tasks, each the work of one 256-thread block of the standalone
// kernels (same bodies: bodies_common.h, bodies_sweep.h, bodies_mfma.h).  A
// block claims the next task of a job's current phase with one 64-bit atomic
// on (phase << 32 | index); the block that completes the last task of a phase
// opens the next one.  Blocks of all jobs interleave on the device, so jobs of
// uneven n, d, eps and MinPts overlap.  No block ever waits for another: a
// block without a claimable task sleeps briefly and retries, and every block
// leaves the loop at the epoch's deadline (device wall clock) or after a run
// of idle polls, so the grid always drains.  Job state stays in device memory
// between epochs; the host admits new jobs between epochs.
#include "bodies_common.h"
#include "bodies_mfma.h"
#include "bodies_sweep.h"
#include "serve_internal.h"

namespace dbk {

constexpr int kServeRows = 16;     // rows per wave of the float32 sweep
constexpr int kIdlePolls = 256;    // idle polls (~0.2 us each) before a block leaves

union ServeLds {
  MfmaLds<5> m;
  MfmaLds<4> m4;  // the largest row-count array: the union covers every MfmaLds<KS>
  int2 q[4][128];
  struct {
    int2 q[4][kListQueue];
    int colcnt[kServeTriChunk];
    unsigned long long xfer[5];
  } t;
};

__device__ __forceinline__ unsigned long long ld_acq(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_acq(const unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_acq(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ SweepScalars plain_scalars(const JobDesc &jd) {
  SweepScalars sc{};
  sc.n = jd.n;
  sc.n_pad = jd.n_pad;
  sc.d = jd.d;
  sc.d_pad = jd.d_pad;
  sc.nchunks = jd.nchunks;
  sc.chunk = jd.chunk;
  sc.lo = jd.lo;
  sc.hi = jd.hi;
  sc.eps2 = jd.eps2;
  sc.edge_cap = jd.pair_cap;
  sc.flags = 0;
  sc.rgroup = jd.rgroup;
  return sc;
}

template <int KS>
__device__ __forceinline__ void mfma_count_task(const JobDesc &jd, int idx, ServeLds &lds) {
  static_assert(sizeof(MfmaLds<KS>) <= sizeof(ServeLds), "served LDS too small");
  MfmaScalars ms{};
  ms.n = jd.n;
  ms.n_pad = jd.n_pad;
  ms.d = jd.d;
  ms.nchunks = jd.nchunks;
  ms.chunk = jd.chunk;
  ms.pair_cap = jd.pair_cap;
  ms.band_cap = jd.band_cap;
  mfma_count_body<_Float16, KS>((const _Float16 *)jd.a_aug, (const _Float16 *)jd.b_aug, jd.counts,
                                jd.pairs, jd.band, jd.st, ms, idx,
                                reinterpret_cast<MfmaLds<KS> &>(lds.m));
}

__device__ __forceinline__ void run_task(const JobDesc &jd, int phase, int idx, ServeLds &lds) {
  switch (phase) {
    case kPhStage:
      if (jd.mfma_ks) {
        mfma_prep_body<_Float16>(jd.pts, jd.n, jd.d, jd.n_pad, jd.mfma_ks * 16,
                                 (_Float16 *)jd.a_aug, (_Float16 *)jd.b_aug, jd.st, idx);
        const int i = idx * 256 + (int)threadIdx.x;
        if (i < jd.n) {
          jd.counts[i] = 0;
          jd.parent[i] = i;
          jd.jstar[i] = kNoNeighbour;
        }
      } else {
        stage_body(jd.pts, jd.n, jd.d, jd.n_pad, jd.d_pad, jd.soa, jd.counts, jd.parent, jd.jstar,
                   jd.st, idx);
      }
      break;
    case kPhThresh:
      if (threadIdx.x == 0)
        mfma_thresholds_body<_Float16>(jd.st, jd.eps2, jd.d, jd.mfma_ks * 16, jd.band_rel);
      break;
    case kPhCount:
      if (jd.mfma_ks) {
        switch (jd.mfma_ks) {
          case 1: mfma_count_task<1>(jd, idx, lds); break;
          case 2: mfma_count_task<2>(jd, idx, lds); break;
          case 3: mfma_count_task<3>(jd, idx, lds); break;
          case 4: mfma_count_task<4>(jd, idx, lds); break;
          default: mfma_count_task<5>(jd, idx, lds); break;
        }
      } else {
        const SweepScalars sc = plain_scalars(jd);
        switch (jd.d) {
          case 1: count_tri_body<1, kServeRows, true>(jd.soa, jd.counts, jd.pairs, jd.st, sc, idx, lds.t.q, lds.t.colcnt, lds.t.xfer); break;
          case 2: count_tri_body<2, kServeRows, true>(jd.soa, jd.counts, jd.pairs, jd.st, sc, idx, lds.t.q, lds.t.colcnt, lds.t.xfer); break;
          case 3: count_tri_body<3, kServeRows, true>(jd.soa, jd.counts, jd.pairs, jd.st, sc, idx, lds.t.q, lds.t.colcnt, lds.t.xfer); break;
          default: count_tri_body<4, kServeRows, true>(jd.soa, jd.counts, jd.pairs, jd.st, sc, idx, lds.t.q, lds.t.colcnt, lds.t.xfer); break;
        }
      }
      break;
    case kPhRecheck: {
      unsigned long long total = ld_acq(&jd.st->band_list);
      if (total > (unsigned long long)jd.band_cap) total = (unsigned long long)jd.band_cap;
      const unsigned long long b = (unsigned long long)idx * kServeSlice;
      const unsigned long long e = b + kServeSlice < total ? b + kServeSlice : total;
      recheck_band_range(jd.pts, jd.d, jd.band, jd.counts, jd.pairs, jd.st, jd.eps2, jd.pair_cap,
                         b, e, lds.q);
      if (threadIdx.x == 0 && e > b) atomicAdd(&jd.st->band_pairs, e - b);
      break;
    }
    case kPhCore:
      core_body(jd.counts, jd.n, jd.n_pad, jd.minpts, jd.core, jd.corebits, jd.st, idx);
      break;
    case kPhMerge: {
      unsigned long long total = ld_acq(&jd.st->edges);
      if (total > (unsigned long long)jd.pair_cap) total = (unsigned long long)jd.pair_cap;
      const unsigned long long b = (unsigned long long)idx * kServeSlice;
      const unsigned long long e = b + kServeSlice < total ? b + kServeSlice : total;
      merge_pairs_range(jd.pairs, jd.corebits, jd.parent, jd.jstar, b, e);
      break;
    }
    case kPhLabels:
      labels_body(jd.n, jd.corebits, jd.jstar, jd.parent, jd.labels, jd.st, idx);
      break;
    default:
      break;
  }
}

__device__ __forceinline__ unsigned slices(unsigned long long total, long long cap) {
  if (total > (unsigned long long)cap) total = (unsigned long long)cap;
  return (unsigned)((total + kServeSlice - 1) / kServeSlice);
}

// Open the phase after `phase` (one thread, after the last task of `phase`).
__device__ void open_next_phase(const JobDesc &jd, JobSched *js, int phase) {
  int p = phase + 1;
  for (;;) {
    const unsigned status = ld_acq(&jd.st->status);
    if (p == kPhRecheck || p == kPhCore) {
      // step 3 needs the complete pair list and an unabridged step 1
      if (status & (kStatusEdgeOverflow | kStatusBandOverflow | kStatusRange)) {
        js->fail_status = (int)status;
        __hip_atomic_store(&js->state, (int)kJobFailed, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&js->claim, (unsigned long long)kPhDone << 32, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    if (p == kPhRecheck)
      js->ntasks[p] = jd.mfma_ks ? slices(ld_acq(&jd.st->band_list), jd.band_cap) : 0u;
    if (p == kPhMerge) js->ntasks[p] = slices(ld_acq(&jd.st->edges), jd.pair_cap);
    if (p == kPhDone) {
      js->fail_status = (int)status;  // kStatusNonFinite is reported to the caller
      js->t_done = wall_clock64();
      __hip_atomic_store(&js->state, (int)kJobDone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&js->claim, (unsigned long long)kPhDone << 32, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (js->ntasks[p] > 0u) {
      __hip_atomic_store(&js->claim, (unsigned long long)p << 32, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    ++p;
  }
}

__global__ __launch_bounds__(256) void k_serve_epoch(const JobDesc *__restrict__ jobs,
                                                     JobSched *__restrict__ sched, int nslots,
                                                     long long deadline) {
  __shared__ ServeLds lds;
  __shared__ int s_job, s_phase, s_idx;
  int idle = 0;
  int start = (int)(blockIdx.x % (unsigned)nslots);
  for (;;) {
    if (threadIdx.x == 0) {
      int job = -1, phase = 0, idx = 0;
      if (wall_clock64() >= deadline) {
        job = -2;
      } else {
        for (int k = 0; k < nslots && job < 0; ++k) {
          const int j = (start + k) % nslots;
          if (ld_acq(&sched[j].state) != kJobActive) continue;
          const unsigned long long c = ld_acq(&sched[j].claim);
          const int ph = (int)(c >> 32);
          if (ph >= kPhDone || (unsigned)c >= ld_acq(&sched[j].ntasks[ph])) continue;
          const unsigned long long old =
              __hip_atomic_fetch_add(&sched[j].claim, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
          const int ph2 = (int)(old >> 32);
          if (ph2 < kPhDone && (unsigned)old < ld_acq(&sched[j].ntasks[ph2])) {
            job = j;
            phase = ph2;
            idx = (int)(unsigned)old;
            start = j;
          }
        }
        if (job < 0) job = (++idle > kIdlePolls) ? -2 : -1;
        else idle = 0;
      }
      s_job = job;
      s_phase = phase;
      s_idx = idx;
    }
    __syncthreads();
    const int job = s_job, phase = s_phase, idx = s_idx;
    __syncthreads();
    if (job == -2) break;
    if (job == -1) {
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    const JobDesc jd = jobs[job];
    run_task(jd, phase, idx, lds);
    __syncthreads();
    if (threadIdx.x == 0) {
      __atomic_thread_fence(__ATOMIC_RELEASE);
      const unsigned d = __hip_atomic_fetch_add(&sched[job].done[phase], 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT) + 1u;
      if (d == ld_acq(&sched[job].ntasks[phase])) open_next_phase(jd, &sched[job], phase);
    }
  }
}

__global__ void k_read_clock(long long *out) {
  if (threadIdx.x == 0) *out = wall_clock64();
}

// ------------------------------------------------------------ host launchers
bool serve_supports(int d, int prec) {
  if (prec == kPrecBf16) return false;  // the served form uses FP16 matrix cores
  if (prec == kPrecFp16) return d <= 76;
  return d <= 4;
}

hipError_t run_serve_epoch(const JobDesc *jobs, JobSched *sched, int nslots, long long deadline,
                           int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_serve_epoch, dim3(blocks), dim3(256), 0, s, jobs, sched, nslots, deadline);
  return hipGetLastError();
}

hipError_t run_read_clock(long long *out, hipStream_t s) {
  hipLaunchKernelGGL(k_read_clock, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

}  // namespace dbk
