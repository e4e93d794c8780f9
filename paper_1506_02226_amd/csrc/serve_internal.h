// Device-side job table of the served form (shared by serve_kernels.hip and
// server.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dbscan_device.h"
#include "dbscan_internal.h"

namespace dbk {

// Phases of one job; every phase is a set of independent block-sized tasks.
enum ServePhase {
  kPhStage = 0,    // staging / low-precision copies, counters cleared
  kPhThresh = 1,   // matrix-core thresholds (one task; none for float32 jobs)
  kPhCount = 2,    // step 1: epsilon tests, counts, neighbour pairs (and band pairs)
  kPhRecheck = 3,  // float64 pass over band pairs (matrix-core jobs)
  kPhCore = 4,     // step 2: core flags
  kPhMerge = 5,    // step 3: union-find and border points from the pair list
  kPhLabels = 6,   // canonical labels
  kPhDone = 7,
  kNumPhases = 8
};

enum ServeState { kJobFree = 0, kJobActive = 1, kJobDone = 2, kJobFailed = 3 };

constexpr int kServeSlice = 4096;  // pairs per task in the list phases
constexpr int kServeTriChunk = 4096;  // columns per float32 step-1 task (LDS tallies)
constexpr int kServeTriRows = 128;    // rows per float32 step-1 task

// Read-only description of one admitted job (written by the host before an
// epoch starts).
struct JobDesc {
  const float *pts;  // caller's points [n][d]
  int32_t *labels;
  uint8_t *core;
  int32_t *counts;
  DevState *st;
  float *soa;        // float32 jobs
  int *parent;
  int *jstar;
  uint32_t *corebits;
  int2 *pairs;
  int2 *band;        // matrix-core jobs
  void *a_aug;
  void *b_aug;
  int n, n_pad, d, d_pad, minpts;
  int mfma_ks;       // 0: float32 direct form; else K/16 of the FP16 matrix-core filter
  double eps2;
  double band_rel;
  float lo, hi;      // float32 band (direct form)
  long long pair_cap, band_cap;
  int nchunks, chunk;  // step-1 split (columns for float32, 32-row tiles for matrix cores)
  int rgroup;          // float32: rows per task of the triangular sweep
};

// Mutable scheduling state of one job slot.
struct JobSched {
  unsigned long long claim;        // (phase << 32) | next task index of that phase
  unsigned int done[kNumPhases];   // completed tasks per phase
  unsigned int ntasks[kNumPhases]; // tasks per phase (list phases filled at run time)
  int state;                       // ServeState
  int fail_status;                 // DevState status bits when the job failed
  long long t_done;                // device wall clock at completion
};

hipError_t run_serve_epoch(const JobDesc *jobs, JobSched *sched, int nslots, long long deadline,
                           int blocks, hipStream_t s);
hipError_t run_read_clock(long long *out, hipStream_t s);
bool serve_supports(int d, int prec);

}  // namespace dbk
