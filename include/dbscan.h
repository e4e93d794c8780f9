/*
 * libdbscan -- DBSCAN on one AMD Instinct MI355X (gfx950), C ABI.
 *
 * The library computes the three steps of the paper "Design and optimization
 * of DBSCAN Algorithm based on CUDA" (Wang et al.):
 *   step 1  the epsilon test of every ordered pair of points, done on squared
 *           distances against eps^2 (Section IV-A) and never stored as an
 *           n x n float matrix (Section IV-B.1 fuses the distance into the
 *           neighbourhood test);
 *   step 2  neighbour counts, core flags and primitive clusters (Section IV-B;
 *           core = "at least MinPts points within eps", Section II);
 *   step 3  merging of primitive clusters whose centres are reachable core
 *           points (Section IV-C; reachability as defined in Section II).
 *
 * Results are exactly those of the plain float64 definition: for each pair
 *   s = 0; for k in 0..d-1 { t = x_ik - x_jk; s = s + t*t }  (float64, each
 *   operation rounded alone), neighbour iff s <= eps*eps (rounded once);
 * counts include the point itself; core iff count >= minpts; labels are
 * canonical: a core point's label is the lowest index of a core point in its
 * cluster, a non-core point with core neighbours takes the label of its
 * lowest-index core neighbour, every other point is noise (-1).  The kernels
 * evaluate the distance in float32 (or on BF16/FP16 matrix cores for d >= 16)
 * only as a filter: every pair whose float32 value lies inside a rigorous
 * rounding band around eps^2 is re-evaluated in float64 on the GPU, so the
 * decisions, and therefore counts, core flags and labels, equal the float64
 * definition bit for bit in every mode.
 *
 * Conventions for every entry point:
 *   - Pointers marked DEVICE must be device memory of the current HIP device
 *     (hipMalloc, or a PyTorch tensor on that device); HOST pointers are
 *     ordinary host memory.  Point arrays are row-major float32, n rows of d
 *     coordinates, C-contiguous.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; the call returns once the work is enqueued
 *     unless a `stats` pointer is given, in which case it waits for the
 *     stream and fills the statistics.
 *   - The caller owns every buffer it passes and must keep them alive and
 *     unmodified until the stream has finished the call's work.
 *   - Return codes: 0 (DBSCAN_OK) on success; negative DBSCAN_E_* codes on
 *     failure.  Arguments are checked before anything is enqueued; an
 *     invalid argument enqueues nothing.  No C++ exception crosses the ABI.
 *   - Calls are re-entrant on distinct streams.
 */
#ifndef DBSCAN_MI355X_H
#define DBSCAN_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBSCAN_OK 0
#define DBSCAN_PENDING 1           /* dbscan_batch_poll: job not finished */
#define DBSCAN_E_INVAL (-22)       /* bad argument (null pointer, size, eps, minpts) */
#define DBSCAN_E_NOMEM (-12)       /* device allocation failed / workspace too small */
#define DBSCAN_E_AGAIN (-11)       /* serving: admission queue full */
#define DBSCAN_E_DEVICE (-1000)    /* a HIP call failed (hip error in stats) */
#define DBSCAN_E_NONFINITE (-1001) /* a coordinate is NaN or +-inf */
#define DBSCAN_E_UNSUPPORTED (-1002)

/* Largest n accepted: 2^31 - 256, so that n rounded up to a multiple of 256
 * (the padded row count) is still an int32 index. */
#define DBSCAN_MAX_N 2147483392LL

/* Device array behind dbscan_fit_noalloc, per GPU (64 MiB). */
#define DBSCAN_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* How the neighbour relation is kept between step 2 and step 3. */
#define DBSCAN_ADJ_AUTO 0     /* bitmask when it fits the limit, else on the fly */
#define DBSCAN_ADJ_BITMASK 1  /* one bit per ordered pair, kept in device memory */
#define DBSCAN_ADJ_ONTHEFLY 2 /* nothing stored; step 3 repeats the epsilon tests */

/* Order in which the rows are processed (results are always returned in the
 * caller's order and are identical either way). */
#define DBSCAN_ORDER_AUTO 0    /* spatial for d <= 128 from n = 16384 (bit matrix),
                                  32768 (matrix cores) or 65536 (on the fly), else input */
#define DBSCAN_ORDER_INPUT 1   /* the caller's order */
#define DBSCAN_ORDER_SPATIAL 2 /* rows permuted on the device so that neighbours sit at
                                  nearby indices -- by a Morton key of the coordinates
                                  (quantised over the bounding box) for d <= 4, by the
                                  nearest of 256 pivot rows (rows taken at a fixed
                                  stride; 128 beyond d = 64) for 5 <= d <= 128 -- so the
                                  sweeps meet their rare neighbour branch far less often
                                  and the bitmask's set bits gather near its diagonal.
                                  d <= 128 only (else DBSCAN_E_UNSUPPORTED). */

/* Arithmetic of the epsilon-test filter (the decision is always float64-exact). */
#define DBSCAN_PREC_AUTO 0 /* FP16 matrix cores for 16 <= d <= 76, else float32 */
#define DBSCAN_PREC_FP32 1 /* float32 direct form (x_i - x_j)^2 summed */
#define DBSCAN_PREC_BF16 2 /* |x|^2 + |y|^2 - 2 x.y on BF16 matrix cores, d <= 76 */
#define DBSCAN_PREC_FP16 3 /* same on FP16 matrix cores, d <= 76; inputs with a
                              coordinate |x| > 30000 fall back to float32 */

typedef struct dbscan_opts {
  int32_t adjacency;          /* DBSCAN_ADJ_*  (0 = auto) */
  int32_t precision;          /* DBSCAN_PREC_* (0 = auto) */
  double band_rel;            /* matrix-core filter: re-check every pair with
                                 |s - eps^2| <= band_rel * eps^2 at least
                                 (0 = 1e-2); widened to the rigorous bound */
  uint64_t bitmask_limit;     /* AUTO uses the bitmask when it needs at most this
                                 many bytes (0 = 16 GiB) */
  void *workspace;            /* DEVICE, optional: caller-owned scratch of at least
                                 dbscan_workspace_size() bytes, 256-byte aligned.
                                 NULL: the library allocates it stream-ordered. */
  uint64_t workspace_bytes;
  uint64_t pair_capacity;     /* on-the-fly form (any d): room for this many
                                 neighbour pairs (i, j), j < i, recorded by step 1
                                 for the merge (8 bytes each; 0 = 128 per point).
                                 If they do not fit, step 3 repeats the epsilon
                                 tests instead; results are identical. */
  uint64_t band_capacity;     /* matrix-core filter: room for this many undecided
                                 pairs awaiting the float64 pass (8 bytes each;
                                 0 = 64 per point).  If they do not fit, step 1
                                 is redone with the float32 direct form. */
  void *events;               /* HOST, optional: hipEvent_t[6] created by the caller.
                                 Recorded on `stream` (no wait): [0] before step 1,
                                 [1]-[3] after steps 1, 2 and 3, [4]/[5] just before
                                 and after the step-1 sweep kernel alone (the
                                 pair-test kernel, without staging or the float64
                                 band pass), so the caller can time the kernels of
                                 a call it does not wait for. */
  int32_t order;              /* DBSCAN_ORDER_* (0 = auto) */
  int32_t prune;              /* 1: skip the epsilon tests of tile pairs whose bounding
                                 boxes are farther apart than eps (float32 forms,
                                 d <= 4; effective with the spatial order).  The
                                 results are identical -- a skipped pair is provably
                                 not a neighbour -- but not every pair is tested, so
                                 sweep1_tests then counts the tests actually made.
                                 0 (default): every pair is tested. */
} dbscan_opts;

typedef struct dbscan_stats {
  int32_t status;         /* DBSCAN_OK, DBSCAN_E_NONFINITE or DBSCAN_E_DEVICE */
  int32_t hip_error;      /* hipError_t of the failing call, else 0 */
  int32_t adjacency_used; /* DBSCAN_ADJ_BITMASK or DBSCAN_ADJ_ONTHEFLY */
  int32_t precision_used; /* DBSCAN_PREC_FP32 / _BF16 / _FP16 */
  int64_t pairs_tested;   /* ordered pairs of the step-1 sweep (n*n) */
  int64_t pairs_rechecked;/* pair tests re-evaluated in float64 (all steps) */
  int64_t core_points;
  float ms_step1;         /* epsilon tests + counts (+ bitmask), device time */
  float ms_step2;         /* core flags */
  float ms_step3;         /* merge, border assignment and labels */
  float ms_total;         /* steps 1-3, device time (input staging excluded) */
  float thr_lo, thr_hi;   /* band thresholds of the filter used (float32 direct
                             form on s32, or matrix-core form on s~) */
  int64_t pairs_listed;   /* neighbour pairs j < i found by step 1 (pair list) */
  int32_t pair_overflow;  /* 1 if they exceeded pair_capacity (step 3 repeated
                             the tests), else 0 */
  int32_t filter_fallback;/* 1 if the matrix-core filter gave up (inputs out of
                             its range or band_capacity exceeded) and step 1 was
                             redone in float32, else 0 */
  float ms_sweep1;        /* the step-1 sweep kernel alone, device time */
  int64_t sweep1_tests;   /* pair tests that kernel makes: about n^2/2 for the
                             triangular float32 sweeps (each unordered pair
                             once, both orders inside 64x64 diagonal blocks)
                             and for the matrix-core tiles (256x256 diagonal
                             zones); with pruning, the tests made (counted on
                             the device) */
  int32_t order_used;     /* DBSCAN_ORDER_INPUT or DBSCAN_ORDER_SPATIAL */
  int32_t pruned;         /* 1 if tile pruning was on (dbscan_opts.prune) */
  int32_t hoisted;        /* 1 if the float32 sweep tested the hoisted form
                             (d <= 4, rows in spatial order;
                             dbscan_hoist_band), 0 for the direct form */
  int32_t reserved0;
} dbscan_stats;

/*
 * dbscan_fit -- cluster n points (Sections II and IV: steps 1-3).
 *   points  DEVICE const float[n*d], row-major, finite values.
 *   n       1 <= n <= DBSCAN_MAX_N;  1 <= d <= 1024.
 *   eps     finite, >= 0 (compared as eps*eps rounded once in float64).
 *   minpts  >= 1 (a point counts itself).
 *   labels  DEVICE int32[n]  out: -1 noise, else canonical cluster id (a point
 *           index); filled with -2 when an input coordinate is not finite.
 *   core    DEVICE uint8[n]  out: 1 for core points, else 0.
 *   counts  DEVICE int32[n]  out: |N_eps(i)|, the point itself included.
 *   stream  hipStream_t as void*.
 * Uses the default options (auto adjacency and precision, library-allocated
 * workspace).  Asynchronous; a non-finite input is reported through labels
 * (-2) -- use dbscan_fit_ex with stats to get DBSCAN_E_NONFINITE returned.
 */
int dbscan_fit(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
               int32_t *labels, uint8_t *core, int32_t *counts, void *stream);

/*
 * dbscan_fit_ex -- dbscan_fit with options and statistics.
 *   opts   HOST, nullable (NULL = defaults).
 *   stats  HOST, nullable.  When given, the call waits for the stream,
 *          fills *stats (per-step device times from HIP events on `stream`)
 *          and returns DBSCAN_E_NONFINITE if an input was not finite.
 */
int dbscan_fit_ex(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
                  int32_t *labels, uint8_t *core, int32_t *counts, void *stream,
                  const dbscan_opts *opts, dbscan_stats *stats);

/*
 * dbscan_fit_noalloc -- dbscan_fit for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and asynchrony as dbscan_fit;
 * the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Its workspace is a library array of DBSCAN_NOALLOC_SCRATCH_BYTES
 * in device memory, one per GPU, held from the library's load until the
 * process ends.  The default plan is used when its workspace fits; otherwise
 * the on-the-fly form runs with pair and band lists sized to the array (a
 * full pair list makes step 3 repeat the epsilon tests; results are the
 * same).  DBSCAN_E_NOMEM when even that does not fit: n above 887,296 at
 * d = 3, 388,608 at d = 16, 120,320 at d = 64.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on one GPU (different streams, or
 * different host threads without ordering) race and must be serialized by
 * the caller.  The array keeps the last call's contents; each call
 * initialises everything it reads.
 */
int dbscan_fit_noalloc(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
                       int32_t *labels, uint8_t *core, int32_t *counts, void *stream);

/*
 * dbscan_workspace_size -- bytes of device scratch dbscan_fit_ex needs for
 * (n, d, opts); *bytes (HOST) receives the size.  The bitmask adjacency keeps
 * one triangle of the relation, n_pad^2 / 16 + 4 n_pad bytes, plus a flag
 * byte per 32 x 64 tile (n_pad^2 / 2048), n_pad = ceil(n/256)*256; the
 * on-the-fly form needs O(n*d).
 */
int dbscan_workspace_size(int64_t n, int32_t d, const dbscan_opts *opts, uint64_t *bytes);

/*
 * dbscan_fp32_band -- the float32 thresholds the direct form uses for eps2
 * (= eps*eps in float64) and d coordinates: a pair whose float32 squared
 * distance s32 (any summation order, with or without fused multiply-add)
 * satisfies s32 <= *lo is a neighbour under the float64 definition, one with
 * s32 > *hi is not, and pairs in between are re-evaluated in float64.  This
 * is the rounding-error bound of a sum of d squared differences (Section
 * IV-B.2 writes the squared distance as that sum).  lo, hi: HOST float*.
 */
int dbscan_fp32_band(double eps2, int32_t d, float *lo, float *hi);

/*
 * dbscan_hoist_band -- the float32 thresholds of one row of the hoisted test
 * that the on-the-fly float32 sweep (d <= 4) makes: Section IV-B.2's
 * T + P[n] - 2 t.p, taken about a local origin c (the centre of the box of
 * the row's block of 16 staged rows).  For the row x, a = fl(x - c) with
 * sq_norm = |a|^2 (float64), and for a column y, b = fl(y - c): the float32
 * value q of |b|^2 - 2 a.b (2d roundings, any order, fused or not) with
 * q <= *lo makes the pair a neighbour under the float64 definition, q > *hi
 * makes it not one, and pairs in between are re-evaluated in float64.
 * *lo is -inf when eps is too small beside |x - c| for a sure "in".
 * Valid while every coordinate is at most 2^60 in magnitude (the sweep takes
 * the direct form otherwise).  d in 1..4; lo, hi: HOST float*.
 */
int dbscan_hoist_band(double sq_norm, int32_t d, double eps2, float *lo, float *hi);

/*
 * dbscan_hoist_gate -- the gate of one 16-row block of that hoisted test
 * (Section IV-B.2's form, evaluated as the sweep does).  Per column the
 * sweep forms, for each row, s = fl(-2 a.b) (a product, then d - 1 fused
 * multiply-adds) and skips the column for the whole block when
 * fl(min over rows of s + P) > *gate, P = fl(|b|^2); only otherwise are the
 * rows' q compared with their thresholds.  hi_max: the largest *hi of the
 * block's rows (dbscan_hoist_band), sq_norm_max: the largest |a|^2 of its
 * rows (float64).  The gate is sound: a column with q <= hi for some row of
 * the block is never skipped.  NaN hi_max (no rows) gives NaN, +inf gives
 * +inf.  d in 1..4; gate: HOST float*.  DBSCAN_E_INVAL for a null pointer,
 * d out of range, a negative or NaN sq_norm_max, or hi_max = -inf.
 */
int dbscan_hoist_gate(float hi_max, double sq_norm_max, int32_t d, float *gate);

/* ------------------------------------------------------------------ serving
 * A server runs the jobs of many callers on one GPU.  Small jobs (n up to
 * 16,384; float32 for d <= 4, FP16 matrix cores for 16 <= d <= 76) share one
 * persistent kernel, relaunched every epoch (a time slice of ~2 ms): they
 * wait in a FIFO until a slot is free and their device-memory footprint fits
 * in the server's arena, their block-sized tasks interleave on the device,
 * and jobs that arrive while others run are admitted at the next epoch.
 * Every other job (larger n, other d, a precision the loop does not run, or
 * a small job whose lists overflowed) runs the dbscan_fit_ex path on one of
 * eight worker streams (float32 jobs with d <= 4 in the spatial order with
 * tile pruning), with its workspace taken from the same arena, so its
 * kernels overlap with the epochs and with the other workers' jobs.  Each
 * job's outputs equal those of dbscan_fit on the same inputs.  All entry
 * points are thread-safe.  The caller's work that produces a job's points
 * must be complete before dbscan_batch_submit (the server reads them on its
 * own streams, unordered with the caller's), and the output buffers must not
 * be used by other work until the job is finished.
 */
typedef struct dbscan_server dbscan_server;

#define DBSCAN_JOB_QUEUED 0
#define DBSCAN_JOB_RUNNING 1
#define DBSCAN_JOB_DONE 2
#define DBSCAN_JOB_FAILED 3

typedef struct dbscan_job {
  const float *points;   /* DEVICE [n*d] row-major float32 (same rules as dbscan_fit) */
  int64_t n;
  int32_t d;
  int32_t minpts;
  double eps;
  int32_t *labels;       /* DEVICE outputs, as in dbscan_fit */
  uint8_t *core;
  int32_t *counts;
  uint64_t tag;          /* caller's value, returned in the status */
  int32_t precision;     /* DBSCAN_PREC_* as in dbscan_opts (AUTO = dbscan_fit's choice) */
  int32_t reserved;      /* 0 */
} dbscan_job;

typedef struct dbscan_job_status {
  int32_t state;         /* DBSCAN_JOB_* */
  int32_t error;         /* DBSCAN_OK or the error of a failed job */
  int64_t t_submit_ns;   /* host steady clock, ns */
  int64_t t_admit_ns;
  int64_t t_done_ns;     /* completion (device clock mapped to the host clock) */
  uint64_t footprint;    /* device bytes held while running */
  uint64_t tag;
  int32_t fallback;      /* 1 if the job ran through the dbscan_fit_ex path on a worker */
  int32_t reserved;
} dbscan_job_status;

typedef struct dbscan_server_stats {
  int64_t jobs_submitted, jobs_admitted, jobs_done;
  int64_t queued, running;
  int64_t epochs;
  int64_t busy_ns;       /* host time spent in epochs */
  int64_t points_done;
  double pairs_done;     /* sum of n^2 over finished jobs */
  uint64_t budget_bytes, arena_used, peak_bytes;
} dbscan_server_stats;

/*
 * dbscan_server_create -- server on HIP device `device` with a device-memory
 * arena of hbm_budget_bytes (0 = 80% of the free memory) and at most
 * max_slots jobs running at once (1..4096).  *out (HOST) receives the handle.
 * Errors: DBSCAN_E_INVAL, DBSCAN_E_NOMEM, DBSCAN_E_DEVICE.
 */
int dbscan_server_create(int device, uint64_t hbm_budget_bytes, int32_t max_slots,
                         dbscan_server **out);

/*
 * dbscan_batch_submit -- queue one job (HOST struct, DEVICE buffers that must
 * stay valid until the job is finished).  *job_id (HOST) receives its id.
 * DBSCAN_E_INVAL for bad arguments, DBSCAN_E_UNSUPPORTED for a precision the
 * job's d does not allow, DBSCAN_E_NOMEM if the job's footprint exceeds the
 * whole arena, DBSCAN_E_AGAIN if the queue is full.
 */
int dbscan_batch_submit(dbscan_server *s, const dbscan_job *job, uint64_t *job_id);

/*
 * dbscan_batch_poll -- status of a job (HOST out).  Returns DBSCAN_OK once the
 * job is finished (state DONE or FAILED), DBSCAN_PENDING before, and
 * DBSCAN_E_INVAL for an unknown id.  A finished job's status is returned
 * once: the server then forgets the job (a later poll gives DBSCAN_E_INVAL),
 * so a long-lived server holds only unfinished and unread jobs.
 */
int dbscan_batch_poll(dbscan_server *s, uint64_t job_id, dbscan_job_status *st);

/* dbscan_batch_wait -- dbscan_batch_poll that blocks up to timeout_ns (the
 * finished status is likewise returned once). */
int dbscan_batch_wait(dbscan_server *s, uint64_t job_id, int64_t timeout_ns,
                      dbscan_job_status *st);

/* dbscan_server_get_stats -- counters of the server (HOST out). */
int dbscan_server_get_stats(dbscan_server *s, dbscan_server_stats *out);

/*
 * dbscan_server_destroy -- finish every queued and running job, then release
 * the server.  Returns DBSCAN_OK or the first device error the server met.
 */
int dbscan_server_destroy(dbscan_server *s);

/* dbscan_strerror -- static description of a return code. */
const char *dbscan_strerror(int code);

/* dbscan_version -- library ABI version (major*10000 + minor*100 + patch). */
int dbscan_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DBSCAN_MI355X_H */
