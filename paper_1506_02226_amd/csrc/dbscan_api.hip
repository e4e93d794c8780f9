// C ABI of libdbscan (declared in include/dbscan.h): argument checks,
// workspace layout, float32 band thresholds, kernel sequence.
#include <errno.h>
#include <float.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "../../include/dbscan.h"
#include "dbscan_internal.h"

namespace {

constexpr int kVersion = 100;  // 0.1.0
constexpr int64_t kPadRows = 256;
constexpr int32_t kMaxD = 1024;
constexpr uint64_t kDefaultBitmaskLimit = 16ull << 30;
constexpr double kDefaultBandRel = 1e-2;
constexpr uint64_t kPairsPerPoint = 128;       // default pair-list capacity per point
constexpr uint64_t kMaxPairs = 2147483647ull;  // 16 GiB of (int, int) pairs
constexpr uint64_t kBandPerPoint = 64;         // default band-list capacity per point
constexpr int32_t kMaxMfmaD = 76;              // contraction length <= 80
// auto order: below these sizes the sort's ~15 launches cost more than they
// save (measured on the blob workloads: the bit-matrix form gains from
// 16,384 points, the matrix cores from 32,768; the on-the-fly float32 form
// only on dense inputs)
constexpr int64_t kSpatialMinN = 65536;
constexpr int64_t kSpatialMinNBitmask = 16384;
constexpr int64_t kSpatialMinNMfma = 32768;

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Layout {
  int64_t n_pad = 0;
  int32_t d_pad = 0;
  int adjacency = DBSCAN_ADJ_ONTHEFLY;
  int precision = DBSCAN_PREC_FP32;
  int order = DBSCAN_ORDER_INPUT;
  bool prune = false;
  uint64_t off_state = 0, off_soa = 0, off_parent = 0, off_jstar = 0, off_corebits = 0,
           off_list = 0, off_adj = 0, off_tflag = 0, off_pairs = 0, off_aaug = 0, off_baug = 0, off_band = 0,
           total = 0;
  // spatial order: sort keys and values (two buffers each), digit histograms,
  // the inverse permutation, staged-order counts and per-root label minima
  uint64_t off_keys[2] = {0, 0}, off_vals[2] = {0, 0}, off_hist = 0, off_inv = 0,
           off_counts = 0, off_rootmin = 0;
  uint64_t off_box = 0;  // tile pruning: per-64-point-block boxes
  uint64_t off_hoist = 0;  // rows of the hoisted float32 test (0: none)
  int64_t edge_cap = 0;  // pair-list entries (on-the-fly form, d <= 4 or matrix cores)
  int64_t band_cap = 0;  // band-list entries (matrix cores)
  int mfma_k = 0;        // contraction length of the matrix-core filter
};

// the words of each 32-row block from its diagonal block on (dbk::adj_index)
uint64_t bitmask_bytes(int64_t n_pad) { return dbk::adj_words((int)n_pad) * 4; }
// one byte per 32 x 64 tile of the bitmask: non-empty or not
uint64_t tile_flag_bytes(int64_t n_pad) { return (uint64_t)n_pad / 64 * (uint64_t)(n_pad / 32); }

int plan(int64_t n, int32_t d, const dbscan_opts *o, Layout *L) {
  L->n_pad = round_up(n, kPadRows);
  const int dc = dbk::coord_chunk(d);
  L->d_pad = (int32_t)round_up(d, dc);
  const int req_adj = o ? o->adjacency : DBSCAN_ADJ_AUTO;
  const int req_prec = o ? o->precision : DBSCAN_PREC_AUTO;
  const uint64_t limit = (o && o->bitmask_limit) ? o->bitmask_limit : kDefaultBitmaskLimit;
  const bool mfma_ok = d <= kMaxMfmaD;
  if (req_prec == DBSCAN_PREC_AUTO)
    L->precision = (d >= 16 && mfma_ok && req_adj != DBSCAN_ADJ_BITMASK) ? DBSCAN_PREC_FP16
                                                                         : DBSCAN_PREC_FP32;
  else if (req_prec == DBSCAN_PREC_FP32)
    L->precision = DBSCAN_PREC_FP32;
  else if (req_prec == DBSCAN_PREC_BF16 || req_prec == DBSCAN_PREC_FP16) {
    if (!mfma_ok) return DBSCAN_E_UNSUPPORTED;
    L->precision = req_prec;
  } else
    return DBSCAN_E_INVAL;
  const bool mfma = L->precision != DBSCAN_PREC_FP32;
  const bool bm_ok = d <= 4 && !mfma;
  if (req_adj == DBSCAN_ADJ_BITMASK) {
    if (!bm_ok) return DBSCAN_E_UNSUPPORTED;
    L->adjacency = DBSCAN_ADJ_BITMASK;
  } else if (req_adj == DBSCAN_ADJ_ONTHEFLY) {
    L->adjacency = DBSCAN_ADJ_ONTHEFLY;
  } else if (req_adj == DBSCAN_ADJ_AUTO) {
    L->adjacency =
        (bm_ok && bitmask_bytes(L->n_pad) <= limit) ? DBSCAN_ADJ_BITMASK : DBSCAN_ADJ_ONTHEFLY;
  } else {
    return DBSCAN_E_INVAL;
  }
  const int req_order = o ? o->order : DBSCAN_ORDER_AUTO;
  const bool order_ok = d <= dbk::order_max_d();
  const int req_prune = o ? o->prune : 0;
  if (req_prune != 0 && req_prune != 1) return DBSCAN_E_INVAL;
  if (req_prune) {
    if (d > 4 || mfma) return DBSCAN_E_UNSUPPORTED;
    L->prune = true;
  }
  if (req_order == DBSCAN_ORDER_AUTO) {
    const int64_t min_n = mfma ? kSpatialMinNMfma
                               : (L->adjacency == DBSCAN_ADJ_BITMASK ? kSpatialMinNBitmask
                                                                     : kSpatialMinN);
    L->order = (order_ok && n >= min_n) ? DBSCAN_ORDER_SPATIAL : DBSCAN_ORDER_INPUT;
  } else if (req_order == DBSCAN_ORDER_INPUT)
    L->order = DBSCAN_ORDER_INPUT;
  else if (req_order == DBSCAN_ORDER_SPATIAL) {
    if (!order_ok) return DBSCAN_E_UNSUPPORTED;
    L->order = DBSCAN_ORDER_SPATIAL;
  } else
    return DBSCAN_E_INVAL;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = off;
    off += (uint64_t)round_up((int64_t)bytes, 256);
    return at;
  };
  L->off_state = take(sizeof(dbk::DevState));  // first: the server reads its status word
  L->off_soa = take((uint64_t)L->d_pad * L->n_pad * 4);
  L->off_parent = take((uint64_t)L->n_pad * 4);
  L->off_jstar = take((uint64_t)L->n_pad * 4);
  L->off_corebits = take((uint64_t)L->n_pad / 8);
  L->off_list = take((uint64_t)L->n_pad * 4);
  L->off_adj = (L->adjacency == DBSCAN_ADJ_BITMASK) ? take(bitmask_bytes(L->n_pad)) : off;
  L->off_tflag = (L->adjacency == DBSCAN_ADJ_BITMASK) ? take(tile_flag_bytes(L->n_pad)) : off;
  if (L->adjacency == DBSCAN_ADJ_ONTHEFLY) {
    const uint64_t req = (o && o->pair_capacity) ? o->pair_capacity : (uint64_t)kPairsPerPoint * n;
    L->edge_cap = (int64_t)(req < kMaxPairs ? req : kMaxPairs);
  }
  L->off_pairs = L->edge_cap ? take((uint64_t)L->edge_cap * 8) : off;
  if (mfma) {
    L->mfma_k = dbk::mfma_k(d);
    L->off_aaug = take(dbk::mfma_a_bytes(L->n_pad, L->mfma_k));
    L->off_baug = take((uint64_t)L->n_pad * L->mfma_k * 2);
    const uint64_t req = (o && o->band_capacity) ? o->band_capacity : (uint64_t)kBandPerPoint * n;
    L->band_cap = (int64_t)(req < kMaxPairs ? req : kMaxPairs);
    L->off_band = take((uint64_t)L->band_cap * 8);
  }
  if (L->order == DBSCAN_ORDER_SPATIAL) {
    for (int k = 0; k < 2; ++k) {
      L->off_keys[k] = take((uint64_t)L->n_pad * 4);
      L->off_vals[k] = take((uint64_t)L->n_pad * 4);
    }
    L->off_hist = take((uint64_t)dbk::order_hist_entries(n) * 4);
    L->off_inv = take((uint64_t)L->n_pad * 4);
    L->off_counts = take((uint64_t)L->n_pad * 4);
    L->off_rootmin = take((uint64_t)L->n_pad * 4);
  }
  // boxes of the 64-point blocks, then of the row groups and of the chunks
  if (L->prune) L->off_box = take((uint64_t)3 * 2 * d * (L->n_pad / 64) * 4);
  // the float32 step-1 sweeps for d <= 4 (on the fly and bitmask) test the
  // hoisted form when the rows are in spatial order: in the caller's order
  // 16 consecutive rows lie anywhere, their origin is far from most of them
  // and a group's gate (its largest threshold) opens on most tiles.  The
  // pruned sweeps keep the direct form: the tiles they visit mostly hold
  // neighbours, so the gate opens there too and the hoisted form's rare
  // branch (per-row thresholds from memory, a second column preparation)
  // costs more than its cheaper test saves (measured on the pruned sweeps:
  // blobs2d_200k 0.60 against 0.27 ms, aniso3d_2m 7.9 against 7.1 ms)
  if (!mfma && d <= 4 && L->order == DBSCAN_ORDER_SPATIAL && !L->prune)
    L->off_hoist = take(dbk::hoist_floats((int)L->n_pad, d) * 4);
  L->total = off;
  return DBSCAN_OK;
}

int check_args(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
               const int32_t *labels, const uint8_t *core, const int32_t *counts) {
  if (!points || !labels || !core || !counts) return DBSCAN_E_INVAL;
  if (n < 1 || n > DBSCAN_MAX_N) return DBSCAN_E_INVAL;
  if (d < 1 || d > kMaxD) return DBSCAN_E_INVAL;
  if (!(eps >= 0.0) || !isfinite(eps)) return DBSCAN_E_INVAL;
  if (minpts < 1) return DBSCAN_E_INVAL;
  return DBSCAN_OK;
}

// float32 thresholds such that, for the float64 value s64 of the definition
// and any float32 evaluation s32 of the same sum (any order, with or without
// fused multiply-add), s32 <= lo implies s64 <= eps2 and s32 > hi implies
// s64 > eps2.  With u = 2^-24 and u' = 2^-53, a sum of d squared differences
// evaluated with d+2 roundings per term satisfies |s32 - S| <= g32*S + a and
// |s64 - S| <= g64*S, S the exact value, g = (d+2)u/(1-(d+2)u); a covers
// gradual underflow.  The double arithmetic below is widened by 4u' and the
// results are rounded outward to float32.
void band_fp32(double eps2, int32_t d, float *lo, float *hi) {
  if (isinf(eps2)) {
    *lo = INFINITY;
    *hi = INFINITY;
    return;
  }
  const double u = 0x1p-24, u64 = 0x1p-53;
  const double g32 = (d + 2) * u / (1.0 - (d + 2) * u);
  const double g64 = (d + 2) * u64 / (1.0 - (d + 2) * u64);
  const double a = (4.0 * d + 4.0) * 0x1p-149;
  const double lo_d = eps2 * (1.0 - g32) / (1.0 + g64) * (1.0 - 4 * u64) - a;
  const double hi_d = eps2 * (1.0 + g32) / (1.0 - g64) * (1.0 + 4 * u64) + a;
  float l = (float)lo_d;
  if ((double)l > lo_d) l = nextafterf(l, -INFINITY);
  float h = (float)hi_d;
  if ((double)h < hi_d) h = nextafterf(h, INFINITY);
  *lo = l;
  *hi = h;
}

struct Chunks {
  int nchunks;
  int chunk;  // columns (multiple of 64) or words
};

// Split `units` column units into chunks so that the grid has enough waves
// and each chunk's coordinates stay small enough for one XCD's L2.
Chunks split(int64_t units, int64_t row_waves, int64_t bytes_per_unit, int64_t min_units) {
  int nch = 1;
  while (nch < 64 && units / (nch * 2) >= min_units &&
         (row_waves * nch < 16384 || (units / nch) * bytes_per_unit > (2ll << 20)))
    nch *= 2;
  Chunks c;
  c.chunk = (int)((units + nch - 1) / nch);
  c.nchunks = (int)((units + c.chunk - 1) / c.chunk);
  return c;
}

// Tiles of a triangular sweep: `rgroup` rows x `chunk` columns per block
// (both multiples of 64, chunk <= max_chunk).  Starts at 512 x max_chunk and
// halves the rows (then the columns) until the upper triangle holds enough
// blocks to fill the chip several times over.
struct Tri {
  int nchunks, chunk, rgroup;
};

Tri tri_split(int64_t n_pad, int max_chunk) {
  int64_t rg = 512, ch = max_chunk;
  auto blocks = [&]() {
    const int64_t g = (n_pad + rg - 1) / rg, c = (n_pad + ch - 1) / ch;
    return g * c / 2 + 1;
  };
  while (blocks() < 4096 && (rg > 64 || ch > 256)) {
    if (rg > 64)
      rg /= 2;
    else
      ch /= 2;
  }
  Tri t;
  t.rgroup = (int)rg;
  t.chunk = (int)ch;
  t.nchunks = (int)((n_pad + ch - 1) / ch);
  return t;
}

// Tiles of the step-1 sweep: triangular for d <= 4, column chunks otherwise.
// For d <= 4 a block's column chunk is at most 2,048 points: every wave
// re-reads the chunk for each 16 rows it holds, and 2,048-point chunks of
// the blocks an XCD runs at once stay in its L2 (measured on the 2M-point
// 3-D workload: 53 GB fetched past the L2 per launch instead of 315 GB,
// same sweep time; 1,024-point chunks were 4% slower).  The pruned sweep
// visits only the column blocks near its rows and keeps 4,096-point chunks
// (fewer blocks to test against the rows' boxes: 6.5 against 7.1 ms on the
// pruned 2M-point sweep).
dbk::SweepScalars sweep_tiles(const dbk::SweepScalars &sc, int64_t npad, int d, bool prune) {
  dbk::SweepScalars t = sc;
  const Tri tr = tri_split(npad, (d <= 4 && !prune) ? 2048 : 4096);
  t.nchunks = tr.nchunks;
  t.chunk = tr.chunk;
  t.rgroup = tr.rgroup;
  return t;
}

// Pair tests made by the step-1 sweep kernel (its tiling, not n^2).
int64_t sweep_tests(int64_t n, int64_t n_pad, int d, bool bitmask, bool mfma) {
  if (mfma) {
    // 256-column groups g test the row tiles from row 256 g on
    const int64_t G = n_pad / 256;
    return 65536 * G * (G + 1) / 2;
  }
  // 32-row (bitmask) or 8-row blocks from row 0 while below n_pad / n, each
  // testing the columns from its own 64-column diagonal block to n_pad
  const int64_t R = bitmask ? 32 : dbk::rows_per_wave(d);
  const int64_t rows_end = bitmask ? n_pad : n;
  int64_t t = 0;
  for (int64_t row0 = 0; row0 < rows_end; row0 += R) t += R * (n_pad - (row0 & ~63LL));
  return t;
}

int hip_fail(hipError_t e, dbscan_stats *stats) {
  if (stats) {
    stats->status = DBSCAN_E_DEVICE;
    stats->hip_error = (int32_t)e;
  }
  return DBSCAN_E_DEVICE;
}

}  // namespace

extern "C" {

int dbscan_version(void) { return kVersion; }

int dbscan_fp32_band(double eps2, int32_t d, float *lo, float *hi) {
  if (!lo || !hi || d < 1 || d > kMaxD || !(eps2 >= 0.0)) return DBSCAN_E_INVAL;
  band_fp32(eps2, d, lo, hi);
  return DBSCAN_OK;
}

int dbscan_hoist_band(double sq_norm, int32_t d, double eps2, float *lo, float *hi) {
  if (!lo || !hi || d < 1 || d > 4 || !(eps2 >= 0.0) || !(sq_norm >= 0.0)) return DBSCAN_E_INVAL;
  dbk::hoist_band(sq_norm, d, eps2, lo, hi);
  return DBSCAN_OK;
}

int dbscan_hoist_gate(float hi_max, double sq_norm_max, int32_t d, float *gate) {
  if (!gate || d < 1 || d > 4 || !(sq_norm_max >= 0.0) || hi_max == -__builtin_inff())
    return DBSCAN_E_INVAL;
  *gate = dbk::hoist_gate(hi_max, sq_norm_max, d);
  return DBSCAN_OK;
}

const char *dbscan_strerror(int code) {
  switch (code) {
    case DBSCAN_OK: return "ok";
    case DBSCAN_PENDING: return "pending";
    case DBSCAN_E_INVAL: return "invalid argument";
    case DBSCAN_E_NOMEM: return "out of device memory or workspace too small";
    case DBSCAN_E_AGAIN: return "admission queue full";
    case DBSCAN_E_DEVICE: return "HIP runtime error";
    case DBSCAN_E_NONFINITE: return "input coordinate is NaN or infinite";
    case DBSCAN_E_UNSUPPORTED: return "unsupported option combination";
    default: return "unknown error";
  }
}

int dbscan_workspace_size(int64_t n, int32_t d, const dbscan_opts *opts, uint64_t *bytes) {
  if (!bytes || n < 1 || n > DBSCAN_MAX_N || d < 1 || d > kMaxD) return DBSCAN_E_INVAL;
  Layout L;
  const int rc = plan(n, d, opts, &L);
  if (rc) return rc;
  *bytes = L.total;
  return DBSCAN_OK;
}

int dbscan_fit_ex(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
                  int32_t *labels, uint8_t *core, int32_t *counts, void *stream,
                  const dbscan_opts *opts, dbscan_stats *stats) {
  int rc = check_args(points, n, d, eps, minpts, labels, core, counts);
  if (rc) return rc;
  Layout L;
  rc = plan(n, d, opts, &L);
  if (rc) return rc;
  if (stats) memset(stats, 0, sizeof(*stats));
  hipStream_t s = (hipStream_t)stream;

  // ---- workspace
  char *ws = nullptr;
  bool owned = false;
  if (opts && opts->workspace) {
    if (opts->workspace_bytes < L.total) return DBSCAN_E_NOMEM;
    if (((uintptr_t)opts->workspace & 255u) != 0) return DBSCAN_E_INVAL;
    ws = (char *)opts->workspace;
  } else {
    hipError_t e = hipMallocAsync((void **)&ws, L.total, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return (e == hipErrorOutOfMemory) ? DBSCAN_E_NOMEM : hip_fail(e, stats);
    }
    owned = true;
  }
  auto *st = (dbk::DevState *)(ws + L.off_state);
  auto *soa = (float *)(ws + L.off_soa);
  auto *parent = (int *)(ws + L.off_parent);
  auto *jstar = (int *)(ws + L.off_jstar);
  auto *corebits = (uint32_t *)(ws + L.off_corebits);
  auto *list = (int *)(ws + L.off_list);
  auto *adjT = (uint32_t *)(ws + L.off_adj);
  auto *pairs = (int2 *)(ws + L.off_pairs);
  void *a_aug = ws + L.off_aaug;
  void *b_aug = ws + L.off_baug;
  auto *band = (int2 *)(ws + L.off_band);
  const bool mfma = L.precision != DBSCAN_PREC_FP32;

  const double eps2 = eps * eps;
  float lo, hi;
  band_fp32(eps2, d, &lo, &hi);
  const int ni = (int)n, npad = (int)L.n_pad;

  hipEvent_t ev[6] = {};
  if (stats) {
    for (auto &e : ev) {
      hipError_t he = hipEventCreate(&e);
      if (he != hipSuccess) return hip_fail(he, stats);
    }
  }
  hipEvent_t *user_ev = (opts && opts->events) ? (hipEvent_t *)opts->events : nullptr;
  auto mark = [&](int k) {
    if (stats) (void)hipEventRecord(ev[k], s);
    if (user_ev) (void)hipEventRecord(user_ev[k], s);
  };

  hipError_t e = hipSuccess;
  auto step = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };

  step(dbk::run_reset(st, L.edge_cap, s));
  // spatial order: the permutation first, then the staging gathers through it
  // and the kernels count into a staged-order array (scattered back by the
  // core-flag pass)
  dbk::Order ord{nullptr, nullptr, nullptr};
  int *counts_k = counts;
  if (L.order == DBSCAN_ORDER_SPATIAL) {
    unsigned *keys[2] = {(unsigned *)(ws + L.off_keys[0]), (unsigned *)(ws + L.off_keys[1])};
    int *vals[2] = {(int *)(ws + L.off_vals[0]), (int *)(ws + L.off_vals[1])};
    int *perm = nullptr;
    step(dbk::run_spatial_order(points, ni, d, keys, vals, (int *)(ws + L.off_hist), st, &perm,
                                s));
    ord.perm = perm;
    ord.inv = (int *)(ws + L.off_inv);
    ord.rootmin = (int *)(ws + L.off_rootmin);
    counts_k = (int *)(ws + L.off_counts);
  }
  // the matrix-core path stages the float32 coordinates only if it falls back
  float *hoist = L.off_hoist ? (float *)(ws + L.off_hoist) : nullptr;
  step(dbk::run_stage(points, ni, d, npad, L.d_pad, mfma ? nullptr : soa, counts_k, parent, jstar,
                      st, ord, s, hoist, eps * eps));
  const double band_rel = (opts && opts->band_rel > 0.0) ? opts->band_rel : kDefaultBandRel;
  if (mfma) {
    step(dbk::run_mfma_prep(points, ord.perm, ni, d, npad, L.precision, a_aug, b_aug, st, s));
    step(dbk::run_mfma_thresholds(st, eps * eps, d, L.precision, band_rel, s));
  }
  mark(0);

  dbk::Buffers bufs{};
  bufs.soa = soa;
  bufs.counts = counts_k;
  bufs.okey = ord.perm;
  bufs.corebits = corebits;
  bufs.parent = parent;
  bufs.jstar = jstar;
  bufs.list = list;
  bufs.adjT = adjT;
  bufs.tflag = (uint8_t *)(ws + L.off_tflag);
  bufs.pairs = pairs;
  bufs.band = band;
  bufs.st = st;
  dbk::SweepScalars sc{};
  sc.n = ni;
  sc.n_pad = npad;
  sc.d = d;
  sc.d_pad = L.d_pad;
  sc.lo = lo;
  sc.hi = hi;
  sc.eps2 = eps2;
  sc.edge_cap = L.edge_cap;
  sc.flags = 0;
  sc.box = nullptr;
  sc.hoist = nullptr;
  if (L.prune) {
    float *box = (float *)(ws + L.off_box);
    step(dbk::run_block_boxes(soa, npad, d, box, s));
    sc.box = box;
  }
  const bool use_pairs = L.edge_cap > 0;

  // ---- step 1 (+ the neighbour counts of step 2)
  const bool bitmask = L.adjacency == DBSCAN_ADJ_BITMASK;
  if (mfma) {
    dbk::MfmaScalars ms{};
    ms.n = ni;
    ms.n_pad = npad;
    ms.d = d;
    // row chunks (fewer tiles for small n): 128 tiles (4096 rows) for FP16,
    // 256 (8192 rows; 128 beyond K = 64) for BF16.  Measured at n = 300,000,
    // d = 64: BF16 8.7 -> 6.7 ms with 256 tiles, FP16 5.5 -> 5.6 ms
    const int tiles = (int)(npad / 32);
    const int lds_most = dbk::mfma_chunk_tiles(dbk::mfma_k(d) / 16);
    const int most = L.precision == DBSCAN_PREC_BF16 ? lds_most : (lds_most < 128 ? lds_most : 128);
    ms.chunk = dbk::mfma_chunk_for(tiles, most);
    ms.nchunks = (tiles + ms.chunk - 1) / ms.chunk;
    ms.pair_cap = L.edge_cap;
    ms.band_cap = L.band_cap;
    mark(4);
    step(dbk::run_mfma_count(a_aug, b_aug, bufs, ms, L.precision, s));
    mark(5);
    step(dbk::run_recheck_band(points, d, bufs, eps2, L.band_cap, L.edge_cap, s));
    // the float32 sweep redoes step 1 only if the filter gave up
    step(dbk::run_filter_fallback(points, ord.perm, ni, d, npad, L.d_pad, soa, counts_k, st, s));
    dbk::SweepScalars f1 = sweep_tiles(sc, npad, d, L.prune);
    f1.flags = dbk::kOnlyOnFilterFail;
    step(dbk::run_count(bufs, f1, false, s));
  } else if (bitmask) {
    // chunks of 2,048 columns: the all-pairs bitmask kernel keeps a chunk's
    // columns in LDS (the pruned one reads them from L2, 4,096 at a time)
    const Tri t = tri_split(npad, L.prune ? 4096 : 2048);
    dbk::SweepScalars b1 = sc;
    b1.hoist = hoist;
    b1.nchunks = t.nchunks;
    b1.chunk = t.chunk;
    b1.rgroup = t.rgroup;
    mark(4);
    step(dbk::run_bitmask(bufs, b1, s));
    mark(5);
  } else {
    dbk::SweepScalars c1 = sweep_tiles(sc, npad, d, L.prune);
    c1.hoist = hoist;
    mark(4);
    step(dbk::run_count(bufs, c1, use_pairs, s));
    mark(5);
  }
  mark(1);
  // ---- step 2: core flags
  // the core-point total is a statistic: counted only when asked for
  // the core points' degree gates the bitmask merge's hook passes in the
  // caller's order (run_merge_bitmask)
  step(dbk::run_core(counts_k, ni, npad, minpts, core, corebits, st, ord, counts,
                     stats != nullptr, s,
                     bitmask && L.order != DBSCAN_ORDER_SPATIAL && npad <= dbk::kHookCallerOrderMax));
  mark(2);
  // ---- step 3: merge (union-find over core-core neighbour pairs) and border
  // points (lowest-index core neighbour)
  const int R = dbk::rows_per_wave(d);
  const int listed_max = ni;  // every point may be non-core
  dbk::SweepScalars b3 = sc;
  {
    const Chunks c = split(npad / 64, (listed_max + R - 1) / R / 8 + 1, 64LL * L.d_pad * 4, 2);
    b3.nchunks = c.nchunks;
    b3.chunk = c.chunk * 64;
  }
  if (bitmask) {
    const Chunks c = split(npad / 32, npad / 64, 1, 8);
    dbk::SweepScalars u3 = sc;
    u3.nchunks = c.nchunks;
    u3.chunk = c.chunk;
    step(dbk::run_merge_bitmask(bufs, u3, s));  // union-find and border points
  } else if (use_pairs) {
    // pair list; the repeated sweeps run only if it overflowed
    step(dbk::run_merge_list(bufs, L.edge_cap, s));
    dbk::SweepScalars f3 = sc;
    f3.flags = dbk::kOnlyOnOverflow;
    b3.flags = dbk::kOnlyOnOverflow;
    step(dbk::run_union(bufs, f3, s));
    step(dbk::run_compact_noncore(corebits, ni, list, st, true, s));
    step(dbk::run_border(bufs, b3, s));
  } else {
    step(dbk::run_union(bufs, sc, s));
    step(dbk::run_compact_noncore(corebits, ni, list, st, false, s));
    step(dbk::run_border(bufs, b3, s));
  }
  step(dbk::run_labels(ni, corebits, jstar, parent, labels, st, ord, s));
  mark(3);

  dbk::DevState hst{};
  if (stats && e == hipSuccess) {
    step(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
  }
  if (owned) step(hipFreeAsync(ws, s));
  if (e != hipSuccess) {
    if (stats)
      for (auto &x : ev) (void)hipEventDestroy(x);
    return hip_fail(e, stats);
  }
  if (!stats) return DBSCAN_OK;

  hipError_t se = hipStreamSynchronize(s);
  if (se != hipSuccess) {
    for (auto &x : ev) (void)hipEventDestroy(x);
    return hip_fail(se, stats);
  }
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0, t45 = 0;
  (void)hipEventElapsedTime(&t45, ev[4], ev[5]);
  (void)hipEventElapsedTime(&t01, ev[0], ev[1]);
  (void)hipEventElapsedTime(&t12, ev[1], ev[2]);
  (void)hipEventElapsedTime(&t23, ev[2], ev[3]);
  (void)hipEventElapsedTime(&t03, ev[0], ev[3]);
  for (auto &x : ev) (void)hipEventDestroy(x);
  stats->adjacency_used = L.adjacency;
  stats->precision_used = L.precision;
  stats->order_used = L.order;
  stats->pairs_tested = (int64_t)n * (int64_t)n;
  stats->pairs_rechecked = (int64_t)hst.band_pairs;
  stats->core_points = (int64_t)hst.core_points;
  stats->ms_step1 = t01;
  stats->ms_step2 = t12;
  stats->ms_step3 = t23;
  stats->ms_total = t03;
  stats->thr_lo = lo;
  stats->thr_hi = hi;
  uint64_t listed = hst.edges;
  for (int g = 0; g < dbk::kPairSegments; ++g) listed += hst.edge_seg[g][0];
  stats->pairs_listed = (int64_t)listed;
  stats->pair_overflow = (hst.status & dbk::kStatusEdgeOverflow) ? 1 : 0;
  stats->filter_fallback = (hst.status & (dbk::kStatusRange | dbk::kStatusBandOverflow)) ? 1 : 0;
  stats->thr_lo = mfma ? hst.thr[0] : lo;
  stats->thr_hi = mfma ? hst.thr[1] : hi;
  stats->ms_sweep1 = t45;
  stats->sweep1_tests = L.prune ? (int64_t)hst.tests
                                 : sweep_tests(n, L.n_pad, d, L.adjacency == DBSCAN_ADJ_BITMASK,
                                               mfma);
  stats->pruned = L.prune ? 1 : 0;
  stats->hoisted = (L.off_hoist && !(hst.status & dbk::kStatusNoHoist)) ? 1 : 0;
  stats->status = (hst.status & dbk::kStatusNonFinite) ? DBSCAN_E_NONFINITE : DBSCAN_OK;
  return stats->status;
}

int dbscan_fit(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
               int32_t *labels, uint8_t *core, int32_t *counts, void *stream) {
  return dbscan_fit_ex(points, n, d, eps, minpts, labels, core, counts, stream, nullptr, nullptr);
}

}  // extern "C"
