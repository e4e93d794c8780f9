// Served form, host side: admission by device-memory footprint, the job
// table, the loop that relaunches the persistent epoch kernel, and the
// workers that run larger jobs through the standalone path.
//
//  * dbscan_batch_submit validates a job, picks its route and footprint and
//    queues it (FIFO per route):
//      - the persistent loop takes small jobs (n <= loop_max_n, default
//        16,384) of the forms it covers (float32 for d <= 4, FP16 matrix
//        cores for 16 <= d <= 76): their footprint is the served sections
//        (staged coordinates or FP16 copies, union-find, core bits, pair
//        list, band list);
//      - every other job runs dbscan_fit_ex on a worker's stream, with its
//        workspace (dbscan_workspace_size for the job's precision) taken
//        from the same arena, so admission bounds it too.
//  * The loop thread admits queued small jobs while a slot is free and the
//    footprint fits (first fit), writes their descriptors to the device job
//    table, and launches one epoch of the persistent kernel (a time slice,
//    2 ms by default) over all admitted jobs.  After the epoch it reads the
//    scheduling table back, releases finished jobs and admits more, so jobs
//    that arrive while others run join at the next epoch boundary and
//    overlap with them on the device.  A small job whose pair or band list
//    overflowed, or whose inputs left the FP16 range, moves to the front of
//    the workers' queue (same results).
//  * Six workers, each with its own stream, admit the larger jobs as
//    arena memory frees up; their kernels overlap with the epochs and with
//    each other on the device.  Float32 jobs with d <= 4 run there in the
//    spatial order with tile pruning.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <math.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "../../include/dbscan.h"
#include "dbscan_internal.h"
#include "serve_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch())
      .count();
}
inline uint64_t round_up(uint64_t v, uint64_t m) { return (v + m - 1) / m * m; }

constexpr uint64_t kServePairsPerPoint = 128;  // as dbscan_fit's default
constexpr uint64_t kServeBandPerPoint = 64;
constexpr int kMaxQueue = 1 << 20;
// streams for jobs outside the loop (default): with six, worker jobs of the
// served recipe queued for a worker at 0.7 x saturation (p99 266 ms against
// 34 ms with eight, same saturation rate)
constexpr int kWorkers = 8;
constexpr int kMaxWorkers = 16;
constexpr int64_t kLoopMaxN = 16384;           // largest job the loop takes by default

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t *off) {
    bytes = round_up(bytes, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = round_up(bytes, 256);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0;
};

struct ServeLayout {
  bool persistent = false;
  int prec = DBSCAN_PREC_FP32;
  int n_pad = 0, d_pad = 0, ks = 0;
  uint64_t off_state = 0, off_soa = 0, off_parent = 0, off_jstar = 0, off_corebits = 0,
           off_pairs = 0, off_band = 0, off_aaug = 0, off_baug = 0, total = 0;
  int64_t pair_cap = 0, band_cap = 0;
};

ServeLayout serve_layout(const dbscan_job &j, int64_t loop_max_n) {
  ServeLayout L;
  const int d = j.d;
  const int req = j.precision;
  L.prec = (d >= 16 && d <= 76 && (req == DBSCAN_PREC_AUTO || req == DBSCAN_PREC_FP16))
               ? DBSCAN_PREC_FP16
               : DBSCAN_PREC_FP32;
  const bool prec_ok = req == DBSCAN_PREC_AUTO || req == L.prec;
  L.persistent = prec_ok && j.n <= loop_max_n &&
                 dbk::serve_supports(d, L.prec == DBSCAN_PREC_FP16 ? dbk::kPrecFp16 : 1);
  if (!L.persistent) return L;
  L.n_pad = (int)round_up((uint64_t)j.n, 256);
  L.d_pad = d;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = off;
    off += round_up(bytes, 256);
    return at;
  };
  L.off_state = take(sizeof(dbk::DevState));
  L.off_parent = take((uint64_t)L.n_pad * 4);
  L.off_jstar = take((uint64_t)L.n_pad * 4);
  L.off_corebits = take((uint64_t)L.n_pad / 8);
  L.pair_cap = (int64_t)(kServePairsPerPoint * (uint64_t)j.n);
  L.off_pairs = take((uint64_t)L.pair_cap * 8);
  if (L.prec == DBSCAN_PREC_FP16) {
    L.ks = dbk::mfma_k(d) / 16;
    L.off_aaug = take(dbk::mfma_a_bytes(L.n_pad, L.ks * 16));
    L.off_baug = take((uint64_t)L.n_pad * L.ks * 16 * 2);
    L.band_cap = (int64_t)(kServeBandPerPoint * (uint64_t)j.n);
    L.off_band = take((uint64_t)L.band_cap * 8);
  } else {
    L.off_soa = take((uint64_t)L.d_pad * L.n_pad * 4);
  }
  L.total = off;
  return L;
}

// Same rule as the standalone path (dbscan_api.hip): float32 band thresholds.
void serve_band(double eps2, int32_t d, float *lo, float *hi) {
  if (isinf(eps2)) {
    *lo = INFINITY;
    *hi = INFINITY;
    return;
  }
  dbscan_fp32_band(eps2, d, lo, hi);
}

// Options of a job run through dbscan_fit_ex on a worker: the job's
// precision and, for float32 jobs with d <= 4, the spatial order with tile
// pruning (same results, far fewer pair tests on clustered data).
dbscan_opts direct_opts(const dbscan_job &j, bool prune) {
  dbscan_opts o{};
  o.precision = j.precision;
  const bool fp32 = j.precision == DBSCAN_PREC_FP32 ||
                    (j.precision == DBSCAN_PREC_AUTO && (j.d <= 4 || j.d > 76 || j.d < 16));
  if (prune && j.d <= 4 && fp32) {
    o.order = DBSCAN_ORDER_SPATIAL;
    o.prune = 1;
  }
  return o;
}

uint64_t direct_bytes(const dbscan_job &j, bool prune, int *rc) {
  const dbscan_opts o = direct_opts(j, prune);
  uint64_t b = 0;
  *rc = dbscan_workspace_size(j.n, j.d, &o, &b);
  return b;
}

struct Record {
  dbscan_job job{};
  dbscan_job_status status{};
  ServeLayout layout;
  bool direct = false;     // runs through dbscan_fit_ex on a worker
  uint64_t need = 0;       // arena bytes while running
  uint64_t held = 0;       // arena bytes held now
  uint64_t arena_off = 0;
  int slot = -1;
};

}  // namespace

struct dbscan_server {
  int device = 0;
  int nslots = 0;
  int epoch_us = 2000;
  int blocks = 0;
  uint64_t budget = 0;
  char *arena_base = nullptr;
  Arena *arena = nullptr;
  dbk::JobDesc *d_jobs = nullptr;
  dbk::JobSched *d_sched = nullptr;
  long long *d_clock = nullptr;
  hipStream_t stream = nullptr;
  std::vector<dbk::JobSched> h_sched;
  std::vector<uint64_t> slot_job;  // job id per slot (0 = free)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;         // jobs for the persistent loop
  std::deque<uint64_t> direct_pending;  // jobs for the workers
  std::unordered_map<uint64_t, Record> records;
  uint64_t next_id = 1;
  bool stopping = false;
  bool loop_done = false;
  int error = DBSCAN_OK;
  int64_t loop_max_n = kLoopMaxN;
  int nworkers = kWorkers;
  bool prune = true;
  int direct_running = 0;
  std::thread worker;                   // the loop thread
  std::vector<std::thread> workers;
  std::vector<hipStream_t> wstreams;
  // clock calibration: host ns = host0 + (ticks - dev0) * ns_per_tick
  int64_t host0 = 0;
  long long dev0 = 0;
  double ns_per_tick = 10.0;
  dbscan_server_stats stats{};

  int64_t dev_to_host(long long ticks) const {
    return host0 + (int64_t)((double)(ticks - dev0) * ns_per_tick);
  }
  long long host_to_dev(int64_t ns) const {
    return dev0 + (long long)((double)(ns - host0) / ns_per_tick);
  }
  void loop();
  void work(int w);
  bool admit_locked(std::vector<int> &fresh);
  void finish_locked(uint64_t id, int32_t state, int32_t error, int64_t t_done, int fallback);
};

void dbscan_server::finish_locked(uint64_t id, int32_t state, int32_t err, int64_t t_done,
                                  int fallback) {
  Record &r = records[id];
  r.status.state = state;
  r.status.error = err;
  // a loop job's completion is the device clock mapped to the host's, which
  // is calibrated to within half a round trip: never before the admission
  r.status.t_done_ns = t_done < r.status.t_admit_ns ? r.status.t_admit_ns : t_done;
  r.status.fallback = fallback;
  if (r.slot >= 0) {
    slot_job[r.slot] = 0;
    r.slot = -1;
  }
  if (r.held) {
    arena->release(r.arena_off, r.held);
    r.held = 0;
  }
  stats.jobs_done += 1;
  stats.points_done += r.job.n;
  stats.pairs_done += (double)r.job.n * (double)r.job.n;
}

// A worker: admits the oldest job of the workers' queue once its workspace
// fits in the arena and runs it through dbscan_fit_ex on the worker's own
// stream (the call waits for that stream, so the device time of one job
// overlaps with the other workers' jobs and with the loop's epochs).
void dbscan_server::work(int w) {
  std::unique_lock<std::mutex> lk(mu);
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    error = DBSCAN_E_DEVICE;  // the other threads fail the queued jobs
    cv.notify_all();
    return;
  }
  const hipStream_t ws = wstreams[w];
  for (;;) {
    uint64_t id = 0, off = 0;
    if (!direct_pending.empty() && error == DBSCAN_OK) {
      Record &r = records[direct_pending.front()];
      if (arena->alloc(r.need, &off)) {
        id = direct_pending.front();
        direct_pending.pop_front();
        r.arena_off = off;
        r.held = r.need;
        r.status.state = DBSCAN_JOB_RUNNING;
        if (!r.status.t_admit_ns) r.status.t_admit_ns = now_ns();
        r.status.footprint = r.need;
        direct_running += 1;
        stats.jobs_admitted += 1;
        if (arena->used() > stats.peak_bytes) stats.peak_bytes = arena->used();
      }
    }
    if (id) {
      const dbscan_job j = records[id].job;
      const uint64_t need = records[id].need;
      lk.unlock();
      dbscan_opts o = direct_opts(j, prune);
      o.workspace = arena_base + off;  // arena offsets are multiples of 256
      o.workspace_bytes = need;
      int rc = dbscan_fit_ex(j.points, j.n, j.d, j.eps, j.minpts, j.labels, j.core, j.counts,
                             (void *)ws, &o, nullptr);
      // the call's device state opens its workspace: its status word says
      // whether an input was not finite
      unsigned status = 0;
      if (rc == DBSCAN_OK) {
        hipError_t e = hipMemcpyAsync(&status, o.workspace, sizeof(status),
                                      hipMemcpyDeviceToHost, ws);
        if (e == hipSuccess) e = hipStreamSynchronize(ws);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          rc = DBSCAN_E_DEVICE;
        } else if (status & dbk::kStatusNonFinite) {
          rc = DBSCAN_E_NONFINITE;
        }
      }
      // a failed call may have left work queued: the arena slice is released
      // only once the stream holds nothing that uses it
      if (rc != DBSCAN_OK && rc != DBSCAN_E_NONFINITE) (void)hipStreamSynchronize(ws);
      const int64_t t = now_ns();
      lk.lock();
      const bool done = rc == DBSCAN_OK || rc == DBSCAN_E_NONFINITE;  // labels -2 if non-finite
      if (rc == DBSCAN_E_DEVICE) error = DBSCAN_E_DEVICE;
      direct_running -= 1;
      finish_locked(id, done ? DBSCAN_JOB_DONE : DBSCAN_JOB_FAILED, rc, t, 1);
      cv.notify_all();
      continue;
    }
    if (stopping && loop_done && direct_pending.empty()) break;
    if (error != DBSCAN_OK) {
      while (!direct_pending.empty()) {
        finish_locked(direct_pending.front(), DBSCAN_JOB_FAILED, error, now_ns(), 1);
        direct_pending.pop_front();
      }
      cv.notify_all();
      if (stopping && loop_done) break;
    }
    cv.wait_for(lk, std::chrono::milliseconds(1));
  }
}

// Move queued jobs into free slots while their footprint fits (FIFO).
bool dbscan_server::admit_locked(std::vector<int> &fresh) {
  while (!pending.empty()) {
    const uint64_t id = pending.front();
    Record &r = records[id];
    int slot = -1;
    for (int s = 0; s < nslots; ++s)
      if (slot_job[s] == 0) {
        slot = s;
        break;
      }
    if (slot < 0) return false;
    uint64_t off = 0;
    if (!arena->alloc(r.layout.total, &off)) return false;
    pending.pop_front();
    r.slot = slot;
    r.arena_off = off;
    r.held = r.layout.total;
    slot_job[slot] = id;
    r.status.state = DBSCAN_JOB_RUNNING;
    r.status.t_admit_ns = now_ns();
    r.status.footprint = r.layout.total;
    fresh.push_back(slot);
    stats.jobs_admitted += 1;
    if (arena->used() > stats.peak_bytes) stats.peak_bytes = arena->used();
  }
  return true;
}

void dbscan_server::loop() {
  if (hipSetDevice(device) != hipSuccess) {
    std::lock_guard<std::mutex> g(mu);
    error = DBSCAN_E_DEVICE;
    while (!pending.empty()) {
      finish_locked(pending.front(), DBSCAN_JOB_FAILED, DBSCAN_E_DEVICE, now_ns(), 0);
      pending.pop_front();
    }
    loop_done = true;
    cv.notify_all();
    return;
  }
  std::vector<int> fresh;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    fresh.clear();
    admit_locked(fresh);
    bool active = false;
    for (int s = 0; s < nslots; ++s) active |= slot_job[s] != 0;
    if (!active && pending.empty()) {
      if (stopping) break;
      cv.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    // descriptors of newly admitted jobs
    struct Upload {
      int slot;
      dbk::JobDesc jd;
      char *state;
    };
    std::vector<Upload> descs;
    for (int s : fresh) {
      const uint64_t id = slot_job[s];
      Record &r = records[id];
      const ServeLayout &L = r.layout;
      char *ws = arena_base + r.arena_off;
      dbk::JobDesc jd{};
      jd.pts = r.job.points;
      jd.labels = r.job.labels;
      jd.core = r.job.core;
      jd.counts = r.job.counts;
      jd.st = (dbk::DevState *)(ws + L.off_state);
      jd.soa = (float *)(ws + L.off_soa);
      jd.parent = (int *)(ws + L.off_parent);
      jd.jstar = (int *)(ws + L.off_jstar);
      jd.corebits = (uint32_t *)(ws + L.off_corebits);
      jd.pairs = (int2 *)(ws + L.off_pairs);
      jd.band = (int2 *)(ws + L.off_band);
      jd.a_aug = ws + L.off_aaug;
      jd.b_aug = ws + L.off_baug;
      jd.n = (int)r.job.n;
      jd.n_pad = L.n_pad;
      jd.d = r.job.d;
      jd.d_pad = L.d_pad;
      jd.minpts = r.job.minpts;
      jd.mfma_ks = L.ks;
      jd.eps2 = r.job.eps * r.job.eps;
      jd.band_rel = 1e-2;
      serve_band(jd.eps2, r.job.d, &jd.lo, &jd.hi);
      jd.pair_cap = L.pair_cap;
      jd.band_cap = L.band_cap;
      dbk::JobSched js{};
      js.claim = 0;
      js.state = dbk::kJobActive;
      const unsigned blocks256 = (unsigned)(L.n_pad / 256);
      js.ntasks[dbk::kPhStage] = blocks256;
      js.ntasks[dbk::kPhThresh] = L.ks ? 1u : 0u;
      if (L.ks) {
        // 256 stationary columns per task, row chunks of <= 128 tiles of 32
        // rows; only the lower triangle of (chunk, column group) is a task
        const int tiles = L.n_pad / 32;
        const int per = dbk::mfma_chunk_for(tiles, 128);
        jd.chunk = per;
        jd.nchunks = (tiles + per - 1) / per;
        js.ntasks[dbk::kPhCount] =
            (unsigned)dbk::mfma_items_before((int)blocks256, jd.nchunks, per / 8);
      } else {
        // triangular sweep: 128 rows x a column chunk of <= 4096 per task
        jd.chunk = L.n_pad < dbk::kServeTriChunk ? L.n_pad : dbk::kServeTriChunk;
        jd.nchunks = (L.n_pad + jd.chunk - 1) / jd.chunk;
        jd.rgroup = dbk::kServeTriRows;
        const unsigned groups = (unsigned)((jd.n + jd.rgroup - 1) / jd.rgroup);
        js.ntasks[dbk::kPhCount] = groups * (unsigned)jd.nchunks;
      }
      js.ntasks[dbk::kPhCore] = blocks256;
      js.ntasks[dbk::kPhLabels] = (unsigned)((jd.n + 255) / 256);
      h_sched[s] = js;
      descs.push_back(Upload{s, jd, ws + L.off_state});
    }
    lk.unlock();
    hipError_t e = hipSuccess;
    static const dbk::DevState zero_state{};
    for (const Upload &u : descs) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(u.state, &zero_state, sizeof(zero_state), hipMemcpyHostToDevice,
                           stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_jobs + u.slot, &u.jd, sizeof(dbk::JobDesc), hipMemcpyHostToDevice,
                           stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_sched + u.slot, &h_sched[u.slot], sizeof(dbk::JobSched),
                           hipMemcpyHostToDevice, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // host staging buffers reused
    bool persistent_active = false;
    lk.lock();
    for (int s = 0; s < nslots; ++s)
      if (slot_job[s]) persistent_active = true;
    lk.unlock();
    if (persistent_active && e == hipSuccess) {
      const int64_t t0 = now_ns();
      const long long deadline = host_to_dev(t0 + (int64_t)epoch_us * 1000);
      e = dbk::run_serve_epoch(d_jobs, d_sched, nslots, deadline, blocks, stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(h_sched.data(), d_sched, sizeof(dbk::JobSched) * nslots,
                           hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      const int64_t t1 = now_ns();
      std::lock_guard<std::mutex> g(mu);
      stats.epochs += 1;
      stats.busy_ns += t1 - t0;
    }
    lk.lock();
    if (e != hipSuccess) {
      error = DBSCAN_E_DEVICE;
      for (int s = 0; s < nslots; ++s)
        if (slot_job[s]) finish_locked(slot_job[s], DBSCAN_JOB_FAILED, DBSCAN_E_DEVICE, now_ns(), 0);
      while (!pending.empty()) {
        finish_locked(pending.front(), DBSCAN_JOB_FAILED, DBSCAN_E_DEVICE, now_ns(), 0);
        pending.pop_front();
      }
      break;
    }
    // harvest
    for (int s = 0; s < nslots; ++s) {
      const uint64_t id = slot_job[s];
      if (!id) continue;
      const dbk::JobSched &js = h_sched[s];
      if (js.state == dbk::kJobDone) {
        const int err = (js.fail_status & dbk::kStatusNonFinite) ? DBSCAN_E_NONFINITE : DBSCAN_OK;
        finish_locked(id, DBSCAN_JOB_DONE, err, dev_to_host(js.t_done), 0);
      } else if (js.state == dbk::kJobFailed) {
        // pair/band list overflow or inputs outside the FP16 range: the job
        // moves to the front of the workers' queue (same results)
        Record &r = records[id];
        slot_job[s] = 0;
        r.slot = -1;
        arena->release(r.arena_off, r.held);
        r.held = 0;
        r.direct = true;
        int rc = DBSCAN_OK;
        r.need = direct_bytes(r.job, prune, &rc);
        if (rc != DBSCAN_OK || r.need > budget) {
          finish_locked(id, DBSCAN_JOB_FAILED, rc != DBSCAN_OK ? rc : DBSCAN_E_NOMEM, now_ns(), 1);
        } else {
          r.status.state = DBSCAN_JOB_QUEUED;
          direct_pending.push_front(id);
        }
      }
    }
    cv.notify_all();
  }
  loop_done = true;
  cv.notify_all();
}

extern "C" {

int dbscan_server_create(int device, uint64_t hbm_budget_bytes, int32_t max_slots,
                         dbscan_server **out) {
  if (!out || max_slots < 1 || max_slots > 4096) return DBSCAN_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return DBSCAN_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return DBSCAN_E_DEVICE;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return DBSCAN_E_DEVICE;
  const uint64_t budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.8 * (double)free_b);
  if (budget > free_b) return DBSCAN_E_NOMEM;
  auto *s = new dbscan_server();
  s->device = device;
  s->nslots = max_slots;
  s->budget = round_up(budget, 256);
  bool ok = hipMalloc((void **)&s->arena_base, s->budget) == hipSuccess &&
            hipMalloc((void **)&s->d_jobs, sizeof(dbk::JobDesc) * max_slots) == hipSuccess &&
            hipMalloc((void **)&s->d_sched, sizeof(dbk::JobSched) * max_slots) == hipSuccess &&
            hipMalloc((void **)&s->d_clock, sizeof(long long)) == hipSuccess &&
            hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
  // tuning: DBSCAN_SERVE_WORKERS (1-16 worker streams), DBSCAN_SERVE_PRUNE=0
  // (no tile pruning on the workers), DBSCAN_SERVE_LOOP_MAX_N (largest n the
  // persistent loop takes)
  if (const char *v = getenv("DBSCAN_SERVE_WORKERS")) {
    const int w = atoi(v);
    if (w >= 1 && w <= kMaxWorkers) s->nworkers = w;
  }
  if (const char *v = getenv("DBSCAN_SERVE_PRUNE")) s->prune = atoi(v) != 0;
  if (const char *v = getenv("DBSCAN_SERVE_LOOP_MAX_N")) {
    const long long m = atoll(v);
    if (m >= 0) s->loop_max_n = m;
  }
  for (int w = 0; ok && w < s->nworkers; ++w) {
    hipStream_t ws = nullptr;
    ok = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) == hipSuccess;
    if (ok) s->wstreams.push_back(ws);
  }
  if (ok) {
    s->h_sched.assign(max_slots, dbk::JobSched{});
    s->slot_job.assign(max_slots, 0);
    ok = hipMemcpy(s->d_sched, s->h_sched.data(), sizeof(dbk::JobSched) * max_slots,
                   hipMemcpyHostToDevice) == hipSuccess;
  }
  int cus = 0, khz = 0;
  if (ok) {
    ok = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) ==
             hipSuccess &&
         hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
         khz > 0;
  }
  if (ok) {
    s->blocks = 3 * cus;
    s->ns_per_tick = 1e6 / (double)khz;
    // the device clock read in the middle of a host interval: the shortest
    // of four round trips (the first one also loads the kernel)
    int64_t best = -1;
    for (int k = 0; ok && k < 4; ++k) {
      long long ticks = 0;
      const int64_t a = now_ns();
      ok = dbk::run_read_clock(s->d_clock, s->stream) == hipSuccess &&
           hipMemcpyAsync(&ticks, s->d_clock, sizeof(long long), hipMemcpyDeviceToHost,
                          s->stream) == hipSuccess &&
           hipStreamSynchronize(s->stream) == hipSuccess;
      const int64_t b = now_ns();
      if (ok && (best < 0 || b - a < best)) {
        best = b - a;
        s->dev0 = ticks;
        s->host0 = (a + b) / 2;
      }
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->d_jobs) (void)hipFree(s->d_jobs);
    if (s->d_sched) (void)hipFree(s->d_sched);
    if (s->d_clock) (void)hipFree(s->d_clock);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    for (hipStream_t ws : s->wstreams) (void)hipStreamDestroy(ws);
    delete s;
    return DBSCAN_E_NOMEM;
  }
  s->arena = new Arena(s->budget);
  s->stats.budget_bytes = s->budget;
  s->worker = std::thread([s] { s->loop(); });
  for (int w = 0; w < s->nworkers; ++w) s->workers.emplace_back([s, w] { s->work(w); });
  *out = s;
  return DBSCAN_OK;
}

int dbscan_batch_submit(dbscan_server *s, const dbscan_job *job, uint64_t *job_id) {
  if (!s || !job || !job_id) return DBSCAN_E_INVAL;
  if (!job->points || !job->labels || !job->core || !job->counts) return DBSCAN_E_INVAL;
  if (job->n < 1 || job->n > DBSCAN_MAX_N || job->d < 1 || job->d > 1024) return DBSCAN_E_INVAL;
  if (!(job->eps >= 0.0) || !isfinite(job->eps) || job->minpts < 1) return DBSCAN_E_INVAL;
  if (job->precision < DBSCAN_PREC_AUTO || job->precision > DBSCAN_PREC_FP16) return DBSCAN_E_INVAL;
  const ServeLayout L = serve_layout(*job, s->loop_max_n);
  uint64_t need = L.total;
  if (!L.persistent) {
    int rc = DBSCAN_OK;
    need = direct_bytes(*job, s->prune, &rc);
    if (rc != DBSCAN_OK) return rc;  // e.g. a matrix-core precision for d > 76
  }
  if (need > s->budget) return DBSCAN_E_NOMEM;  // could never be admitted
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != DBSCAN_OK) return s->error;
  if ((int)(s->pending.size() + s->direct_pending.size()) >= kMaxQueue) return DBSCAN_E_AGAIN;
  const uint64_t id = s->next_id++;
  Record &r = s->records[id];
  r.job = *job;
  r.layout = L;
  r.direct = !L.persistent;
  r.need = need;
  r.status.state = DBSCAN_JOB_QUEUED;
  r.status.t_submit_ns = now_ns();
  r.status.footprint = need;
  r.status.tag = job->tag;
  (r.direct ? s->direct_pending : s->pending).push_back(id);
  s->stats.jobs_submitted += 1;
  *job_id = id;
  s->cv.notify_all();
  return DBSCAN_OK;
}

int dbscan_batch_poll(dbscan_server *s, uint64_t job_id, dbscan_job_status *st) {
  if (!s || !st) return DBSCAN_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->records.find(job_id);
  if (it == s->records.end()) return DBSCAN_E_INVAL;
  *st = it->second.status;
  if (st->state == DBSCAN_JOB_DONE || st->state == DBSCAN_JOB_FAILED) {
    s->records.erase(it);  // a finished job's status is returned once
    return DBSCAN_OK;
  }
  return DBSCAN_PENDING;
}

int dbscan_batch_wait(dbscan_server *s, uint64_t job_id, int64_t timeout_ns,
                      dbscan_job_status *st) {
  if (!s || !st) return DBSCAN_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto until = Clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? 0 : timeout_ns);
  for (;;) {
    auto it = s->records.find(job_id);
    if (it == s->records.end()) return DBSCAN_E_INVAL;
    *st = it->second.status;
    if (st->state == DBSCAN_JOB_DONE || st->state == DBSCAN_JOB_FAILED) {
      s->records.erase(it);  // a finished job's status is returned once
      return DBSCAN_OK;
    }
    if (s->error != DBSCAN_OK) return s->error;
    if (s->cv.wait_until(lk, until) == std::cv_status::timeout) {
      it = s->records.find(job_id);
      *st = it->second.status;
      if (st->state == DBSCAN_JOB_DONE || st->state == DBSCAN_JOB_FAILED) {
        s->records.erase(it);
        return DBSCAN_OK;
      }
      return DBSCAN_PENDING;
    }
  }
}

int dbscan_server_get_stats(dbscan_server *s, dbscan_server_stats *out) {
  if (!s || !out) return DBSCAN_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued = (int64_t)(s->pending.size() + s->direct_pending.size());
  int running = s->direct_running;
  for (int i = 0; i < s->nslots; ++i) running += s->slot_job[i] != 0;
  out->running = running;
  out->arena_used = s->arena->used();
  return DBSCAN_OK;
}

int dbscan_server_destroy(dbscan_server *s) {
  if (!s) return DBSCAN_E_INVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &w : s->workers)
    if (w.joinable()) w.join();
  const int err = s->error;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  for (hipStream_t ws : s->wstreams) {
    (void)hipStreamSynchronize(ws);
    (void)hipStreamDestroy(ws);
  }
  (void)hipFree(s->arena_base);
  (void)hipFree(s->d_jobs);
  (void)hipFree(s->d_sched);
  (void)hipFree(s->d_clock);
  (void)hipStreamDestroy(s->stream);
  delete s->arena;
  delete s;
  return err;
}

}  // extern "C"
