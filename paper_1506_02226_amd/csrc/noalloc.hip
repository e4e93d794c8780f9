// dbscan_fit_noalloc: dbscan_fit for callers that cannot allocate device
// memory.  The workspace of every call is one file-scope device array per
// GPU (DBSCAN_NOALLOC_SCRATCH_BYTES), held from the code object's load until
// the process ends; its device address is looked up once per device and the
// kernels receive that address, never the array's host-side name.
#include <mutex>

#include <hip/hip_runtime.h>

#include "../../include/dbscan.h"

static __device__ __align__(256) unsigned char scratch[DBSCAN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch`, per device

// Device address of the current device's copy of `scratch`.
int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return DBSCAN_E_DEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) return DBSCAN_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return DBSCAN_E_DEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return DBSCAN_OK;
}

uint64_t size_for(int64_t n, int32_t d, const dbscan_opts &o, int *rc) {
  uint64_t b = 0;
  *rc = dbscan_workspace_size(n, d, &o, &b);
  return b;
}

}  // namespace

extern "C" {

int dbscan_fit_noalloc(const float *points, int64_t n, int32_t d, double eps, int32_t minpts,
                       int32_t *labels, uint8_t *core, int32_t *counts, void *stream) {
  if (!points || !labels || !core || !counts) return DBSCAN_E_INVAL;
  if (n < 1 || n > DBSCAN_MAX_N || d < 1 || d > 1024) return DBSCAN_E_INVAL;
  const uint64_t room = DBSCAN_NOALLOC_SCRATCH_BYTES;
  dbscan_opts o = {};
  int rc = DBSCAN_OK;
  uint64_t need = size_for(n, d, o, &rc);
  if (rc) return rc;
  if (need > room) {
    // the default plan does not fit: no bit matrix, and pair / band lists
    // sized to the room that remains (a full pair list makes step 3 repeat
    // the epsilon tests instead, with the same results)
    o.adjacency = DBSCAN_ADJ_ONTHEFLY;
    o.pair_capacity = 1;
    o.band_capacity = 1;
    const uint64_t fixed = size_for(n, d, o, &rc);
    if (rc) return rc;
    if (fixed + 1024 > room) return DBSCAN_E_NOMEM;  // (n, d) beyond the array
    o.band_capacity = 1 + 64;
    const bool band = size_for(n, d, o, &rc) != fixed;  // matrix-core filter in use
    if (rc) return rc;
    const uint64_t spare = room - fixed - 1024;  // slack for 256-byte rounding
    o.pair_capacity = band ? spare / 8 * 2 / 3 : spare / 8;
    o.band_capacity = band ? spare / 8 / 3 : 1;
    if (o.pair_capacity < 1) o.pair_capacity = 1;
    if (o.band_capacity < 1) o.band_capacity = 1;
    need = size_for(n, d, o, &rc);
    if (rc) return rc;
    if (need > room) return DBSCAN_E_NOMEM;
  }
  rc = scratch_address(&o.workspace);
  if (rc) return rc;
  o.workspace_bytes = room;
  return dbscan_fit_ex(points, n, d, eps, minpts, labels, core, counts, stream, &o, nullptr);
}

}  // extern "C"
