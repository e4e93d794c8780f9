"""DBSCAN on one AMD Instinct MI355X (gfx950).

``fit(points, eps, minpts)`` runs the three steps of Wang et al., "Design and
optimization of DBSCAN Algorithm based on CUDA" -- the all-pairs epsilon test
(Section IV-A), neighbour counts, core flags and primitive clusters
(Section IV-B) and the merge of reachable core points (Section IV-C) -- in the
HIP kernels of ``libdbscan.so`` behind its C ABI (``include/dbscan.h``).
PyTorch only provides device memory and the stream.

Outputs equal the float64 definition bit for bit: ``counts`` include the point
itself, ``core = counts >= minpts``, and ``labels`` are canonical (-1 noise;
a core point's label is the lowest core index in its cluster; a border point
takes the label of its lowest-index core neighbour).
"""
from __future__ import annotations

import ctypes

from . import _lib

__all__ = ["fit", "workspace_size", "version", "DbscanError", "Server"]

DbscanError = _lib.DbscanError


def version() -> int:
    return int(_lib.load().dbscan_version())


def workspace_size(n: int, d: int, adjacency: str = "auto", precision: str = "auto",
                   bitmask_limit: int = 0, pair_capacity: int = 0, band_capacity: int = 0,
                   order: str = "auto", prune: bool = False) -> int:
    L = _lib.load()
    opts = _lib.make_opts(adjacency, precision, bitmask_limit=bitmask_limit,
                          pair_capacity=pair_capacity, band_capacity=band_capacity, order=order,
                          prune=prune)
    out = ctypes.c_uint64(0)
    rc = L.dbscan_workspace_size(int(n), int(d), ctypes.byref(opts), ctypes.byref(out))
    if rc != _lib.DBSCAN_OK:
        raise DbscanError(rc, "dbscan_workspace_size")
    return int(out.value)


def _check_points(points):
    import torch
    if not isinstance(points, torch.Tensor):
        raise TypeError("points must be a torch.Tensor on a ROCm device")
    if points.device.type != "cuda":
        raise ValueError("points must live on the GPU (device 'cuda')")
    if points.dtype != torch.float32 or points.dim() != 2:
        raise ValueError("points must be a 2-D float32 tensor (n, d)")
    return points.contiguous()


def fit(points, eps: float, minpts: int, *, adjacency: str = "auto", precision: str = "auto",
        band_rel: float = 0.0, bitmask_limit: int = 0, pair_capacity: int = 0,
        band_capacity: int = 0, stats: bool = False, out=None, workspace=None, events: int = 0,
        order: str = "auto", prune: bool = False):
    """Cluster `points` (torch float32 (n, d) on the GPU).

    Returns (labels int32[n], core uint8[n], counts int32[n]) as GPU tensors,
    plus a statistics dict when ``stats=True`` (the call then waits for the
    stream).  ``out`` may pass preallocated (labels, core, counts) tensors and
    ``workspace`` a uint8 GPU tensor of at least ``workspace_size`` bytes.
    ``events`` is the address of a caller-created hipEvent_t[6] that the
    library records around the steps (see dbscan_opts.events).  ``order``
    is "auto", "input" or "spatial" (dbscan_opts.order); ``prune`` skips
    the tests of tile pairs whose boxes are farther apart than eps
    (dbscan_opts.prune)."""
    import torch
    L = _lib.load()
    x = _check_points(points)
    n, d = int(x.shape[0]), int(x.shape[1])
    dev = x.device
    if out is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
        core = torch.empty(n, dtype=torch.uint8, device=dev)
        counts = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        labels, core, counts = out
    if workspace is None:
        # a caller-supplied workspace is checked against the size by the library
        ws_bytes = workspace_size(n, d, adjacency, precision, bitmask_limit, pair_capacity,
                                  band_capacity, order, prune)
        workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) // 256 * 256
    avail = workspace.numel() - (aligned - base)
    opts = _lib.make_opts(adjacency, precision, band_rel, bitmask_limit, aligned, avail, events,
                          pair_capacity, band_capacity, order, prune)
    st = _lib.Stats()
    stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        rc = L.dbscan_fit_ex(x.data_ptr(), n, d, float(eps), int(minpts), labels.data_ptr(),
                             core.data_ptr(), counts.data_ptr(), stream, ctypes.byref(opts),
                             ctypes.byref(st) if stats else None)
    if rc != _lib.DBSCAN_OK:
        raise DbscanError(rc, "dbscan_fit_ex")
    if stats:
        return labels, core, counts, st.as_dict()
    return labels, core, counts


class Server:
    """Continuously batched DBSCAN jobs on one GPU (dbscan_server_* ABI).

    ``submit`` queues a job on device tensors and returns its id; ``poll`` /
    ``wait`` return the status dict once the job is finished (None while it
    is pending; a finished status is returned once).  Jobs are admitted by
    device-memory footprint: small ones run together in the server's
    persistent kernel, the others on its worker streams beside it.  The
    caller keeps the input and output tensors alive until the job is
    finished (``submit`` also keeps a reference)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, max_slots: int = 256):
        self._L = _lib.load()
        h = ctypes.c_void_p()
        rc = self._L.dbscan_server_create(int(device), int(hbm_budget), int(max_slots),
                                          ctypes.byref(h))
        if rc != _lib.DBSCAN_OK:
            raise DbscanError(rc, "dbscan_server_create")
        self._h = h
        self._keep = {}

    def submit(self, points, eps: float, minpts: int, out=None, tag: int = 0,
               precision: str = "auto") -> int:
        import torch
        x = _check_points(points)
        n, d = int(x.shape[0]), int(x.shape[1])
        if out is None:
            out = (torch.empty(n, dtype=torch.int32, device=x.device),
                   torch.empty(n, dtype=torch.uint8, device=x.device),
                   torch.empty(n, dtype=torch.int32, device=x.device))
        labels, core, counts = out
        # the server reads the points on its own streams: the work that made
        # them (and any copy `_check_points` queued) must be complete
        torch.cuda.current_stream(x.device).synchronize()
        job = _lib.Job(x.data_ptr(), n, d, int(minpts), float(eps), labels.data_ptr(),
                       core.data_ptr(), counts.data_ptr(), int(tag), _lib.PREC[precision], 0)
        jid = ctypes.c_uint64()
        rc = self._L.dbscan_batch_submit(self._h, ctypes.byref(job), ctypes.byref(jid))
        if rc != _lib.DBSCAN_OK:
            raise DbscanError(rc, "dbscan_batch_submit")
        self._keep[int(jid.value)] = (x, out)
        return int(jid.value)

    def outputs(self, job_id: int):
        return self._keep[job_id][1]

    def poll(self, job_id: int):
        st = _lib.JobStatus()
        rc = self._L.dbscan_batch_poll(self._h, int(job_id), ctypes.byref(st))
        if rc == _lib.DBSCAN_PENDING:
            return None
        if rc != _lib.DBSCAN_OK:
            raise DbscanError(rc, "dbscan_batch_poll")
        return st.as_dict()

    def wait(self, job_id: int, timeout: float = 60.0):
        st = _lib.JobStatus()
        rc = self._L.dbscan_batch_wait(self._h, int(job_id), int(timeout * 1e9), ctypes.byref(st))
        if rc == _lib.DBSCAN_PENDING:
            return None
        if rc != _lib.DBSCAN_OK:
            raise DbscanError(rc, "dbscan_batch_wait")
        return st.as_dict()

    def release(self, job_id: int) -> None:
        self._keep.pop(job_id, None)

    def stats(self) -> dict:
        st = _lib.ServerStats()
        rc = self._L.dbscan_server_get_stats(self._h, ctypes.byref(st))
        if rc != _lib.DBSCAN_OK:
            raise DbscanError(rc, "dbscan_server_get_stats")
        return st.as_dict()

    def close(self) -> None:
        if self._h is not None:
            rc = self._L.dbscan_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            if rc != _lib.DBSCAN_OK:
                raise DbscanError(rc, "dbscan_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
