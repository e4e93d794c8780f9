"""ctypes binding of libdbscan.so (the C ABI declared in include/dbscan.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library.  There is no CPU fallback -- if the library is
missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbscan.so")

DBSCAN_OK = 0
DBSCAN_PENDING = 1
DBSCAN_E_INVAL = -22
DBSCAN_E_NOMEM = -12
DBSCAN_E_AGAIN = -11
DBSCAN_E_DEVICE = -1000
DBSCAN_E_NONFINITE = -1001
DBSCAN_E_UNSUPPORTED = -1002

ADJ = {"auto": 0, "bitmask": 1, "onthefly": 2}
PREC = {"auto": 0, "fp32": 1, "bf16": 2, "fp16": 3}
ORDER = {"auto": 0, "input": 1, "spatial": 2}
ADJ_NAMES = {v: k for k, v in ADJ.items()}
PREC_NAMES = {v: k for k, v in PREC.items()}
ORDER_NAMES = {v: k for k, v in ORDER.items()}

# Every symbol include/dbscan.h and include/dbscan_paper.h declare.
EXPORTS = (
    "dbscan_fit",
    "dbscan_fit_ex",
    "dbscan_fit_noalloc",
    "dbscan_workspace_size",
    "dbscan_strerror",
    "dbscan_version",
    "dbscan_fp32_band",
    "dbscan_hoist_band",
    "dbscan_hoist_gate",
    "dbscan_server_create",
    "dbscan_batch_submit",
    "dbscan_batch_poll",
    "dbscan_batch_wait",
    "dbscan_server_get_stats",
    "dbscan_server_destroy",
    "dbscan_paper_distance",
    "dbscan_paper_cluster",
    "dbscan_paper_merge",
)

JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3


class Opts(ctypes.Structure):
    _fields_ = [
        ("adjacency", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("band_rel", ctypes.c_double),
        ("bitmask_limit", ctypes.c_uint64),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
        ("pair_capacity", ctypes.c_uint64),
        ("band_capacity", ctypes.c_uint64),
        ("events", ctypes.c_void_p),
        ("order", ctypes.c_int32),
        ("prune", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("hip_error", ctypes.c_int32),
        ("adjacency_used", ctypes.c_int32),
        ("precision_used", ctypes.c_int32),
        ("pairs_tested", ctypes.c_int64),
        ("pairs_rechecked", ctypes.c_int64),
        ("core_points", ctypes.c_int64),
        ("ms_step1", ctypes.c_float),
        ("ms_step2", ctypes.c_float),
        ("ms_step3", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("thr_lo", ctypes.c_float),
        ("thr_hi", ctypes.c_float),
        ("pairs_listed", ctypes.c_int64),
        ("pair_overflow", ctypes.c_int32),
        ("filter_fallback", ctypes.c_int32),
        ("ms_sweep1", ctypes.c_float),
        ("sweep1_tests", ctypes.c_int64),
        ("order_used", ctypes.c_int32),
        ("pruned", ctypes.c_int32),
        ("hoisted", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["adjacency_used"] = ADJ_NAMES.get(d["adjacency_used"], d["adjacency_used"])
        d["precision_used"] = PREC_NAMES.get(d["precision_used"], d["precision_used"])
        d["order_used"] = ORDER_NAMES.get(d["order_used"], d["order_used"])
        return d


class Job(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int32),
        ("minpts", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("labels", ctypes.c_void_p),
        ("core", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
        ("tag", ctypes.c_uint64),
        ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class JobStatus(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32),
        ("error", ctypes.c_int32),
        ("t_submit_ns", ctypes.c_int64),
        ("t_admit_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64),
        ("footprint", ctypes.c_uint64),
        ("tag", ctypes.c_uint64),
        ("fallback", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("jobs_submitted", ctypes.c_int64),
        ("jobs_admitted", ctypes.c_int64),
        ("jobs_done", ctypes.c_int64),
        ("queued", ctypes.c_int64),
        ("running", ctypes.c_int64),
        ("epochs", ctypes.c_int64),
        ("busy_ns", ctypes.c_int64),
        ("points_done", ctypes.c_int64),
        ("pairs_done", ctypes.c_double),
        ("budget_bytes", ctypes.c_uint64),
        ("arena_used", ctypes.c_uint64),
        ("peak_bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class DbscanError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        msg = load().dbscan_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})" if where else f"{msg} ({code})")


_lib = None


def load(path: str | None = None):
    """Load libdbscan.so (raises if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_1506_02226_amd/build.py`")
    L = ctypes.CDLL(p)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.dbscan_fit.argtypes = [vp, i64, i32, dbl, i32, vp, vp, vp, vp]
    L.dbscan_fit.restype = ctypes.c_int
    L.dbscan_fit_ex.argtypes = [vp, i64, i32, dbl, i32, vp, vp, vp, vp,
                                ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
    L.dbscan_fit_ex.restype = ctypes.c_int
    L.dbscan_fit_noalloc.argtypes = [vp, i64, i32, dbl, i32, vp, vp, vp, vp]
    L.dbscan_fit_noalloc.restype = ctypes.c_int
    L.dbscan_workspace_size.argtypes = [i64, i32, ctypes.POINTER(Opts),
                                        ctypes.POINTER(ctypes.c_uint64)]
    L.dbscan_workspace_size.restype = ctypes.c_int
    L.dbscan_strerror.argtypes = [ctypes.c_int]
    L.dbscan_strerror.restype = ctypes.c_char_p
    L.dbscan_version.argtypes = []
    L.dbscan_version.restype = ctypes.c_int
    L.dbscan_fp32_band.argtypes = [dbl, i32, ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float)]
    L.dbscan_fp32_band.restype = ctypes.c_int
    L.dbscan_hoist_band.argtypes = [dbl, i32, dbl, ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(ctypes.c_float)]
    L.dbscan_hoist_band.restype = ctypes.c_int
    L.dbscan_hoist_gate.argtypes = [ctypes.c_float, dbl, i32, ctypes.POINTER(ctypes.c_float)]
    L.dbscan_hoist_gate.restype = ctypes.c_int
    sp = ctypes.c_void_p
    L.dbscan_server_create.argtypes = [ctypes.c_int, ctypes.c_uint64, i32, ctypes.POINTER(sp)]
    L.dbscan_server_create.restype = ctypes.c_int
    L.dbscan_batch_submit.argtypes = [sp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
    L.dbscan_batch_submit.restype = ctypes.c_int
    L.dbscan_batch_poll.argtypes = [sp, ctypes.c_uint64, ctypes.POINTER(JobStatus)]
    L.dbscan_batch_poll.restype = ctypes.c_int
    L.dbscan_batch_wait.argtypes = [sp, ctypes.c_uint64, i64, ctypes.POINTER(JobStatus)]
    L.dbscan_batch_wait.restype = ctypes.c_int
    L.dbscan_server_get_stats.argtypes = [sp, ctypes.POINTER(ServerStats)]
    L.dbscan_server_get_stats.restype = ctypes.c_int
    L.dbscan_server_destroy.argtypes = [sp]
    L.dbscan_server_destroy.restype = ctypes.c_int
    u8p = ctypes.c_void_p
    L.dbscan_paper_distance.argtypes = [vp, i64, i32, i32, vp, vp]
    L.dbscan_paper_distance.restype = ctypes.c_int
    L.dbscan_paper_cluster.argtypes = [vp, vp, i64, i32, dbl, i32, i32, vp, vp, vp,
                                       ctypes.POINTER(ctypes.c_uint64), vp]
    L.dbscan_paper_cluster.restype = ctypes.c_int
    L.dbscan_paper_merge.argtypes = [u8p, vp, i64, i32, vp, vp, ctypes.POINTER(ctypes.c_int64), vp]
    L.dbscan_paper_merge.restype = ctypes.c_int
    if path is None:
        _lib = L
    return L


def make_opts(adjacency: str = "auto", precision: str = "auto", band_rel: float = 0.0,
              bitmask_limit: int = 0, workspace: int = 0, workspace_bytes: int = 0,
              events: int = 0, pair_capacity: int = 0, band_capacity: int = 0,
              order: str = "auto", prune: bool = False) -> Opts:
    return Opts(ADJ[adjacency], PREC[precision], float(band_rel), int(bitmask_limit),
                int(workspace) or None, int(workspace_bytes), int(pair_capacity),
                int(band_capacity), int(events) or None, ORDER[order], 1 if prune else 0)
