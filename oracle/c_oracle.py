"""ctypes wrapper for the C oracle (``dbscan_oracle.c``) -- TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_dbscan.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_int32, _i32p, _u8p, _i32p, ctypes.c_int]
        L.oracle_dbscan.restype = ctypes.c_int
        L.oracle_row_counts.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                        _i64p, ctypes.c_int64, _i32p, ctypes.c_int]
        L.oracle_row_counts.restype = ctypes.c_int
        L.oracle_row_neighbours.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_int64, _u8p]
        L.oracle_row_neighbours.restype = ctypes.c_int
        L.oracle_first_core_neighbour.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int32,
                                                  ctypes.c_double, _u8p, ctypes.c_int64]
        L.oracle_first_core_neighbour.restype = ctypes.c_int64
        L.oracle_max_threads.argtypes = [ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _pts(points):
    x = np.ascontiguousarray(points, dtype=np.float32)
    if x.ndim != 2:
        raise ValueError("points must be (n, d)")
    return x


def threads(requested: int = 0) -> int:
    """Threads the oracle will use (all host cores when requested == 0)."""
    return int(lib().oracle_max_threads(int(requested)))


def dbscan(points, eps: float, minpts: int, threads: int = 0):
    x = _pts(points)
    n, d = x.shape
    labels = np.empty(n, np.int32)
    core = np.empty(n, np.uint8)
    counts = np.empty(n, np.int32)
    rc = lib().oracle_dbscan(x.ctypes.data_as(_f32p), n, d, float(eps), int(minpts),
                             labels.ctypes.data_as(_i32p), core.ctypes.data_as(_u8p),
                             counts.ctypes.data_as(_i32p), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_dbscan failed: {rc}")
    return labels, core.astype(bool), counts


def row_counts(points, eps: float, rows, threads: int = 0) -> np.ndarray:
    x = _pts(points)
    n, d = x.shape
    r = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(r.shape[0], np.int32)
    rc = lib().oracle_row_counts(x.ctypes.data_as(_f32p), n, d, float(eps), r.ctypes.data_as(_i64p),
                                 r.shape[0], out.ctypes.data_as(_i32p), int(threads))
    if rc != 0:
        raise RuntimeError("oracle_row_counts failed")
    return out


def row_neighbours(points, eps: float, i: int) -> np.ndarray:
    x = _pts(points)
    n, d = x.shape
    out = np.empty(n, np.uint8)
    rc = lib().oracle_row_neighbours(x.ctypes.data_as(_f32p), n, d, float(eps), int(i),
                                     out.ctypes.data_as(_u8p))
    if rc != 0:
        raise RuntimeError("oracle_row_neighbours failed")
    return out.astype(bool)


def first_core_neighbour(points, eps: float, core, i: int) -> int:
    x = _pts(points)
    n, d = x.shape
    c = np.ascontiguousarray(core, dtype=np.uint8)
    return int(lib().oracle_first_core_neighbour(x.ctypes.data_as(_f32p), n, d, float(eps),
                                                 c.ctypes.data_as(_u8p), int(i)))
