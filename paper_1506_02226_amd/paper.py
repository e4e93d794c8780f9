"""The paper's own three-step design on the GPU, as measured ablations of the
main path (``include/dbscan_paper.h``): the float distance matrix of
Section IV-A (Table III's four kernels), the byte cluster matrix of Section
IV-B (from the matrix, fused, fused with the hoisted form; Table IV) and the
merges of Section IV-C (targets) and Section VI (Warshall closure).

Argument marshalling only: every step runs in the HIP kernels of
``libdbscan.so``."""
from __future__ import annotations

import ctypes

from . import _lib

DIST_KERNELS = {"baseline": 1, "coalesced": 2, "shared": 3, "unrolled": 4}
CLUSTER_KERNELS = {"from_dist": 5, "fused": 6, "hoisted": 7}
MERGE_KERNELS = {"targets": 8, "warshall": 9}


def _points(points):
    import torch
    if not (isinstance(points, torch.Tensor) and points.device.type == "cuda"
            and points.dtype == torch.float32 and points.dim() == 2):
        raise ValueError("points must be a 2-D float32 tensor on the GPU")
    return points.contiguous()


def _stream(dev):
    import torch
    return torch.cuda.current_stream(dev).cuda_stream


def distance(points, kernel: str = "unrolled", out=None):
    """n x n float32 squared distances (Section IV-A)."""
    import torch
    x = _points(points)
    n, d = x.shape
    dist = out if out is not None else torch.empty((n, n), dtype=torch.float32, device=x.device)
    with torch.cuda.device(x.device):
        rc = _lib.load().dbscan_paper_distance(x.data_ptr(), n, d, DIST_KERNELS[kernel],
                                               dist.data_ptr(), _stream(x.device))
    if rc != _lib.DBSCAN_OK:
        raise _lib.DbscanError(rc, "dbscan_paper_distance")
    return dist


def cluster(points, eps: float, minpts: int, kernel: str = "hoisted", dist=None, out=None,
            rechecked: bool = False):
    """(cluster uint8 n x n, valid uint8[n], counts int32[n]) of Section IV-B,
    plus the float64 re-evaluation count when ``rechecked`` (waits)."""
    import torch
    x = _points(points)
    n, d = x.shape
    if out is None:
        out = (torch.empty((n, n), dtype=torch.uint8, device=x.device),
               torch.empty(n, dtype=torch.uint8, device=x.device),
               torch.empty(n, dtype=torch.int32, device=x.device))
    cl, valid, counts = out
    r = ctypes.c_uint64(0)
    with torch.cuda.device(x.device):
        rc = _lib.load().dbscan_paper_cluster(
            x.data_ptr(), dist.data_ptr() if dist is not None else None, n, d, float(eps),
            int(minpts), CLUSTER_KERNELS[kernel], cl.data_ptr(), valid.data_ptr(),
            counts.data_ptr(), ctypes.byref(r) if rechecked else None, _stream(x.device))
    if rc != _lib.DBSCAN_OK:
        raise _lib.DbscanError(rc, "dbscan_paper_cluster")
    return (cl, valid, counts, int(r.value)) if rechecked else (cl, valid, counts)


def merge(cluster_matrix, valid, kernel: str = "targets", labels=None, alive: bool = False):
    """Canonical labels from the cluster matrix (Section IV-C targets, merged
    in place, or the Warshall closure of Section VI).  Returns (labels,
    launches) or (labels, alive, launches).  Synchronous."""
    import torch
    n = int(valid.shape[0])
    dev = valid.device
    lab = labels if labels is not None else torch.empty(n, dtype=torch.int32, device=dev)
    al = torch.empty(n, dtype=torch.uint8, device=dev) if alive else None
    nl = ctypes.c_int64(0)
    with torch.cuda.device(dev):
        rc = _lib.load().dbscan_paper_merge(cluster_matrix.data_ptr(), valid.data_ptr(), n,
                                            MERGE_KERNELS[kernel], lab.data_ptr(),
                                            al.data_ptr() if al is not None else None,
                                            ctypes.byref(nl), _stream(dev))
    if rc != _lib.DBSCAN_OK:
        raise _lib.DbscanError(rc, "dbscan_paper_merge")
    return (lab, al, int(nl.value)) if alive else (lab, int(nl.value))
