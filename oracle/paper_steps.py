"""Plain CPU oracle for the paper's own intermediate products -- TEST
INFRASTRUCTURE ONLY (tests and the benchmark's CPU leg; never the product).

The paper's design (Section IV) materialises two n x n matrices and merges
primitive clusters by targets.  These functions compute those products from
their definitions, for the GPU kernels that reproduce that design as
ablations of the main path:

* ``distance_matrix_f32`` -- Section IV-A: the squared distance of every
  ordered pair, the float ("floating point", Section V-B) matrix the
  distance kernels write.  Reading taken: float32 arithmetic, the direct
  form of Section IV-B.2 summed over the coordinates in order 0..d-1, every
  operation rounded on its own (no fused multiply-add).
* ``cluster_matrix`` -- Section IV-B: cluster[i][j] = 1 iff point j lies in
  the eps-neighbourhood of point i, decided as the float64 definition decides
  it (the oracle's neighbour relation), and valid[i] = (count >= MinPts).
* ``target_merge`` -- Section IV-C: for each target (a valid cluster, taken
  in ascending index order), every other valid cluster that shares a core
  point with it is merged into it (its row ORed into the target's row) and
  made invalid; this repeats until nothing merges.  Reading taken for the
  criterion, which the paper does not state: two primitive clusters merge iff
  they share a core point (nothing is reachable from a non-core point,
  Section II).
"""
from __future__ import annotations

import numpy as np

from . import dbscan_oracle as orc

__all__ = ["distance_matrix_f32", "cluster_matrix", "target_merge", "labels_from_merge"]


def distance_matrix_f32(points: np.ndarray) -> np.ndarray:
    """n x n float32 squared distances, coordinate order, unfused."""
    x = np.asarray(points, dtype=np.float32)
    if x.ndim != 2:
        raise ValueError("points must be (n, d)")
    s = None
    for k in range(x.shape[1]):
        t = x[:, k][:, None] - x[None, :, k]  # float32, rounded once
        tt = t * t                             # float32, rounded once
        s = tt if s is None else s + tt        # float32, rounded once
    return s


def cluster_matrix(points: np.ndarray, eps: float, minpts: int):
    """(cluster uint8[n][n], valid bool[n], counts int64[n]) of Section IV-B."""
    adj = orc.neighbour_matrix(points, eps)
    counts = orc.counts_from_matrix(adj)
    return adj.astype(np.uint8), counts >= minpts, counts


def target_merge(cluster: np.ndarray, valid: np.ndarray):
    """Section IV-C on a copy of the primitive cluster matrix.

    Returns (merged uint8[n][n], alive bool[n]): the rows of the surviving
    clusters after every target has absorbed the clusters that share a core
    point with it, and which clusters survive."""
    core = np.asarray(valid, dtype=bool)
    rows = np.array(cluster, dtype=bool)
    alive = core.copy()
    n = rows.shape[0]
    for t in range(n):
        if not alive[t]:
            continue
        while True:
            merged = False
            for c in range(n):
                if c == t or not alive[c]:
                    continue
                if (rows[c] & rows[t] & core).any():
                    rows[t] |= rows[c]
                    alive[c] = False
                    merged = True
            if not merged:
                break
    return rows.astype(np.uint8), alive


def labels_from_merge(prim: np.ndarray, merged: np.ndarray, alive: np.ndarray,
                      valid: np.ndarray) -> np.ndarray:
    """Canonical labels from the merge: a core point takes the surviving
    target whose row holds it; a non-core point takes the label of its
    lowest-index core neighbour (its primitive row), else -1."""
    core = np.asarray(valid, dtype=bool)
    n = core.shape[0]
    labels = np.full(n, -1, dtype=np.int64)
    for t in np.flatnonzero(alive):
        members = np.flatnonzero(merged[t].astype(bool) & core)
        labels[members] = t
    for j in range(n):
        if core[j]:
            continue
        nb = np.flatnonzero(prim[j].astype(bool) & core)
        if nb.size:
            labels[j] = labels[nb.min()]
    return labels
