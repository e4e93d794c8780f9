"""Plain CPU oracle for DBSCAN (numpy, float64) -- TEST INFRASTRUCTURE ONLY.

This module is the reference that the GPU path is checked against.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
it; the product path never calls it and never falls back to it.

What it computes follows the paper directly, with no blocking or reordering
beyond the definitions:

* Section II, definitions 1-3: the eps-neighbourhood of p is every point
  within distance eps of p (p itself included, at distance 0); p is a core
  point when at least MinPts points lie in that neighbourhood; only core
  points make other points reachable.
* Section II, the cluster definition (maximality and connectivity): a cluster
  is a connected component of the eps-graph restricted to core points,
  together with the non-core points reachable from it.
* Section IV-A: the test is carried out on squared distances against eps^2
  (no square root); Section IV-B writes the test as distance <= eps^2, so a
  pair exactly eps apart is a neighbour.
* Section II, serial algorithm steps 1-3: distances of every pair, core
  points and their neighbourhoods (primitive clusters), then merging of
  reachable core points; the merge here is a breadth-first search.

Readings taken where the paper is silent or inconsistent:

* squared distance in float64: s = 0; for k = 0..d-1: t = x_ik - x_jk;
  s = s + t*t; each operation rounded on its own (numpy never fuses a
  multiply into an add), coordinates widened exactly from float32, and
  eps^2 rounded once from the caller's double eps;
* core test is count >= MinPts (Section II's "at least"), not the
  "greater than" wording of Section IV-B;
* cluster id = the lowest index of a core point in the component (BFS runs
  from each unvisited core point in ascending index order);
* a non-core point with core neighbours takes the cluster of its
  lowest-index core neighbour; every other point is noise, labelled -1.
"""
from __future__ import annotations

from collections import deque

import numpy as np

__all__ = [
    "eps_squared",
    "sq_dist_row",
    "neighbour_row",
    "neighbour_matrix",
    "counts_from_matrix",
    "bfs_labels",
    "warshall_labels",
    "dbscan",
    "row_counts",
]


def eps_squared(eps: float) -> float:
    """eps^2 rounded once in float64 (Section IV-A compares against eps^2)."""
    e = np.float64(eps)
    return float(e * e)


def _as64(points: np.ndarray) -> np.ndarray:
    x = np.asarray(points)
    if x.ndim != 2:
        raise ValueError("points must be (n, d)")
    return x.astype(np.float64)


def _sq_block(xr: np.ndarray, xc: np.ndarray) -> np.ndarray:
    """Squared distances between every row of xr and every row of xc, the
    direct form of dist(t, p[n]) in Section IV-B.2, summed over the
    coordinates in order 0..d-1 with each float64 operation rounded alone."""
    s = np.zeros((xr.shape[0], xc.shape[0]), dtype=np.float64)
    for k in range(xr.shape[1]):
        t = xr[:, k][:, None] - xc[None, :, k]
        s = s + t * t
    return s


def sq_dist_row(x64: np.ndarray, i: int, cols: np.ndarray | slice = slice(None)) -> np.ndarray:
    """Squared distances from point i to the points `cols`."""
    return _sq_block(x64[i : i + 1], x64[cols])[0]


def neighbour_row(x64: np.ndarray, i: int, eps2: float) -> np.ndarray:
    """Boolean eps-neighbourhood of point i (Section II, definition 1)."""
    return sq_dist_row(x64, i) <= eps2


def neighbour_matrix(points: np.ndarray, eps: float, block: int = 512) -> np.ndarray:
    """Full n x n boolean neighbour matrix (the paper's cluster matrix,
    Section IV-B), for small n only."""
    x64 = _as64(points)
    n = x64.shape[0]
    eps2 = eps_squared(eps)
    adj = np.zeros((n, n), dtype=bool)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        adj[r0:r1] = _sq_block(x64[r0:r1], x64) <= eps2
    return adj


def counts_from_matrix(adj: np.ndarray) -> np.ndarray:
    return adj.sum(axis=1).astype(np.int64)


def _border_labels(adj_rows, core: np.ndarray, labels: np.ndarray) -> np.ndarray:
    n = core.shape[0]
    for i in range(n):
        if core[i]:
            continue
        nb = np.flatnonzero(adj_rows(i) & core)
        if nb.size:
            labels[i] = labels[nb.min()]
    return labels


def bfs_labels(adj: np.ndarray, core: np.ndarray) -> np.ndarray:
    """Merge step by breadth-first search over core points (Section II, serial
    step 3), then border assignment; returns canonical labels."""
    n = adj.shape[0]
    labels = np.full(n, -1, dtype=np.int64)
    for s in range(n):
        if not core[s] or labels[s] != -1:
            continue
        labels[s] = s
        queue = deque([s])
        while queue:
            p = queue.popleft()
            for q in np.flatnonzero(adj[p] & core):
                if labels[q] == -1:
                    labels[q] = s
                    queue.append(q)
    return _border_labels(lambda i: adj[i], core, labels)


def warshall_labels(adj: np.ndarray, core: np.ndarray) -> np.ndarray:
    """Independent merge via the transitive closure of the core-core relation
    (the Warshall formulation of Section VI); tiny inputs only."""
    n = adj.shape[0]
    reach = adj & core[:, None] & core[None, :]
    for k in range(n):
        reach = reach | (reach[:, k : k + 1] & reach[k : k + 1, :])
    labels = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        if core[i]:
            labels[i] = int(np.flatnonzero(reach[i]).min())
    return _border_labels(lambda i: adj[i], core, labels)


def dbscan(points: np.ndarray, eps: float, minpts: int, merge: str = "bfs"):
    """Full DBSCAN on a small point set.

    Returns (labels int64[n], core bool[n], counts int64[n])."""
    if minpts < 1:
        raise ValueError("minpts must be >= 1")
    adj = neighbour_matrix(points, eps)
    counts = counts_from_matrix(adj)
    core = counts >= minpts
    if merge == "bfs":
        labels = bfs_labels(adj, core)
    elif merge == "warshall":
        labels = warshall_labels(adj, core)
    else:
        raise ValueError(merge)
    return labels, core, counts


def row_counts(points: np.ndarray, eps: float, rows) -> np.ndarray:
    """|N_eps(i)| for selected rows i, computed one row at a time (for
    sampled checks at sizes where the full oracle is too slow)."""
    x64 = _as64(points)
    eps2 = eps_squared(eps)
    return np.array([int(neighbour_row(x64, int(i), eps2).sum()) for i in rows], dtype=np.int64)
