"""The C oracle agrees bit for bit with the numpy oracle, and with the
hand-worked example.  CPU only."""
import numpy as np
import pytest

from oracle import c_oracle, dbscan_oracle as orc
from paper_1506_02226_amd import workloads


def test_c_oracle_handworked(handworked):
    pts, eps, minpts, counts, core, labels = handworked
    lab, c, cnt = c_oracle.dbscan(pts, eps, minpts, threads=2)
    np.testing.assert_array_equal(cnt, counts)
    np.testing.assert_array_equal(c, core)
    np.testing.assert_array_equal(lab, labels)


def test_c_oracle_matches_numpy_blobs2d_small():
    w = workloads.blobs2d_small(0)
    a = orc.dbscan(w.points, w.eps, w.minpts)
    b = c_oracle.dbscan(w.points, w.eps, w.minpts)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(np.asarray(x).astype(np.int64), np.asarray(y).astype(np.int64))


@pytest.mark.parametrize("seed,d", [(1, 1), (2, 3), (3, 16), (4, 64)])
def test_c_oracle_matches_numpy_random(seed, d):
    rng = np.random.default_rng(seed)
    n = 700
    pts = (rng.standard_normal((n, d)) * rng.uniform(0.5, 2.0, size=(1, d))).astype(np.float32)
    eps = float(np.sqrt(d) * 0.6)
    minpts = 4
    a = orc.dbscan(pts, eps, minpts)
    b = c_oracle.dbscan(pts, eps, minpts, threads=3)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(np.asarray(x).astype(np.int64), np.asarray(y).astype(np.int64))


def test_c_oracle_thread_count_invariant():
    w = workloads.blobs2d_small(1)
    a = c_oracle.dbscan(w.points, w.eps, w.minpts, threads=1)
    b = c_oracle.dbscan(w.points, w.eps, w.minpts, threads=7)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_c_row_helpers_match_numpy():
    w = workloads.blobs2d_small(0)
    rows = np.array([0, 5, 77, 1999])
    np.testing.assert_array_equal(c_oracle.row_counts(w.points, w.eps, rows),
                                  orc.row_counts(w.points, w.eps, rows))
    x64 = w.points.astype(np.float64)
    nb = c_oracle.row_neighbours(w.points, w.eps, 77)
    np.testing.assert_array_equal(nb, orc.neighbour_row(x64, 77, orc.eps_squared(w.eps)))
    lab, core, cnt = orc.dbscan(w.points, w.eps, w.minpts)
    for i in np.flatnonzero(~core)[:20]:
        j = c_oracle.first_core_neighbour(w.points, w.eps, core, int(i))
        corenb = np.flatnonzero(orc.neighbour_row(x64, int(i), orc.eps_squared(w.eps)) & core)
        assert j == (corenb.min() if corenb.size else -1)
