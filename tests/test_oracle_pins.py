"""Pins for the CPU oracle: each test checks it against something other than
itself (a hand-worked example, exact arithmetic, an independent algorithm, a
textbook reduction or a closed form).  CPU only."""
from fractions import Fraction
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import dbscan_oracle as orc


# --------------------------------------------------------------------------
# Hand-worked example (tests/golden/handworked_d2.txt)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("merge", ["bfs", "warshall"])
def test_handworked_fixture(handworked, merge):
    pts, eps, minpts, counts, core, labels = handworked
    lab, c, cnt = orc.dbscan(pts, eps, minpts, merge=merge)
    np.testing.assert_array_equal(cnt, counts)
    np.testing.assert_array_equal(c, core)
    np.testing.assert_array_equal(lab, labels)


def _fixture_matches(handworked, lab, c, cnt):
    _, _, _, counts, core, labels = handworked
    return (np.array_equal(cnt, counts) and np.array_equal(c, core)
            and np.array_equal(lab, labels))


# Planted mistakes: each plausible slip in the oracle must break the fixture.
def _plant_sq(monkeypatch, fn):
    monkeypatch.setattr(orc, "_sq_block", fn)


def test_fixture_rejects_dropped_term(handworked, monkeypatch):
    def dropped(xr, xc):  # forgets the last coordinate
        s = np.zeros((xr.shape[0], xc.shape[0]))
        for k in range(xr.shape[1] - 1):
            t = xr[:, k][:, None] - xc[None, :, k]
            s = s + t * t
        return s
    _plant_sq(monkeypatch, dropped)
    pts, eps, minpts = handworked[:3]
    assert not _fixture_matches(handworked, *orc.dbscan(pts, eps, minpts))


def test_fixture_rejects_sign_error(handworked, monkeypatch):
    def plus(xr, xc):  # x_i + x_j instead of x_i - x_j
        s = np.zeros((xr.shape[0], xc.shape[0]))
        for k in range(xr.shape[1]):
            t = xr[:, k][:, None] + xc[None, :, k]
            s = s + t * t
        return s
    _plant_sq(monkeypatch, plus)
    pts, eps, minpts = handworked[:3]
    assert not _fixture_matches(handworked, *orc.dbscan(pts, eps, minpts))


def test_fixture_rejects_transposed_coordinate(handworked, monkeypatch):
    def swapped(xr, xc):  # pairs coordinate k of i with coordinate d-1-k of j
        s = np.zeros((xr.shape[0], xc.shape[0]))
        d = xr.shape[1]
        for k in range(d):
            t = xr[:, k][:, None] - xc[None, :, d - 1 - k]
            s = s + t * t
        return s
    _plant_sq(monkeypatch, swapped)
    pts, eps, minpts = handworked[:3]
    assert not _fixture_matches(handworked, *orc.dbscan(pts, eps, minpts))


def test_fixture_rejects_strict_less(handworked):
    # All squared distances are integers, so "s < 4" is "s <= 3.5"
    pts, eps, minpts = handworked[:3]
    assert not _fixture_matches(handworked, *orc.dbscan(pts, math.sqrt(3.5), minpts))


def test_fixture_rejects_greater_than_minpts(handworked):
    # "count > MinPts" (Section IV-B wording) is "count >= MinPts + 1";
    # so is "the point does not count itself"
    pts, eps, minpts = handworked[:3]
    assert not _fixture_matches(handworked, *orc.dbscan(pts, eps, minpts + 1))


def test_fixture_rejects_other_border_rules(handworked, monkeypatch):
    pts, eps, minpts = handworked[:3]

    def lowest_cluster_id(adj_rows, core, labels):
        for i in range(core.shape[0]):
            if not core[i]:
                nb = np.flatnonzero(adj_rows(i) & core)
                if nb.size:
                    labels[i] = labels[nb].min()
        return labels

    def highest_index_neighbour(adj_rows, core, labels):
        for i in range(core.shape[0]):
            if not core[i]:
                nb = np.flatnonzero(adj_rows(i) & core)
                if nb.size:
                    labels[i] = labels[nb.max()]
        return labels

    for planted in (lowest_cluster_id, highest_index_neighbour):
        monkeypatch.setattr(orc, "_border_labels", planted)
        assert not _fixture_matches(handworked, *orc.dbscan(pts, eps, minpts))


def test_fixture_rejects_merge_through_border(handworked, monkeypatch):
    # Merging every point reachable from a core point (border points included)
    # would join the two clusters through point 4.
    pts, eps, minpts = handworked[:3]

    def leaky_bfs(adj, core):
        n = adj.shape[0]
        labels = np.full(n, -1, dtype=np.int64)
        for s in range(n):
            if not core[s] or labels[s] != -1:
                continue
            labels[s] = s
            stack = [s]
            while stack:
                p = stack.pop()
                for q in np.flatnonzero(adj[p]):
                    if labels[q] == -1:
                        labels[q] = s
                        stack.append(q)
        return labels

    monkeypatch.setattr(orc, "bfs_labels", leaky_bfs)
    assert not _fixture_matches(handworked, *orc.dbscan(pts, eps, minpts))


# --------------------------------------------------------------------------
# Brute force on tiny integer inputs with exact arithmetic and an independent
# merge (union-find), against both oracle merges (BFS and Warshall closure).
# --------------------------------------------------------------------------
def _exact_dbscan(pts_int, eps_sq: Fraction, minpts: int):
    n = len(pts_int)
    adj = [[sum((a - b) ** 2 for a, b in zip(pts_int[i], pts_int[j])) <= eps_sq
            for j in range(n)] for i in range(n)]
    counts = [sum(r) for r in adj]
    core = [c >= minpts for c in counts]
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for i in range(n):
        for j in range(n):
            if core[i] and core[j] and adj[i][j]:
                a, b = find(i), find(j)
                if a != b:
                    parent[max(a, b)] = min(a, b)
    labels = [-1] * n
    for i in range(n):
        if core[i]:
            labels[i] = find(i)
    for i in range(n):
        if not core[i]:
            for j in range(n):  # ascending: lowest-index core neighbour
                if core[j] and adj[i][j]:
                    labels[i] = labels[j]
                    break
    return labels, core, counts


EXACT_EPS = [0.0, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0]  # squares exact in binary


@settings(max_examples=150, deadline=None)
@given(
    d=st.integers(1, 3),
    n=st.integers(1, 12),
    data=st.data(),
    eps=st.sampled_from(EXACT_EPS),
    minpts=st.integers(1, 6),
)
def test_tiny_bruteforce_exact(d, n, data, eps, minpts):
    coords = data.draw(st.lists(st.lists(st.integers(-5, 5), min_size=d, max_size=d),
                                min_size=n, max_size=n))
    pts = np.array(coords, dtype=np.float32).reshape(n, d)
    lab_e, core_e, cnt_e = _exact_dbscan(coords, Fraction(eps) ** 2, minpts)
    for merge in ("bfs", "warshall"):
        lab, core, cnt = orc.dbscan(pts, eps, minpts, merge=merge)
        assert list(cnt) == cnt_e
        assert list(core) == core_e
        assert list(lab) == lab_e


# --------------------------------------------------------------------------
# Float64 decisions against exact rational arithmetic
# --------------------------------------------------------------------------
def test_sq_distance_within_rounding_bound():
    rng = np.random.default_rng(7)
    u = 2.0 ** -53
    for d in (1, 2, 3, 16, 64):
        gamma = (d + 2) * u / (1 - (d + 2) * u)
        x = (rng.standard_normal((40, d)) * rng.choice([1e-3, 1.0, 300.0])).astype(np.float32)
        x64 = x.astype(np.float64)
        for i in range(0, 40, 7):
            s = orc.sq_dist_row(x64, i)
            for j in range(40):
                exact = sum((Fraction(float(a)) - Fraction(float(b))) ** 2
                            for a, b in zip(x[i], x[j]))
                assert abs(Fraction(float(s[j])) - exact) <= gamma * exact


def test_near_boundary_decisions_exact():
    """Pairs constructed to straddle eps^2 by one float32 ulp of a coordinate:
    the oracle's float64 decision equals the exact one whenever the exact
    squared distance is farther from eps^2 than the float64 rounding bound."""
    rng = np.random.default_rng(11)
    eps = 0.25
    eps2 = orc.eps_squared(eps)
    checked = 0
    for _ in range(400):
        d = int(rng.integers(1, 4))
        a = rng.uniform(0, 200, size=d).astype(np.float32)
        v = rng.standard_normal(d)
        v /= np.linalg.norm(v)
        b = (a.astype(np.float64) + eps * v).astype(np.float32)
        for shift in (-2, -1, 0, 1, 2):
            b2 = b.copy()
            b2[0] = np.nextafter(b2[0], np.float32(np.inf) if shift > 0 else np.float32(-np.inf))
            if shift == 0:
                b2 = b
            pts = np.stack([a, b2])
            s = orc.sq_dist_row(pts.astype(np.float64), 0)[1]
            exact = sum((Fraction(float(p)) - Fraction(float(q))) ** 2 for p, q in zip(a, b2))
            bound = (d + 2) * 2.0 ** -53 * 1.01 * exact
            if abs(exact - Fraction(eps2)) > bound:
                assert (s <= eps2) == (exact <= Fraction(eps2))
                checked += 1
    assert checked > 1000


def test_eps_squared_rounds_once():
    for eps in (0.1, 0.25, 0.3, 6.0, 1e-3, 123.456):
        exact = Fraction(eps) ** 2
        e2 = orc.eps_squared(eps)
        assert abs(Fraction(e2) - exact) <= Fraction(2.0 ** -53) * exact
        assert e2 == eps * eps


# --------------------------------------------------------------------------
# Textbook reductions and closed forms
# --------------------------------------------------------------------------
def _canonical_components(labels_raw):
    out = np.empty_like(labels_raw)
    first = {}
    for i, c in enumerate(labels_raw):
        first.setdefault(int(c), i)
        out[i] = first[int(c)]
    return out


def test_minpts_one_is_connected_components():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(3)
    for trial in range(5):
        pts = rng.uniform(0, 10, size=(300, 2)).astype(np.float32)
        eps = 0.5 + 0.1 * trial
        lab, core, cnt = orc.dbscan(pts, eps, 1)
        assert core.all()
        d2 = ((pts[:, None, :].astype(np.float64) - pts[None, :, :]) ** 2).sum(-1)
        _, comp = connected_components(csr_matrix(d2 <= eps * eps), directed=False)
        np.testing.assert_array_equal(lab, _canonical_components(comp))


def test_minpts_above_n_is_all_noise():
    rng = np.random.default_rng(4)
    pts = rng.uniform(0, 1, size=(50, 3)).astype(np.float32)
    lab, core, cnt = orc.dbscan(pts, 10.0, 51)
    assert (cnt == 50).all() and not core.any() and (lab == -1).all()


def test_eps_above_diameter_is_one_cluster():
    rng = np.random.default_rng(5)
    pts = rng.uniform(-3, 3, size=(64, 2)).astype(np.float32)
    lab, core, cnt = orc.dbscan(pts, 100.0, 64)
    assert (cnt == 64).all() and core.all() and (lab == 0).all()


def test_eps_zero_duplicates_only():
    pts = np.array([[0, 0], [1, 0], [0, 0], [1, 0], [1, 0], [2, 2]], np.float32)
    lab, core, cnt = orc.dbscan(pts, 0.0, 2)
    np.testing.assert_array_equal(cnt, [2, 3, 2, 3, 3, 1])
    np.testing.assert_array_equal(lab, [0, 1, 0, 1, 1, -1])


def _one_d_closed_form(x, eps, minpts):
    """1-D DBSCAN by sorting and binary search: counts from a window, clusters
    as runs of consecutive core points closer than eps (in 1-D no chain can
    jump a gap between consecutive core points wider than eps)."""
    n = len(x)
    order = np.argsort(x, kind="stable")
    xs = x[order]
    lo = np.searchsorted(xs, xs - eps, side="left")
    hi = np.searchsorted(xs, xs + eps, side="right")
    counts_s = hi - lo
    core_s = counts_s >= minpts
    counts = np.empty(n, np.int64)
    counts[order] = counts_s
    core = np.empty(n, bool)
    core[order] = core_s
    labels = np.full(n, -1, np.int64)
    run = []
    prev = None
    runs = []
    for p in range(n):
        if not core_s[p]:
            continue
        if prev is not None and xs[p] - xs[prev] > eps:
            runs.append(run)
            run = []
        run.append(order[p])
        prev = p
    if run:
        runs.append(run)
    for r in runs:
        labels[r] = min(r)
    for p in range(n):
        i = order[p]
        if core[i]:
            continue
        nb = [order[q] for q in range(lo[p], hi[p]) if core_s[q]]
        if nb:
            labels[i] = labels[min(nb)]
    return labels, core, counts


@pytest.mark.parametrize("seed", range(6))
def test_one_d_closed_form(seed):
    rng = np.random.default_rng(100 + seed)
    x = rng.integers(0, 120, size=90).astype(np.float32)  # integers: exact
    eps = float(rng.integers(1, 4))
    minpts = int(rng.integers(2, 5))
    lab, core, cnt = orc.dbscan(x[:, None], eps, minpts)
    lab2, core2, cnt2 = _one_d_closed_form(x.astype(np.float64), eps, minpts)
    np.testing.assert_array_equal(cnt, cnt2)
    np.testing.assert_array_equal(core, core2)
    np.testing.assert_array_equal(lab, lab2)


# --------------------------------------------------------------------------
# Invariants and an external cross-check away from border ties
# --------------------------------------------------------------------------
def _check_invariants(pts, eps, minpts, lab, core, cnt):
    adj = orc.neighbour_matrix(pts, eps)
    n = len(pts)
    assert (np.diag(adj)).all() and (adj == adj.T).all()
    assert cnt.sum() == n + 2 * int(np.triu(adj, 1).sum())
    for i in range(n):
        corenb = np.flatnonzero(adj[i] & core)
        if core[i]:
            assert lab[i] == lab[corenb].min() == lab[corenb].max()
            assert lab[i] <= i and core[lab[i]] and lab[lab[i]] == lab[i]
        elif corenb.size:
            assert lab[i] == lab[corenb.min()]
        else:
            assert lab[i] == -1


def test_invariants_on_blobs():
    from paper_1506_02226_amd.workloads import blobs2d_small
    w = blobs2d_small(0)
    lab, core, cnt = orc.dbscan(w.points, w.eps, w.minpts)
    _check_invariants(w.points, w.eps, w.minpts, lab, core, cnt)
    assert 0 < core.sum() < w.n and (lab == -1).sum() > 0


def test_sklearn_agrees_away_from_ties():
    sk = pytest.importorskip("sklearn.cluster")
    from paper_1506_02226_amd.workloads import blobs2d_small
    w = blobs2d_small(0)
    lab, core, cnt = orc.dbscan(w.points, w.eps, w.minpts)
    ref = sk.DBSCAN(eps=w.eps, min_samples=w.minpts).fit(w.points.astype(np.float64))
    sk_core = np.zeros(w.n, bool)
    sk_core[ref.core_sample_indices_] = True
    np.testing.assert_array_equal(core, sk_core)
    # same partition of core points
    for c in np.unique(lab[core]):
        members = core & (lab == c)
        assert len(np.unique(ref.labels_[members])) == 1
    # noise agrees; border points agree where all core neighbours share a cluster
    np.testing.assert_array_equal(lab == -1, ref.labels_ == -1)
