"""Pins of the oracle for the paper's intermediate products (oracle/paper_steps):
the float32 distance matrix of Section IV-A, the cluster matrix of Section
IV-B and the target merge of Section IV-C.  CPU only."""
from fractions import Fraction as Q

import numpy as np
import pytest
from hypothesis import given, settings, strategies as hs

from oracle import dbscan_oracle as orc
from oracle import paper_steps as ps


def rn32(x: Q) -> np.float32:
    """Round a rational to the nearest float32, ties to even (normal and
    subnormal range; overflow to +-inf), from its exact value."""
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Q(2) ** e > a:
        e -= 1
    while Q(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)             # subnormals share the smallest exponent
    ulp = Q(2) ** (e - 23)
    m = a / ulp                  # in [2^23, 2^24) for normals
    f = int(m)
    r = m - f
    if r > Q(1, 2) or (r == Q(1, 2) and f % 2 == 1):
        f += 1
    v = f * ulp
    if v >= Q(2) ** 128:
        return np.float32(sign * np.inf)
    return np.float32(sign * float(v))


def exact_f32_distance(a, b):
    s = None
    for x, y in zip(a, b):
        t = rn32(Q(float(x)) - Q(float(y)))
        tt = rn32(Q(float(t)) * Q(float(t)))
        s = tt if s is None else rn32(Q(float(s)) + Q(float(tt)))
    return s


def test_rn32_matches_numpy_on_exactly_representable_cases():
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b = rng.standard_normal(2).astype(np.float32)
        # a float32 product is exact in float64, so one rounding to float32
        assert rn32(Q(float(a)) * Q(float(b))) == np.float32(np.float64(a) * np.float64(b))


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_distance_matrix_equals_exact_rounding(d):
    rng = np.random.default_rng(d)
    pts = np.concatenate([rng.uniform(-50, 50, size=(12, d)),
                          rng.uniform(-1e-20, 1e-20, size=(4, d)),   # subnormal squares
                          rng.uniform(-1e19, 1e19, size=(3, d))]).astype(np.float32)  # overflow
    D = ps.distance_matrix_f32(pts)
    assert D.dtype == np.float32
    for i in range(len(pts)):
        for j in range(len(pts)):
            want = exact_f32_distance(pts[i], pts[j])
            assert D[i, j] == want or (np.isinf(D[i, j]) and np.isinf(want)), (i, j)


def test_distance_matrix_symmetric_zero_diagonal_and_bounded():
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 60, size=(300, 3)).astype(np.float32)
    D = ps.distance_matrix_f32(pts)
    assert (D.view(np.uint32) == D.T.view(np.uint32)).all()
    assert (np.diag(D) == 0).all()
    S = orc._sq_block(pts.astype(np.float64), pts.astype(np.float64))
    gamma = 5 * 2.0**-24 / (1 - 5 * 2.0**-24)  # d + 2 roundings per term
    assert (np.abs(D.astype(np.float64) - S) <= gamma * S + 1e-300).all()


def _fused(a, b):
    s = Q(0)
    for x, y in zip(a, b):
        t = rn32(Q(float(x)) - Q(float(y)))
        s = Q(float(rn32(Q(float(t)) * Q(float(t)) + s)))
    return np.float32(float(s))


def test_planted_fused_or_reversed_distance_fails():
    """Seeded pairs where fusing the multiply into the add, or summing the
    coordinates in reverse, changes the float32 value: the oracle must give
    the unfused coordinate-order value."""
    rng = np.random.default_rng(11)
    fused_seen = reversed_seen = 0
    for _ in range(4000):
        a = rng.uniform(-4, 4, 3).astype(np.float32)
        b = (a + rng.uniform(-1, 1, 3)).astype(np.float32)
        D = ps.distance_matrix_f32(np.stack([a, b]))
        seq = exact_f32_distance(a, b)
        assert D[0, 1] == seq
        fused_seen += int(_fused(a, b) != seq)
        reversed_seen += int(exact_f32_distance(a[::-1], b[::-1]) != seq)
    assert fused_seen > 0 and reversed_seen > 0


def test_cluster_matrix_rows_and_valid():
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, 10, size=(200, 3)).astype(np.float32)
    C, valid, counts = ps.cluster_matrix(pts, 1.2, 6)
    assert C.dtype == np.uint8 and (C == C.T).all() and (np.diag(C) == 1).all()
    assert (C.sum(axis=1) == counts).all()
    assert (valid == (counts >= 6)).all()


def _check_merge(pts, eps, minpts):
    C, valid, _ = ps.cluster_matrix(pts, eps, minpts)
    merged, alive = ps.target_merge(C, valid)
    lab = ps.labels_from_merge(C, merged, alive, valid)
    ref = orc.dbscan(pts, eps, minpts)[0]
    np.testing.assert_array_equal(lab, ref)
    # closed form of the merged state: a surviving row is the union of the
    # primitive rows of its component's core points; survivors are the
    # components' smallest core indices
    core = valid.astype(bool)
    for t in np.flatnonzero(alive):
        members = np.flatnonzero((ref == t) & core)
        assert members.min() == t
        np.testing.assert_array_equal(merged[t].astype(bool), C[members].astype(bool).any(axis=0))
    assert set(np.flatnonzero(alive)) == set(np.unique(ref[core]))


def test_target_merge_handworked(handworked):
    pts, eps, minpts, counts, core, labels = handworked
    C, valid, cnt = ps.cluster_matrix(pts, eps, minpts)
    np.testing.assert_array_equal(cnt, counts)
    merged, alive = ps.target_merge(C, valid)
    np.testing.assert_array_equal(ps.labels_from_merge(C, merged, alive, valid), labels)
    _check_merge(pts, eps, minpts)


def test_planted_merge_on_shared_border_point_fails(handworked, monkeypatch):
    """Merging clusters that share any point (not a core point) joins the two
    clusters of the fixture through border point 4."""
    pts, eps, minpts, counts, core, labels = handworked

    def wrong(cluster, valid):
        return ps.target_merge(cluster, np.ones_like(valid))[0], np.asarray(valid, bool) & \
            ps.target_merge(cluster, np.ones_like(valid))[1]

    C, valid, _ = ps.cluster_matrix(pts, eps, minpts)
    merged, alive = wrong(C, valid)
    assert not np.array_equal(ps.labels_from_merge(C, merged, alive, valid), labels)


@settings(max_examples=60, deadline=None)
@given(n=hs.integers(1, 14), d=hs.integers(1, 3), seed=hs.integers(0, 10**6),
       minpts=hs.integers(1, 5), eps=hs.sampled_from([0.0, 1.0, 1.5, 2.0, 3.0]))
def test_target_merge_equals_bfs_on_random_integer_inputs(n, d, seed, minpts, eps):
    pts = np.random.default_rng(seed).integers(0, 6, size=(n, d)).astype(np.float32)
    _check_merge(pts, eps, minpts)


def test_target_merge_on_blobs():
    from paper_1506_02226_amd import workloads as wl
    w = wl.blobs2d_small(0, n=600)
    _check_merge(w.points, w.eps, w.minpts)
