"""GPU parity of the paper's own three-step design (include/dbscan_paper.h),
kept as ablations of the main path: the float distance matrix of Section
IV-A (Table III's four kernels) bit for bit against the oracle's float32
matrix, the byte cluster matrix of Section IV-B (three kernels of Table IV)
element by element against the oracle's neighbour relation, and the merges
of Sections IV-C and VI against the oracle's labels and merged state."""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1506_02226_amd as pkg
from paper_1506_02226_amd import paper
from paper_1506_02226_amd import workloads as wl
from oracle import c_oracle, dbscan_oracle as orc
from oracle import paper_steps as ps

pytestmark = pytest.mark.gpu

DIST = ("baseline", "coalesced", "shared", "unrolled")
CLUSTER = ("from_dist", "fused", "hoisted")
SMALL = [(1, 3), (2, 1), (63, 3), (65, 2), (700, 3), (2049, 1), (3001, 4)]


def _blobs(n, d, seed):
    rng = np.random.default_rng(seed)
    k = max(1, n // 80)
    c = rng.uniform(0, 12, size=(k, d))
    pts = c[rng.integers(0, k, size=n)] + 0.4 * rng.standard_normal((n, d))
    return pts.astype(np.float32)


def _gpu(pts):
    return torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).to("cuda:0")


def _cluster(x, eps, minpts, kernel):
    dist = paper.distance(x, "unrolled") if kernel == "from_dist" else None
    cl, valid, counts, rech = paper.cluster(x, eps, minpts, kernel, dist=dist, rechecked=True)
    torch.cuda.synchronize()
    return cl, valid, counts, rech


@pytest.mark.parametrize("n,d", SMALL)
@pytest.mark.parametrize("kernel", DIST)
def test_distance_matrix_bit_exact(n, d, kernel):
    pts = _blobs(n, d, 10 * n + d)
    D = paper.distance(_gpu(pts), kernel).cpu().numpy()
    ref = ps.distance_matrix_f32(pts)
    np.testing.assert_array_equal(D.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("n,d", SMALL)
@pytest.mark.parametrize("kernel", CLUSTER)
def test_cluster_matrix_equals_oracle(n, d, kernel):
    pts = _blobs(n, d, 7 * n + d)
    eps, minpts = 0.5 * np.sqrt(d), 4
    cl, valid, counts, _ = _cluster(_gpu(pts), eps, minpts, kernel)
    C, v, cnt = ps.cluster_matrix(pts, eps, minpts)
    np.testing.assert_array_equal(cl.cpu().numpy(), C)
    np.testing.assert_array_equal(valid.cpu().numpy().astype(bool), v)
    np.testing.assert_array_equal(counts.cpu().numpy(), cnt)


@pytest.mark.parametrize("kernel", CLUSTER)
def test_cluster_matrix_ties_and_offsets(kernel):
    """Neighbours exactly at eps on an integer grid (every one decided in
    float64), and the same grid moved far from the origin, where the
    hoisted form's cancellation widens its band."""
    g = np.stack(np.meshgrid(np.arange(30), np.arange(20), np.arange(3)), -1).reshape(-1, 3)
    g = g[np.random.default_rng(2).permutation(len(g))].astype(np.float32)
    for pts in (g, (g + 4096.0).astype(np.float32)):
        for eps, minpts in ((1.0, 5), (np.sqrt(2.0), 9)):
            cl, valid, counts, rech = _cluster(_gpu(pts), eps, minpts, kernel)
            C, v, cnt = ps.cluster_matrix(pts, eps, minpts)
            np.testing.assert_array_equal(cl.cpu().numpy(), C)
            np.testing.assert_array_equal(counts.cpu().numpy(), cnt)
            assert rech > 0


@pytest.mark.parametrize("n,d", [(1, 2), (65, 3), (700, 3), (1500, 2)])
@pytest.mark.parametrize("kernel", ["targets", "warshall"])
def test_merge_equals_oracle(n, d, kernel):
    pts = _blobs(n, d, 3 * n + d)
    eps, minpts = 0.5 * np.sqrt(d), 4
    cl, valid, counts, _ = _cluster(_gpu(pts), eps, minpts, "fused")
    prim = cl.cpu().numpy()
    C, v, cnt = ps.cluster_matrix(pts, eps, minpts)
    ref = orc.dbscan(pts, eps, minpts)[0]
    if kernel == "targets":
        lab, alive, _ = paper.merge(cl, valid, kernel, alive=True)
        merged, ref_alive = ps.target_merge(C, v)
        np.testing.assert_array_equal(alive.cpu().numpy().astype(bool), ref_alive)
        np.testing.assert_array_equal(cl.cpu().numpy(), merged)
    else:
        lab, _ = paper.merge(cl, valid, kernel)
        np.testing.assert_array_equal(cl.cpu().numpy(), prim)  # unchanged
    np.testing.assert_array_equal(lab.cpu().numpy(), ref)


def test_merge_handworked(handworked):
    pts, eps, minpts, counts, core, labels = handworked
    for kernel in ("targets", "warshall"):
        cl, valid, cnt, _ = _cluster(_gpu(pts), eps, minpts, "hoisted")
        np.testing.assert_array_equal(cnt.cpu().numpy(), counts)
        lab, _ = paper.merge(cl, valid, kernel)
        np.testing.assert_array_equal(lab.cpu().numpy(), labels)


@functools.lru_cache(maxsize=1)
def _paper3d_ref(n):
    w = wl.paper3d(0, n)
    return w, c_oracle.dbscan(w.points, w.eps, w.minpts)


@pytest.mark.parametrize("n", [5061, 23040])
@pytest.mark.parametrize("kernel", CLUSTER)
def test_paper_sizes_pipeline(n, kernel):
    """At the paper's sizes: counts, valid flags and labels of the whole
    ablation pipeline equal the C oracle (and so dbscan_fit)."""
    w, (lab_ref, core_ref, cnt_ref) = _paper3d_ref(n)
    x = _gpu(w.points)
    cl, valid, counts, _ = _cluster(x, w.eps, w.minpts, kernel)
    np.testing.assert_array_equal(counts.cpu().numpy(), cnt_ref)
    np.testing.assert_array_equal(valid.cpu().numpy().astype(bool), core_ref)
    # the matrix itself: row sums are the counts, and it is symmetric
    C = cl.cpu().numpy()
    assert (C.sum(axis=1) == cnt_ref).all() and (C == C.T).all()
    lab, launches = paper.merge(cl, valid, "targets")
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_ref)
    assert launches >= 3
    main = pkg.fit(x, w.eps, w.minpts)
    np.testing.assert_array_equal(main[0].cpu().numpy(), lab_ref)


def test_paper_size_cluster_matrix_elementwise():
    """n = 5,061: the cluster matrix of every kernel against the oracle's
    relation, element by element."""
    w = wl.paper3d(0, 5061)
    C, v, cnt = ps.cluster_matrix(w.points, w.eps, w.minpts)
    x = _gpu(w.points)
    for kernel in CLUSTER:
        cl, valid, counts, _ = _cluster(x, w.eps, w.minpts, kernel)
        np.testing.assert_array_equal(cl.cpu().numpy(), C, err_msg=kernel)


def test_warshall_paper_size():
    w, (lab_ref, core_ref, cnt_ref) = _paper3d_ref(5061)
    cl, valid, counts, _ = _cluster(_gpu(w.points), w.eps, w.minpts, "fused")
    lab, launches = paper.merge(cl, valid, "warshall")
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_ref)
    assert launches == 5061 + 3


def test_distance_matrix_paper_size_bit_exact():
    w = wl.paper3d(0, 5061)
    ref = ps.distance_matrix_f32(w.points).view(np.uint32)
    x = _gpu(w.points)
    for kernel in DIST:
        D = paper.distance(x, kernel).cpu().numpy()
        np.testing.assert_array_equal(D.view(np.uint32), ref, err_msg=kernel)
