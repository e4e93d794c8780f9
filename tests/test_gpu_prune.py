"""GPU parity of tile pruning (dbscan_opts.prune).

With pruning the sweeps skip tile pairs whose bounding boxes are farther
apart than eps; a skipped pair is provably not a neighbour, so counts, core
flags and labels must still equal the oracle's bit for bit.  The tests made
(counted on the device) must not exceed the unpruned sweep's, and on
clustered data in spatial order they must be far fewer."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import c_oracle, dbscan_oracle as orc
from paper_1506_02226_amd import workloads as wl
from test_gpu_parity import assert_same, run

pytestmark = pytest.mark.gpu

MODES = ("bitmask", "onthefly")


@pytest.mark.parametrize("order", ["input", "spatial"])
@pytest.mark.parametrize("n", [1, 2, 65, 257, 2049, 4099])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_prune_ragged(order, n, d):
    rng = np.random.default_rng(9100 * n + d)
    k = max(1, n // 40)
    centres = rng.uniform(0, 30, size=(k, d))
    pts = (centres[rng.integers(0, k, size=n)] + 0.3 * rng.standard_normal((n, d))).astype(np.float32)
    eps = float(0.35 * np.sqrt(d))
    minpts = int(rng.integers(1, 8))
    ref = orc.dbscan(pts, eps, minpts)
    for mode in MODES:
        full = run(pts, eps, minpts, adjacency=mode, order=order, stats=True)
        gpu = run(pts, eps, minpts, adjacency=mode, order=order, prune=True, stats=True)
        assert gpu[3]["pruned"] == 1 and full[3]["pruned"] == 0
        assert gpu[3]["sweep1_tests"] <= full[3]["sweep1_tests"]
        assert_same(gpu, ref, f"n={n} d={d} {mode} {order}")


@pytest.mark.parametrize("mode", MODES)
def test_prune_ties_duplicates_and_far_points(mode):
    """Neighbours at exactly eps (box gaps equal to eps must not be skipped),
    duplicated points, and a few points near the float32 limits."""
    g = np.stack(np.meshgrid(np.arange(40), np.arange(30)), -1).reshape(-1, 2).astype(np.float32)
    rng = np.random.default_rng(21)
    g = g[rng.permutation(len(g))]
    g = np.concatenate([g, g[:200], np.float32([[3e38, -3e38], [-3e38, 3e38]])])
    for eps, minpts in ((1.0, 5), (np.sqrt(2.0), 9), (2.0, 13)):
        ref = orc.dbscan(g, eps, minpts)
        for order in ("input", "spatial"):
            assert_same(run(g, eps, minpts, adjacency=mode, order=order, prune=True), ref,
                        f"eps={eps} {order}")


def test_prune_nonfinite_reported():
    pts = np.random.default_rng(4).uniform(0, 1, size=(500, 2)).astype(np.float32)
    pts[10, 0] = np.nan
    lab, _, _ = run(pts, 0.05, 3, prune=True, order="spatial")
    assert (lab == -2).all()


@pytest.mark.parametrize("cap", [1, 0])
def test_prune_pair_overflow(cap):
    w = wl.aniso3d_2m(0, n=20_000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", order="spatial", prune=True,
              pair_capacity=cap, stats=True)
    assert_same(gpu, ref, f"cap={cap}")
    assert gpu[3]["pair_overflow"] == (1 if cap == 1 else 0)


@pytest.mark.parametrize("name", ["blobs2d_200k", "aniso3d_2m"])
def test_prune_scaled_recipes(name):
    w = wl.by_name(name, 0, 30_000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    for mode in MODES:
        gpu = run(w.points, w.eps, w.minpts, adjacency=mode, order="spatial", prune=True,
                  stats=True)
        assert_same(gpu, ref, f"{name} {mode}")
        # clustered data in spatial order: most tile pairs are far apart
        assert gpu[3]["sweep1_tests"] < 0.25 * w.n * w.n / 2
