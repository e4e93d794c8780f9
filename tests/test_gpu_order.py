"""GPU parity of the two row orders (dbscan_opts.order).

The spatial order permutes the rows on the device before step 1 and maps
every output back; counts, core flags and labels must equal the oracle's --
and therefore each other's -- bit for bit, in both adjacency forms, on the
fallback sweeps the on-the-fly form runs when its pair list overflows, and on
inputs whose keys tie or cannot be formed (duplicates, an unbounded box,
non-finite coordinates)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1506_02226_amd as pkg
from oracle import c_oracle, dbscan_oracle as orc
from paper_1506_02226_amd import workloads as wl
from test_gpu_parity import assert_same, run

pytestmark = pytest.mark.gpu

MODES = ("bitmask", "onthefly")
ORDERS = ("input", "spatial")


def forms(d):
    """(adjacency, precision) pairs that apply at dimension d."""
    if d <= 4:
        return [("bitmask", "fp32"), ("onthefly", "fp32")]
    if d < 16:
        return [("onthefly", "fp32")]
    return [("onthefly", "fp32"), ("onthefly", "fp16"), ("onthefly", "bf16")]


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("n", [1, 2, 65, 257, 2049, 4099])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 16, 64])
def test_orders_ragged(order, n, d):
    rng = np.random.default_rng(7000 * n + d)
    k = max(1, n // 40)
    centres = rng.uniform(0, 10, size=(k, d))
    pts = (centres[rng.integers(0, k, size=n)] + 0.3 * rng.standard_normal((n, d))).astype(np.float32)
    eps = float(0.35 * np.sqrt(d))
    minpts = int(rng.integers(1, 8))
    ref = orc.dbscan(pts, eps, minpts)
    for adj, prec in forms(d):
        gpu = run(pts, eps, minpts, adjacency=adj, precision=prec, order=order, stats=True)
        assert gpu[3]["order_used"] == order
        assert_same(gpu, ref, f"n={n} d={d} {adj} {prec} {order}")


def test_auto_order_choice():
    rng = np.random.default_rng(3)
    p2 = rng.uniform(0, 1, size=(500, 2)).astype(np.float32)
    big = rng.uniform(0, 1, size=(70_000, 2)).astype(np.float32)
    p16 = rng.uniform(0, 1, size=(500, 16)).astype(np.float32)
    assert run(p2, 0.05, 3, stats=True)[3]["order_used"] == "input"  # small n
    assert run(big, 0.004, 3, stats=True)[3]["order_used"] == "spatial"
    assert run(p16, 0.5, 3, stats=True)[3]["order_used"] == "input"  # small n
    big16 = rng.uniform(0, 1, size=(70_000, 16)).astype(np.float32)
    st = run(big16, 0.3, 3, stats=True)[3]
    assert st["order_used"] == "spatial" and st["precision_used"] == "fp16"
    p130 = rng.uniform(0, 1, size=(300, 130)).astype(np.float32)
    with pytest.raises(pkg.DbscanError) as ei:
        run(p130, 0.5, 3, order="spatial")
    assert ei.value.code == pkg._lib.DBSCAN_E_UNSUPPORTED


@pytest.mark.parametrize("cap", [1, 0])
def test_spatial_order_pair_overflow(cap):
    """Overflow of the pair list: the merge and the border pass repeat the
    epsilon tests in the staged order and must still return the caller's
    lowest-index core neighbour of each border point."""
    w = wl.aniso3d_2m(0, n=20_000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    for order in ORDERS:
        gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", pair_capacity=cap,
                  order=order, stats=True)
        assert_same(gpu, ref, f"cap={cap} {order}")
        assert gpu[3]["pair_overflow"] == (1 if cap == 1 else 0)


@pytest.mark.parametrize("mode", MODES)
def test_spatial_order_ties_and_duplicates(mode):
    """Integer grid (every neighbour at exactly eps, so all decided in float64)
    with duplicated points: equal sort keys keep the input order."""
    g = np.stack(np.meshgrid(np.arange(40), np.arange(30)), -1).reshape(-1, 2).astype(np.float32)
    rng = np.random.default_rng(11)
    g = g[rng.permutation(len(g))]
    g = np.concatenate([g, g[:300], g[:50]])
    for eps, minpts in ((1.0, 5), (1.0, 7), (np.sqrt(2.0), 10)):
        ref = orc.dbscan(g, eps, minpts)
        for order in ORDERS:
            assert_same(run(g, eps, minpts, adjacency=mode, order=order), ref,
                        f"eps={eps} minpts={minpts} {order}")


@pytest.mark.parametrize("mode", MODES)
def test_spatial_order_unbounded_box(mode):
    """Coordinates near the float32 limits: the box width overflows, every
    key is the same cell, and the order degenerates to the input order."""
    rng = np.random.default_rng(13)
    pts = rng.uniform(0, 3, size=(700, 2)).astype(np.float32)
    pts[:3] = np.float32([[-3e38, 3e38], [3e38, -3e38], [3e38, 3e38]])
    ref = orc.dbscan(pts, 0.2, 4)
    assert_same(run(pts, 0.2, 4, adjacency=mode, order="spatial"), ref, mode)


def test_spatial_order_nonfinite_reported():
    pts = np.random.default_rng(2).uniform(0, 1, size=(300, 3)).astype(np.float32)
    pts[17, 1] = np.nan
    pts[200, 0] = np.inf
    for mode in MODES:
        with pytest.raises(pkg.DbscanError) as ei:
            run(pts, 0.1, 3, adjacency=mode, order="spatial", stats=True)
        assert ei.value.code == pkg._lib.DBSCAN_E_NONFINITE
        lab, _, _ = run(pts, 0.1, 3, adjacency=mode, order="spatial")
        assert (lab == -2).all()


@pytest.mark.parametrize("name,n", [("blobs2d_200k", 30_000), ("aniso3d_2m", 30_000),
                                    ("mix64d_300k_q50", 6_000), ("mix64d_300k", 6_000)])
def test_orders_scaled_recipes(name, n):
    w = wl.by_name(name, 0, n)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    for adj, prec in forms(w.d):
        for order in ORDERS:
            assert_same(run(w.points, w.eps, w.minpts, adjacency=adj, precision=prec, order=order),
                        ref, f"{name} {adj} {prec} {order}")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_pivot_order_fallbacks(prec):
    """d > 4 in spatial order through the fallbacks: pair-list overflow (the
    merge and the border pass repeat the tests, keyed by caller index) and,
    for the matrix cores, band-list overflow (step 1 redone in float32 from
    the points in staged order)."""
    w = wl.by_name("mix64d_300k_q50", 0, 6_000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", precision=prec, order="spatial",
              pair_capacity=1, stats=True)
    assert gpu[3]["pair_overflow"] == 1
    assert_same(gpu, ref, f"{prec} pair overflow")
    if prec == "fp16":
        gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", precision=prec,
                  order="spatial", band_capacity=1, stats=True)
        assert gpu[3]["filter_fallback"] == 1
        assert_same(gpu, ref, "band overflow")
