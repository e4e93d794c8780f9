"""GPU parity on the method's numeric edge cases.

* The float64 evaluation order: pairs whose sequential, unfused float64 sum
  (the reading taken for Section IV-B.2's direct form) and a fused, reversed,
  pairwise or exactly rounded sum fall on opposite sides of eps^2.  The GPU
  must decide each of them the sequential way, through its float64 recheck.
* Scales where float32 squared differences underflow, so that only the
  band's absolute allowance keeps the float32 test sound.
* The 16-bit matrix-core filters at coordinates in FP16's subnormal range and
  beyond the BF16 filter's range guard, and eps = 0 with duplicates.
Every output is compared with the float64 oracle element by element."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import fp64_order as fo
from oracle import dbscan_oracle as orc
from paper_1506_02226_amd import workloads as wl
from test_gpu_parity import assert_same, run

pytestmark = pytest.mark.gpu


def _order_dataset(c, n=600, rows=(37, 411)):
    """The case's pair at two rows of different tiles, among filler points
    far enough away (offset 1000 in every coordinate) never to meet it."""
    d = c["a"].shape[0]
    rng = np.random.default_rng(17)
    pts = (1000.0 + rng.uniform(0, 20, size=(n, d))).astype(np.float32)
    pts[rows[0]] = c["a"]
    pts[rows[1]] = c["b"]
    return pts


def _forms(d):
    if d <= 4:
        return [dict(adjacency=a, order=o) for a in ("bitmask", "onthefly")
                for o in ("input", "spatial")]
    return [dict(precision=p) for p in ("fp32", "fp16", "bf16")]


@pytest.mark.parametrize("d", [2, 3, 8, 16])
def test_fp64_order_decided_sequentially(d):
    for c in fo.cases(d):
        pts = _order_dataset(c)
        ref = orc.dbscan(pts, c["eps"], 2)
        want = 2 if c["in"] else 1
        assert ref[2][37] == ref[2][411] == want
        for form in _forms(d):
            gpu = run(pts, c["eps"], 2, stats=True, **form)
            what = f"d={d} {c['variant']} {c['direction']} {form}"
            assert gpu[2][37] == gpu[2][411] == want, what
            assert_same(gpu, ref, what)
            assert gpu[3]["pairs_rechecked"] > 0, what


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("scale", [1e-31, 1e-20])
def test_float32_underflow_scale(d, scale):
    """Coordinates near 1e-30 (or 1e-19): squared differences underflow in
    float32 (to zero or subnormals) but not in float64."""
    w = wl.blobs2d_small(0) if d == 2 else wl.aniso3d_2m(0, n=3000)
    pts = (w.points.astype(np.float64) * scale).astype(np.float32)
    eps = w.eps * scale
    ref = orc.dbscan(pts, eps, w.minpts)
    for mode in ("bitmask", "onthefly"):
        for order in ("input", "spatial"):
            gpu = run(pts, eps, w.minpts, adjacency=mode, order=order, stats=True)
            assert_same(gpu, ref, f"scale={scale} {mode} {order}")
            assert gpu[3]["pairs_rechecked"] > 0


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("scale", [1e-5, 1e-6])
def test_mfma_tiny_coordinates(prec, scale):
    """The 16-bit filters at coordinates in FP16's subnormal range."""
    w = wl.mix64d_300k(0, n=3000, eps_rule="q50")
    pts = (w.points.astype(np.float64) * scale).astype(np.float32)
    eps = w.eps * scale
    ref = orc.dbscan(pts, eps, w.minpts)
    gpu = run(pts, eps, w.minpts, precision=prec, stats=True)
    assert gpu[3]["precision_used"] == prec
    assert_same(gpu, ref, f"{prec} scale={scale} fallback={gpu[3]['filter_fallback']}")


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("d", [16, 64])
def test_mfma_eps_zero_duplicates(prec, d):
    rng = np.random.default_rng(d)
    base = rng.normal(0, 3, size=(300, d)).astype(np.float32)
    pts = np.concatenate([base, base[:150], base[:40], base[:5]])
    pts = pts[rng.permutation(len(pts))]
    for minpts in (1, 2, 3, 4):
        ref = orc.dbscan(pts, 0.0, minpts)
        gpu = run(pts, 0.0, minpts, precision=prec, stats=True)
        assert gpu[3]["filter_fallback"] == 0
        assert_same(gpu, ref, f"{prec} d={d} minpts={minpts}")


def test_bf16_range_guard():
    """BF16 inputs beyond the filter's range (|x| > 1e17, where its FP32 norms
    could overflow) fall back to the float32 sweep; large but in range, the
    filter still decides; and an eps whose square exceeds FLT_MAX."""
    w = wl.mix64d_300k(0, n=2000, eps_rule="q50")
    for scale, fallback in ((1e18, 1), (1e15, 0)):
        pts = (w.points.astype(np.float64) * scale).astype(np.float32)
        eps = w.eps * scale
        ref = orc.dbscan(pts, eps, w.minpts)
        gpu = run(pts, eps, w.minpts, precision="bf16", stats=True)
        assert gpu[3]["filter_fallback"] == fallback, scale
        assert_same(gpu, ref, f"scale={scale}")
    pts = (w.points.astype(np.float64) * 1e15).astype(np.float32)
    for eps in (1e20, 1e30):
        ref = orc.dbscan(pts, eps, w.minpts)
        gpu = run(pts, eps, w.minpts, precision="bf16", stats=True)
        assert gpu[3]["filter_fallback"] == 0
        assert_same(gpu, ref, f"eps={eps}")
        assert (ref[0] == 0).all()
