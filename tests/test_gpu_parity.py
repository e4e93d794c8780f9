"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Counts, core flags and labels must be bit-identical to the float64 oracle.
Sizes stay where the oracle finishes in seconds but span several tiles and
ragged tails; the full-size workloads are compared element by element in
test_gpu_full_size.py."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1506_02226_amd as pkg
from oracle import c_oracle, dbscan_oracle as orc
from paper_1506_02226_amd import workloads as wl

pytestmark = pytest.mark.gpu

MODES = ("bitmask", "onthefly")


def _gpu(points):
    return torch.from_numpy(np.ascontiguousarray(points, dtype=np.float32)).to("cuda:0")


def run(points, eps, minpts, **kw):
    out = pkg.fit(_gpu(points), eps, minpts, **kw)
    torch.cuda.synchronize()
    res = [t.cpu().numpy() for t in out[:3]]
    res[1] = res[1].astype(bool)
    if kw.get("stats"):
        return (*res, out[3])
    return tuple(res)


def assert_same(gpu, ref, what=""):
    lab, core, cnt = gpu[:3]
    rl, rc, rn = ref
    np.testing.assert_array_equal(cnt, np.asarray(rn), err_msg=f"counts {what}")
    np.testing.assert_array_equal(core, np.asarray(rc).astype(bool), err_msg=f"core {what}")
    np.testing.assert_array_equal(lab, np.asarray(rl), err_msg=f"labels {what}")


def modes_for(d):
    return MODES if d <= 4 else ("onthefly",)


@pytest.mark.parametrize("mode", MODES)
def test_handworked_fixture(handworked, mode):
    pts, eps, minpts, counts, core, labels = handworked
    assert_same(run(pts, eps, minpts, adjacency=mode), (labels, core, counts), mode)


@pytest.mark.parametrize("mode", MODES)
def test_blobs2d_small(mode):
    w = wl.blobs2d_small(0)
    gpu = run(w.points, w.eps, w.minpts, adjacency=mode, stats=True)
    assert_same(gpu, orc.dbscan(w.points, w.eps, w.minpts), mode)
    st = gpu[3]
    assert st["adjacency_used"] == mode and st["pairs_tested"] == w.n * w.n
    # the triangular sweep tests each unordered pair once (both orders only
    # inside the 64x64 diagonal blocks): between n(n+1)/2 and n(n+1)/2 + 64 n_pad
    n_pad = -(-w.n // 256) * 256
    assert w.n * (w.n + 1) // 2 <= st["sweep1_tests"] <= n_pad * (n_pad + 1) // 2 + 64 * n_pad
    assert st["ms_sweep1"] > 0.0 and st["ms_sweep1"] <= st["ms_step1"] + 1e-3


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 1000, 4099])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 16, 64])
def test_ragged_random(n, d):
    rng = np.random.default_rng(1000 * n + d)
    k = max(1, n // 50)
    centres = rng.uniform(0, 10, size=(k, d))
    pts = (centres[rng.integers(0, k, size=n)] + 0.3 * rng.standard_normal((n, d))).astype(np.float32)
    eps = float(0.35 * np.sqrt(d))
    minpts = int(rng.integers(1, 8))
    ref = orc.dbscan(pts, eps, minpts)
    for mode in modes_for(d):
        assert_same(run(pts, eps, minpts, adjacency=mode), ref, f"n={n} d={d} {mode}")


@pytest.mark.parametrize("d", [77, 300, 1024])
def test_wide_float32(d):
    """Dimensions beyond the matrix-core range run the float32 sweep with
    rows staged in LDS (d up to the documented maximum of 1024)."""
    rng = np.random.default_rng(d)
    k = 6
    centres = rng.uniform(0, 4, size=(k, d))
    pts = centres[rng.integers(0, k, size=650)] + 0.05 * rng.standard_normal((650, d))
    pts = np.concatenate([pts, rng.uniform(0, 4, size=(50, d))]).astype(np.float32)
    eps = float(0.08 * np.sqrt(d))
    ref = orc.dbscan(pts, eps, 4)
    gpu = run(pts, eps, 4, stats=True)
    assert gpu[3]["precision_used"] == "fp32"
    assert_same(gpu, ref, f"d={d}")


@pytest.mark.parametrize("order", ["input", "spatial"])
@pytest.mark.parametrize("mode", MODES)
def test_integer_grid_ties(mode, order):
    """Every neighbour pair of a unit grid sits exactly at eps: all of them
    fall in the float32 band (direct form in the caller's order, hoisted
    form in spatial order) and are decided in float64."""
    g = np.stack(np.meshgrid(np.arange(40), np.arange(30)), -1).reshape(-1, 2).astype(np.float32)
    rng = np.random.default_rng(5)
    g = g[rng.permutation(len(g))]
    g = np.concatenate([g, g[:100]])  # duplicates
    for eps, minpts in ((1.0, 5), (1.0, 6), (np.sqrt(2.0), 9), (2.0, 13)):
        gpu = run(g, eps, minpts, adjacency=mode, order=order, stats=True)
        assert_same(gpu, orc.dbscan(g, eps, minpts), f"eps={eps} minpts={minpts}")
        assert gpu[3]["hoisted"] == (1 if order == "spatial" else 0)
        if eps == 1.0:
            assert gpu[3]["pairs_rechecked"] > 0


@pytest.mark.parametrize("mode", MODES)
def test_hoisted_form_falls_back_beyond_its_range(mode):
    """A coordinate beyond 2^60 makes the sweep take the direct form (the
    hoisted form's products could overflow); near 2^59 it keeps the hoisted
    form.  Outputs equal the oracle either way."""
    rng = np.random.default_rng(21)
    for base, hoisted in ((3.0e18, 0), (5.0e17, 1)):
        centres = rng.uniform(-1, 1, size=(20, 3)) * base
        pts = (centres[rng.integers(0, 20, 400)] +
               rng.standard_normal((400, 3)) * base * 1e-6).astype(np.float32)
        eps = float(base * 3e-6)
        ref = orc.dbscan(pts, eps, 4)
        gpu = run(pts, eps, 4, adjacency=mode, order="spatial", stats=True)
        assert_same(gpu, ref, f"base={base} {mode}")
        assert gpu[3]["hoisted"] == hoisted, base


@pytest.mark.parametrize("order", ["input", "spatial"])
@pytest.mark.parametrize("mode", MODES)
def test_degenerate_cases(mode, order):
    rng = np.random.default_rng(9)
    pts = rng.uniform(0, 5, size=(300, 2)).astype(np.float32)
    same = np.zeros((200, 3), np.float32) + 1.5
    for p, eps, minpts in ((pts, 0.0, 1), (pts, 0.0, 2), (pts, 100.0, 300), (pts, 100.0, 301),
                           (pts, 0.4, 1), (same, 0.0, 200), (same, 0.0, 201),
                           (np.float32([[3.0, 4.0]]), 1.0, 1), (np.float32([[3.0, 4.0]]), 1.0, 2)):
        if p.shape[1] > 4 and mode == "bitmask":
            continue
        assert_same(run(p, eps, minpts, adjacency=mode, order=order), orc.dbscan(p, eps, minpts),
                    f"eps={eps} minpts={minpts} n={len(p)} {order}")


def test_large_coordinates_and_tiny_eps():
    rng = np.random.default_rng(12)
    base = rng.uniform(-1e6, 1e6, size=(50, 3))
    pts = (base[rng.integers(0, 50, 600)] + rng.standard_normal((600, 3)) * 0.05).astype(np.float32)
    for eps, minpts in ((0.1, 3), (1e-3, 2), (0.0625, 4)):
        ref = orc.dbscan(pts, eps, minpts)
        for mode in MODES:
            for order in ("input", "spatial"):
                assert_same(run(pts, eps, minpts, adjacency=mode, order=order), ref,
                            f"eps={eps} {mode} {order}")


def test_nonfinite_input_reported():
    pts = np.random.default_rng(0).uniform(0, 1, size=(100, 2)).astype(np.float32)
    pts[17, 1] = np.nan
    with pytest.raises(pkg.DbscanError) as ei:
        pkg.fit(_gpu(pts), 0.1, 3, stats=True)
    assert ei.value.code == pkg._lib.DBSCAN_E_NONFINITE
    labels, core, counts = pkg.fit(_gpu(pts), 0.1, 3)
    torch.cuda.synchronize()
    assert (labels.cpu().numpy() == -2).all()


def test_invalid_arguments_raise():
    x = _gpu(np.zeros((10, 2), np.float32))
    with pytest.raises(pkg.DbscanError):
        pkg.fit(x, -1.0, 3)
    with pytest.raises(pkg.DbscanError):
        pkg.fit(x, 1.0, 0)
    with pytest.raises(pkg.DbscanError):
        pkg.fit(_gpu(np.zeros((10, 8), np.float32)), 1.0, 3, adjacency="bitmask")


def test_library_allocated_workspace_and_side_stream():
    """dbscan_fit (library-owned, stream-ordered workspace) on a side stream."""
    w = wl.blobs2d_small(3)
    L = pkg._lib.load()
    x = _gpu(w.points)
    n = w.n
    labels = torch.empty(n, dtype=torch.int32, device="cuda:0")
    core = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    rc = L.dbscan_fit(x.data_ptr(), n, 2, w.eps, w.minpts, labels.data_ptr(), core.data_ptr(),
                      counts.data_ptr(), s.cuda_stream)
    assert rc == 0
    s.synchronize()
    assert_same((labels.cpu().numpy(), core.cpu().numpy().astype(bool), counts.cpu().numpy()),
                orc.dbscan(w.points, w.eps, w.minpts))


def test_repeatable():
    w = wl.blobs2d_200k(0, n=20_000)
    a = run(w.points, w.eps, w.minpts, adjacency="bitmask")
    b = run(w.points, w.eps, w.minpts, adjacency="bitmask")
    c = run(w.points, w.eps, w.minpts, adjacency="onthefly")
    for x, y, z in zip(a, b, c):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x, z)


@pytest.mark.parametrize("name,n", [("blobs2d_200k", 30_000), ("aniso3d_2m", 30_000),
                                    ("mix64d_300k_q50", 6_000)])
def test_scaled_recipes_full_parity(name, n):
    """Each workload recipe at a size the C oracle finishes in seconds."""
    w = wl.by_name(name, 0, n)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    for mode in modes_for(w.d):
        assert_same(run(w.points, w.eps, w.minpts, adjacency=mode), ref, f"{name} {mode}")


@pytest.mark.parametrize("cap", [1, 100, 0])
def test_pair_list_overflow_falls_back(cap):
    """The on-the-fly form records neighbour pairs for the merge; when they do
    not fit it repeats the epsilon tests instead, with identical results."""
    w = wl.aniso3d_2m(0, n=20_000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", pair_capacity=cap, stats=True)
    assert_same(gpu, ref, f"cap={cap}")
    st = gpu[3]
    half_edges = (int(ref[2].sum()) - w.n) // 2
    assert st["pairs_listed"] == half_edges
    assert st["pair_overflow"] == (1 if 0 < cap < half_edges else 0)


@pytest.mark.parametrize("cap", [1, 0])
def test_pair_list_wide_float32(cap):
    """d > 4 in float32 (rows staged in LDS) records the pair list the same
    way, and falls back to repeated tests when it overflows."""
    w = wl.by_name("mix64d_300k_q50", n=6000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", precision="fp32",
              pair_capacity=cap, stats=True)
    assert_same(gpu, ref, f"cap={cap}")
    st = gpu[3]
    half_edges = (int(ref[2].sum()) - w.n) // 2
    assert half_edges > 0 and st["pairs_listed"] == half_edges
    assert st["pair_overflow"] == (1 if cap == 1 else 0)


# ------------------------------------------------------------ matrix cores
PRECS = ("bf16", "fp16")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,d", [(1, 16), (70, 16), (1000, 16), (777, 32), (2050, 64), (513, 70)])
def test_mfma_random(prec, n, d):
    rng = np.random.default_rng(31 * n + d)
    k = max(1, n // 60)
    centres = rng.uniform(-5, 5, size=(k, d))
    pts = (centres[rng.integers(0, k, size=n)] + 0.35 * rng.standard_normal((n, d))).astype(np.float32)
    eps = float(0.4 * np.sqrt(d))
    minpts = int(rng.integers(1, 8))
    ref = orc.dbscan(pts, eps, minpts)
    gpu = run(pts, eps, minpts, precision=prec, stats=True)
    assert gpu[3]["precision_used"] == prec and gpu[3]["filter_fallback"] == 0
    assert_same(gpu, ref, f"n={n} d={d} {prec}")


@pytest.mark.parametrize("prec", PRECS)
def test_mfma_integer_ties(prec):
    """Integer coordinates: many pairs exactly at eps, all decided in float64."""
    rng = np.random.default_rng(8)
    base = rng.integers(-3, 4, size=(40, 16))
    pts = np.concatenate([base + rng.integers(-1, 2, size=(40, 16)) * (rng.random((40, 16)) < 0.1)
                          for _ in range(20)]).astype(np.float32)
    for eps, minpts in ((1.0, 3), (np.sqrt(2.0), 5), (2.0, 8)):
        gpu = run(pts, eps, minpts, precision=prec, stats=True)
        assert_same(gpu, orc.dbscan(pts, eps, minpts), f"eps={eps}")
        assert gpu[3]["pairs_rechecked"] > 0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("cap", [1, 500])
def test_mfma_pair_overflow(prec, cap):
    """Matrix-core filter that decides every pair, but a pair list too small
    for the merge: step 3 repeats the tests in float32 from coordinates the
    matrix-core path stages only for this case."""
    w = wl.by_name("mix64d_300k_q50", 0, 4000)
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    for order in ("input", "spatial"):
        gpu = run(w.points, w.eps, w.minpts, adjacency="onthefly", precision=prec, order=order,
                  pair_capacity=cap, stats=True)
        st = gpu[3]
        assert st["precision_used"] == prec and st["filter_fallback"] == 0
        assert st["pair_overflow"] == 1
        assert_same(gpu, ref, f"{prec} cap={cap} {order}")


@pytest.mark.parametrize("prec", PRECS)
def test_mfma_band_overflow_and_range_fallback(prec):
    w = wl.mix64d_300k(0, n=3000, eps_rule="q50")
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    gpu = run(w.points, w.eps, w.minpts, precision=prec, band_capacity=1, stats=True)
    assert gpu[3]["filter_fallback"] == 1
    assert_same(gpu, ref, "band overflow")
    gpu = run(w.points, w.eps, w.minpts, precision=prec, pair_capacity=5, stats=True)
    assert gpu[3]["pair_overflow"] == 1
    assert_same(gpu, ref, "pair overflow")
    if prec == "fp16":
        # coordinates beyond the FP16 range of the filter (|x| <= 30000)
        big = (w.points * 10000.0).astype(np.float32)
        assert np.abs(big).max() > 30000.0
        refb = c_oracle.dbscan(big, w.eps * 10000.0, w.minpts)
        gpu = run(big, w.eps * 10000.0, w.minpts, precision=prec, stats=True)
        assert gpu[3]["filter_fallback"] == 1
        assert_same(gpu, refb, "range")
        # large but in range: the norms are float32, so the filter still runs
        mid = (w.points * 3000.0).astype(np.float32)
        assert np.abs(mid).max() < 30000.0
        refm = c_oracle.dbscan(mid, w.eps * 3000.0, w.minpts)
        gpu = run(mid, w.eps * 3000.0, w.minpts, precision=prec, stats=True)
        assert gpu[3]["filter_fallback"] == 0
        assert_same(gpu, refm, "large in range")


@pytest.mark.parametrize("prec", PRECS + ("fp32",))
def test_mix64d_scaled_parity(prec):
    w = wl.mix64d_300k(0, n=8000, eps_rule="q50")
    ref = c_oracle.dbscan(w.points, w.eps, w.minpts)
    assert_same(run(w.points, w.eps, w.minpts, precision=prec), ref, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d", [2, 3, 9])
def test_mfma_small_d_on_request(prec, d):
    rng = np.random.default_rng(d)
    pts = rng.uniform(0, 4, size=(900, d)).astype(np.float32)
    eps, minpts = 0.3 * np.sqrt(d), 4
    assert_same(run(pts, eps, minpts, precision=prec), orc.dbscan(pts, eps, minpts), f"d={d}")


@pytest.mark.parametrize("n", [2000, 6000, 16000])
@pytest.mark.parametrize("recipe", ["paper3d", "blobs2d_200k", "blobs2d_small"])
def test_bitmask_merge_caller_order_hook_gate(recipe, n):
    """In the caller's order, up to 16,384 rows, the bitmask merge runs its
    hook and compress passes only when the core points' counts sum to at
    least 4 per point, a decision taken on the device; the pair pass follows
    it.  These recipes and sizes fall on both sides (paper3d at 2,000 has no
    core point, blobs2d_small is dense): every output equals the oracle's."""
    w = wl.by_name(recipe, 0, n)
    gpu = run(w.points, w.eps, w.minpts, adjacency="bitmask", order="input", stats=True)
    assert gpu[3]["adjacency_used"] == "bitmask" and gpu[3]["order_used"] == "input"
    assert_same(gpu, c_oracle.dbscan(w.points, w.eps, w.minpts), f"{recipe} n={n}")
