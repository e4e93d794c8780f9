"""Seeded synthetic workloads: determinism and recipe.  CPU only."""
import numpy as np

from paper_1506_02226_amd import workloads as wl


def test_blob_sizes():
    assert wl.blob_sizes(10, 3) == [4, 3, 3]
    assert sum(wl.blob_sizes(1800, 5)) == 1800


def test_blobs2d_small_recipe_and_determinism():
    a = wl.blobs2d_small(0)
    b = wl.blobs2d_small(0)
    assert a.points.dtype == np.float32 and a.points.flags.c_contiguous
    assert a.points.shape == (2000, 2) and a.eps == 0.3 and a.minpts == 5
    np.testing.assert_array_equal(a.points, b.points)
    assert not np.array_equal(a.points, wl.blobs2d_small(1).points)
    assert a.points.min() > -5 and a.points.max() < 25


def test_scaled_recipes_shapes():
    assert wl.blobs2d_200k(0, n=5000).points.shape == (5000, 2)
    w3 = wl.aniso3d_2m(0, n=4000)
    assert w3.points.shape == (4000, 3) and w3.eps == 0.4 and w3.minpts == 20
    w4 = wl.mix64d_300k(0, n=3000)
    assert w4.points.shape == (3000, 64) and w4.eps == 6.0 and w4.minpts == 15


def test_served_job_deterministic():
    a = wl.served_job(3)
    b = wl.served_job(3)
    np.testing.assert_array_equal(a.points, b.points)
    assert a.eps == b.eps and a.minpts == b.minpts
    assert 1000 <= a.n <= 200000 and a.d in (2, 3, 16, 64) and a.minpts in (5, 10, 20)
    assert a.eps == wl.round_sig(a.eps)


def test_arrivals_poisson():
    t = wl.served_arrivals(2000, 100.0, seed=0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 2000 - 0.01) < 0.002


def test_served_recipes_by_dimension():
    """2-D/3-D jobs follow the 2-D blob recipe (box 200); 16-D/64-D jobs the
    high-dimensional mixture recipe, whose squared norms stay inside the
    half-precision range the matrix-core filter needs."""
    seen = set()
    for j in range(40):
        w = wl.served_job(j, eps_sample=64)
        x = w.points.astype(np.float64)
        nrm2 = (x * x).sum(axis=1).max()
        if w.d <= 3:
            assert w.points.min() > -10 and w.points.max() < 210
        else:
            assert nrm2 < 30000.0
        seen.add(w.d)
    assert seen == {2, 3, 16, 64}


def test_mixture_recipe_matches_mix64d():
    a = wl._mix64d_points(0, 2000)
    b = wl.mixture_blobs(np.random.default_rng(0), 2000, 64, 100, 0.02)
    np.testing.assert_array_equal(a, b)
