"""dbscan_fit_noalloc (the entry point for callers that cannot allocate
device memory) against dbscan_fit_ex, the entry point it shares its kernels
with: every output equal, on two calls in a row, the second with a smaller
input (the array keeps the first call's contents), and sizes beyond the
array rejected before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1506_02226_amd as pkg
from paper_1506_02226_amd import _lib
from paper_1506_02226_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _noalloc(x, eps, minpts):
    L = _lib.load()
    n, d = int(x.shape[0]), int(x.shape[1])
    out = (torch.full((n,), 7, dtype=torch.int32, device=x.device),
           torch.full((n,), 7, dtype=torch.uint8, device=x.device),
           torch.full((n,), 7, dtype=torch.int32, device=x.device))
    stream = torch.cuda.current_stream(x.device).cuda_stream
    rc = L.dbscan_fit_noalloc(x.data_ptr(), n, d, float(eps), int(minpts), out[0].data_ptr(),
                              out[1].data_ptr(), out[2].data_ptr(), stream)
    assert rc == _lib.DBSCAN_OK, rc
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _ex(x, eps, minpts):
    out = pkg.fit(x, eps, minpts)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


CASES = [
    # (first workload, second smaller workload): bitmask form, on the fly
    # with the spatial order and lists sized to the array, matrix cores
    (("blobs2d_200k", 20_000), ("blobs2d_small", 2_000)),
    (("aniso3d_2m", 800_000), ("aniso3d_2m", 30_000)),
    (("mix64d_300k_q50", 100_000), ("mix64d_300k_q50", 5_000)),
]


@pytest.mark.parametrize("first,second", CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_noalloc_equals_fit_ex_twice(first, second):
    for name, n in (first, second):
        w = wl.by_name(name, 0, n)
        x = torch.from_numpy(w.points).to("cuda:0")
        got = _noalloc(x, w.eps, w.minpts)
        want = _ex(x, w.eps, w.minpts)
        for g, e, what in zip(got, want, ("labels", "core", "counts")):
            np.testing.assert_array_equal(g, e, err_msg=f"{name} n={n} {what}")


def test_noalloc_rejects_sizes_beyond_the_array():
    L = _lib.load()
    # rejected on the host before any device work: the pointers are never read
    for n, d in ((887_297, 3), (388_609, 16), (120_321, 64)):
        rc = L.dbscan_fit_noalloc(0x1000, n, d, 1.0, 5, 0x2000, 0x3000, 0x4000, None)
        assert rc == _lib.DBSCAN_E_NOMEM, (n, d, rc)
    rc = L.dbscan_fit_noalloc(None, 10, 2, 1.0, 5, 0x2000, 0x3000, 0x4000, None)
    assert rc == _lib.DBSCAN_E_INVAL
