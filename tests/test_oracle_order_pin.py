"""Pin of the float64 evaluation order of the oracle's squared distance.

Reading taken (the paper states neither the precision nor the order of the
direct sum of Section IV-B.2): sequential over the coordinates, every
operation rounded on its own, no fused multiply-add.  The cases of
``fp64_order`` put that value and a fused, reversed, pairwise (np.sum) or
exactly rounded sum on opposite sides of eps^2, so both oracles must decide
each pair the sequential way, and a planted variant of the numpy oracle's
distance must fail."""
import numpy as np
import pytest

import fp64_order as fo
from oracle import c_oracle, dbscan_oracle as orc


@pytest.fixture(scope="module", params=[2, 3, 8, 16])
def order_cases(request):
    return fo.cases(request.param)


def _pair(c):
    return np.stack([c["a"], c["b"]]).astype(np.float32)


def test_cases_separate_every_variant(order_cases):
    seen = {(c["variant"], c["direction"]) for c in order_cases}
    assert seen == {(v, dr) for v in fo.variants_for(len(order_cases[0]["a"]))
                    for dr in ("in", "out")}
    for c in order_cases:
        e2 = orc.eps_squared(c["eps"])
        assert (c["seq"] <= e2) == c["in"] and (c["alt"] <= e2) != c["in"]
        assert c["in"] == (c["direction"] == "in")


def test_numpy_oracle_decides_sequentially(order_cases):
    for c in order_cases:
        p = _pair(c)
        assert orc.sq_dist_row(p.astype(np.float64), 0)[1] == c["seq"]
        adj = orc.neighbour_matrix(p, c["eps"])
        assert adj[0, 1] == adj[1, 0] == c["in"], (c["variant"], c["direction"])
        lab, core, cnt = orc.dbscan(p, c["eps"], 2)
        assert list(cnt) == ([2, 2] if c["in"] else [1, 1])


def test_c_oracle_decides_sequentially(order_cases):
    for c in order_cases:
        p = _pair(c)
        assert c_oracle.row_neighbours(p, c["eps"], 0)[1] == c["in"]
        assert c_oracle.row_neighbours(p, c["eps"], 1)[0] == c["in"]
        lab, core, cnt = c_oracle.dbscan(p, c["eps"], 2)
        assert list(lab) == ([0, 0] if c["in"] else [-1, -1])


def _planted_npsum(xr, xc):
    t = xr[:, None, :] - xc[None, :, :]
    return (t * t).sum(axis=2)


def _planted_reversed(xr, xc):
    s = np.zeros((xr.shape[0], xc.shape[0]))
    for k in reversed(range(xr.shape[1])):
        t = xr[:, k][:, None] - xc[None, :, k]
        s = s + t * t
    return s


def _planted_fused(xr, xc):
    from fractions import Fraction as Q
    s = np.zeros((xr.shape[0], xc.shape[0]))
    for i in range(xr.shape[0]):
        for j in range(xc.shape[0]):
            acc = 0.0
            for k in range(xr.shape[1]):
                t = float(xr[i, k] - xc[j, k])
                acc = float(Q(t) * Q(t) + Q(acc))
            s[i, j] = acc
    return s


@pytest.mark.parametrize("variant,planted", [("pairwise", _planted_npsum),
                                             ("reversed", _planted_reversed),
                                             ("fused", _planted_fused)])
def test_planted_order_mistakes_fail(order_cases, monkeypatch, variant, planted):
    monkeypatch.setattr(orc, "_sq_block", planted)
    wrong = 0
    for c in order_cases:
        if c["variant"] != variant:
            continue
        adj = orc.neighbour_matrix(_pair(c), c["eps"])
        wrong += int(adj[0, 1] != c["in"])
    if not any(c["variant"] == variant for c in order_cases):
        pytest.skip(f"{variant} equals the sequential sum at this d")
    assert wrong == 2  # both directions flip
