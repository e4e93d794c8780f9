"""Shared checks of GPU results against the oracle (imported by the GPU test
modules; not a test module itself)."""
import json
import os
import sys

import numpy as np


GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLDEN_DIR not in sys.path:
    sys.path.insert(0, GOLDEN_DIR)
import make_full_size as mfs  # noqa: E402  (digest layout shared with the writer)


def golden(name: str) -> dict:
    """The committed oracle digests of a full-size workload
    (tests/golden/full_size/<name>.json, written by make_full_size.py)."""
    path = os.path.join(GOLDEN_DIR, "full_size", f"{name}.json")
    if not os.path.exists(path):
        import pytest
        pytest.skip(f"no oracle digests for {name} (tests/golden/make_full_size.py {name})")
    with open(path) as f:
        return json.load(f)


def golden_job(j: int) -> dict:
    rec = golden("served_jobs")
    return rec["records"][rec["jobs"].index(j)]


def assert_golden(rec: dict, points, gpu, what: str = "") -> None:
    """Every element of (labels, core, counts) equals the oracle's: the
    SHA-256 of each whole array must match the digest the oracle's outputs
    gave.  On a mismatch, the index blocks whose digests differ are named."""
    assert mfs.sha(np.asarray(points, dtype="<f4")) == rec["points_sha256"], \
        f"{what}: input points differ from those the digests were taken on"
    lab, cor, cnt = mfs.canonical(*gpu[:3])
    assert lab.shape[0] == rec["n"]
    bad = []
    for key, arr in (("counts", cnt), ("core", cor), ("labels", lab)):
        if mfs.sha(arr) == rec[f"{key}_sha256"]:
            continue
        blocks = [b for b, (lo, hi) in enumerate(rec["blocks"])
                  if mfs.sha(arr[lo:hi])[:16] != rec["block_sha256_16"][key][b]]
        bad.append(f"{key}: {len(blocks)} of {len(rec['blocks'])} index blocks differ, first "
                   f"{[tuple(rec['blocks'][b]) for b in blocks[:4]]}")
    assert not bad, f"{what}: " + "; ".join(bad)
    s = rec["summary"]
    assert int(cor.sum()) == s["core_points"] and int((lab == -1).sum()) == s["noise"]
