#!/usr/bin/env python3
"""Write the expected outputs of the full-size workloads from the C oracle.

Each workload's counts, core flags and labels come from ``oracle/c_oracle``
(float64 brute force, breadth-first merge, lowest-index border rule) and
nothing else; the GPU path is not involved.  The arrays are stored as SHA-256
digests -- of the whole array and of 64 contiguous index blocks, so that a
mismatch can be located -- together with a digest of the input points (a
change of the seeded generator shows up as a mismatch there, not as a
clustering error) and a few summary numbers.

    python tests/golden/make_full_size.py [name ...] [--threads T]

Names: blobs2d_small, blobs2d_200k, aniso3d_2m, mix64d_300k, mix64d_300k_q50,
served_jobs (jobs 0..31 of the served workload, one file).  Files are written
to tests/golden/full_size/<name>.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "full_size")
BLOCKS = 64
SERVED_JOBS = tuple(range(32))
NAMES = ("blobs2d_small", "blobs2d_200k", "served_jobs", "mix64d_300k", "mix64d_300k_q50",
         "aniso3d_2m")


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def canonical(labels, core, counts):
    """The byte layout every digest is taken over: int32 labels, uint8 core
    flags (0/1), int32 counts, little-endian."""
    return (np.asarray(labels, dtype="<i4"), np.asarray(core, dtype=bool).astype(np.uint8),
            np.asarray(counts, dtype="<i4"))


def block_bounds(n: int, blocks: int = BLOCKS):
    edges = np.linspace(0, n, blocks + 1).round().astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:])]


def digest(points, eps, minpts, labels, core, counts) -> dict:
    lab, cor, cnt = canonical(labels, core, counts)
    n = lab.shape[0]
    bounds = block_bounds(n)
    return {
        "n": int(n), "d": int(points.shape[1]), "eps": float(eps), "eps_hex": float(eps).hex(),
        "minpts": int(minpts),
        "points_sha256": sha(np.asarray(points, dtype="<f4")),
        "labels_sha256": sha(lab), "core_sha256": sha(cor), "counts_sha256": sha(cnt),
        "blocks": bounds,
        "block_sha256_16": {k: [sha(a[lo:hi])[:16] for lo, hi in bounds]
                            for k, a in (("labels", lab), ("core", cor), ("counts", cnt))},
        "summary": {"core_points": int(cor.sum()), "noise": int((lab == -1).sum()),
                    "clusters": int(np.unique(lab[lab >= 0]).size),
                    "sum_counts": int(cnt.astype(np.int64).sum())},
    }


def run_one(w, threads: int) -> dict:
    from oracle import c_oracle
    t0 = time.perf_counter()
    labels, core, counts = c_oracle.dbscan(w.points, w.eps, w.minpts, threads=threads)
    dt = time.perf_counter() - t0
    rec = digest(w.points, w.eps, w.minpts, labels, core, counts)
    rec.update({"workload": w.name, "oracle_seconds": round(dt, 1),
                "oracle_threads": c_oracle.threads(threads)})
    return rec


def make(name: str, threads: int) -> str:
    from paper_1506_02226_amd import workloads as wl
    if name == "served_jobs":
        recs = []
        for j in SERVED_JOBS:
            recs.append(run_one(wl.served_job(j), threads))
            print(f"  served_job {j}: n={recs[-1]['n']} d={recs[-1]['d']} "
                  f"{recs[-1]['oracle_seconds']} s", flush=True)
        payload = {"workload": "served_jobs", "jobs": list(SERVED_JOBS), "records": recs}
    else:
        payload = run_one(wl.by_name(name), threads)
    payload["command"] = f"python tests/golden/make_full_size.py {name}"
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, f"{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(payload, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    return path


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("names", nargs="*", default=list(NAMES))
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args(argv)
    for name in args.names:
        if name not in NAMES:
            raise SystemExit(f"unknown workload {name}; choose from {NAMES}")
        t0 = time.perf_counter()
        path = make(name, args.threads)
        print(f"{name}: {time.perf_counter() - t0:.1f} s -> {os.path.relpath(path, ROOT)}",
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
