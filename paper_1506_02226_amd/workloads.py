"""Seeded synthetic DBSCAN workloads (Gaussian blobs plus uniform noise).

This module only draws input points and picks the (eps, MinPts) parameters of
each workload; it contains none of DBSCAN's own arithmetic (no epsilon test, no
counting, no merging).  Both the GPU path and the CPU oracle are fed from here.

The paper evaluates on an unnamed 3-D point set that is not published
(Section IV, Table I; Section V, Tables III-V), so every input is synthetic:

* ``blobs2d_small``   n=2,000,   d=2,  5 isotropic blobs (std 0.5) + 10% noise,
                      eps=0.3,  MinPts=5.
* ``blobs2d_200k``    n=200,000, d=2,  50 blobs (std ~ U[0.2, 1.0]) + 5% noise,
                      eps=0.25, MinPts=10.
* ``aniso3d_2m``      n=2,000,000, d=3, 200 anisotropic blobs in [0,500]^3
                      (covariance Q diag(lambda) Q^T, lambda ~ U[0.1, 1]) + 5%
                      noise, eps=0.4, MinPts=20.
* ``mix64d_300k``     n=300,000, d=64, 100 components with centres 10*g/|g|,
                      unit per-coordinate std, + 2% noise in the bounding box,
                      eps=6.0, MinPts=15 (``mix64d_300k_q50``: same points, eps
                      set to the median sampled core distance).
* ``served_job(j)``   the jobs of the served workload (n log-uniform in
                      [1e3, 2e5], d in {2,3,16,64}, 5-50 blobs, 5% noise).

Draw order is fixed: centres, per-blob parameters, blob points in blob order,
noise, then a single ``rng.permutation`` shuffle so that index order carries no
spatial locality.  Blob sizes are floor(n_blob / k) with the remainder given to
the first blobs.  Values are drawn in float64 and cast to float32 at the end.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "blob_sizes",
    "blobs2d_small",
    "blobs2d_200k",
    "aniso3d_2m",
    "mix64d_300k",
    "served_job",
    "served_arrivals",
    "by_name",
    "WORKLOADS",
    "round_sig",
]


@dataclass
class Workload:
    name: str
    points: np.ndarray  # float32, C-contiguous, shape (n, d)
    eps: float
    minpts: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def d(self) -> int:
        return int(self.points.shape[1])


def round_sig(x: float, sig: int = 4) -> float:
    """Round a positive parameter to `sig` significant digits.

    Parameters chosen from data (eps quantiles) are rounded so that they do not
    depend on the last bits of a BLAS reduction on a particular host.
    """
    if x == 0.0 or not math.isfinite(x):
        return float(x)
    return float(f"{x:.{sig - 1}e}")


def blob_sizes(n_blob: int, k: int) -> list[int]:
    base, rem = divmod(n_blob, k)
    return [base + (1 if b < rem else 0) for b in range(k)]


def _finish(rng: np.random.Generator, blob_pts: list[np.ndarray], noise: np.ndarray) -> np.ndarray:
    pts = np.concatenate(blob_pts + [noise], axis=0)
    pts = pts[rng.permutation(pts.shape[0])]
    return np.ascontiguousarray(pts.astype(np.float32))


def isotropic_blobs(
    rng: np.random.Generator,
    n: int,
    d: int,
    k: int,
    box: float,
    noise_frac: float,
    sigma_lo: float,
    sigma_hi: float | None = None,
) -> np.ndarray:
    """k isotropic Gaussian blobs with centres ~ U[0, box]^d plus uniform noise."""
    n_noise = int(round(noise_frac * n))
    n_blob = n - n_noise
    centres = rng.uniform(0.0, box, size=(k, d))
    if sigma_hi is None:
        sigmas = np.full(k, sigma_lo)
    else:
        sigmas = rng.uniform(sigma_lo, sigma_hi, size=k)
    blob_pts = []
    for b, m in enumerate(blob_sizes(n_blob, k)):
        blob_pts.append(centres[b] + sigmas[b] * rng.standard_normal((m, d)))
    noise = rng.uniform(0.0, box, size=(n_noise, d))
    return _finish(rng, blob_pts, noise)


def blobs2d_small(seed: int = 0, n: int = 2000) -> Workload:
    rng = np.random.default_rng(seed)
    pts = isotropic_blobs(rng, n, 2, 5, 20.0, 0.10, 0.5)
    return Workload("blobs2d_small", pts, 0.3, 5, {"seed": seed, "blobs": 5, "noise": 0.10})


def blobs2d_200k(seed: int = 0, n: int = 200_000) -> Workload:
    rng = np.random.default_rng(seed)
    pts = isotropic_blobs(rng, n, 2, 50, 200.0, 0.05, 0.2, 1.0)
    return Workload("blobs2d_200k", pts, 0.25, 10, {"seed": seed, "blobs": 50, "noise": 0.05})


def _haar_rotation(rng: np.random.Generator, d: int) -> np.ndarray:
    a = rng.standard_normal((d, d))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def aniso3d_2m(seed: int = 0, n: int = 2_000_000) -> Workload:
    rng = np.random.default_rng(seed)
    d, k, box = 3, 200, 500.0
    n_noise = int(round(0.05 * n))
    n_blob = n - n_noise
    centres = rng.uniform(0.0, box, size=(k, d))
    rots = [_haar_rotation(rng, d) for _ in range(k)]
    lams = rng.uniform(0.1, 1.0, size=(k, d))
    blob_pts = []
    for b, m in enumerate(blob_sizes(n_blob, k)):
        z = rng.standard_normal((m, d)) * np.sqrt(lams[b])[None, :]
        blob_pts.append(centres[b] + z @ rots[b].T)
    noise = rng.uniform(0.0, box, size=(n_noise, d))
    pts = _finish(rng, blob_pts, noise)
    return Workload("aniso3d_2m", pts, 0.4, 20, {"seed": seed, "blobs": k, "noise": 0.05})


def paper3d(seed: int = 0, n: int = 23_040) -> Workload:
    """3-D points at the paper's own sizes (N = 5,061 / 23,040 / 60,032 in
    Tables I and III-V; its dataset is not published): 20 anisotropic
    Gaussian blobs (covariance Q diag(lambda) Q^T, lambda ~ U[0.1, 1]) with
    centres in [0, 60]^3, plus 5% uniform noise; eps = 0.4, MinPts = 20."""
    rng = np.random.default_rng(seed)
    d, k, box = 3, 20, 60.0
    n_noise = int(round(0.05 * n))
    centres = rng.uniform(0.0, box, size=(k, d))
    rots = [_haar_rotation(rng, d) for _ in range(k)]
    lams = rng.uniform(0.1, 1.0, size=(k, d))
    blob_pts = []
    for b, m in enumerate(blob_sizes(n - n_noise, k)):
        z = rng.standard_normal((m, d)) * np.sqrt(lams[b])[None, :]
        blob_pts.append(centres[b] + z @ rots[b].T)
    noise = rng.uniform(0.0, box, size=(n_noise, d))
    pts = _finish(rng, blob_pts, noise)
    return Workload("paper3d", pts, 0.4, 20, {"seed": seed, "blobs": k, "noise": 0.05})


def mixture_blobs(
    rng: np.random.Generator, n: int, d: int, k: int, noise_frac: float, radius: float = 10.0
) -> np.ndarray:
    """k unit-variance Gaussian components whose centres are random unit
    vectors scaled by `radius`, plus uniform noise over the bounding box of
    the component points."""
    n_noise = int(round(noise_frac * n))
    n_blob = n - n_noise
    g = rng.standard_normal((k, d))
    centres = radius * g / np.linalg.norm(g, axis=1, keepdims=True)
    blob_pts = []
    for b, m in enumerate(blob_sizes(n_blob, k)):
        blob_pts.append(centres[b] + rng.standard_normal((m, d)))
    allb = np.concatenate(blob_pts, axis=0)
    lo, hi = allb.min(axis=0), allb.max(axis=0)
    noise = rng.uniform(lo, hi, size=(n_noise, d))
    return _finish(rng, blob_pts, noise)


def _mix64d_points(seed: int, n: int, d: int = 64, k: int = 100) -> np.ndarray:
    return mixture_blobs(np.random.default_rng(seed), n, d, k, 0.02)


def core_distance_quantile(
    pts: np.ndarray, minpts: int, q: float, sample: int, rng: np.random.Generator
) -> float:
    """q-quantile over a point sample of each point's distance to its
    MinPts-th nearest point (itself counted).  Used only to choose eps; the
    distances come from a float64 Gram product and the result is rounded to
    four significant digits."""
    n = pts.shape[0]
    m = min(n, sample)
    idx = np.sort(rng.choice(n, size=m, replace=False))
    x = pts.astype(np.float64)
    nx = np.einsum("ij,ij->i", x, x)
    out = np.empty(m)
    for s0 in range(0, m, 64):
        s = x[idx[s0 : s0 + 64]]
        d2 = nx[idx[s0 : s0 + 64], None] + nx[None, :] - 2.0 * (s @ x.T)
        np.maximum(d2, 0.0, out=d2)
        kth = np.partition(d2, minpts - 1, axis=1)[:, minpts - 1]
        out[s0 : s0 + 64] = np.sqrt(kth)
    return round_sig(float(np.quantile(out, q)))


def mix64d_300k(seed: int = 0, n: int = 300_000, eps_rule: str = "literal") -> Workload:
    pts = _mix64d_points(seed, n)
    minpts = 15
    if eps_rule == "literal":
        eps = 6.0
        name = "mix64d_300k"
    elif eps_rule == "q50":
        eps = core_distance_quantile(pts, minpts, 0.5, 1000, np.random.default_rng(seed + 1000))
        name = "mix64d_300k_q50"
    else:
        raise ValueError(eps_rule)
    return Workload(name, pts, eps, minpts, {"seed": seed, "blobs": 100, "noise": 0.02, "eps_rule": eps_rule})


SERVED_D = (2, 3, 16, 64)
SERVED_MINPTS = (5, 10, 20)


def served_job(j: int, eps_sample: int = 256) -> Workload:
    """Job j of the served workload (drawn from seed j+1)."""
    rng = np.random.default_rng(j + 1)
    n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
    d = int(SERVED_D[rng.integers(0, len(SERVED_D))])
    k = int(rng.integers(5, 51))
    minpts = int(SERVED_MINPTS[rng.integers(0, len(SERVED_MINPTS))])
    if d <= 3:  # the 2-D recipe: centres in [0, 200]^d, std in [0.2, 1]
        pts = isotropic_blobs(rng, n, d, k, 200.0, 0.05, 0.2, 1.0)
    else:  # the high-dimensional mixture recipe: centres at radius 10, std 1
        pts = mixture_blobs(rng, n, d, k, 0.05)
    eps = core_distance_quantile(pts, minpts, 0.02, eps_sample, rng)
    return Workload(f"served_job_{j}", pts, eps, minpts, {"job": j, "blobs": k})


def served_arrivals(num_jobs: int, rate: float, seed: int = 0) -> np.ndarray:
    """Poisson arrival times (seconds from start) at `rate` jobs/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=num_jobs))


WORKLOADS = {
    "blobs2d_small": blobs2d_small,
    "blobs2d_200k": blobs2d_200k,
    "aniso3d_2m": aniso3d_2m,
    "mix64d_300k": mix64d_300k,
    "mix64d_300k_q50": lambda seed=0, n=300_000: mix64d_300k(seed, n, "q50"),
    "paper3d": paper3d,
}


def by_name(name: str, seed: int = 0, n: int | None = None) -> Workload:
    fn = WORKLOADS[name]
    return fn(seed) if n is None else fn(seed, n)
