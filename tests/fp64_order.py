"""Pairs of float32 points whose float64 decision depends on the order and
fusion of the squared-distance sum (shared by the CPU pin of the oracle and
the GPU parity test; not a test module itself).

The reading taken for the paper's distance (Section IV-B.2 writes it as the
direct sum of squared coordinate differences; the precision, order and
fusion are not stated) is: coordinates widened exactly from float32, then
for k = 0..d-1: t = x_ik - x_jk, s = s + t*t, each operation rounded on its
own, neighbour iff s <= eps^2 with eps^2 rounded once.  Each case below is a
pair (a, b) and an eps for which that sequential, unfused value and one
plausible alternative fall on opposite sides of fl(eps*eps):

  fused     s = fma(t, t, s)             (one rounding per coordinate)
  reversed  k = d-1 .. 0
  pairwise  numpy's np.sum order (eight partial sums for d >= 8)
  exact     the exactly rounded sum (math.fsum of the rounded squares)

Every value is computed here from exact rationals with one explicit
round-to-nearest-even per operation (``float(Fraction)`` is correctly
rounded), independently of numpy's and the C compiler's arithmetic.  The
search is seeded, so the cases are the same on every run.
"""
from __future__ import annotations

import math
from fractions import Fraction as Q

import numpy as np

VARIANTS = ("fused", "reversed", "pairwise", "exact")


def _rn(x: Q) -> float:
    return float(x)  # correctly rounded to the nearest double, ties to even


def _diffs(a, b):
    # float32 -> float64 is exact; the difference is rounded once
    return [_rn(Q(float(x)) - Q(float(y))) for x, y in zip(a, b)]


def _sq(t: float) -> float:
    return _rn(Q(t) * Q(t))


def sequential(a, b) -> float:
    s = 0.0
    for t in _diffs(a, b):
        s = _rn(Q(s) + Q(_sq(t)))
    return s


def fused(a, b) -> float:
    s = 0.0
    for t in _diffs(a, b):
        s = _rn(Q(t) * Q(t) + Q(s))
    return s


def reversed_order(a, b) -> float:
    s = 0.0
    for t in reversed(_diffs(a, b)):
        s = _rn(Q(s) + Q(_sq(t)))
    return s


def pairwise(a, b) -> float:
    """numpy's pairwise summation for fewer than 128 terms: eight running
    partial sums, combined as ((r0+r1)+(r2+r3))+((r4+r5)+(r6+r7)), then the
    remainder added in order (sequential below 8 terms)."""
    v = [_sq(t) for t in _diffs(a, b)]
    add = lambda x, y: _rn(Q(x) + Q(y))
    if len(v) < 8:
        s = 0.0
        for x in v:
            s = add(s, x)
        return s
    r = v[:8]
    i = 8
    while i + 8 <= len(v):
        r = [add(r[j], v[i + j]) for j in range(8)]
        i += 8
    s = add(add(add(r[0], r[1]), add(r[2], r[3])), add(add(r[4], r[5]), add(r[6], r[7])))
    while i < len(v):
        s = add(s, v[i])
        i += 1
    return s


def exact(a, b) -> float:
    return _rn(sum((Q(_sq(t)) for t in _diffs(a, b)), Q(0)))


ALT = {"fused": fused, "reversed": reversed_order, "pairwise": pairwise, "exact": exact}


def _eps_with_square(target: float):
    """A double eps with fl(eps * eps) == target, or None."""
    r = math.sqrt(target)
    cands = [r]
    up, dn = r, r
    for _ in range(6):
        up, dn = float(np.nextafter(up, np.inf)), float(np.nextafter(dn, 0.0))
        cands += [up, dn]
    for e in cands:
        if _rn(Q(e) * Q(e)) == target:
            return e
    return None


def variants_for(d: int):
    """The alternatives that can differ from the sequential sum at this d:
    below 8 terms numpy's pairwise order is the sequential one, and with two
    terms only fusion changes the result (addition is commutative)."""
    if d <= 2:
        return ("fused",)
    if d < 8:
        return ("fused", "reversed", "exact")
    return VARIANTS


def cases(d: int, seed: int = 2024):
    """One case per (variant, direction) of ``variants_for(d)``: direction
    "in" means the sequential value is a neighbour and the variant's is not;
    "out" the reverse.  Returns a list of dicts with float32 arrays a, b, the
    double eps, the variant, the sequential decision and both values."""
    rng = np.random.default_rng(seed + d)
    want = {(v, dr) for v in variants_for(d) for dr in ("in", "out")}
    out = []
    for _ in range(200_000):
        if not want:
            break
        a = rng.uniform(-4, 4, d).astype(np.float32)
        b = (a.astype(np.float64) + rng.uniform(-1, 1, d)).astype(np.float32)
        s = sequential(a, b)
        for v in variants_for(d):
            alt = ALT[v](a, b)
            if alt == s:
                continue
            direction = "in" if s < alt else "out"
            if (v, direction) not in want:
                continue
            eps = _eps_with_square(min(s, alt))
            if eps is None:
                continue
            want.discard((v, direction))
            out.append({"a": a, "b": b, "eps": eps, "variant": v, "direction": direction,
                        "seq": s, "alt": alt, "in": s <= _rn(Q(eps) * Q(eps))})
    if want:
        raise RuntimeError(f"no case found for {sorted(want)} at d={d}")
    return out
