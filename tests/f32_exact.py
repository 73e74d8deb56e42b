"""Exact rational model of the pinned binary32 collision predicate.

Every binary32 value is a rational number, so each step of the pinned sequence
(the float32 collision predicate of the interact() test, Section 4, with the
reading that fixes its order of operations) can be computed exactly with
``fractions.Fraction`` and then rounded to the nearest binary32 value, ties to
even, subnormals kept.  That model shares nothing with the C oracle or the GPU
kernels: it is the IEEE 754 definition of each operation written out.

``near_boundary_pairs`` draws pairs of spheres whose distance lies within a few
units in the last place of the sum of their radii, where the order and the
rounding of the steps decide the answer, and reports, for each pair, the
pinned answer and the answers of plausible wrong sequences (plain products, a
reordered chain, exact real arithmetic, flushed subnormals).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

_HALF = Fraction(1, 2)
_TWO = Fraction(2)
_FLT_OVERFLOW = (_TWO ** 24 - _HALF) * _TWO ** 104  # halfway between FLT_MAX and 2^128


def exact(v) -> Fraction:
    """The exact rational value of a float32 (or float64) number."""
    return Fraction(float(v))


def round_binary32(q: Fraction) -> Fraction:
    """Nearest binary32 value to q, ties to the even significand; subnormals are
    kept (spacing 2^-149 below 2^-126).  Raises OverflowError past FLT_MAX."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = -q if q < 0 else q
    if a >= _FLT_OVERFLOW:
        raise OverflowError("rounds to infinity")
    # e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if _TWO ** e > a:
        e -= 1
    elif _TWO ** (e + 1) <= a:
        e += 1
    ulp = _TWO ** (max(e, -126) - 23)
    m = a / ulp
    k = m.numerator // m.denominator
    rem = m - k
    if rem > _HALF or (rem == _HALF and k % 2 == 1):
        k += 1
    return sign * k * ulp


def flush(q: Fraction) -> Fraction:
    """q with subnormal magnitudes replaced by zero (flush to zero)."""
    return Fraction(0) if abs(q) < _TWO ** -126 else q


def pinned_hit(pi, pj) -> bool:
    """The pinned sequence: dx = fl(xi - xj) (dy, dz likewise),
    d2 = fl(fma(dz, dz, fl(fma(dy, dy, fl(dx * dx))))), R = fl(ri + rj),
    hit iff d2 <= fl(R * R)."""
    rn = round_binary32
    xi, yi, zi, ri = (exact(v) for v in pi)
    xj, yj, zj, rj = (exact(v) for v in pj)
    dx, dy, dz = rn(xi - xj), rn(yi - yj), rn(zi - zj)
    d2 = rn(dx * dx)
    d2 = rn(dy * dy + d2)
    d2 = rn(dz * dz + d2)
    R = rn(ri + rj)
    return d2 <= rn(R * R)


def variant_hits(pi, pj) -> dict:
    """Answers of sequences that a plausible mistake would compute instead."""
    rn = round_binary32
    xi, yi, zi, ri = (exact(v) for v in pi)
    xj, yj, zj, rj = (exact(v) for v in pj)
    dx, dy, dz = rn(xi - xj), rn(yi - yj), rn(zi - zj)
    R = rn(ri + rj)
    R2 = rn(R * R)
    out = {}
    # separate products and sums, no fused multiply-add
    d2 = rn(rn(rn(dx * dx) + rn(dy * dy)) + rn(dz * dz))
    out["plain"] = d2 <= R2
    # the fused chain in the other order: fma(dx, dx, fma(dy, dy, dz * dz))
    d2 = rn(dx * dx + rn(dy * dy + rn(dz * dz)))
    out["reordered"] = d2 <= R2
    # exact real arithmetic on the float32 inputs
    out["exact"] = (xi - xj) ** 2 + (yi - yj) ** 2 + (zi - zj) ** 2 <= (ri + rj) ** 2
    # every intermediate flushed to zero when subnormal
    fdx, fdy, fdz = (flush(v) for v in (dx, dy, dz))
    d2 = flush(rn(fdx * fdx))
    d2 = flush(rn(fdy * fdy + d2))
    d2 = flush(rn(fdz * fdz + d2))
    fR = flush(R)
    out["flushed"] = d2 <= flush(rn(fR * fR))
    return out


def near_boundary_pairs(n: int, seed: int, scale: float = 1.0):
    """n pairs (pi, pj) of float32 spheres, pj placed at distance (r_i + r_j)
    times 1 + delta from pi along a random direction, |delta| <= 4e-7.
    scale multiplies coordinates and radii (1e-20 puts every squared distance
    into the subnormal range)."""
    rng = np.random.default_rng(seed)
    p = rng.random((n, 3)) * scale
    r = rng.uniform(0.005, 0.02, (n, 2)) * scale
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    delta = rng.uniform(-4e-7, 4e-7, n)
    q = p + u * ((r[:, 0] + r[:, 1]) * (1.0 + delta))[:, None]
    pi = np.concatenate([p, r[:, :1]], axis=1).astype(np.float32)
    pj = np.concatenate([q, r[:, 1:]], axis=1).astype(np.float32)
    return pi, pj


def discriminating_pairs(n: int, seed: int, scale: float = 1.0):
    """Pairs from near_boundary_pairs for which at least one wrong sequence
    disagrees with the pinned one, with the pinned answers:
    (pi, pj, hits, disagreements by variant name)."""
    pi, pj = near_boundary_pairs(n, seed, scale)
    keep, hits = [], []
    tally = {"plain": 0, "reordered": 0, "exact": 0, "flushed": 0}
    for k in range(n):
        h = pinned_hit(pi[k], pj[k])
        v = variant_hits(pi[k], pj[k])
        differs = [name for name, ans in v.items() if ans != h]
        if differs:
            keep.append(k)
            hits.append(h)
            for name in differs:
                tally[name] += 1
    keep = np.array(keep, dtype=np.int64)
    return pi[keep], pj[keep], np.array(hits, dtype=bool), tally
