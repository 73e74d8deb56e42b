"""Pin of the float32 collision oracle's rounding sequence.

The float32 count decides each pair by one fixed binary32 sequence (the
reading of the paper's unspecified float collision test, Section 4 and
Section 5's floating-point spheres).  Inputs where every order is exact cannot
tell a wrong sequence from the right one, so these tests use pairs at the
touching distance, where one rounding more or less flips the answer, and check
the oracle against an exact rational model of each IEEE operation
(tests/f32_exact.py).  The pairs are chosen so that the plain-product chain,
the reordered fused chain, exact arithmetic and flushed subnormals each
disagree with the pinned sequence on several of them: any of those mistakes in
the oracle fails here.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from f32_exact import (discriminating_pairs, exact, pinned_hit, round_binary32,
                       variant_hits)


def test_rounding_model_matches_ieee_conversion():
    # numpy's float64 -> float32 conversion is IEEE round to nearest even,
    # subnormals included: the model must give the same value for any double
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.normal(size=2000),
        rng.normal(size=500) * 1e-39,           # subnormal binary32 range
        rng.normal(size=500) * 1e-45,           # around the smallest subnormal
        rng.normal(size=500) * 1e37,
        # exact ties between two binary32 values: 1 + (2k + 1) 2^-24
        1.0 + (2 * np.arange(200) + 1) * 2.0 ** -24,
        (2 * np.arange(200) + 1) * 2.0 ** -150,  # ties between subnormals
    ])
    for v in vals:
        assert round_binary32(Fraction(float(v))) == exact(np.float32(v)), v


def test_rounding_model_hand_values():
    assert round_binary32(Fraction(1) + Fraction(1, 2 ** 24)) == 1  # tie to even (down)
    assert round_binary32(Fraction(1) + Fraction(3, 2 ** 24)) == 1 + Fraction(2, 2 ** 23)
    assert round_binary32(Fraction(1, 2 ** 150)) == 0                # tie to even zero
    assert round_binary32(Fraction(3, 2 ** 150)) == Fraction(2, 2 ** 149)
    assert round_binary32(Fraction(-5, 2 ** 151)) == -Fraction(1, 2 ** 149)
    with pytest.raises(OverflowError):
        round_binary32(Fraction(2) ** 128)


@pytest.fixture(scope="module")
def pairs_unit():
    return discriminating_pairs(6000, seed=11)


@pytest.fixture(scope="module")
def pairs_subnormal():
    return discriminating_pairs(600, seed=12, scale=1e-20)


def test_pairs_discriminate_every_wrong_sequence(pairs_unit, pairs_subnormal):
    _, _, _, t1 = pairs_unit
    _, _, _, t2 = pairs_subnormal
    assert t1["plain"] >= 5 and t1["reordered"] >= 5 and t1["exact"] >= 5
    assert t2["flushed"] >= 5


def _oracle_pair(pi, pj):
    x, y, z, r = (np.array([pi[a], pj[a]], np.float32) for a in range(4))
    return oracle.count_f32(x, y, z, r)


@pytest.mark.parametrize("which", ["unit", "subnormal"])
def test_oracle_f32_follows_pinned_sequence(which, pairs_unit, pairs_subnormal):
    pi, pj, hits, _ = pairs_unit if which == "unit" else pairs_subnormal
    assert len(hits) > 0 and hits.any() and not hits.all()
    for k in range(len(hits)):
        assert _oracle_pair(pi[k], pj[k]) == int(hits[k]), k
        # the other orientation: fl(a - b) = -fl(b - a), same answer
        assert _oracle_pair(pj[k], pi[k]) == int(hits[k]), k


def test_pinned_model_is_orientation_symmetric(pairs_unit):
    pi, pj, hits, _ = pairs_unit
    for k in range(min(200, len(hits))):
        assert pinned_hit(pj[k], pi[k]) == hits[k]
        v = variant_hits(pi[k], pj[k])
        assert set(v) == {"plain", "reordered", "exact", "flushed"}
