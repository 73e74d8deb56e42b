"""Pins of the lattice-bead oracle (collision and contact counts, Section 3).

The oracle is the plain pairwise definition (oracle_lattice_counts in
oracle/pairs_oracle.c).  These tests check it against facts fixed outside
it: closed forms of regular bead arrangements, a hand-worked walk (a fixture
under tests/golden/), counts from site multiplicities (Section 3 counts from
site occupancy; here each occupied site's multiplicity is found with
np.unique and neighbouring sites by a sorted search), and invariants.  A swapped predicate (collision for contact), a missing axis, a
diagonal counted as a contact, a halving error or a pair counted twice each
fail one of them.  All run on the CPU.
"""
import json
import os
from math import comb

import numpy as np
import pytest

import oracle
import workloads as w


def beads(points):
    p = np.asarray(points, dtype=np.int32).reshape(-1, 3)
    return [np.ascontiguousarray(p[:, k]) for k in range(3)]


# ------------------------------------------------------------- closed forms --

@pytest.mark.parametrize("n", [0, 1, 2, 5, 64, 257])
def test_all_beads_on_one_site(n):
    # every pair collides, none is a contact
    assert oracle.lattice_counts(*beads([[3, -4, 9]] * n)) == (comb(n, 2), 0)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [1, 2, 10, 333])
def test_straight_line(axis, n):
    # a straight chain: consecutive beads touch, nothing else
    p = np.zeros((n, 3), np.int32)
    p[:, axis] = np.arange(n) - 7
    assert oracle.lattice_counts(*beads(p)) == (0, max(n - 1, 0))


@pytest.mark.parametrize("n", [2, 3, 8, 101])
def test_chain_folded_back_and_forth(n):
    # a chain stepping +x, -x, +x, ...: ceil(n/2) beads on site A, floor(n/2) on B
    p = np.zeros((n, 3), np.int32)
    p[1::2, 0] = 1
    a, b = (n + 1) // 2, n // 2
    assert oracle.lattice_counts(*beads(p)) == (comb(a, 2) + comb(b, 2), a * b)


@pytest.mark.parametrize("k,m", [(1, 1), (2, 1), (3, 1), (4, 2), (5, 3)])
def test_full_cube(k, m):
    # k^3 sites with m beads each: 3 k^2 (k-1) neighbouring site pairs
    g = np.stack(np.meshgrid(*[np.arange(k)] * 3, indexing="ij"), -1).reshape(-1, 3)
    p = np.repeat(g, m, axis=0) + np.array([100, -50, 7])
    assert oracle.lattice_counts(*beads(p)) == (k ** 3 * comb(m, 2),
                                                3 * k * k * (k - 1) * m * m)


def test_diagonal_and_distance_two_are_not_contacts():
    for d in ([1, 1, 0], [1, 0, 1], [0, 1, 1], [1, 1, 1], [2, 0, 0], [0, -2, 0], [0, 0, 2]):
        assert oracle.lattice_counts(*beads([[0, 0, 0], d])) == (0, 0)
    for d in ([1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]):
        assert oracle.lattice_counts(*beads([[0, 0, 0], d])) == (0, 1)


def test_extreme_coordinates():
    # differences beyond int32 must not wrap into a collision or contact
    lo, hi = -2 ** 31, 2 ** 31 - 1
    assert oracle.lattice_counts(*beads([[lo, 0, 0], [hi, 0, 0]])) == (0, 0)
    assert oracle.lattice_counts(*beads([[hi, hi, hi], [hi, hi, hi - 1], [hi, hi, hi]])) == (1, 2)
    assert oracle.lattice_counts(*beads([[lo, lo, lo], [lo + 1, lo, lo]])) == (0, 1)


# ------------------------------------------------------------- hand-worked --

def test_hand_worked_walks(golden_dir):
    with open(os.path.join(golden_dir, "lattice_hand.json")) as f:
        cases = json.load(f)["cases"]
    assert len(cases) >= 3
    for c in cases:
        got = oracle.lattice_counts(*beads(c["beads"]))
        assert got == (c["collisions"], c["contacts"]), c["name"]


# --------------------------------------- site multiplicities (Section 3) --
#
# Section 3 counts both quantities from the occupancy of lattice sites.  The
# same numbers follow from the multiplicity m(s) of each occupied site s:
# the beads sharing a site give C(m(s), 2) collisions, and a site and its
# neighbour one unit further along an axis give m(s) m(s + e) contacts (each
# unordered pair of neighbouring sites taken once, from its lower site).


def site_multiplicities(p):
    sites, mult = np.unique(np.asarray(p, np.int64), axis=0, return_counts=True)
    return sites, mult.astype(np.int64)


def collisions_from_multiplicities(p):
    _, m = site_multiplicities(p)
    return int(np.sum(m * (m - 1) // 2))


def contacts_from_multiplicities(p):
    sites, m = site_multiplicities(p)
    # encode each site as one integer so that membership is a sorted search
    lo = sites.min(axis=0) - 1
    span = sites.max(axis=0) - lo + 2
    key = ((sites[:, 0] - lo[0]) * span[1] + (sites[:, 1] - lo[1])) * span[2] + (sites[:, 2] - lo[2])
    order = np.argsort(key)
    key, m = key[order], m[order]
    total = 0
    for step in (span[1] * span[2], span[2], 1):  # +x, +y, +z neighbours
        at = np.searchsorted(key, key + step)
        found = (at < len(key)) & (key[np.minimum(at, len(key) - 1)] == key + step)
        total += int(np.sum(m[found] * m[at[found]]))
    return total


@pytest.mark.parametrize("seed", range(6))
def test_matches_site_multiplicity_counts(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 300))
    if seed % 2:
        b = w.lattice_walks(1, n, seed)
        p = np.stack(b.objs.arrays(), 1).astype(np.int64)
    else:
        p = np.rint(rng.normal(0, 1.5, (n, 3))).astype(np.int64)
    got = oracle.lattice_counts(*beads(p))
    assert got == (collisions_from_multiplicities(p), contacts_from_multiplicities(p))


# --------------------------------------------------------------- invariants --

def test_invariant_under_translation_and_permutation():
    b = w.lattice_walks(1, 500, 3)
    p = np.stack(b.objs.arrays(), 1)
    ref = oracle.lattice_counts(*beads(p))
    rng = np.random.default_rng(1)
    q = p[rng.permutation(len(p))] + np.array([12345, -999, 70000], np.int32)
    assert oracle.lattice_counts(*beads(q)) == ref


def test_walks_touch_along_the_chain():
    # consecutive beads of a chain are always one unit apart
    b = w.lattice_walks(20, 200, 4)
    coll, cont = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    assert np.all(cont >= 199)
    # a step straight back lands on the site two beads before: a collision
    x, y, z = b.objs.arrays()
    for s in range(20):
        sl = slice(b.offsets[s], b.offsets[s + 1])
        p = np.stack([x[sl], y[sl], z[sl]], 1)
        backs = int(np.sum(np.all(p[2:] == p[:-2], axis=1)))
        assert coll[s] >= backs


def test_batched_equals_single_vectors():
    b = w.lattice_walks(7, [0, 1, 2, 3, 50, 129, 400], 9)
    coll, cont = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    x, y, z = b.objs.arrays()
    for s in range(7):
        sl = slice(b.offsets[s], b.offsets[s + 1])
        assert (int(coll[s]), int(cont[s])) == oracle.lattice_counts(x[sl], y[sl], z[sl])


def test_generator_recipe():
    # chains from the origin by unit steps along one axis
    b = w.lattice_walks(30, 64, 2)
    p = np.stack(b.objs.arrays(), 1).astype(np.int64)
    off = b.offsets
    assert np.all(p[off[:-1]] == 0)
    for s in range(30):
        d = np.abs(np.diff(p[off[s]:off[s + 1]], axis=0)).sum(axis=1)
        assert np.all(d == 1)
