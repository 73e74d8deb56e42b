"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle (oracle/pairs_oracle.c) against a closed form, an
independent algorithm, a library routine, brute force on tiny inputs or an
invariant of the mathematics, chosen so that a dropped term, a wrong sign or
index, a strict instead of non-strict comparison or a double-counted pair makes
one of them fail.  All run on the CPU.
"""
import itertools
import json
import math
import os
from math import comb

import numpy as np
import pytest
from scipy.spatial.distance import cdist, pdist

import oracle
import workloads as w

EPS2 = np.float32(1e-4)


def i32(*arrs):
    return [np.asarray(a, dtype=np.int32) for a in arrs]


# ----------------------------------------------------------- integer counts --

@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 64, 301])
def test_coincident_spheres_all_collide(n):
    # every pair is at distance 0 <= (r_i + r_j)^2: C(N, 2)
    x, y, z = (np.full(n, 7, np.int32) for _ in range(3))
    r = np.arange(n, dtype=np.int32) % 5
    assert oracle.count_i32(x, y, z, r) == comb(n, 2)


def touching_chain(n, seed, gap):
    """Spheres on a line, neighbours at distance exactly r_k + r_{k+1} + gap."""
    rng = np.random.default_rng(seed)
    r = rng.integers(1, 1000, n).astype(np.int64)
    pos = np.zeros(n, np.int64)
    pos[1:] = np.cumsum(r[:-1] + r[1:] + gap)
    return pos.astype(np.int32), r.astype(np.int32)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_chain_touching_counts_neighbours(axis):
    # contact at exactly r_i + r_j counts (<=); non-neighbours are farther apart
    n = 200
    pos, r = touching_chain(n, seed=axis + 10, gap=0)
    zero = np.zeros(n, np.int32)
    coords = [zero, zero, zero]
    coords[axis] = pos
    rng = np.random.default_rng(axis)
    perm = rng.permutation(n)
    assert oracle.count_i32(*coords, r) == n - 1
    assert oracle.count_i32(*(c[perm] for c in coords), r[perm]) == n - 1
    # one unit of clearance separates every neighbour pair
    pos1, r1 = touching_chain(n, seed=axis + 10, gap=1)
    coords[axis] = pos1
    assert oracle.count_i32(*coords, r1) == 0


def test_chain_off_axis_term_matters():
    # neighbours touch along x, and an added y offset of 1 on every other sphere
    # separates every pair: a dropped y term would still count N - 1
    n = 50
    pos, r = touching_chain(n, seed=3, gap=0)
    y = (np.arange(n) % 2).astype(np.int32)
    z = np.zeros(n, np.int32)
    assert oracle.count_i32(pos, y, z, r) == 0
    assert oracle.count_i32(pos, z, y, r) == 0


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_cubic_lattice_face_neighbours(m):
    # m^3 lattice, spacing 2r, radius r: only face neighbours touch, 3 m^2 (m-1)
    rad = 5
    g = np.arange(m) * 2 * rad
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = (a.ravel().astype(np.int32) for a in (X, Y, Z))
    r = np.full(x.shape[0], rad, np.int32)
    assert oracle.count_i32(x, y, z, r) == 3 * m * m * (m - 1)
    # a lattice translated far from the origin (in the negative range) too
    assert oracle.count_i32(x - 2 ** 30, y - 12345, z + 2 ** 29, r) == 3 * m * m * (m - 1)


def collisions_by_site(x, y, z):
    """Collisions of point beads from their site multiplicities (Section 3
    counts collisions from the occupancy of lattice sites): the m beads that
    share a site give C(m, 2) pairs."""
    _, m = np.unique(np.stack([x, y, z], 1), axis=0, return_counts=True)
    return int(sum(comb(int(k), 2) for k in m))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_point_beads_match_site_multiplicities(seed):
    # radius 0: a collision is two beads on the same site; counting site
    # multiplicities is an independent way to count them
    rng = np.random.default_rng(seed)
    n = 3000
    # random walk of beads, as in the paper's experiments (Section 5)
    steps = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    walk = np.cumsum(steps[rng.integers(0, 6, n)], axis=0)
    walk[0] = 0
    x, y, z = (walk[:, k].astype(np.int32) for k in range(3))
    r = np.zeros(n, np.int32)
    expect = collisions_by_site(x, y, z)
    assert expect > 0
    assert oracle.count_i32(x, y, z, r) == expect


def pdist_count(x, y, z, r):
    """Count with scipy's pairwise squared distances (float64, exact below 2^53)."""
    p = np.stack([x, y, z], 1).astype(np.float64)
    d2 = pdist(p, "sqeuclidean")
    ri = np.asarray(r, np.int64)
    rr = (ri[:, None] + ri[None, :])
    iu = np.triu_indices(len(ri), 1)
    R2 = (rr[iu].astype(np.float64)) ** 2
    return int(np.count_nonzero(d2 <= R2))


@pytest.mark.parametrize("seed,n,coord_hi,rad_hi", [
    (1, 500, 2 ** 10, 2 ** 6), (2, 1200, 2 ** 16, 2 ** 12), (3, 2001, 2 ** 20, 2 ** 17),
    (4, 800, 64, 4)])
def test_count_matches_scipy_pdist(seed, n, coord_hi, rad_hi):
    s = w.spheres_i32(n, seed, coord_hi, rad_hi)
    assert oracle.count_i32(*s.arrays()) == pdist_count(*s.arrays())


def test_count_brute_force_tiny():
    rng = np.random.default_rng(7)
    for n in range(0, 40):
        x, y, z = (rng.integers(-20, 20, n).astype(np.int32) for _ in range(3))
        r = rng.integers(0, 12, n).astype(np.int32)
        expect = 0
        for i, j in itertools.combinations(range(n), 2):
            d2 = sum((int(a[i]) - int(a[j])) ** 2 for a in (x, y, z))
            expect += d2 <= (int(r[i]) + int(r[j])) ** 2
        assert oracle.count_i32(x, y, z, r) == expect


def test_int32_domain_extremes():
    lo, hi = -2 ** 31, 2 ** 31 - 1
    big = 2 ** 31 - 1
    # distance 2^32 - 1 against reach 2^32 - 2: apart
    x, y, z, r = i32([lo, hi], [0, 0], [0, 0], [big, big])
    assert oracle.count_i32(x, y, z, r) == 0
    # distance 2^32 - 2 = reach: touching
    x, y, z, r = i32([lo, hi - 1], [0, 0], [0, 0], [big, big])
    assert oracle.count_i32(x, y, z, r) == 1
    # all three axes at full span: d^2 = 3 (2^32 - 1)^2 > (2^32 - 2)^2
    x, y, z, r = i32([lo, hi], [lo, hi], [hi, lo], [big, big])
    assert oracle.count_i32(x, y, z, r) == 0


def test_count_invariances():
    s = w.spheres_i32(900, 11, 2 ** 12, 2 ** 8)
    x, y, z, r = s.arrays()
    c = oracle.count_i32(x, y, z, r)
    assert c > 0
    perm = np.random.default_rng(1).permutation(len(x))
    assert oracle.count_i32(x[perm], y[perm], z[perm], r[perm]) == c
    assert oracle.count_i32(x + 1000, y - 77777, z + 3, r) == c      # translation
    assert oracle.count_i32(z, x, y, r) == c                         # axis swap
    assert oracle.count_i32(-x, y, -z, r) == c                       # reflection
    assert oracle.count_i32(3 * x, 3 * y, 3 * z, 3 * r) == c         # scaling


@pytest.mark.parametrize("split", [0, 1, 137, 450, 899])
def test_count_partition_identity(split):
    # C(A u B) = C(A) + C(B) + cross(A, B)
    s = w.spheres_i32(900, 12, 2 ** 11, 2 ** 8)
    a = [v[:split] for v in s.arrays()]
    b = [v[split:] for v in s.arrays()]
    cross = oracle.cross_count_i32(a, b)
    total = oracle.count_i32(*s.arrays())
    assert total == oracle.count_i32(*a) + oracle.count_i32(*b) + cross


def test_cross_count_matches_scipy_cdist():
    sa = w.spheres_i32(300, 21, 2 ** 10, 2 ** 7)
    sb = w.spheres_i32(410, 22, 2 ** 10, 2 ** 7)
    pa = np.stack(sa.arrays()[:3], 1).astype(np.float64)
    pb = np.stack(sb.arrays()[:3], 1).astype(np.float64)
    d2 = cdist(pa, pb, "sqeuclidean")
    R2 = (sa.r.astype(np.float64)[:, None] + sb.r.astype(np.float64)[None, :]) ** 2
    assert oracle.cross_count_i32(sa.arrays(), sb.arrays()) == int(np.count_nonzero(d2 <= R2))


def test_threads_do_not_change_counts():
    s = w.spheres_i32(1500, 5, 2 ** 12, 2 ** 8)
    assert oracle.count_i32(*s.arrays(), threads=1) == oracle.count_i32(*s.arrays(), threads=3)


# -------------------------------------------------------- float32 counts ----

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_f32_count_equals_integer_count_on_dyadic_inputs(seed):
    # coordinates k * 2^-10 with |k| < 2^10 and radii m * 2^-10: every step of
    # the pinned binary32 sequence is exact, so it decides like the integers
    rng = np.random.default_rng(seed)
    n = 700
    k = rng.integers(0, 2 ** 10, (n, 3)).astype(np.int32)
    m = rng.integers(0, 2 ** 6, n).astype(np.int32)
    expect = oracle.count_i32(k[:, 0], k[:, 1], k[:, 2], m)
    f = [np.ldexp(k[:, a].astype(np.float32), -10) for a in range(3)]
    rf = np.ldexp(m.astype(np.float32), -10)
    assert oracle.count_f32(*f, rf) == expect
    assert expect > 0


def test_f32_count_orientation_and_permutation():
    b = w.moving_sets(n_sets=1, seed=9, size_hi=4096)
    x, y, z, r = b.objs.arrays()
    c = oracle.count_f32(x, y, z, r)
    perm = np.random.default_rng(2).permutation(len(x))
    assert oracle.count_f32(x[perm], y[perm], z[perm], r[perm]) == c
    assert oracle.count_f32(x[::-1].copy(), y[::-1].copy(), z[::-1].copy(), r) == c


def test_f32_touching_pair_counts():
    # two spheres of radius 0.25 at distance 0.5 (all exact in binary32)
    x = np.array([0.0, 0.5], np.float32)
    zero = np.zeros(2, np.float32)
    r = np.full(2, 0.25, np.float32)
    assert oracle.count_f32(x, zero, zero, r) == 1
    x[1] = np.nextafter(np.float32(0.5), np.float32(1))
    assert oracle.count_f32(x, zero, zero, r) == 0


# -------------------------------------------------------------- energies ----

def test_energy_two_particles_closed_form():
    x = np.array([0.0, 0.75], np.float32)
    y = np.array([0.0, 1.0], np.float32)
    z = np.zeros(2, np.float32)
    d2 = 0.75 ** 2 + 1.0
    expect = 1.0 / math.sqrt(d2 + float(EPS2))
    assert oracle.energy_total(x, y, z, EPS2) == pytest.approx(expect, rel=1e-15)
    E = oracle.energy_rows(x, y, z, EPS2)
    assert E == pytest.approx([expect, expect], rel=1e-15)


@pytest.mark.parametrize("n", [2, 3, 100, 1001])
def test_energy_coincident_closed_form(n):
    x, y, z = (np.full(n, 0.3, np.float32) for _ in range(3))
    inv = 1.0 / math.sqrt(float(EPS2))
    assert oracle.energy_total(x, y, z, EPS2) == pytest.approx(comb(n, 2) * inv, rel=1e-14)
    E = oracle.energy_rows(x, y, z, EPS2)
    np.testing.assert_allclose(E, (n - 1) * inv, rtol=1e-14)


def test_energy_matches_scipy_with_exact_sum():
    p = w.particles_f32(1500, 31)
    x, y, z = p.arrays()
    pts = np.stack([x, y, z], 1).astype(np.float64)
    e = 1.0 / np.sqrt(pdist(pts, "sqeuclidean") + float(EPS2))
    expect = math.fsum(e.tolist())
    assert oracle.energy_total(x, y, z, EPS2) == pytest.approx(expect, rel=1e-13)
    D = cdist(pts, pts, "sqeuclidean")
    M = 1.0 / np.sqrt(D + float(EPS2))
    np.fill_diagonal(M, 0.0)
    rows = [math.fsum(row.tolist()) for row in M]
    np.testing.assert_allclose(oracle.energy_rows(x, y, z, EPS2), rows, rtol=1e-13)


def test_energy_sum_identity_and_permutation():
    p = w.particles_f32(2000, 32)
    x, y, z = p.arrays()
    tot = oracle.energy_total(x, y, z, EPS2)
    E = oracle.energy_rows(x, y, z, EPS2)
    assert math.fsum(E.tolist()) == pytest.approx(2 * tot, rel=1e-13)
    perm = np.random.default_rng(0).permutation(len(x))
    assert oracle.energy_total(x[perm], y[perm], z[perm], EPS2) == pytest.approx(tot, rel=1e-13)
    sub = np.array([0, 5, 1999, 1000])
    np.testing.assert_allclose(oracle.energy_rows(x, y, z, EPS2, rows=sub), E[sub], rtol=0)


def test_energy_uniform_cube_sanity():
    # sanity only: the mean softened inverse distance of two uniform points in
    # the unit cube is about 1.88
    p = w.particles_f32(3000, 33)
    tot = oracle.energy_total(*p.arrays(), EPS2)
    assert 1.80 < tot / comb(3000, 2) < 1.96


# --------------------------------------------------------------- batches ----

def test_batched_equals_single_sets_with_edge_sizes():
    rng = np.random.default_rng(3)
    sizes = np.array([0, 1, 2, 3, 0, 64, 65, 200, 1, 513], np.int64)
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(int(off[-1]), 4, 2 ** 9, 2 ** 5)
    got = oracle.count_i32_batched(*s.arrays(), off)
    for k in range(len(sizes)):
        sl = slice(off[k], off[k + 1])
        assert got[k] == oracle.count_i32(*(a[sl] for a in s.arrays()))
    assert got[0] == got[1] == got[4] == got[8] == 0
    perm = rng.permutation(len(sizes))
    # reordering the sets permutes the outputs
    parts = [[a[off[k]:off[k + 1]] for a in s.arrays()] for k in perm]
    cat = [np.concatenate([p[c] for p in parts]) for c in range(4)]
    off2 = w.offsets_from_sizes(sizes[perm])
    np.testing.assert_array_equal(oracle.count_i32_batched(*cat, off2), got[perm])


def test_energy_count_batched_equals_single_sets():
    b = w.moving_sets(n_sets=40, seed=12, size_hi=300)
    x, y, z, r = b.objs.arrays()
    e, c = oracle.energy_count_f32_batched(x, y, z, r, b.offsets, EPS2)
    for k in range(b.n_sets):
        sl = slice(b.offsets[k], b.offsets[k + 1])
        assert e[k] == pytest.approx(oracle.energy_total(x[sl], y[sl], z[sl], EPS2), rel=1e-15)
        assert c[k] == oracle.count_f32(x[sl], y[sl], z[sl], r[sl])


# ---------------------------------------------------------------- jitter ----

def test_philox_known_answers(golden_dir):
    with open(os.path.join(golden_dir, "philox_kat.json")) as f:
        g = json.load(f)
    for v in g["vectors"]:
        ctr = [int(a, 16) for a in v["ctr"]]
        key = [int(a, 16) for a in v["key"]]
        out = [int(a, 16) for a in v["out"]]
        assert oracle.philox4x32_10(ctr, key).tolist() == out


def test_jitter_statistics_and_determinism():
    n = 200_000
    zero = np.zeros(n, np.float32)
    sigma = 1e-3
    x, y, z = oracle.jitter_f32(zero, zero, zero, seed=6, step=0, sigma=sigma)
    for a in (x, y, z):
        assert abs(float(a.mean())) < 5 * sigma / math.sqrt(n)
        assert float(a.std()) == pytest.approx(sigma, rel=0.01)
        assert float(np.abs(a).max()) <= 2 * math.sqrt(3) * sigma * (1 + 1e-6)
    x2, _, _ = oracle.jitter_f32(zero, zero, zero, seed=6, step=0, sigma=sigma)
    np.testing.assert_array_equal(x, x2)
    x3, _, _ = oracle.jitter_f32(zero, zero, zero, seed=6, step=1, sigma=sigma)
    assert np.count_nonzero(x3 == x) < n // 1000
    # object k of a sub-range is object first_index + k of the whole
    xs, _, _ = oracle.jitter_f32(zero[:100], zero[:100], zero[:100], 6, 0, sigma,
                                 first_index=5000)
    np.testing.assert_array_equal(xs, x[5000:5100])
