"""Single sets whose tiling has more wave tasks than one launch holds
(2^24 waves): the kernels' waves then stride over the tasks.  Results are
checked against closed forms at any size, against the CPU oracle on sampled
rows, and against identities that hold at any size (sum of the per-object
energies = twice the total)."""
import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

EPS2 = np.float32(1e-4)


def cubic_lattice(m, spacing, dtype, seed):
    """m^3 points on a cubic lattice, permuted; the collision count at radius
    spacing/2 is 3 m^2 (m - 1): face neighbours touch, diagonals do not."""
    g = np.arange(m, dtype=np.int64) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    perm = np.random.default_rng(seed).permutation(m ** 3)
    return [a.reshape(-1)[perm].astype(dtype) for a in (X, Y, Z)]


def strides(kind, n):
    tasks, blocks, threads = P.pairs_debug_single_launch(kind, n)
    return tasks > blocks * threads // 64


@pytest.fixture
def small_tiles():
    """Force the smallest single-set shape (64 rows, 64 partners per task) so
    that a set of a few 10^5 objects already needs the grid stride."""
    kinds = []

    def force(kind):
        kinds.append(kind)
        P.pairs_set_shapes(kind, False, [(0, 1, 64)])

    yield force
    for k in kinds:
        P.pairs_set_shapes(k, False, None)


def test_count_i32_cubic_lattice_204():
    # 204^3 = 8 489 664 objects (> 2^23) with the default shapes
    m = 204
    x, y, z = cubic_lattice(m, 10, np.int32, 1)
    r = np.full(m ** 3, 5, np.int32)
    assert strides(P.KIND_COUNT_I32, m ** 3)
    announce("count_i32 cubic lattice", m)
    assert P.count_i32(*dev(x, y, z, r)) == 3 * m * m * (m - 1)


def test_count_i32_grid_stride_small_tiles(small_tiles):
    small_tiles(P.KIND_COUNT_I32)
    m = 74
    x, y, z = cubic_lattice(m, 6, np.int32, 2)
    r = np.full(m ** 3, 3, np.int32)
    assert strides(P.KIND_COUNT_I32, m ** 3)
    announce("count_i32 grid stride, shape (1, 64)", m)
    assert P.count_i32(*dev(x, y, z, r)) == 3 * m * m * (m - 1)
    # one sphere grown to radius 9 (reach 12 = two spacings) gains the lattice
    # points within 12 of it beyond its 6 face neighbours: 12 edge and 8
    # corner diagonals and 6 second-shell points along the axes
    r2 = r.copy()
    centre = int(np.flatnonzero((x == 30 * 6) & (y == 30 * 6) & (z == 30 * 6))[0])
    r2[centre] = 9
    assert P.count_i32(*dev(x, y, z, r2)) == 3 * m * m * (m - 1) + 26


def test_count_i32_matrix_form_grid_stride():
    """The matrix-core form with 64-partner chunks: 405 224 objects need the
    grid stride; the lattice's closed form with one grown sphere."""
    P.pairs_set_shapes(P.KIND_COUNT_I32, False, [(0, 1, 64, P.FORM_MATRIX)])
    try:
        m = 74
        x, y, z = cubic_lattice(m, 6, np.int32, 4)
        r = np.full(m ** 3, 3, np.int32)
        assert strides(P.KIND_COUNT_I32, m ** 3)
        announce("count_i32 matrix form grid stride", m)
        assert P.count_i32(*dev(x, y, z, r)) == 3 * m * m * (m - 1)
        centre = int(np.flatnonzero((x == 40 * 6) & (y == 20 * 6) & (z == 50 * 6))[0])
        r[centre] = 9
        assert P.count_i32(*dev(x, y, z, r)) == 3 * m * m * (m - 1) + 26
    finally:
        P.pairs_set_shapes(P.KIND_COUNT_I32, False, None)


def test_count_f32_grid_stride_small_tiles(small_tiles):
    small_tiles(P.KIND_COUNT_F32)
    m = 74
    x, y, z = cubic_lattice(m, 0.25, np.float32, 3)   # dyadic: every step exact
    r = np.full(m ** 3, 0.125, np.float32)
    assert strides(P.KIND_COUNT_F32, m ** 3)
    announce("count_f32 grid stride, shape (1, 64)", m)
    assert P.count_f32(*dev(x, y, z, r)) == 3 * m * m * (m - 1)


def particles(n, seed):
    rng = np.random.default_rng(seed)
    return [a.copy() for a in rng.random((3, n), dtype=np.float32)]


def sampled_rows(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, 1, n // 2 - 1, n // 2, n - 2, n - 1],
                                     rng.integers(0, n, k)]))


def check_energy(arrays, n, E, tot, rows):
    want = oracle.energy_rows(*arrays, EPS2, rows=rows)
    got = E[rows]
    assert np.max(np.abs(got - want) / want) <= 1e-5
    # every pair is counted once in the total and twice over the objects
    assert abs(E.sum() - 2 * tot) <= 1e-6 * 2 * tot


def test_energy_f32_above_2p22():
    n = 2 ** 22 + 1
    a = particles(n, 11)
    assert strides(P.KIND_ENERGY_F32, n)
    announce("energy_f32", n)
    E, tot = P.energy_f32(*dev(*a), eps2=float(EPS2))
    check_energy(a, n, E.cpu().numpy(), tot, sampled_rows(n, 58, 12))


def test_energy_f32_grid_stride_small_tiles(small_tiles):
    small_tiles(P.KIND_ENERGY_F32)
    n = 400_003
    a = particles(n, 13)
    assert strides(P.KIND_ENERGY_F32, n)
    announce("energy_f32 grid stride, shape (1, 64)", n)
    E, tot = P.energy_f32(*dev(*a), eps2=float(EPS2))
    check_energy(a, n, E.cpu().numpy(), tot, sampled_rows(n, 60, 14))
    _, tot2 = P.energy_f32(*dev(*a), eps2=float(EPS2), per_particle=False)
    assert abs(tot2 - tot) <= 1e-6 * tot


def test_energy_f64_grid_stride_small_tiles(small_tiles):
    import torch
    small_tiles(P.KIND_ENERGY_F32)    # the double-precision call runs these shapes
    n = 400_003
    a = [v.astype(np.float64) for v in particles(n, 15)]
    assert strides(P.KIND_ENERGY_F64, n)
    announce("energy_f64 grid stride, shape (1, 64)", n)
    E = torch.empty(n, dtype=torch.float64, device="cuda")
    tot = torch.empty(1, dtype=torch.float64, device="cuda")
    P.pairs_energy_f64(*dev(*a), 1e-4, E, tot)
    E = E.cpu().numpy()
    rows = sampled_rows(n, 60, 16)
    want = oracle.energy_f64_rows(*a, 1e-4, rows=rows)
    assert np.max(np.abs(E[rows] - want) / want) <= 1e-12
    assert abs(E.sum() - 2 * float(tot)) <= 1e-12 * 2 * float(tot)


def test_force_f32_grid_stride_small_tiles(small_tiles):
    import torch
    small_tiles(P.KIND_ENERGY_F32)    # the force call runs these shapes
    n = 400_003
    a = particles(n, 17)
    assert strides(P.KIND_FORCE_F32, n)
    announce("force_f32 grid stride, shape (1, 64)", n)
    F = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    P.pairs_force_f32(*dev(*a), float(EPS2), *F)
    got = np.stack([f.cpu().numpy() for f in F], axis=1)
    rows = sampled_rows(n, 40, 18)
    want, S = oracle.force_rows(*a, EPS2, rows=rows)
    assert np.all(np.abs(got[rows] - want).max(axis=1) <= 1e-5 * S)
