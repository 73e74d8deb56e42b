"""Pins of the force oracle (oracle_force_rows): the forces of the softened
potential e_ij = 1/sqrt(|p_i - p_j|^2 + eps2), f_ij = (p_i - p_j)/(d^2 + eps2)^1.5.

Checked against a closed form (two particles), the negative gradient of the
potential by central differences (written here in numpy over float64
positions, so a wrong sign, exponent or factor fails), Newton's third law
(the forces of a set sum to zero), symmetric arrangements, the triangle
inequality against the norm sum S, and translation invariance.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as w

EPS2 = np.float32(1e-4)


def f32(*a):
    return [np.asarray(v, dtype=np.float32) for v in a]


def test_two_particles_closed_form():
    for d, eps2 in [(1.0, EPS2), (0.25, EPS2), (3.0, np.float32(0.5))]:
        x, y, z = f32([0.0, d], [0.0, 0.0], [0.0, 0.0])
        F, S = oracle.force_rows(x, y, z, eps2)
        e2 = float(np.float32(eps2))
        want = d / (d * d + e2) ** 1.5
        assert F[0, 0] == pytest.approx(-want, rel=1e-14)
        assert F[1, 0] == pytest.approx(want, rel=1e-14)
        assert F[0, 1] == 0.0 and F[0, 2] == 0.0
        assert S[0] == pytest.approx(want, rel=1e-14)


def potential(p, eps2):
    d = p[:, None, :] - p[None, :, :]
    r2 = (d * d).sum(-1) + eps2
    iu = np.triu_indices(p.shape[0], 1)
    return float((1.0 / np.sqrt(r2[iu])).sum())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_minus_gradient_of_the_potential(seed):
    p = w.particles_f32(40, seed)
    x, y, z = p.arrays()
    F, _ = oracle.force_rows(x, y, z, EPS2)
    pos = np.stack([x, y, z], 1).astype(np.float64)
    eps2 = float(EPS2)
    h = 1e-5
    for i in (0, 7, 39):
        for a in range(3):
            q1, q2 = pos.copy(), pos.copy()
            q1[i, a] += h
            q2[i, a] -= h
            g = (potential(q1, eps2) - potential(q2, eps2)) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=2e-6, abs=1e-6 * abs(F[i]).sum())


@pytest.mark.parametrize("n", [2, 3, 17, 200])
def test_newtons_third_law(n):
    p = w.particles_f32(n, 10 + n)
    F, S = oracle.force_rows(*p.arrays(), EPS2)
    assert np.all(np.abs(F.sum(axis=0)) <= 1e-12 * S.sum())


def test_symmetric_arrangements():
    # centre of a cube of eight particles, and the middle of three in a row
    c = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], np.float32) * 2 - 1
    pts = np.vstack([np.zeros((1, 3), np.float32), c])
    F, S = oracle.force_rows(*[np.ascontiguousarray(pts[:, a]) for a in range(3)], EPS2)
    assert np.all(np.abs(F[0]) <= 1e-15 * S[0]) and S[0] > 0
    x, y, z = f32([-1.0, 0.0, 1.0], [0, 0, 0], [0, 0, 0])
    F, S = oracle.force_rows(x, y, z, EPS2)
    assert F[1, 0] == 0.0 and S[1] > 0
    assert F[0, 0] < 0 < F[2, 0]  # repulsive: the outer ones are pushed out


def test_triangle_inequality_and_rows():
    p = w.particles_f32(300, 5)
    F, S = oracle.force_rows(*p.arrays(), EPS2)
    assert np.all(np.linalg.norm(F, axis=1) <= S * (1 + 1e-12))
    rows = np.array([299, 0, 150], np.int64)
    Fr, Sr = oracle.force_rows(*p.arrays(), EPS2, rows=rows)
    np.testing.assert_array_equal(Fr, F[rows])
    np.testing.assert_array_equal(Sr, S[rows])


def test_translation_invariance():
    p = w.particles_f32(100, 6)
    # coordinates on a 2^-10 grid, so that the shifted ones stay exact
    x, y, z = (np.round(v * 1024) / np.float32(1024) for v in p.arrays())
    F, _ = oracle.force_rows(x, y, z, EPS2)
    F2, _ = oracle.force_rows(x + np.float32(4), y - np.float32(2), z + np.float32(8), EPS2)
    np.testing.assert_allclose(F2, F, rtol=0, atol=1e-9 * np.abs(F).max())
