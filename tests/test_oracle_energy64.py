"""Pins of the double-input energy oracle (oracle_energy_f64_*): the
potential of the double-precision variant.

Checked against the float32-input oracle on float32-representable inputs
(both promote to the same doubles, so the results must be identical), against
sums of 1/sqrt(d^2 + eps2) evaluated with Python's decimal module at 40
digits, and against the two-particle closed form.  CPU only."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
import workloads as w


def test_equals_the_float32_oracle_on_float32_inputs():
    p = w.particles_f32(500, 3)
    x, y, z = p.arrays()
    eps2 = np.float32(1e-4)
    t32 = oracle.energy_total(x, y, z, eps2)
    t64 = oracle.energy_f64_total(x.astype(np.float64), y.astype(np.float64),
                                  z.astype(np.float64), float(eps2))
    assert t64 == t32
    r = np.array([0, 17, 499])
    np.testing.assert_array_equal(
        oracle.energy_f64_rows(x.astype(np.float64), y.astype(np.float64), z.astype(np.float64),
                               float(eps2), rows=r),
        oracle.energy_rows(x, y, z, eps2, rows=r))


def decimal_energy(pts, eps2):
    getcontext().prec = 40
    e = Decimal(eps2)
    tot = Decimal(0)
    rows = [Decimal(0)] * len(pts)
    P = [[Decimal(float(c)) for c in p] for p in pts]
    for i in range(len(P)):
        for j in range(i + 1, len(P)):
            d2 = sum((P[i][a] - P[j][a]) ** 2 for a in range(3))
            v = 1 / (d2 + e).sqrt()
            tot += v
            rows[i] += v
            rows[j] += v
    return float(tot), [float(r) for r in rows]


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_a_40_digit_evaluation(seed):
    rng = np.random.default_rng(seed)
    pts = rng.normal(0, 10, (40, 3))  # full-precision doubles, not float32 values
    eps2 = 1e-3
    tot, rows = decimal_energy(pts, eps2)
    x, y, z = (np.ascontiguousarray(pts[:, a]) for a in range(3))
    assert oracle.energy_f64_total(x, y, z, eps2) == pytest.approx(tot, rel=1e-15)
    np.testing.assert_allclose(oracle.energy_f64_rows(x, y, z, eps2), rows, rtol=1e-15)


def test_two_particles():
    x = np.array([0.0, 0.1], np.float64)
    z = np.zeros(2)
    e = oracle.energy_f64_total(x, z, z, 0.01)
    assert e == pytest.approx(1 / np.sqrt(0.01 + 0.01), rel=1e-15)
