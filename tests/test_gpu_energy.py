"""GPU softened-potential sums against the FP64 oracle, within the stated
tolerances: relative error of the total <= 1e-6, of each per-particle sum <= 1e-5."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

EPS2 = np.float32(1e-4)
TOL_TOTAL = 1e-6
TOL_PARTICLE = 1e-5

SIZES = [2, 3, 4, 5, 63, 64, 65, 127, 129, 255, 257, 511, 512, 513, 1025, 4095, 4096, 8193,
         20000, 65537]


@pytest.mark.parametrize("n", SIZES)
def test_energy_matches_oracle(n):
    p = w.particles_f32(n, 2000 + n)
    announce("energy_f32", n)
    E, tot = P.energy_f32(*dev(*p.arrays()), eps2=float(EPS2))
    want_tot = oracle.energy_total(*p.arrays(), EPS2)
    assert abs(tot - want_tot) <= TOL_TOTAL * want_tot
    want_E = oracle.energy_rows(*p.arrays(), EPS2)
    got_E = E.cpu().numpy()
    assert np.max(np.abs(got_E - want_E) / want_E) <= TOL_PARTICLE
    # the total-only path
    _, tot2 = P.energy_f32(*dev(*p.arrays()), eps2=float(EPS2), per_particle=False)
    assert abs(tot2 - want_tot) <= TOL_TOTAL * want_tot


@pytest.mark.parametrize("K,U", [(1, 64), (2, 128), (4, 256), (8, 1024)])
def test_energy_every_shape(K, U):
    P.pairs_set_shapes(P.KIND_ENERGY_F32, False, [(0, K, U)])
    try:
        for n in (2, 64 * K - 1, 64 * K + 1, 2 * 64 * K + 5, 3001):
            p = w.particles_f32(n, 100 + n)
            E, tot = P.energy_f32(*dev(*p.arrays()), eps2=float(EPS2))
            want_tot = oracle.energy_total(*p.arrays(), EPS2)
            assert abs(tot - want_tot) <= TOL_TOTAL * want_tot, (K, U, n)
            want_E = oracle.energy_rows(*p.arrays(), EPS2)
            assert np.max(np.abs(E.cpu().numpy() - want_E) / want_E) <= TOL_PARTICLE, (K, U, n)
    finally:
        P.pairs_set_shapes(P.KIND_ENERGY_F32, False, None)


@pytest.mark.parametrize("K,U", [(1, 64), (1, 2048), (2, 256), (8, 1024)])
def test_energy_total_only_every_shape(K, U):
    """The total-only table (mode SHAPES_TOTAL_ONLY) drives calls without
    per-object output, and only those."""
    P.pairs_set_shapes(P.KIND_ENERGY_F32, P.SHAPES_TOTAL_ONLY, [(0, K, U)])
    try:
        assert P.pairs_get_shapes(P.KIND_ENERGY_F32, P.SHAPES_TOTAL_ONLY) == \
            [(0, K, U, P.FORM_BROADCAST)]
        for n in (2, 64 * K - 1, 64 * K + 1, 2 * 64 * K + 5, 3001, 20000):
            p = w.particles_f32(n, 300 + n)
            announce("energy_f32 total only", K, U, n)
            _, tot = P.energy_f32(*dev(*p.arrays()), eps2=float(EPS2), per_particle=False)
            want_tot = oracle.energy_total(*p.arrays(), EPS2)
            assert abs(tot - want_tot) <= TOL_TOTAL * want_tot, (K, U, n)
            _, tot_r = P.energy_f32(*dev(*p.arrays()), eps2=float(EPS2), per_particle=False,
                                    deterministic=True)
            assert abs(tot_r - want_tot) <= TOL_TOTAL * want_tot, (K, U, n)
    finally:
        P.pairs_set_shapes(P.KIND_ENERGY_F32, P.SHAPES_TOTAL_ONLY, None)


@pytest.mark.parametrize("n", [0, 1])
def test_energy_no_pairs(n):
    p = w.particles_f32(n, 1)
    E, tot = P.energy_f32(*dev(*p.arrays()))
    assert tot == 0.0
    assert E.shape[0] == n and (n == 0 or float(E[0]) == 0.0)


def test_energy_coincident_closed_form():
    n = 3000
    x = np.full(n, 0.25, np.float32)
    E, tot = P.energy_f32(*dev(x, x, x), eps2=float(EPS2))
    inv = 1.0 / math.sqrt(float(EPS2))
    assert tot == pytest.approx(n * (n - 1) / 2 * inv, rel=TOL_TOTAL)
    np.testing.assert_allclose(E.cpu().numpy(), (n - 1) * inv, rtol=TOL_PARTICLE)


def test_energy_particles_2p18_full_size():
    with open(os.path.join(os.path.dirname(__file__), "golden", "workload_values.json")) as f:
        g = json.load(f)
    p = w.particles_unit_cube()
    announce("energy_f32 2^18 particles")
    E, tot = P.energy_f32(*dev(*p.arrays()), eps2=float(EPS2))
    got_E = E.cpu().numpy()
    rows = np.random.default_rng(4).choice(p.n, 384, replace=False)
    rows = np.concatenate([rows, [0, 1, p.n // 2 - 1, p.n // 2, p.n - 1]])
    want = oracle.energy_rows(*p.arrays(), EPS2, rows=rows)
    assert np.max(np.abs(got_E[rows] - want) / want) <= TOL_PARTICLE
    # the per-particle sums add to twice the total
    assert math.fsum(got_E.tolist()) == pytest.approx(2 * tot, rel=1e-9)
    if "particles_2p18_energy_total" in g:
        want_tot = g["particles_2p18_energy_total"]
        assert abs(tot - want_tot) <= TOL_TOTAL * want_tot
