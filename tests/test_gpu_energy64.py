"""The double-precision potential on the GPU (pairs_energy_f64) against the
CPU oracle (oracle_energy_f64_*), relative error at most 1e-12 for totals and
per particle.  The kernel's per-term error is a few units in the last place
after the Newton step, and its double sums of at most a few hundred thousand
positive terms add at most n u, far below 1e-12 for the sizes here."""
import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

TOL = 1e-12


def points(n, seed):
    rng = np.random.default_rng(seed)
    return [np.ascontiguousarray(v) for v in rng.normal(0.0, 3.0, (3, n))]


def gpu_energy(arrays, eps2, per_object=True):
    import torch
    x, y, z = dev(*arrays)
    n = int(arrays[0].shape[0])
    E = torch.full((n,), 7.0, dtype=torch.float64, device="cuda") if per_object else None
    tot = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    P.pairs_energy_f64(x, y, z, eps2, E, tot)
    torch.cuda.synchronize()
    return (None if E is None else E.cpu().numpy()), float(tot.item())


@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 4097, 30000])
def test_energy64_matches_oracle(n):
    a = points(n, 500 + n)
    announce("energy64", n)
    E, tot = gpu_energy(a, 1e-4)
    if n < 2:
        assert tot == 0.0 and np.all(E == 0.0)
        return
    want = oracle.energy_f64_total(*a, 1e-4)
    assert abs(tot - want) <= TOL * want
    rows = np.unique(np.r_[0, n - 1, np.random.default_rng(n).integers(0, n, 64)])
    wr = oracle.energy_f64_rows(*a, 1e-4, rows=rows)
    assert np.all(np.abs(E[rows] - wr) <= TOL * wr)
    _, tot_only = gpu_energy(a, 1e-4, per_object=False)
    assert abs(tot_only - want) <= TOL * want


def test_energy64_coincident_points_and_softening():
    base = points(400, 7)
    a = [np.concatenate([v, v[:100], np.zeros(30)]) for v in base]
    for eps2 in (1e-12, 0.5):
        announce("energy64 coincident", eps2)
        E, tot = gpu_energy(a, eps2)
        want = oracle.energy_f64_total(*a, eps2)
        assert abs(tot - want) <= TOL * want
        wr = oracle.energy_f64_rows(*a, eps2)
        assert np.all(np.abs(E - wr) <= TOL * wr)


def test_energy64_agrees_with_float32_path_on_float32_inputs():
    # on float32 values the double kernel and the float32 kernel compute the
    # same potential; the float32 one within its own 1e-6
    p = w.particles_f32(5000, 9)
    a32 = p.arrays()
    a64 = [v.astype(np.float64) for v in a32]
    announce("energy64 vs energy32")
    _, t64 = gpu_energy(a64, float(np.float32(1e-4)))
    want = oracle.energy_total(*a32, np.float32(1e-4))
    assert abs(t64 - want) <= TOL * want
