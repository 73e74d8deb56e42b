"""Batched forces (pairs_force_f32_batched) and batched double-precision
energies (pairs_energy_f64_batched) against the CPU oracle run set by set:
every force component within 1e-5 of the object's norm sum S_i, set totals
and per-object sums within 1e-12; empty and one-object sets give zeros;
objects never feel objects of other sets."""
import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

EPS2 = np.float32(1e-4)
SIZES = [0, 1, 2, 3, 5, 64, 65, 127, 128, 129, 200, 0, 1, 257, 1024, 1025, 1500, 4097, 2, 33]


def T():
    import torch
    return torch


def batch_f32(sizes, seed):
    off = w.offsets_from_sizes(np.array(sizes, np.int64))
    rng = np.random.default_rng(seed)
    n = int(off[-1])
    return off, [a.copy() for a in rng.random((3, n), dtype=np.float32)]


def gpu_forces(off, a, flags=0):
    torch = T()
    n = int(off[-1])
    F = [torch.full((n,), 7.0, dtype=torch.float64, device="cuda") for _ in range(3)]
    P.pairs_force_f32_batched(*dev(*a), *dev(off), float(EPS2), *F, flags=flags)
    torch.cuda.synchronize()
    return np.stack([f.cpu().numpy() for f in F], axis=1)


@pytest.mark.parametrize("seed", [1, 2])
def test_forces_batched_match_oracle(seed):
    off, a = batch_f32(SIZES, 90 + seed)
    announce("batched forces", seed)
    got = gpu_forces(off, a)
    for s in range(len(off) - 1):
        lo, hi = int(off[s]), int(off[s + 1])
        if hi - lo < 2:
            assert np.all(got[lo:hi] == 0.0)
            continue
        F, S = oracle.force_rows(*[v[lo:hi] for v in a], EPS2)
        assert np.all(np.abs(got[lo:hi] - F).max(axis=1) <= 1e-5 * S), s
        # an isolated set: its forces sum to zero
        assert np.all(np.abs(got[lo:hi].sum(axis=0)) <= 1e-5 * S.sum())


def test_forces_batched_lognormal_and_deterministic():
    b = w.moving_sets(n_sets=800, seed=44, size_hi=2000)
    a = list(b.objs.arrays()[:3])
    announce("batched forces, 800 lognormal sets")
    got = gpu_forces(b.offsets, a)
    rng = np.random.default_rng(3)
    for s in rng.choice(800, 40, replace=False):
        lo, hi = int(b.offsets[s]), int(b.offsets[s + 1])
        if hi - lo < 2:
            continue
        F, S = oracle.force_rows(*[v[lo:hi] for v in a], EPS2)
        assert np.all(np.abs(got[lo:hi] - F).max(axis=1) <= 1e-5 * S), s
    d0 = gpu_forces(b.offsets, a, P.FLAG_DETERMINISTIC)
    d1 = gpu_forces(b.offsets, a, P.FLAG_DETERMINISTIC)
    np.testing.assert_array_equal(d0.view(np.uint64), d1.view(np.uint64))
    assert np.max(np.abs(d0 - got)) <= 1e-9 * np.max(np.abs(got))


def energy64(off, a, per_object, flags=0):
    torch = T()
    n, m = int(off[-1]), len(off) - 1
    Es = torch.full((m,), 3.0, dtype=torch.float64, device="cuda")
    E = torch.full((n,), 5.0, dtype=torch.float64, device="cuda") if per_object else None
    P.pairs_energy_f64_batched(*dev(*a), *dev(off), 1e-4, Es, E, flags=flags)
    torch.cuda.synchronize()
    return Es.cpu().numpy(), (E.cpu().numpy() if per_object else None)


@pytest.mark.parametrize("per_object", [True, False])
def test_energy_f64_batched_match_oracle(per_object):
    off, a32 = batch_f32(SIZES, 7)
    a = [v.astype(np.float64) for v in a32]
    announce("batched energy_f64", per_object)
    Es, E = energy64(off, a, per_object)
    for s in range(len(off) - 1):
        lo, hi = int(off[s]), int(off[s + 1])
        if hi - lo < 2:
            assert Es[s] == 0.0
            if per_object:
                assert np.all(E[lo:hi] == 0.0)
            continue
        sub = [v[lo:hi] for v in a]
        want = oracle.energy_f64_total(*sub, 1e-4)
        assert abs(Es[s] - want) <= 1e-12 * want, s
        if per_object:
            rows = oracle.energy_f64_rows(*sub, 1e-4)
            assert np.max(np.abs(E[lo:hi] - rows) / rows) <= 1e-12, s
    d0, e0 = energy64(off, a, True, P.FLAG_DETERMINISTIC)
    d1, e1 = energy64(off, a, True, P.FLAG_DETERMINISTIC)
    np.testing.assert_array_equal(d0.view(np.uint64), d1.view(np.uint64))
    np.testing.assert_array_equal(e0.view(np.uint64), e1.view(np.uint64))
    nz = d0 > 0
    assert np.max(np.abs(d0[nz] - Es[nz]) / d0[nz]) <= 1e-12


def test_batched_forces_in_a_graph():
    """Captured once, replayed three times with eager work in between; each
    replay equals an eager call bit for bit under the deterministic flag."""
    torch = T()
    off, a = batch_f32(SIZES, 12)
    n = int(off[-1])
    ta, toff = dev(*a), dev(off)[0]
    F = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    ws = torch.empty(P.pairs_batched_workspace_size(len(SIZES), n), dtype=torch.uint8,
                     device="cuda")
    want = gpu_forces(off, a, P.FLAG_DETERMINISTIC)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.pairs_force_f32_batched(*ta, toff, float(EPS2), *F, ws=ws,
                                  flags=P.FLAG_DETERMINISTIC)
    announce("batched forces graph replays")
    for _ in range(3):
        for f in F:
            f.fill_(9.0)
        g.replay()
        torch.cuda.synchronize()
        got = np.stack([f.cpu().numpy() for f in F], axis=1)
        np.testing.assert_array_equal(got.view(np.uint64), want.view(np.uint64))
        P.count_f32(*[v[:50].contiguous() for v in ta], ta[0][:50].contiguous())


def test_batched_x_validation():
    torch = T()
    off, a = batch_f32([3, 4], 1)
    F = [torch.empty(7, dtype=torch.float64, device="cuda") for _ in range(3)]
    bad = off.copy()
    bad[1] = 9
    with pytest.raises(P.PairsError):
        P.pairs_force_f32_batched(*dev(*a), *dev(bad), float(EPS2), *F,
                                  flags=P.FLAG_VALIDATE)
    x = a[0].copy()
    x[2] = np.inf
    with pytest.raises(P.PairsError) as e:
        P.pairs_force_f32_batched(*dev(x, a[1], a[2]), *dev(off), float(EPS2), *F,
                                  flags=P.FLAG_VALIDATE)
    assert e.value.status == -2
    with pytest.raises(P.PairsError):
        P.pairs_force_f32_batched(*dev(*a), *dev(off), 0.0, *F)
    torch.cuda.synchronize()
