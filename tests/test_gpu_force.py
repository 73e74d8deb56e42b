"""Forces of the softened potential on the GPU (pairs_force_f32) against the
CPU oracle (oracle_force_rows): every component within 1e-5 of the object's
norm sum S_i = sum_j |f_ij|, the scale that cancellation in F_i is measured
against.  The kernel evaluates each pair once in float32 (error per term a
few units in the last place, about 1e-6) and folds float32 partials of 16
terms into double sums (at most about 16 u of S), well inside 1e-5."""
import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

EPS2 = np.float32(1e-4)
TOL = 1e-5


def gpu_forces(arrays, eps2=EPS2):
    import torch
    x, y, z = dev(*arrays)
    n = int(arrays[0].shape[0])
    F = [torch.full((n,), 7.0, dtype=torch.float64, device="cuda") for _ in range(3)]
    P.pairs_force_f32(x, y, z, float(eps2), *F)
    torch.cuda.synchronize()
    return np.stack([f.cpu().numpy() for f in F], axis=1)


def check(got, want, S):
    err = np.abs(got - want).max(axis=1)
    assert np.all(err <= TOL * S + 1e-300), (err / np.maximum(S, 1e-300)).max()


@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000,
                               4095, 4097, 20000])
def test_forces_match_oracle(n):
    p = w.particles_f32(n, 300 + n)
    announce("force", n)
    got = gpu_forces(p.arrays())
    if n < 2:
        assert np.all(got == 0.0)
        return
    F, S = oracle.force_rows(*p.arrays(), EPS2)
    check(got, F, S)


def test_newtons_third_law_on_the_gpu():
    p = w.particles_f32(5000, 7)
    announce("force third law")
    got = gpu_forces(p.arrays())
    F, S = oracle.force_rows(*p.arrays(), EPS2)
    check(got, F, S)
    # the forces of an isolated set sum to zero: the residual is bounded by
    # the per-object tolerance summed over the set
    assert np.all(np.abs(got.sum(axis=0)) <= TOL * S.sum())


def test_coincident_and_clustered_particles():
    rng = np.random.default_rng(3)
    base = rng.random((300, 3), dtype=np.float32)
    pts = np.vstack([base, base[:50], np.full((20, 3), 0.5, np.float32)])
    arrays = [np.ascontiguousarray(pts[:, a]) for a in range(3)]
    announce("force coincident")
    got = gpu_forces(arrays)
    F, S = oracle.force_rows(*arrays, EPS2)
    check(got, F, S)


@pytest.mark.parametrize("eps2", [np.float32(1e-8), np.float32(0.25)])
def test_softening_values(eps2):
    p = w.particles_f32(3000, 11)
    announce("force eps2", float(eps2))
    got = gpu_forces(p.arrays(), eps2)
    F, S = oracle.force_rows(*p.arrays(), eps2)
    check(got, F, S)


def test_particles_2p18_sampled_rows():
    # N = 2^18 particles of the energy workload; 257 rows checked one by one
    p = w.particles_unit_cube()
    announce("force 2^18")
    got = gpu_forces(p.arrays())
    rows = np.unique(np.r_[0, 1, 2 ** 17, p.n - 1,
                          np.random.default_rng(0).integers(0, p.n, 253)])
    F, S = oracle.force_rows(*p.arrays(), EPS2, rows=rows)
    check(got[rows], F, S)


def test_force_calls_captured_in_a_graph():
    import torch
    p = w.particles_f32(3000, 21)
    q = w.particles_f32(1000, 22)
    F, S = oracle.force_rows(*p.arrays(), EPS2)
    Fq, Sq = oracle.force_rows(*q.arrays(), EPS2)
    t = dev(*p.arrays())
    tq = dev(*q.arrays())
    out = [torch.empty(3000, dtype=torch.float64, device="cuda") for _ in range(3)]
    outq = [torch.empty(1000, dtype=torch.float64, device="cuda") for _ in range(3)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.pairs_force_f32(*t, float(EPS2), *out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    announce("force graph capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(4):
            P.pairs_force_f32(*t, float(EPS2), *out)
    for rep in range(3):
        for o in out:
            o.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        check(np.stack([o.cpu().numpy() for o in out], 1), F, S)
        P.pairs_force_f32(*tq, float(EPS2), *outq)
        torch.cuda.synchronize()
        check(np.stack([o.cpu().numpy() for o in outq], 1), Fq, Sq)
