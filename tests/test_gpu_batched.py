"""GPU parity of the batched path (unplanned calls and plans), the jitter step
and the graph-captured repeated steps, against the CPU oracle."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

EPS2 = np.float32(1e-4)
TOL_SET = 1e-6


def torch():
    import torch as t
    return t


def run_count_i32(x, y, z, r, off, planned):
    T = torch()
    tx = dev(x, y, z, r)
    counts = T.empty(len(off) - 1, dtype=T.int64, device="cuda")
    if planned:
        plan = P.Plan(P.KIND_COUNT_I32, off)
        plan.execute(tx, (counts,))
        T.cuda.synchronize()
        plan.close()
    else:
        (toff,) = dev(off)
        P.pairs_count_i32_batched(*tx, toff, counts)
    return counts.cpu().numpy().astype(np.uint64)


EDGE_SIZES = [0, 1, 2, 3, 0, 64, 65, 200, 1, 256, 257, 513, 1024, 1025, 4096, 4097, 5000, 8192,
              2, 63, 127, 129]


@pytest.mark.parametrize("planned", [False, True])
def test_batched_count_i32_edge_sizes(planned):
    sizes = np.array(EDGE_SIZES, np.int64)
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(int(off[-1]), 41, 64, 5, radius_lo=0)
    announce("batched count_i32 edge sizes", planned)
    got = run_count_i32(*s.arrays(), off, planned)
    want = oracle.count_i32_batched(*s.arrays(), off)
    np.testing.assert_array_equal(got, want)
    assert got[0] == got[1] == got[4] == got[8] == 0


@pytest.mark.parametrize("planned", [False, True])
def test_batched_count_i32_lognormal(planned):
    b = w.binned_sets(n_sets=3000, seed=17)
    announce("batched count_i32 lognormal 3000 sets", planned)
    got = run_count_i32(*b.objs.arrays(), b.offsets, planned)
    want = oracle.count_i32_batched(*b.objs.arrays(), b.offsets)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("planned", [False, True])
def test_batched_count_i32_full_domain(planned):
    """Sets of every form (packs of small sets, stepping row blocks) whose
    objects span the whole exact domain, some sets entirely inside the plain
    test's box: each wave takes the plain or the wide test per task."""
    lo, hi, rmax = -(2 ** 30), 2 ** 30 - 1, 2 ** 30
    sizes = np.array(EDGE_SIZES + [3, 5, 17, 40, 300, 2000], np.int64)
    off = w.offsets_from_sizes(sizes)
    n = int(off[-1])
    rng = np.random.default_rng(23)
    x, y, z = (rng.integers(lo, hi, n, endpoint=True).astype(np.int32) for _ in range(3))
    r = rng.integers(0, rmax, n, endpoint=True).astype(np.int32)
    # every third set stays dense inside the box (collisions among small values)
    dense = w.spheres_i32(n, 24, 64, 5, radius_lo=0)
    for k in range(0, len(sizes), 3):
        a, b = off[k], off[k + 1]
        x[a:b], y[a:b], z[a:b], r[a:b] = (v[a:b] for v in dense.arrays())
    # touching pairs across the span at the start of every set of two or more
    for k in range(1, len(sizes), 3):
        a = off[k]
        if sizes[k] >= 2:
            x[a], x[a + 1], y[a], y[a + 1], z[a], z[a + 1] = lo, hi, 0, 0, 0, 0
            r[a], r[a + 1] = rmax, rmax - 1
    announce("batched count_i32 full domain", planned)
    got = run_count_i32(x, y, z, r, off, planned)
    want = oracle.count_i32_batched(x, y, z, r, off)
    np.testing.assert_array_equal(got, want)


def test_batched_permuted_sets_permute_outputs():
    rng = np.random.default_rng(8)
    sizes = rng.integers(0, 700, 60).astype(np.int64)
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(int(off[-1]), 9, 40, 4, radius_lo=0)
    base = run_count_i32(*s.arrays(), off, True)
    perm = rng.permutation(len(sizes))
    parts = [[a[off[k]:off[k + 1]] for a in s.arrays()] for k in perm]
    cat = [np.concatenate([p[c] for p in parts]) for c in range(4)]
    got = run_count_i32(*cat, w.offsets_from_sizes(sizes[perm]), False)
    np.testing.assert_array_equal(got, base[perm])


def test_batched_equals_single_set_calls():
    sizes = np.array([5, 700, 4100, 66, 2], np.int64)
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(int(off[-1]), 10, 200, 20, radius_lo=0)
    got = run_count_i32(*s.arrays(), off, False)
    for k in range(len(sizes)):
        sl = slice(off[k], off[k + 1])
        assert got[k] == P.count_i32(*dev(*(a[sl] for a in s.arrays())))


def test_batched_count_f32():
    T = torch()
    b = w.moving_sets(n_sets=500, seed=21, size_hi=3000, radius=0.02)
    x, y, z, r = b.objs.arrays()
    counts = T.empty(b.n_sets, dtype=T.int64, device="cuda")
    (toff,) = dev(b.offsets)
    P.pairs_count_f32_batched(*dev(x, y, z, r), toff, counts)
    _, want = oracle.energy_count_f32_batched(x, y, z, r, b.offsets, EPS2)
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), want)


@pytest.mark.parametrize("with_count", [False, True])
@pytest.mark.parametrize("planned", [False, True])
def test_batched_energy(with_count, planned):
    T = torch()
    b = w.moving_sets(n_sets=700, seed=22, size_hi=5000, radius=0.02)
    x, y, z, r = b.objs.arrays()
    energy = T.empty(b.n_sets, dtype=T.float64, device="cuda")
    counts = T.empty(b.n_sets, dtype=T.int64, device="cuda") if with_count else None
    tx = dev(x, y, z, r)
    announce("batched energy", with_count, planned)
    if planned:
        plan = P.Plan(P.KIND_ENERGY_F32, b.offsets)
        plan.execute((tx[0], tx[1], tx[2], tx[3] if with_count else None), (energy, counts),
                     eps2=float(EPS2))
        T.cuda.synchronize()
        plan.close()
    else:
        (toff,) = dev(b.offsets)
        P.pairs_energy_f32_batched(tx[0], tx[1], tx[2], tx[3] if with_count else None, toff,
                                   float(EPS2), energy, counts)
    want_e, want_c = oracle.energy_count_f32_batched(x, y, z, r, b.offsets, EPS2)
    got_e = energy.cpu().numpy()
    nz = want_e > 0
    assert np.all(got_e[~nz] == 0)
    assert np.max(np.abs(got_e[nz] - want_e[nz]) / want_e[nz]) <= TOL_SET
    if with_count:
        np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), want_c)


def test_batched_validation():
    T = torch()
    sizes = np.array([3, 4, 5], np.int64)
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(12, 1, 100, 5)
    counts = T.empty(3, dtype=T.int64, device="cuda")
    bad = off.copy()
    bad[2] = 1  # not non-decreasing
    with pytest.raises(P.PairsError) as e:
        P.pairs_count_i32_batched(*dev(*s.arrays()), *dev(bad), counts, flags=P.FLAG_VALIDATE)
    assert e.value.status == -1
    # malformed offsets without validation: no fault, just some result
    P.pairs_count_i32_batched(*dev(*s.arrays()), *dev(bad), counts)
    T.cuda.synchronize()
    x = s.x.copy()
    x[0] = -(2 ** 30) - 1
    with pytest.raises(P.PairsError) as e:
        P.pairs_count_i32_batched(*dev(x, s.y, s.z, s.r), *dev(off), counts,
                                  flags=P.FLAG_VALIDATE)
    assert e.value.status == -2
    P.pairs_count_i32_batched(*dev(*s.arrays()), *dev(off), counts, flags=P.FLAG_VALIDATE)
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64),
                                  oracle.count_i32_batched(*s.arrays(), off))


def test_binned_sets_200k_full_size():
    b = w.binned_sets()
    announce("200 000 binned sets, full size (plan)")
    got = run_count_i32(*b.objs.arrays(), b.offsets, True)
    want = oracle.count_i32_batched(*b.objs.arrays(), b.offsets)
    np.testing.assert_array_equal(got, want)
    with open(os.path.join(os.path.dirname(__file__), "golden", "workload_values.json")) as f:
        g = json.load(f)["binned_sets_200k_counts"]
    assert int(got.sum()) == g["total"]
    assert hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == g["sha256_le_u64"]
    announce("200 000 binned sets, full size (unplanned)")
    got2 = run_count_i32(*b.objs.arrays(), b.offsets, False)
    np.testing.assert_array_equal(got2, want)


# ------------------------------------------------------------------ jitter --

def test_jitter_bit_exact():
    n = 100_003
    p = w.particles_f32(n, 5)
    tx = dev(*p.arrays())
    ox, oy, oz = p.arrays()
    for step in range(3):
        P.pairs_jitter_f32(*tx, seed=123456789012345, step=step, sigma=1e-3)
        ox, oy, oz = oracle.jitter_f32(ox, oy, oz, 123456789012345, step, 1e-3)
    for g, o in zip(tx, (ox, oy, oz)):
        np.testing.assert_array_equal(g.cpu().numpy().view(np.uint32), o.view(np.uint32))
    # a sub-range with its global index offset matches too
    sub = dev(*(a[:1000].copy() for a in p.arrays()))
    P.pairs_jitter_f32(*sub, seed=7, step=0, sigma=1e-3, first_index=50_000)
    sx, _, _ = oracle.jitter_f32(*(a[:1000] for a in p.arrays()), 7, 0, 1e-3, first_index=50_000)
    np.testing.assert_array_equal(sub[0].cpu().numpy().view(np.uint32), sx.view(np.uint32))


# ---------------------------------------------------------- repeated steps --

def oracle_steps(b, sets, steps, seed, sigma):
    """Oracle energy/count of the given sets after each listed step (positions
    jittered by the oracle itself from the initial ones)."""
    x, y, z, r = b.objs.arrays()
    out = {}
    last = max(steps)
    for s in sets:
        a, e = int(b.offsets[s]), int(b.offsets[s + 1])
        px, py, pz = x[a:e].copy(), y[a:e].copy(), z[a:e].copy()
        for k in range(last + 1):
            px, py, pz = oracle.jitter_f32(px, py, pz, seed, k, sigma, first_index=a)
            if k in steps:
                en = oracle.energy_total(px, py, pz, EPS2, threads=1)
                cn = oracle.count_f32(px, py, pz, r[a:e], threads=1)
                out[(s, k)] = (en, cn)
    return out


def check_steps(b, E, C, sets, steps, ref, n_sets):
    for s in sets:
        for k in steps:
            en, cn = ref[(s, k)]
            ge = float(E[k * n_sets + s])
            if en == 0:
                assert ge == 0
            else:
                assert abs(ge - en) <= TOL_SET * en, (s, k, ge, en)
            assert int(C[k * n_sets + s]) == cn, (s, k)


def test_graph_steps_small():
    T = torch()
    b = w.moving_sets(n_sets=400, seed=23, size_hi=2000)
    x, y, z, r = b.objs.arrays()
    tx = dev(x, y, z, r)
    steps = 6
    E = T.zeros(steps * b.n_sets, dtype=T.float64, device="cuda")
    C = T.zeros(steps * b.n_sets, dtype=T.int64, device="cuda")
    plan = P.Plan(P.KIND_ENERGY_F32, b.offsets)
    g = plan.capture_steps(tx[0], tx[1], tx[2], tx[3], seed=6, sigma=1e-3, first_step=0,
                           n_steps=steps, eps2=float(EPS2), energy=E, counts=C)
    announce("graph steps small")
    g.launch()
    T.cuda.synchronize()
    En, Cn = E.cpu().numpy(), C.cpu().numpy()
    sets = list(range(b.n_sets))
    ref = oracle_steps(b, sets, set(range(steps)), 6, 1e-3)
    check_steps(b, En, Cn, sets, range(steps), ref, b.n_sets)
    # positions after the steps equal the oracle's, bit for bit
    ox, oy, oz = x, y, z
    for k in range(steps):
        ox, oy, oz = oracle.jitter_f32(ox, oy, oz, 6, k, 1e-3)
    np.testing.assert_array_equal(tx[0].cpu().numpy().view(np.uint32), ox.view(np.uint32))
    # a second launch replays the same steps on the moved positions, and eager
    # work in between does not disturb it
    P.count_f32(tx[0][:100].contiguous(), tx[1][:100].contiguous(),
                tx[2][:100].contiguous(), tx[3][:100].contiguous())
    g.launch()
    T.cuda.synchronize()
    for k in range(steps):
        ox, oy, oz = oracle.jitter_f32(ox, oy, oz, 6, k, 1e-3)
    np.testing.assert_array_equal(tx[2].cpu().numpy().view(np.uint32), oz.view(np.uint32))
    want_e, want_c = oracle.energy_count_f32_batched(ox, oy, oz, r, b.offsets, EPS2)
    last = E.cpu().numpy()[(steps - 1) * b.n_sets:]
    nz = want_e > 0
    assert np.max(np.abs(last[nz] - want_e[nz]) / want_e[nz]) <= TOL_SET
    np.testing.assert_array_equal(C.cpu().numpy()[(steps - 1) * b.n_sets:].astype(np.uint64),
                                  want_c)
    g.close()
    plan.close()


def test_moving_sets_50k_full_graph_sampled():
    T = torch()
    b = w.moving_sets()
    x, y, z, r = b.objs.arrays()
    tx = dev(x, y, z, r)
    steps = 100
    E = T.zeros(steps * b.n_sets, dtype=T.float64, device="cuda")
    C = T.zeros(steps * b.n_sets, dtype=T.int64, device="cuda")
    plan = P.Plan(P.KIND_ENERGY_F32, b.offsets)
    g = plan.capture_steps(tx[0], tx[1], tx[2], tx[3], seed=6, sigma=1e-3, first_step=0,
                           n_steps=steps, eps2=float(EPS2), energy=E, counts=C)
    announce("50 000 moving sets, full graph, 100 steps")
    g.launch()
    T.cuda.synchronize()
    En, Cn = E.cpu().numpy(), C.cpu().numpy()
    sizes = np.diff(b.offsets)
    rng = np.random.default_rng(0)
    sets = sorted(set(rng.choice(b.n_sets, 24, replace=False).tolist() +
                      [int(np.argmax(sizes)), int(np.argmin(sizes)), 0, b.n_sets - 1]))
    check_steps(b, En, Cn, sets, [0, 1, 49, 99],
                oracle_steps(b, sets, {0, 1, 49, 99}, 6, 1e-3), b.n_sets)
    g.close()
    plan.close()


# ------------------------------------------------------- every task form --
#
# Forced batched shape tables: the broadcast sweep, the row-stepping form
# (row blocks and, in plans, packs of equal-size small sets) and a mix, on a
# batch with many repeated small sizes (multi-set packs), ragged sizes and
# dense collisions.

B, S = P.FORM_BROADCAST, P.FORM_STEPPING
FORM_TABLES = {
    "bcast-1x256": [(0, 1, 256, B)],
    "bcast-8x512": [(0, 8, 512, B)],
    "step-1x16": [(0, 1, 16, S)],
    "step-1x192": [(0, 1, 192, S)],
    "step-1x288": [(0, 1, 288, S)],
    "step-2x16": [(0, 2, 16, S)],
    "step-2x48": [(0, 2, 48, S)],
    "step-2x144": [(0, 2, 144, S)],
    "step-2x272": [(0, 2, 272, S)],
    "mixed": [(1000, 4, 1024, B), (100, 2, 144, S), (0, 1, 64, S)],
}


def form_batch(seed):
    rng = np.random.default_rng(seed)
    small = np.repeat(np.arange(0, 140), 3)                  # every small size, 3 times
    ragged = rng.integers(140, 1200, 25)
    sizes = np.concatenate([small, ragged, [2048, 1, 0, 2]]).astype(np.int64)
    rng.shuffle(sizes)
    return sizes, w.offsets_from_sizes(sizes)


@pytest.fixture
def forced_batched():
    kinds = []

    def set_(kind, table):
        kinds.append(kind)
        P.pairs_set_shapes(kind, True, table)
    yield set_
    for k in kinds:
        P.pairs_set_shapes(k, True, None)


@pytest.mark.parametrize("name", list(FORM_TABLES))
@pytest.mark.parametrize("planned", [False, True])
def test_batched_count_i32_every_form(forced_batched, name, planned):
    forced_batched(P.KIND_COUNT_I32, FORM_TABLES[name])
    sizes, off = form_batch(31)
    s = w.spheres_i32(int(off[-1]), 32, 48, 4, radius_lo=0)
    announce("batched count_i32 form", name, planned)
    got = run_count_i32(*s.arrays(), off, planned)
    want = oracle.count_i32_batched(*s.arrays(), off)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("name", ["bcast-1x256", "step-1x192", "step-2x48", "step-2x272",
                                  "mixed"])
@pytest.mark.parametrize("planned", [False, True])
def test_batched_energy_count_every_form(forced_batched, name, planned):
    T = torch()
    forced_batched(P.KIND_ENERGY_F32, FORM_TABLES[name])
    sizes, off = form_batch(33)
    n = int(off[-1])
    p = w.particles_f32(n, 34)
    x, y, z = p.arrays()
    x, y, z = x * 0.3, y * 0.3, z * 0.3                      # dense: many contacts
    r = np.full(n, 0.02, np.float32)
    tx = dev(x, y, z, r)
    energy = T.empty(len(sizes), dtype=T.float64, device="cuda")
    counts = T.empty(len(sizes), dtype=T.int64, device="cuda")
    announce("batched energy+count form", name, planned)
    if planned:
        plan = P.Plan(P.KIND_ENERGY_F32, off)
        plan.execute(tx, (energy, counts), eps2=float(EPS2))
        T.cuda.synchronize()
        plan.close()
    else:
        (toff,) = dev(off)
        P.pairs_energy_f32_batched(*tx, toff, float(EPS2), energy, counts)
    want_e, want_c = oracle.energy_count_f32_batched(x, y, z, r, off, EPS2)
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), want_c)
    got_e = energy.cpu().numpy()
    nz = want_e > 0
    assert np.all(got_e[~nz] == 0.0)
    rel = np.abs(got_e[nz] - want_e[nz]) / want_e[nz]
    assert rel.max() <= TOL_SET, rel.max()


@pytest.mark.parametrize("name", ["step-1x16", "step-1x288", "step-2x272", "mixed"])
def test_batched_count_f32_every_form(forced_batched, name):
    T = torch()
    forced_batched(P.KIND_COUNT_F32, FORM_TABLES[name])
    sizes, off = form_batch(35)
    n = int(off[-1])
    p = w.particles_f32(n, 36)
    x, y, z = (a * np.float32(0.25) for a in p.arrays())
    r = np.full(n, 0.02, np.float32)
    counts = T.empty(len(sizes), dtype=T.int64, device="cuda")
    for planned in (False, True):
        if planned:
            plan = P.Plan(P.KIND_COUNT_F32, off)
            plan.execute(dev(x, y, z, r), (counts,))
            T.cuda.synchronize()
            plan.close()
        else:
            (toff,) = dev(off)
            P.pairs_count_f32_batched(*dev(x, y, z, r), toff, counts)
        _, want = oracle.energy_count_f32_batched(x, y, z, r, off, EPS2)
        np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), want)


def test_energy_per_set_without_count_every_form(forced_batched):
    T = torch()
    for name in ("step-1x288", "step-2x272"):
        forced_batched(P.KIND_ENERGY_F32, FORM_TABLES[name])
        sizes, off = form_batch(37)
        n = int(off[-1])
        x, y, z = w.particles_f32(n, 38).arrays()
        energy = T.empty(len(sizes), dtype=T.float64, device="cuda")
        plan = P.Plan(P.KIND_ENERGY_F32, off)
        tx = dev(x, y, z)
        plan.execute((tx[0], tx[1], tx[2], None), (energy, None), eps2=float(EPS2))
        T.cuda.synchronize()
        plan.close()
        want_e, _ = oracle.energy_count_f32_batched(x, y, z, np.zeros(n, np.float32), off, EPS2)
        got = energy.cpu().numpy()
        nz = want_e > 0
        assert np.all(got[~nz] == 0.0)
        assert (np.abs(got[nz] - want_e[nz]) / want_e[nz]).max() <= TOL_SET
