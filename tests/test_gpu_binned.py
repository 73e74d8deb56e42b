"""The binned collision count (pairs_count_i32_binned) against the oracle's
plain pairwise count: bit-exact over densities from one object per cell to
one cell holding everything, coordinates on cell boundaries and at the domain
edges, radii up to half the cell, and the 2^20-sphere set at full size."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu


def binned(arrays, cell, flags=0):
    import torch
    t = dev(*arrays)
    out = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    P.pairs_count_i32_binned(*t, cell, out, flags=flags)
    torch.cuda.synchronize()
    return int(out.item())


def spheres(n, seed, lo, hi, rmax):
    rng = np.random.default_rng(seed)
    xyz = rng.integers(lo, hi, (n, 3), dtype=np.int32)
    r = rng.integers(0, rmax, n, dtype=np.int32, endpoint=True)
    return [np.ascontiguousarray(xyz[:, k]) for k in range(3)] + [r]


@pytest.mark.parametrize("n,span,cell", [(0, 100, 32), (1, 100, 32), (2, 64, 32),
                                          (100, 1000, 64), (1000, 2000, 64),
                                          (5000, 4096, 256), (20000, 1 << 20, 1 << 12),
                                          (20000, 4096, 4096), (3000, 200, 32)])
def test_binned_matches_oracle(n, span, cell):
    a = spheres(n, n + cell, -span, span, cell // 2)
    announce("binned", n, span, cell)
    assert binned(a, cell) == oracle.count_i32(*a)


# cells of 32 give the widest keys (21 bits per axis, 63 in all), cells of
# 2^15 the 33-bit keys of the 2^20 set, cells of 2^16 keys of 30 bits and
# cells of 2^25 keys of 6 bits
@pytest.mark.parametrize("cell", [32, 64, 1 << 15, 1 << 16, 1 << 25])
def test_cell_boundaries_and_domain_edges(cell):
    # objects exactly on cell faces and at both ends of the domain, touching
    # across faces with radii of exactly half a cell
    B = 1 << 24
    base = np.array([-B, -B + cell - 1, -B + cell, -1, 0, cell - 1, cell, cell + 1, B - cell,
                     B - 1, B], np.int64)
    base = np.clip(base, -B, B)
    g = np.stack(np.meshgrid(base, base[::3], base[::5], indexing="ij"), -1).reshape(-1, 3)
    x, y, z = (np.ascontiguousarray(g[:, k].astype(np.int32)) for k in range(3))
    r = np.full(x.shape[0], cell // 2, np.int32)
    announce("binned boundaries", cell)
    assert binned([x, y, z, r], cell) == oracle.count_i32(x, y, z, r)


@pytest.mark.parametrize("cell", [32, 1 << 16, 1 << 25])
def test_corner_clusters_over_the_whole_domain(cell):
    # a third of the objects spread over the whole domain and a third in a
    # block of 6 x 6 x 6 cells at each corner, where the cell keys take
    # their lowest and highest values
    B = 1 << 24
    rng = np.random.default_rng(cell)
    k = 6000
    side = min(6 * cell, 2 * B)
    spread = rng.integers(-B, B, (k, 3), endpoint=True)
    low = rng.integers(-B, -B + side, (k, 3), endpoint=True)
    high = rng.integers(B - side, B, (k, 3), endpoint=True)
    xyz = np.vstack([spread, low, high]).astype(np.int32)
    r = rng.integers(0, cell // 2, xyz.shape[0], dtype=np.int32, endpoint=True)
    a = [np.ascontiguousarray(xyz[:, j]) for j in range(3)] + [r]
    announce("binned corner clusters", cell)
    want = oracle.count_i32(*a)
    assert want > 1000
    assert binned(a, cell) == want


def test_workspace_reused_by_calls_in_a_row():
    # one workspace for several calls: every call clears what it needs at the
    # start (count, sizes, table tags and claims, big-cell count), so what an
    # earlier call left there must not change a later count; the later calls
    # are smaller, with other cell sizes, and one has big cells
    import torch
    cases = [(20000, 1 << 16, 1 << 12, 31), (3000, 60, 32, 32), (5000, 4096, 256, 33),
             (20000, 1 << 16, 1 << 12, 31)]
    ws = torch.empty(P.pairs_binned_workspace_size(20000), dtype=torch.uint8, device="cuda")
    ws.fill_(0xA5)
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    for n, span, cell, seed in cases:
        a = spheres(n, seed, -span, span, cell // 2)
        announce("binned reuse", n, span, cell)
        P.pairs_count_i32_binned(*dev(*a), cell, out, ws)
        torch.cuda.synchronize()
        assert int(out.item()) == oracle.count_i32(*a)


def test_one_dense_cell_and_clusters():
    rng = np.random.default_rng(4)
    c1 = rng.integers(0, 50, (3000, 3))           # one crowded cell
    c2 = rng.integers(1000, 1400, (4000, 3))      # a block of busy cells
    c3 = rng.integers(-60000, 60000, (5000, 3))   # sparse background
    xyz = np.vstack([c1, c2, c3]).astype(np.int32)
    r = rng.integers(0, 32, xyz.shape[0], dtype=np.int32, endpoint=True)
    a = [np.ascontiguousarray(xyz[:, k]) for k in range(3)] + [r]
    announce("binned clusters")
    assert binned(a, 64) == oracle.count_i32(*a)


def test_validation():
    a = spheres(100, 1, -1000, 1000, 40)  # radii above cell/2 = 32
    announce("binned validation")
    with pytest.raises(P.PairsError) as e:
        binned(a, 64, flags=P.FLAG_VALIDATE)
    assert e.value.status == -2
    b = spheres(100, 2, -1000, 1000, 32)
    assert binned(b, 64, flags=P.FLAG_VALIDATE) == oracle.count_i32(*b)


def test_spheres_2p20_full_size(golden_dir):
    # N = 2^20 spheres with radii up to 2^14: cells of 2^15
    with open(os.path.join(golden_dir, "workload_values.json")) as f:
        want = json.load(f)["spheres_2p20_count"]
    s = w.spheres_2p24(2 ** 20)
    announce("binned 2^20 spheres")
    assert binned(s.arrays(), 1 << 15) == want


def test_one_cell_above_2p16():
    """70 000 objects in one cell (more than 2^16): the cell's pairs are tiled
    into bounded tasks shared by every wave, where one wave per cell would do
    2.4e9 pair tests alone."""
    a = spheres(70_000, 81, 0, 4000, 8)
    announce("binned one cell of 70000 objects")
    assert binned(a, 1 << 14) == oracle.count_i32(*a)


def test_big_cells_next_to_small_and_big():
    """Big cells (more than 64 objects) next to small cells and next to each
    other along every forward direction, with isolated small cells between:
    every pair of ranges with a big side goes through the work items."""
    cell = 1024
    rng = np.random.default_rng(82)
    parts = []
    for cx, cy, cz, m in [(0, 0, 0, 300), (1, 0, 0, 5), (0, 1, 1, 200), (1, 1, 1, 90),
                          (5, 5, 5, 2), (5, 5, 6, 150), (6, 6, 6, 40), (9, 0, 0, 65),
                          (9, 1, 0, 64), (9, 0, 1, 66)]:
        xyz = rng.integers(0, cell, (m, 3)) + np.array([cx, cy, cz]) * cell
        parts.append(xyz)
    xyz = np.concatenate(parts)
    perm = rng.permutation(len(xyz))
    xyz = xyz[perm]
    x, y, z = (np.ascontiguousarray(xyz[:, k].astype(np.int32)) for k in range(3))
    r = rng.integers(0, cell // 2, len(x), endpoint=True).astype(np.int32)
    announce("binned big cells next to small and big", len(x))
    assert binned([x, y, z, r], cell) == oracle.count_i32(x, y, z, r)


# ------------------------------------------------------------ CSR batches --

def binned_batched(arrays, off, cell, flags=0, ws=None):
    import torch
    t = dev(*arrays)
    toff = dev(off)[0]
    out = torch.full((len(off) - 1,), -1, dtype=torch.int64, device="cuda")
    P.pairs_count_i32_binned_batched(*t, toff, cell, out, ws=ws, flags=flags)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def overlapping_batch(sizes, seed, span, cell):
    """Sets that all occupy the same region, so that pairs across sets touch
    as often as pairs within one: a count that leaked across sets would be
    far off."""
    off = w.offsets_from_sizes(np.array(sizes, np.int64))
    a = spheres(int(off[-1]), seed, -span, span, cell // 2)
    return off, a


@pytest.mark.parametrize("sizes,span,cell", [
    ([0, 1, 2, 3, 0, 50, 0], 100, 64),
    ([2000, 1, 0, 3000, 17, 2], 600, 64),           # crowded cells: work items
    ([500] * 40, 1 << 12, 256),
    ([150, 180], 2000, 32),                          # cells of 32: 63 key bits and 1 set bit
])
def test_batched_matches_oracle_per_set(sizes, span, cell):
    off, a = overlapping_batch(sizes, len(sizes) + cell, span, cell)
    announce("binned batched", len(sizes), span, cell)
    got = binned_batched(a, off, cell)
    for s in range(len(sizes)):
        lo, hi = int(off[s]), int(off[s + 1])
        assert got[s] == oracle.count_i32(*[v[lo:hi] for v in a]), s


def test_batched_one_set_equals_single_call():
    a = spheres(30000, 5, -(1 << 14), 1 << 14, 128)
    off = np.array([0, 30000], np.int64)
    announce("binned batched one set")
    assert binned_batched(a, off, 256)[0] == binned(a, 256) == oracle.count_i32(*a)


def test_batched_binned_sets_200k_full_size(golden_dir):
    """The 200 000 binned sets, each the content of one 2^14 cell, binned
    again inside each set: cells of 2^14 (one cell per set, so every set of
    more than 64 objects is a work item) and of 4096 (up to 64 cells per
    set); the per-set counts equal the stored oracle counts."""
    import hashlib
    with open(os.path.join(golden_dir, "workload_values.json")) as f:
        g = json.load(f)["binned_sets_200k_counts"]
    b = w.binned_sets()
    for cell in (1 << 14, 4096):
        announce("binned batched 200 000 sets", cell)
        got = binned_batched(b.objs.arrays(), b.offsets, cell)
        assert int(got.sum()) == g["total"]
        assert hashlib.sha256(got.astype("<u8").tobytes()).hexdigest() == g["sha256_le_u64"]


def test_batched_validation_and_key_bits():
    off, a = overlapping_batch([10, 20, 30], 3, 100, 32)
    announce("binned batched validation")
    # cells of 32: 63 key bits, no room for three sets
    with pytest.raises(P.PairsError) as e:
        binned_batched(a, off, 32)
    assert e.value.status == -1
    bad = off.copy()
    bad[1] = 25  # offsets must not decrease
    bad[2] = 20
    with pytest.raises(P.PairsError):
        binned_batched(a, bad, 64, flags=P.FLAG_VALIDATE)
    big = [v.copy() for v in a]
    big[3][7] = 40  # radius above cell / 2
    with pytest.raises(P.PairsError) as e:
        binned_batched(big, off, 64, flags=P.FLAG_VALIDATE)
    assert e.value.status == -2
    got = binned_batched(a, off, 64, flags=P.FLAG_VALIDATE)
    for s in range(3):
        lo, hi = int(off[s]), int(off[s + 1])
        assert got[s] == oracle.count_i32(*[v[lo:hi] for v in a])


def test_binned_calls_in_a_graph():
    """A single-set and a batched binned count captured into one graph and
    replayed three times, with eager binned calls of other sizes on the same
    workspaces in between and the outputs overwritten before each replay:
    every replay gives the oracle's counts."""
    import torch
    a = spheres(20000, 61, -(1 << 13), 1 << 13, 64)
    off, b = overlapping_batch([3000, 0, 1, 5000, 700], 62, 3000, 128)
    ta, tb, toff = dev(*a), dev(*b), dev(off)[0]
    wa = torch.empty(P.pairs_binned_workspace_size(20000), dtype=torch.uint8, device="cuda")
    wb = torch.empty(P.pairs_binned_workspace_size(int(off[-1])), dtype=torch.uint8,
                     device="cuda")
    oa = torch.empty(1, dtype=torch.int64, device="cuda")
    ob = torch.empty(len(off) - 1, dtype=torch.int64, device="cuda")
    want_a = oracle.count_i32(*a)
    want_b = [oracle.count_i32(*[v[int(off[s]):int(off[s + 1])] for v in b])
              for s in range(len(off) - 1)]
    # warm the library's device state outside the capture
    P.pairs_count_i32_binned(*ta, 128, oa, wa)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.pairs_count_i32_binned(*ta, 128, oa, wa)
        P.pairs_count_i32_binned_batched(*tb, toff, 128, ob, wb)
    announce("binned graph replays")
    other = spheres(5000, 63, -500, 500, 16)
    for rep in range(3):
        oa.fill_(-7)
        ob.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert int(oa.item()) == want_a, rep
        assert list(ob.cpu().numpy()) == want_b, rep
        # eager work on the same workspaces between replays
        P.pairs_count_i32_binned(*dev(*other), 32, oa, wa)
        P.pairs_count_i32_binned_batched(*dev(*other), dev(np.array([0, 2500, 5000]))[0], 64,
                                         ob[:2], wb)
        torch.cuda.synchronize()
        assert int(oa.item()) == oracle.count_i32(*other)
