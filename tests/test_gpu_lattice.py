"""Lattice-bead collision and contact counts on the GPU (Section 3) against
the CPU oracle's plain pairwise definition, bit for bit.

Covers the LDS path at every table size (ragged vector lengths around the
thread and table boundaries), the batched global path for vectors longer than
the LDS tables, the single-vector grid-wide path, optional outputs, extreme
coordinates, the domain and length errors, and the paper's own scale (1000
chains of 1920 beads)."""
import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

BAD = -1  # UINT64_MAX read back as int64


def run_batched(b, max_n, want=(True, True), flags=0):
    import torch
    x, y, z = dev(*b.objs.arrays())
    off, = dev(b.offsets)
    coll = torch.full((b.n_sets,), 7, dtype=torch.int64, device="cuda") if want[0] else None
    cont = torch.full((b.n_sets,), 7, dtype=torch.int64, device="cuda") if want[1] else None
    P.pairs_lattice_count_batched(x, y, z, off, max_n, coll, cont, flags=flags)
    torch.cuda.synchronize()
    return (None if coll is None else coll.cpu().numpy().astype(np.uint64),
            None if cont is None else cont.cpu().numpy().astype(np.uint64))


def run_single(arrays, want=(True, True), flags=0):
    import torch
    x, y, z = dev(*arrays)
    coll = torch.full((1,), 7, dtype=torch.int64, device="cuda") if want[0] else None
    cont = torch.full((1,), 7, dtype=torch.int64, device="cuda") if want[1] else None
    P.pairs_lattice_count(x, y, z, coll, cont, flags=flags)
    torch.cuda.synchronize()
    return (None if coll is None else int(coll.item()), None if cont is None else int(cont.item()))


RAGGED = [0, 1, 2, 3, 4, 31, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1000,
          1023, 1024, 1025, 1920, 2047, 2048, 2049, 3000, 4095, 4096]


@pytest.mark.parametrize("max_n", ["exact", 0, 4096])
def test_batched_walks_ragged(max_n):
    b = w.lattice_walks(len(RAGGED), RAGGED, 21)
    m = max(RAGGED) if max_n == "exact" else max_n
    announce("lattice batched ragged", max_n)
    coll, cont = run_batched(b, m)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    np.testing.assert_array_equal(coll, c0)
    np.testing.assert_array_equal(cont, c1)


@pytest.mark.parametrize("n,max_n", [(16, 16), (128, 128), (200, 256), (768, 768),
                                     (1920, 1920), (1920, 4000)])
def test_batched_table_sizes(n, max_n):
    # every (beads per thread, table size) pair the host picks
    b = w.lattice_walks(300, n, 1000 + n)
    announce("lattice batched", n, max_n)
    coll, cont = run_batched(b, max_n)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    np.testing.assert_array_equal(coll, c0)
    np.testing.assert_array_equal(cont, c1)


@pytest.mark.parametrize("sigma", [0.6, 2.0, 20.0])
def test_batched_normal_coordinates(sigma):
    # dense clouds: many beads per site, long probe sequences
    b = w.lattice_normal(100, 1500, sigma, 31)
    announce("lattice normal", sigma)
    coll, cont = run_batched(b, 1500)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    np.testing.assert_array_equal(coll, c0)
    np.testing.assert_array_equal(cont, c1)


def test_one_output_only():
    b = w.lattice_walks(64, 700, 5)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    announce("lattice collisions only")
    coll, cont = run_batched(b, 700, want=(True, False))
    assert cont is None
    np.testing.assert_array_equal(coll, c0)
    announce("lattice contacts only")
    coll, cont = run_batched(b, 700, want=(False, True))
    np.testing.assert_array_equal(cont, c1)


def test_batched_long_vectors_global_path():
    sizes = [5000, 100, 12000, 4097, 3, 0, 9000]
    b = w.lattice_walks(len(sizes), sizes, 8)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    for want in [(True, True), (True, False)]:
        announce("lattice batched global", want)
        coll, cont = run_batched(b, 0, want=want)
        np.testing.assert_array_equal(coll, c0)
        if want[1]:
            np.testing.assert_array_equal(cont, c1)


@pytest.mark.parametrize("n", [0, 1, 2, 100, 4096, 4097, 30000])
def test_single_vector(n):
    b = w.lattice_walks(1, n, 40 + n)
    a = b.objs.arrays()
    announce("lattice single", n)
    assert run_single(a) == oracle.lattice_counts(*a)


def test_single_vector_global_one_output():
    b = w.lattice_normal(1, 20000, 5.0, 3)
    a = b.objs.arrays()
    want = oracle.lattice_counts(*a)
    announce("lattice single global collisions only")
    assert run_single(a, want=(True, False))[0] == want[0]
    announce("lattice single global contacts only")
    assert run_single(a, want=(False, True))[1] == want[1]


def test_extreme_coordinates():
    # chains translated next to both ends of int32; only the box matters
    b = w.lattice_walks(4, 900, 12)
    x, y, z = (v.astype(np.int64) for v in b.objs.arrays())
    shift = [(2 ** 31 - 1 - 1000, 0, 0), (-2 ** 31 + 1000, 2 ** 31 - 1000, 5),
             (0, -2 ** 31 + 1000, 2 ** 31 - 1000), (123, -456, 789)]
    xs, ys, zs = x.copy(), y.copy(), z.copy()
    for s, (a, c, d) in enumerate(shift):
        sl = slice(b.offsets[s], b.offsets[s + 1])
        xs[sl] += a
        ys[sl] += c
        zs[sl] += d
    arrs = [v.astype(np.int32) for v in (xs, ys, zs)]
    bb = w.Batch(b.offsets, w.Beads(*arrs))
    announce("lattice extreme coordinates")
    coll, cont = run_batched(bb, 900)
    c0, c1 = oracle.lattice_counts_batched(*arrs, b.offsets)
    np.testing.assert_array_equal(coll, c0)
    np.testing.assert_array_equal(cont, c1)


def test_domain_and_length_errors():
    import torch
    # vector 1 spans 2^31 on every axis: its padded box exceeds 2^40 sites
    good = w.lattice_walks(1, 50, 1)
    gx, gy, gz = good.objs.arrays()
    far = np.array([-2 ** 30, 2 ** 30, 0, 7], np.int32)
    x = np.concatenate([gx, far, gx])
    y = np.concatenate([gy, far, gy])
    z = np.concatenate([gz, far[::-1].copy(), gz])
    off = np.array([0, 50, 54, 104], np.int64)
    b = w.Batch(off, w.Beads(x, y, z))
    announce("lattice domain error")
    coll, cont = run_batched(b, 64)
    want = oracle.lattice_counts(gx, gy, gz)
    assert (int(coll[0]), int(cont[0])) == want and (int(coll[2]), int(cont[2])) == want
    assert coll[1] == np.uint64(2 ** 64 - 1) and cont[1] == np.uint64(2 ** 64 - 1)
    with pytest.raises(P.PairsError) as e:
        run_batched(b, 64, flags=P.FLAG_VALIDATE)
    assert e.value.status == -2
    # a vector longer than the max_n the call was given
    b2 = w.lattice_walks(3, [100, 300, 100], 2)
    announce("lattice length error")
    coll, cont = run_batched(b2, 100)
    assert coll[1] == np.uint64(2 ** 64 - 1)
    c0, _ = oracle.lattice_counts_batched(*b2.objs.arrays(), b2.offsets)
    assert coll[0] == c0[0] and coll[2] == c0[2]
    with pytest.raises(P.PairsError) as e:
        run_batched(b2, 100, flags=P.FLAG_VALIDATE)
    assert e.value.status == -1
    # a valid batch passes validation
    announce("lattice validate ok")
    coll, cont = run_batched(good, 50, flags=P.FLAG_VALIDATE)
    assert (int(coll[0]), int(cont[0])) == want
    torch.cuda.synchronize()


def test_paper_scale_1000_chains_of_1920():
    # the linear-time experiments count 1000 bead vectors per execution,
    # up to 1920 beads each (Section 5)
    b = w.lattice_walks(1000, 1920, 77)
    announce("lattice paper scale")
    coll, cont = run_batched(b, 1920)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    np.testing.assert_array_equal(coll, c0)
    np.testing.assert_array_equal(cont, c1)


def test_repeated_calls_reuse_nothing():
    # a second call on other data must not see the first call's tables
    b1 = w.lattice_normal(50, 2000, 1.0, 1)
    b2 = w.lattice_walks(50, 2000, 2)
    announce("lattice repeated")
    run_batched(b1, 2000)
    coll, cont = run_batched(b2, 2000)
    c0, c1 = oracle.lattice_counts_batched(*b2.objs.arrays(), b2.offsets)
    np.testing.assert_array_equal(coll, c0)
    np.testing.assert_array_equal(cont, c1)


def test_large_workload_matches_stored_oracle_values(golden_dir):
    # 65536 chains of 1920 beads; the expected per-vector counts were written
    # by tests/golden/make_golden.py from the oracle
    import hashlib
    import json
    import os
    with open(os.path.join(golden_dir, "workload_values.json")) as f:
        g = json.load(f)["lattice_large_counts"]
    b = w.lattice_large()
    announce("lattice large stored values")
    coll, cont = run_batched(b, 1920)
    assert hashlib.sha256(coll.astype("<u8").tobytes()).hexdigest() == g["collisions_sha256_le_u64"]
    assert hashlib.sha256(cont.astype("<u8").tobytes()).hexdigest() == g["contacts_sha256_le_u64"]


@pytest.mark.parametrize("want", [(True, True), (True, False), (False, True)])
def test_far_vectors_take_the_box_pass(want):
    # beads more than ~1000 sites from their vector's first bead cannot use
    # the near keys; such vectors are recounted with box-based 64-bit keys.
    # Mixed with near vectors, and with either output alone (the marker then
    # lives in the other output).
    near = w.lattice_walks(20, 700, 4)
    # sigma 800: beads thousands of sites from the first one, while the box
    # stays inside the 2^40-site domain
    far = w.lattice_normal(20, 700, 800.0, 5)
    dense_far = w.lattice_normal(20, 700, 1.5, 6)
    for v in dense_far.objs.arrays():
        v += 50_000  # a dense cloud whose first bead is an outlier
    for v, s in zip(dense_far.objs.arrays(), (-40_000, 0, 40_000)):
        v[dense_far.offsets[:-1]] += s
    parts = [near, far, dense_far]
    arrs = [np.concatenate([p.objs.arrays()[a] for p in parts]) for a in range(3)]
    sizes = np.concatenate([np.diff(p.offsets) for p in parts])
    b = w.Batch(w.offsets_from_sizes(sizes), w.Beads(*arrs))
    announce("lattice far vectors", want)
    coll, cont = run_batched(b, 700, want=want)
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    if want[0]:
        np.testing.assert_array_equal(coll, c0)
    if want[1]:
        np.testing.assert_array_equal(cont, c1)


def test_batched_calls_captured_in_a_graph():
    # with max_n within the LDS tables a call needs no workspace and
    # synchronises nothing: a graph holds it, and each replay, with eager
    # calls on other data in between, gives the oracle's counts
    import torch
    b = w.lattice_walks(200, 1000, 13)
    o = w.lattice_normal(50, 900, 3.0, 14)
    c0, k0 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    c1, k1 = oracle.lattice_counts_batched(*o.objs.arrays(), o.offsets)
    x, y, z = dev(*b.objs.arrays())
    off, = dev(b.offsets)
    ox, oy, oz = dev(*o.objs.arrays())
    ooff, = dev(o.offsets)
    coll = torch.empty(200, dtype=torch.int64, device="cuda")
    cont = torch.empty_like(coll)
    oc = torch.empty(50, dtype=torch.int64, device="cuda")
    ok = torch.empty_like(oc)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.pairs_lattice_count_batched(x, y, z, off, 1000, coll, cont)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    announce("lattice graph capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(5):
            P.pairs_lattice_count_batched(x, y, z, off, 1000, coll, cont)
    for rep in range(3):
        coll.fill_(-1)
        cont.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(coll.cpu().numpy().astype(np.uint64), c0)
        np.testing.assert_array_equal(cont.cpu().numpy().astype(np.uint64), k0)
        P.pairs_lattice_count_batched(ox, oy, oz, ooff, 900, oc, ok)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(oc.cpu().numpy().astype(np.uint64), c1)
        np.testing.assert_array_equal(ok.cpu().numpy().astype(np.uint64), k1)


@pytest.mark.parametrize("max_n", [64, 128, 256])
def test_short_vectors_one_wave_each(max_n):
    # vectors of at most 256 beads are counted one per wave, four tables per
    # workgroup; ragged lengths, dense clouds, and far vectors (box pass)
    sizes = [s for s in [0, 1, 2, 3, 31, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256]
             if s <= max_n]
    walks = w.lattice_walks(len(sizes) * 7, sizes * 7, 30 + max_n)
    dense = w.lattice_normal(40, max_n, 1.0, 31)
    far = w.lattice_normal(9, max_n, 800.0, 32)
    parts = [walks, dense, far]
    arrs = [np.concatenate([p.objs.arrays()[a] for p in parts]) for a in range(3)]
    szs = np.concatenate([np.diff(p.offsets) for p in parts])
    b = w.Batch(w.offsets_from_sizes(szs), w.Beads(*arrs))
    c0, c1 = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    for want in [(True, True), (True, False), (False, True)]:
        announce("lattice per-wave", max_n, want)
        coll, cont = run_batched(b, max_n, want=want)
        if want[0]:
            np.testing.assert_array_equal(coll, c0)
        if want[1]:
            np.testing.assert_array_equal(cont, c1)
