"""GPU parity of the collision counts against the CPU oracle (bit-exact)."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu

# sizes around every tile edge of the single-set shapes (64 to 512 rows per
# wave), ragged tails, both parities, and the size-class switches of the
# default tables (4096, 8192, 16384, 65536)
SIZES = [0, 1, 2, 3, 4, 5, 6, 7, 63, 64, 65, 66, 127, 128, 129, 255, 256, 257, 511, 512, 513,
         1000, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 8194,
         12345, 16383, 16384, 16385, 30001, 65535, 65536, 65537, 65538]


def dense_i32(n, seed):
    # many collisions: centres in a 48-cube, radii 0..6
    return w.spheres_i32(n, seed, 48, 6, radius_lo=0)


def sparse_i32(n, seed):
    return w.spheres_i32(n, seed, 2 ** 16, 2 ** 9)


@pytest.mark.parametrize("n", SIZES)
def test_count_i32_matches_oracle(n):
    for kind, gen in (("dense", dense_i32), ("sparse", sparse_i32)):
        s = gen(n, 1000 + n)
        announce("count_i32", kind, n)
        expect = oracle.count_i32(*s.arrays())
        got = P.count_i32(*dev(*s.arrays()))
        assert got == expect, (kind, n)


def test_count_i32_spheres_4096():
    s = w.spheres_4096()
    announce("count_i32 4096 spheres")
    assert P.count_i32(*dev(*s.arrays())) == oracle.count_i32(*s.arrays())


@pytest.fixture
def forced_shape():
    """Force one single-set tile shape for a kind; restores the defaults after."""
    kinds = []

    def force(kind, rows_per_lane, chunk, form=P.FORM_BROADCAST):
        kinds.append(kind)
        P.pairs_set_shapes(kind, False, [(0, rows_per_lane, chunk, form)])

    yield force
    for k in kinds:
        P.pairs_set_shapes(k, False, None)


@pytest.mark.parametrize("K,U", [(1, 64), (1, 256), (2, 128), (4, 64), (4, 1024), (8, 512)])
def test_count_i32_every_shape(forced_shape, K, U):
    # both predicate forms (64-bit integer for K <= 2, double for K >= 4),
    # across tile edges
    forced_shape(P.KIND_COUNT_I32, K, U)
    for n in (2, 3, 64 * K - 1, 64 * K, 64 * K + 1, 3 * 64 * K + 7, 2500):
        s = dense_i32(n, 7 * n + K)
        announce("count_i32 forced shape", K, U, n)
        assert P.count_i32(*dev(*s.arrays())) == oracle.count_i32(*s.arrays()), (K, U, n)


@pytest.mark.parametrize("U", [64, 128, 1024])
def test_count_i32_matrix_form(forced_shape, U):
    """The matrix-core form (16-row tiles on v_mfma_f64_16x16x4f64) at tile
    edges, ragged tails, the band's two edges and the even-n extra step."""
    forced_shape(P.KIND_COUNT_I32, 1, U, P.FORM_MATRIX)
    for n in (2, 3, 15, 16, 17, 63, 64, 65, 127, 128, 129, 2 * U + 1, 2500, 8193, 16384):
        for kind, gen in (("dense", dense_i32), ("sparse", sparse_i32)):
            s = gen(n, 11 * n + U)
            announce("count_i32 matrix form", kind, U, n)
            assert P.count_i32(*dev(*s.arrays())) == oracle.count_i32(*s.arrays()), (kind, U, n)


def test_count_i32_matrix_form_spheres_4096(forced_shape):
    forced_shape(P.KIND_COUNT_I32, 1, 512, P.FORM_MATRIX)
    s = w.spheres_4096()
    announce("count_i32 matrix form 4096 spheres")
    assert P.count_i32(*dev(*s.arrays())) == oracle.count_i32(*s.arrays())


LO, HI, RMAX = -(2 ** 30), 2 ** 30 - 1, 2 ** 30   # the exact domain


def domain_set(n, seed, lo, hi, rmax):
    rng = np.random.default_rng(seed)
    x, y, z = (rng.integers(lo, hi, n, endpoint=True).astype(np.int32) for _ in range(3))
    r = rng.integers(0, rmax, n, endpoint=True).astype(np.int32)
    return x, y, z, r


@pytest.mark.parametrize("K", [1, 2, 4, 8, "matrix"])
@pytest.mark.parametrize("L", [2 ** 22, 2 ** 24, 2 ** 29, 2 ** 30])
def test_count_i32_domain_edges(forced_shape, K, L):
    """Coordinates in [-L, L) and radii in [0, L] up to the domain's edges,
    with no flag: the plain Gram tests hold up to 2^24 (double form, K >= 4,
    and the matrix form) and 2^29 (integer form, K <= 2); beyond, waves
    switch to the wide test."""
    K = force_k_or_matrix(forced_shape, K, 256)
    n = 3001
    x, y, z, r = domain_set(n, 5 + K, -L, L - 1, L)
    # pin a few objects to the extreme corners
    x[:4] = [-L, L - 1, -L, L - 1]
    y[:4] = [-L, L - 1, L - 1, -L]
    z[:4] = [L - 1, -L, -L, L - 1]
    r[:4] = [L, L, 0, L]
    announce("count_i32 domain edges", K, L, n)
    assert P.count_i32(*dev(x, y, z, r)) == oracle.count_i32(x, y, z, r)
    assert P.count_i32(*dev(x, y, z, r), validate=True) == oracle.count_i32(x, y, z, r)
    # touching and one-apart pairs across the full span
    for gap, expect in ((0, 1), (1, 0)):
        a = np.array([-L, L - 1], np.int32)
        zero = np.zeros(2, np.int32)
        rr = np.array([L, L - 1 - gap], np.int32)
        assert P.count_i32(*dev(a, zero, zero, rr)) == expect, (gap, L)


def force_k_or_matrix(forced_shape, K, U):
    """Force K rows per lane in the broadcast form, or the matrix form for
    K = "matrix"; returns an integer standing for K in seeds."""
    if K == "matrix":
        forced_shape(P.KIND_COUNT_I32, 1, U, P.FORM_MATRIX)
        return 16
    forced_shape(P.KIND_COUNT_I32, K, U)
    return K


@pytest.mark.parametrize("K", [1, 2, 4, 8, "matrix"])
def test_count_i32_extreme_pairs(forced_shape, K):
    """Pairs at the largest distances and radii of the domain, decided at exact
    equality: the squared distance 3 (2^31 - 1)^2 and the squared radius sum
    2^62 sit at the edges of the wide test's modulo-2^64 window."""
    K = force_k_or_matrix(forced_shape, K, 64)
    pts = []
    # opposite corners: d^2 = 3 (2^31 - 1)^2 > (2^31)^2, never touching
    pts.append(((LO, LO, LO, RMAX), (HI, HI, HI, RMAX)))
    # along one axis: d = 2^31 - 1 against R = 2^31 (hit), 2^31 - 1 (hit), 2^31 - 2 (miss)
    pts.append(((LO, 0, 0, RMAX), (HI, 0, 0, RMAX)))
    pts.append(((LO, 0, 0, RMAX - 1), (HI, 0, 0, RMAX)))
    pts.append(((LO, 0, 0, RMAX - 1), (HI, 0, 0, RMAX - 1)))
    # two axes: d^2 = 2 (2^31 - 1)^2 against (2^31)^2 (miss)
    pts.append(((LO, LO, 0, RMAX), (HI, HI, 0, RMAX)))
    # a Pythagorean triple scaled to the span: (3k, 4k) at distance 5k
    k = (2 ** 31 - 1) // 5
    pts.append(((-(2 ** 30), -(2 ** 30), 7, (5 * k) // 2), (-(2 ** 30) + 3 * k, -(2 ** 30) + 4 * k,
                                                          7, 5 * k - (5 * k) // 2)))
    pts.append(((-(2 ** 30), -(2 ** 30), 7, (5 * k) // 2), (-(2 ** 30) + 3 * k, -(2 ** 30) + 4 * k,
                                                          7, 5 * k - (5 * k) // 2 - 1)))
    for a, b in pts:
        x, y, z, r = (np.array([a[c], b[c]], np.int32) for c in range(4))
        want = oracle.count_i32(x, y, z, r)
        announce("count_i32 extreme pair", K, a, b, want)
        assert P.count_i32(*dev(x, y, z, r)) == want, (a, b)
    # all of them in one set, shuffled among ordinary objects
    rng = np.random.default_rng(K)
    obj = [c for ab in pts for c in ab]
    x, y, z, r = domain_set(2000, 40 + K, LO, HI, RMAX)
    for i, o in enumerate(obj):
        x[i], y[i], z[i], r[i] = o
    perm = rng.permutation(2000)
    x, y, z, r = x[perm], y[perm], z[perm], r[perm]
    assert P.count_i32(*dev(x, y, z, r)) == oracle.count_i32(x, y, z, r)


@pytest.mark.parametrize("K", [1, 2, 4, 8, "matrix"])
def test_count_i32_mixed_boxes(forced_shape, K):
    """Dense objects inside the plain tests' boxes with a few far outside:
    tasks and partner groups take the plain and the wide test side by side."""
    K = force_k_or_matrix(forced_shape, K, 128)
    n = 5000
    s = dense_i32(n, 90 + K)
    x, y, z, r = [a.copy() for a in s.arrays()]
    rng = np.random.default_rng(K)
    far = rng.choice(n, 9, replace=False)
    x[far[:3]] = [HI, LO, HI]
    y[far[3:6]] = [LO, HI, LO]
    r[far[6:]] = [RMAX, 2 ** 29, 2 ** 24 + 1]     # huge spheres reach everything nearby
    announce("count_i32 mixed boxes", K, n)
    assert P.count_i32(*dev(x, y, z, r)) == oracle.count_i32(x, y, z, r)


def test_count_i32_validate_rejects_out_of_domain():
    import torch
    s = sparse_i32(100, 3)
    for axis, v in ((0, 2 ** 30), (1, -(2 ** 30) - 1), (2, 2 ** 31 - 1)):
        a = [c.copy() for c in (s.x, s.y, s.z)]
        a[axis][17] = v
        with pytest.raises(P.PairsError) as e:
            P.count_i32(*dev(*a, s.r), validate=True)
        assert e.value.status == -2
    for bad_r in (-1, 2 ** 30 + 1):
        r = s.r.copy()
        r[3] = bad_r
        with pytest.raises(P.PairsError):
            P.count_i32(*dev(s.x, s.y, s.z, r), validate=True)
    # the domain's own edges pass validation
    x = s.x.copy()
    x[5], x[6] = -(2 ** 30), 2 ** 30 - 1
    r = s.r.copy()
    r[7] = 2 ** 30
    assert P.count_i32(*dev(x, s.y, s.z, r), validate=True) == oracle.count_i32(x, s.y, s.z, r)
    torch.cuda.synchronize()


def test_count_i32_invariances_and_partition():
    s = dense_i32(5000, 77)
    x, y, z, r = s.arrays()
    c = P.count_i32(*dev(x, y, z, r))
    perm = np.random.default_rng(0).permutation(len(x))
    assert P.count_i32(*dev(x[perm], y[perm], z[perm], r[perm])) == c
    assert P.count_i32(*dev(x - 1000, y + 5, z, r)) == c
    for split in (1, 64, 1777, 4999):
        a = [v[:split] for v in (x, y, z, r)]
        b = [v[split:] for v in (x, y, z, r)]
        cross = oracle.cross_count_i32(a, b)
        assert P.count_i32(*dev(*a)) + P.count_i32(*dev(*b)) + cross == c
    assert all(P.count_i32(*dev(x, y, z, r)) == c for _ in range(3))


def golden():
    with open(os.path.join(os.path.dirname(__file__), "golden", "workload_values.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("n,key", [(2 ** 20, "spheres_2p20_count"),
                                   (2 ** 20 - 1, "spheres_2p20m1_count")])
def test_count_i32_spheres_2p20_full_size(n, key):
    g = golden()
    if key not in g:
        pytest.skip(f"{key} not yet in tests/golden/workload_values.json")
    s = w.spheres_2p24(n)
    announce("count_i32 spheres", n)
    assert P.count_i32(*dev(*s.arrays())) == g[key]


F32_SIZES = [0, 1, 2, 3, 64, 65, 127, 129, 511, 513, 1000, 4096, 8193, 20011]


@pytest.mark.parametrize("K,U", [(1, 64), (2, 128), (4, 256), (8, 512)])
def test_count_f32_every_shape(forced_shape, K, U):
    forced_shape(P.KIND_COUNT_F32, K, U)
    rng = np.random.default_rng(K)
    for n in (2, 64 * K - 1, 64 * K + 1, 2 * 64 * K + 5, 3001):
        x, y, z = (rng.random(n, dtype=np.float32) for _ in range(3))
        r = np.full(n, np.float32(0.07))
        assert P.count_f32(*dev(x, y, z, r)) == oracle.count_f32(x, y, z, r), (K, U, n)


@pytest.mark.parametrize("n", F32_SIZES)
def test_count_f32_matches_oracle(n):
    rng = np.random.default_rng(n)
    # unit cube, radius 0.05: a few percent of pairs hit
    x, y, z = (rng.random(n, dtype=np.float32) for _ in range(3))
    r = np.full(n, np.float32(0.05))
    announce("count_f32", n)
    assert P.count_f32(*dev(x, y, z, r)) == oracle.count_f32(x, y, z, r)
    # per-object radii and a subnormal-scale cluster
    r2 = rng.random(n, dtype=np.float32) * np.float32(0.1)
    xs = (x * np.float32(1e-38)).astype(np.float32)
    assert P.count_f32(*dev(x, y, z, r2)) == oracle.count_f32(x, y, z, r2)
    rs = (r2 * np.float32(1e-38)).astype(np.float32)
    assert P.count_f32(*dev(xs, y * 0, z * 0, rs)) == oracle.count_f32(xs, y * 0, z * 0, rs)


def test_count_f32_validate_rejects_nonfinite():
    n = 50
    x = np.zeros(n, np.float32)
    x[7] = np.inf
    z = np.zeros(n, np.float32)
    with pytest.raises(P.PairsError):
        P.count_f32(*dev(x, z, z, z), validate=True)


def test_count_i32_calls_captured_in_a_graph():
    """Single-set calls allocate and synchronise nothing, so a HIP graph can
    hold them: each replay, with eager calls on other data in between, gives
    the oracle's count."""
    import torch
    s = w.spheres_4096()
    want = oracle.count_i32(*s.arrays())
    t = dev(*s.arrays())
    other = dev(*w.spheres_i32(777, 5, 32, 3, radius_lo=0).arrays())
    want_other = oracle.count_i32(*w.spheres_i32(777, 5, 32, 3, radius_lo=0).arrays())
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    out2 = torch.empty(1, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.pairs_count_i32(*t, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(10):
            P.pairs_count_i32(*t, out)
    for rep in range(3):
        out.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert int(out.item()) == want, rep
        P.pairs_count_i32(*other, out2)
        torch.cuda.synchronize()
        assert int(out2.item()) == want_other
