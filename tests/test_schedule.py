"""The library's wave tasks cover the paper's balanced assignment exactly once.

pairs_debug_task_ranges (host-only, no GPU) lists the tasks the kernels run
for a set of n objects: rows [ra, ra + 64K) and virtual partners u in
[u0, u1).  Expanding them with the paper's rule -- row i evaluates
(i + s) mod n for s = 1 .. floor((n-1)/2), plus s = n/2 for i < n/2 when n is
even -- must give every unordered pair exactly once (Propositions 1 and 2).
"""
import numpy as np
import pytest

import paper_1901_11204_amd as P


def steps(n, i):
    return (n - 1) // 2 + (1 if n % 2 == 0 and i < n // 2 else 0)


def expand(n, K, U):
    tasks = P.pairs_debug_task_ranges(n, K, U)
    seen = np.zeros((n, n), np.int32)
    rows = 64 * K
    for ra, u0, u1 in tasks:
        for i in range(ra, min(ra + rows, n)):
            lo = max(u0, i + 1)
            hi = min(u1, i + steps(n, i) + 1)
            for u in range(lo, hi):
                j = u % n
                a, b = (i, j) if i < j else (j, i)
                seen[a, b] += 1
    return tasks, seen


@pytest.mark.parametrize("K,U", [(1, 64), (1, 256), (2, 128), (4, 64), (4, 1024), (8, 512)])
def test_tasks_cover_every_pair_once(K, U):
    sizes = sorted(set([0, 1, 2, 3, 4, 5, 63, 64, 65, 127, 128, 129, 200, 257, 511, 512, 513,
                        64 * K - 1, 64 * K, 64 * K + 1, 2 * 64 * K + 3, 1000, 1025]))
    for n in sizes:
        tasks, seen = expand(n, K, U)
        iu = np.triu_indices(n, 1)
        assert np.all(seen[iu] == 1), (n, K, U)
        assert seen.sum() == n * (n - 1) // 2
        # u ranges stay inside [1, 2n) and chunks never exceed U
        for ra, u0, u1 in tasks:
            if u0 < u1:
                assert 1 <= u0 and u1 <= 2 * n and u1 - u0 <= U
                assert ra % (64 * K) == 0 and ra < n


def test_task_count_of_large_sets():
    # N = 2^20 with 512 rows x 8192 partners per task: 2048 row blocks of
    # ceil((512 - 1 + 2^19) / 8192) = 65 chunks
    t = P.pairs_debug_task_ranges(2 ** 20, 8, 8192)
    assert t.shape == (2048 * 65, 3)
    assert int(np.maximum(t[:, 2] - t[:, 1], 0).max()) == 8192


def test_bad_shapes_rejected():
    with pytest.raises(P.PairsError):
        P.pairs_debug_task_ranges(100, 3, 64)
    with pytest.raises(P.PairsError):
        P.pairs_debug_task_ranges(100, 1, 100)
    with pytest.raises(P.PairsError):
        P.pairs_debug_task_ranges(-1, 1, 64)


# ----------------------------------------------------------- stepping form --
#
# pairs_debug_step_ranges lists the stepping-form tasks (the paper's per-row
# form): rows [r0, r0 + 64K) run the steps [s0, s0 + T) and, when x is 1, the
# rows below n/2 run the extra step s0 + T.

def expand_steps(n, K, U):
    tasks = P.pairs_debug_step_ranges(n, K, U)
    seen = np.zeros((n, n), np.int32)
    for r0, s0, T, x in tasks:
        for i in range(r0, min(r0 + 64 * K, n)):
            ss = list(range(s0, s0 + T))
            if x and n % 2 == 0 and i < n // 2:
                ss.append(s0 + T)
            for s in ss:
                j = (i + s) % n
                a, b = (i, j) if i < j else (j, i)
                seen[a, b] += 1
    return tasks, seen


@pytest.mark.parametrize("K,U", [(1, 16), (1, 192), (1, 288), (2, 16), (2, 48), (2, 144), (2, 272)])
def test_step_tasks_cover_every_pair_once(K, U):
    sizes = sorted(set([0, 1, 2, 3, 4, 5, 6, 7, 8, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200,
                        257, 289, 290, 511, 512, 513, 64 * K + 1, 1000, 1025]))
    for n in sizes:
        tasks, seen = expand_steps(n, K, U)
        iu = np.triu_indices(n, 1)
        assert np.all(seen[iu] == 1), (n, K, U)
        assert seen.sum() == n * (n - 1) // 2
        for r0, s0, T, x in tasks:
            assert r0 % (64 * K) == 0 and r0 < n
            assert s0 >= 1 and 0 <= T and T + x <= U and x in (0, 1)
            assert s0 + T + x - 1 <= n // 2


def test_step_shapes_rejected():
    with pytest.raises(P.PairsError):
        P.pairs_debug_step_ranges(100, 4, 64)
    with pytest.raises(P.PairsError):
        P.pairs_debug_step_ranges(100, 1, 0)
    bad = [(0, 4, 64, P.FORM_STEPPING)]          # stepping takes 1 or 2 rows per lane
    with pytest.raises(P.PairsError):
        P.pairs_set_shapes(P.KIND_COUNT_I32, True, bad)
    with pytest.raises(P.PairsError):         # chunk above the window capacity
        P.pairs_set_shapes(P.KIND_COUNT_I32, True, [(0, 2, 288, P.FORM_STEPPING)])
    with pytest.raises(P.PairsError):         # single-set tables are broadcast only
        P.pairs_set_shapes(P.KIND_COUNT_I32, False, [(0, 1, 64, P.FORM_STEPPING)])
    P.pairs_set_shapes(P.KIND_COUNT_I32, True, [(0, 1, 192, P.FORM_STEPPING)])
    assert P.pairs_get_shapes(P.KIND_COUNT_I32, True) == [(0, 1, 192, P.FORM_STEPPING)]
    P.pairs_set_shapes(P.KIND_COUNT_I32, True, None)


def test_total_only_shape_mode():
    """Mode 2 holds the float32 energy's total-only table (one row per lane
    for large sets by default); other kinds and modes beyond 2 are rejected."""
    E = P.KIND_ENERGY_F32
    default = P.pairs_get_shapes(E, P.SHAPES_TOTAL_ONLY)
    assert default[0][1] == 1 and default[0][0] >= 65536
    assert P.pairs_get_shapes(E, P.SHAPES_SINGLE) != default
    P.pairs_set_shapes(E, P.SHAPES_TOTAL_ONLY, [(0, 2, 512)])
    assert P.pairs_get_shapes(E, P.SHAPES_TOTAL_ONLY) == [(0, 2, 512, P.FORM_BROADCAST)]
    assert P.pairs_get_shapes(E, P.SHAPES_SINGLE) != [(0, 2, 512, P.FORM_BROADCAST)]
    P.pairs_set_shapes(E, P.SHAPES_TOTAL_ONLY, None)
    assert P.pairs_get_shapes(E, P.SHAPES_TOTAL_ONLY) == default
    for kind in (P.KIND_COUNT_I32, P.KIND_COUNT_F32):
        with pytest.raises(P.PairsError):
            P.pairs_get_shapes(kind, P.SHAPES_TOTAL_ONLY)
        with pytest.raises(P.PairsError):
            P.pairs_set_shapes(kind, P.SHAPES_TOTAL_ONLY, [(0, 1, 256)])
    for mode in (3, -1):
        with pytest.raises(P.PairsError):
            P.pairs_get_shapes(E, mode)
        with pytest.raises(P.PairsError):
            P.pairs_set_shapes(E, mode, None)
    with pytest.raises(P.PairsError):   # the stepping form is for batches only
        P.pairs_set_shapes(E, P.SHAPES_TOTAL_ONLY, [(0, 1, 64, P.FORM_STEPPING)])


def test_matrix_shapes_rejected():
    """The matrix form takes single-set int32 count tables only, with one row
    per lane and chunks that are multiples of 64."""
    M = P.FORM_MATRIX
    for kind, batched, entry in ((P.KIND_COUNT_I32, True, (0, 1, 256, M)),
                                 (P.KIND_COUNT_F32, False, (0, 1, 256, M)),
                                 (P.KIND_ENERGY_F32, False, (0, 1, 256, M)),
                                 (P.KIND_COUNT_I32, False, (0, 2, 256, M)),
                                 (P.KIND_COUNT_I32, False, (0, 1, 96, M)),
                                 (P.KIND_COUNT_I32, False, (0, 1, 32, M)),
                                 (P.KIND_COUNT_I32, False, (0, 1, 2 ** 23, M))):
        with pytest.raises(P.PairsError):
            P.pairs_set_shapes(kind, batched, [entry])
    table = [(65536, 8, 1024, P.FORM_BROADCAST), (0, 1, 512, M)]
    P.pairs_set_shapes(P.KIND_COUNT_I32, False, table)
    assert P.pairs_get_shapes(P.KIND_COUNT_I32, False) == table
    P.pairs_set_shapes(P.KIND_COUNT_I32, False, None)
    assert all(e[3] == P.FORM_BROADCAST for e in P.pairs_get_shapes(P.KIND_COUNT_I32, False))


# The window indexing of a stepping task, emulated lane by lane exactly as the
# kernel computes it (segments of w lanes, K-interleaved window of S entries
# per residue, sweep positions split into the unmasked core and the masked
# extra step).  Checks that every window entry a lane reads was staged by the
# task, lies inside the wave's window, and holds the partner the paper's rule
# assigns; together with the coverage test above, every pair is tested once.

STEP_CAP = 416


def window_entries(K, w, T, x):
    return w + (T + x + K - 1 + K - 1) // K


def sweep_positions(K, T, x):
    """(tau, k, masked) in the order the kernel tests them."""
    out = []
    if K == 1:
        out += [(t, 0, False) for t in range(T)]
        if x:
            out.append((T, 0, True))
        return out
    if T > 0:
        out.append((0, 0, False))
    for t in range(1, T):
        out += [(t, 0, False), (t, 1, False)]
    if T > 0:
        out.append((T, 1, False))
    if x:
        out += [(T, 0, True), (T + 1, 1, True)]
    return out


def emulate(n, K, r0, s0, T, x, m, w, pack=False):
    S = window_entries(K, w, T, x)
    assert m * K * S <= STEP_CAP and m * w <= 64
    assert S <= w * (6 if K == 1 else 4)                      # staging slots per lane
    staged = {}
    for lane in range(64):
        j, l = divmod(lane, w)
        if j >= m:
            continue
        if pack:
            # whole sets: each row o is written to window positions o - 1, o - 1 + n
            assert r0 == 0 and s0 == 1
            for k in range(K):
                o = K * l + k
                if o < n:
                    for v in (o - 1, o - 1 + n):
                        if 0 <= v < K * S:
                            staged[(j * K + v % K) * S + v // K] = (j, o)
            continue
        for c in range(K):
            for i in range((S + w - 1) // w):
                q = l + w * i
                if q < S:
                    o = r0 + s0 + K * q + c
                    o = o - n if o >= n else o
                    staged[(j * K + c) * S + q] = (j, o if o < n else None)
    pairs = []
    for lane in range(64):
        j, l = divmod(lane, w)
        live = j < m
        if not live:
            j, l = 0, 0
        e0 = (j * K) * S + l
        for tau, k, masked in sweep_positions(K, T, x):
            e = e0 + (tau % K) * S + tau // K
            assert 0 <= e < m * K * S <= STEP_CAP
            row = r0 + K * l + k
            if not live:
                continue                     # idle lanes report nothing
            seg, o = staged[e]               # live lanes, padding rows included, read staged entries
            assert seg == j
            if row >= n:
                continue
            if masked and not (n % 2 == 0 and row < n // 2):
                continue
            s = s0 + tau - k
            assert o == (row + s) % n, (n, K, row, s, o)
            pairs.append((j, row, o))
    return pairs


@pytest.mark.parametrize("K", [1, 2])
def test_step_window_emulation_blocks(K):
    for n in [2, 3, 5, 64, 65, 70, 129, 130, 256, 301, 1000]:
        for U in [16, 48, 272 if K == 2 else 288]:
            for r0, s0, T, x in P.pairs_debug_step_ranges(n, K, U):
                emulate(n, K, int(r0), int(s0), int(T), int(x), 1, 64)


@pytest.mark.parametrize("K", [1, 2])
def test_step_window_emulation_packs(K):
    for n in range(2, 64 * K + 1):
        Kp = 1 if n < 4 * K else K
        w = -(-n // Kp)
        h, x = (n - 1) // 2, 1 if n % 2 == 0 else 0
        S = window_entries(Kp, w, h, x)
        m = max(1, min(64 // w, STEP_CAP // (Kp * S)))
        pairs = emulate(n, Kp, 0, 1, h, x, m, w, pack=True)
        for j in range(m):
            got = sorted(tuple(sorted((r, o))) for (jj, r, o) in pairs if jj == j)
            assert got == [(a, b) for a in range(n) for b in range(a + 1, n)], (n, Kp, j)


# ------------------------------------------------------ launch geometry --
#
# A single-set call launches one wave per task up to 2^22 blocks and strides
# over the rest, so every n up to PAIRS_MAX_SET_SIZE = 2^30 launches within
# the 2^32 work-item limit of one dispatch.

KINDS = [P.KIND_COUNT_I32, P.KIND_COUNT_F32, P.KIND_ENERGY_F32, P.KIND_ENERGY_F64,
         P.KIND_FORCE_F32]
LARGE = [2, 3, 4095, 4096, 2 ** 20, 2 ** 22, 2 ** 22 + 1, 2 ** 23, 204 ** 3, 2 ** 27 - 1,
         2 ** 27, 2 ** 29 + 7, 2 ** 30 - 1, 2 ** 30]


@pytest.mark.parametrize("kind", KINDS)
def test_single_launch_fits_one_dispatch(kind):
    assert P.pairs_debug_single_launch(kind, 0) == (0, 0, 256)
    assert P.pairs_debug_single_launch(kind, 1) == (0, 0, 256)
    for n in LARGE:
        tasks, blocks, threads = P.pairs_debug_single_launch(kind, n)
        assert tasks >= 1 and 1 <= blocks <= 2 ** 22, (kind, n)
        assert blocks * threads < 2 ** 32, (kind, n)
        waves = blocks * threads // 64
        if tasks <= 4 * 2 ** 22:
            assert blocks == -(-tasks // 4)           # one wave per task
        else:
            assert waves == 2 ** 24 and tasks > waves  # grid stride


def test_single_launch_rejects_bad_kind_and_size():
    with pytest.raises(P.PairsError):
        P.pairs_debug_single_launch(0, 10)
    with pytest.raises(P.PairsError):
        P.pairs_debug_single_launch(6, 10)
    with pytest.raises(P.PairsError):
        P.pairs_debug_single_launch(P.KIND_COUNT_I32, 2 ** 30 + 1)


def grouped_indices(nblocks, nchunks, b):
    """Task indices of row block b's chunks 0..nchunks-1 in the single-set
    kernels' order: 16 groups of R = ceil(nblocks / 16) blocks, chunk-major
    inside a group."""
    R = -(-nblocks // 16)
    g, j = divmod(b, R)
    rg = min(R, nblocks - g * R)
    return g * R * nchunks + np.arange(nchunks, dtype=np.int64) * rg + j


@pytest.mark.parametrize("n,K,U", [(2, 1, 64), (7, 1, 64), (1000, 1, 64), (5000, 2, 128),
                                   (12345, 8, 512), (70001, 4, 256), (2 ** 17, 8, 1024),
                                   (17 * 512 + 3, 8, 64)])
def test_grouped_task_order_is_a_permutation(n, K, U):
    """The kernels' grouped order decodes every task of the block-major list
    exactly once, and groups of consecutive indices stay inside one group of
    row blocks, chunk by chunk."""
    listed = P.pairs_debug_task_ranges(n, K, U).astype(np.int64)
    total = len(listed)
    got = P.pairs_debug_task_at(n, K, U, np.arange(total))
    key = lambda t: sorted(map(tuple, t.tolist()))
    assert key(got) == key(listed)
    rows = 64 * K
    nblocks = -(-n // rows)
    nchunks = total // nblocks
    assert nblocks * nchunks == total
    for b in sorted({0, nblocks // 2, nblocks - 1}):
        t = P.pairs_debug_task_at(n, K, U, grouped_indices(nblocks, nchunks, b))
        np.testing.assert_array_equal(t, listed[b * nchunks:(b + 1) * nchunks])


@pytest.mark.parametrize("n", [2 ** 27, 2 ** 27 + 1, 2 ** 30 - 1, 2 ** 30])
@pytest.mark.parametrize("K,U", [(8, 1024), (1, 64)])
def test_task_decode_at_the_size_limit(n, K, U):
    """Row blocks at both ends and around the wrap of a set too large to list:
    the chunks of each block tile its virtual partners [ra+1, rlast +
    steps(rlast)] exactly, in 32-bit indices."""
    rows = 64 * K
    nblocks = -(-n // rows)
    span = min(rows, n) - 1 + steps(n, 0)
    nchunks = -(-span // U)
    picks = sorted(set([0, 1, nblocks // 2 - 1, nblocks // 2, nblocks // 2 + 1, nblocks - 2,
                        nblocks - 1]))
    for b in picks:
        if K == 1 and b not in (0, nblocks - 1):
            continue   # 2^23 chunks per block at K = 1: the two ends suffice
        t = P.pairs_debug_task_at(n, K, U, grouped_indices(nblocks, nchunks, b))
        ra = b * rows
        rlast = min(ra + rows, n) - 1
        uend = rlast + steps(n, rlast) + 1
        assert np.all(t[:, 0] == ra)
        live = t[t[:, 1] < t[:, 2]]
        assert live[0, 1] == ra + 1 and live[-1, 2] == uend, (n, b)
        assert np.all(live[1:, 1] == live[:-1, 2])         # contiguous, disjoint
        assert np.all(live[:, 2] - live[:, 1] <= U)
        assert int(t[:, 1:].max()) < 2 ** 31 and uend <= 2 * n
    with pytest.raises(P.PairsError):
        P.pairs_debug_task_at(n, K, U, [nblocks * nchunks])
