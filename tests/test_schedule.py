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
