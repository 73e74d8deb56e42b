"""pairs_count_i32_batched_noalloc, the batched count whose workspace is the
library's static device scratch (for callers that cannot allocate), against
pairs_count_i32_batched with a caller workspace and against the CPU oracle:
two calls in a row, the second with a smaller batch, so the second runs on
the scratch the first left behind."""
import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu


def both(arrays, off):
    import torch
    t = dev(*arrays)
    (d_off,) = dev(off)
    n_sets = len(off) - 1
    ref = torch.full((n_sets,), -1, dtype=torch.int64, device="cuda")
    got = torch.full((n_sets,), -2, dtype=torch.int64, device="cuda")
    P.pairs_count_i32_batched(*t, d_off, ref)
    P.pairs_count_i32_batched_noalloc(*t, d_off, got)
    torch.cuda.synchronize()
    return got.cpu().numpy().astype(np.uint64), ref.cpu().numpy().astype(np.uint64)


def test_noalloc_two_calls_second_smaller():
    big = w.binned_sets(n_sets=20_000, seed=31)
    announce("noalloc batched count, 20000 sets")
    got, ref = both(big.objs.arrays(), big.offsets)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got, oracle.count_i32_batched(*big.objs.arrays(), big.offsets))

    sizes = np.array([0, 1, 2, 3, 64, 65, 300, 2000, 5, 0], np.int64)
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(int(off[-1]), 32, 48, 5, radius_lo=0)
    announce("noalloc batched count, 10 sets after 20000")
    got, ref = both(s.arrays(), off)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got, oracle.count_i32_batched(*s.arrays(), off))


def test_noalloc_limit():
    import torch
    n_sets = P.NOALLOC_MAX_SETS
    sizes = np.full(n_sets, 2, np.int64)
    sizes[::7] = 3
    off = w.offsets_from_sizes(sizes)
    s = w.spheres_i32(int(off[-1]), 33, 16, 3, radius_lo=0)
    announce("noalloc batched count at the set limit", n_sets)
    got, ref = both(s.arrays(), off)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got, oracle.count_i32_batched(*s.arrays(), off))
    # one set more is refused before anything is enqueued
    off2 = w.offsets_from_sizes(np.full(n_sets + 1, 2, np.int64))
    s2 = w.spheres_i32(int(off2[-1]), 34, 16, 3)
    counts = torch.full((n_sets + 1,), 7, dtype=torch.int64, device="cuda")
    with pytest.raises(P.PairsError) as e:
        P.pairs_count_i32_batched_noalloc(*dev(*s2.arrays()), *dev(off2), counts)
    assert e.value.status == -5
    torch.cuda.synchronize()
    assert int(counts.min()) == 7 and int(counts.max()) == 7
