"""GPU float32 counts on pairs at the touching distance, against the exact
rational model of the pinned binary32 sequence (tests/f32_exact.py), which
shares nothing with the oracle or the kernels.  Every pair is one where a
plain-product chain, a reordered fused chain, exact arithmetic or flushed
subnormals would give the other answer."""
import numpy as np
import pytest

import paper_1901_11204_amd as P
from f32_exact import discriminating_pairs
from gpu_util import announce, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pairs():
    a = discriminating_pairs(6000, seed=11)
    b = discriminating_pairs(600, seed=12, scale=1e-20)
    pi = np.concatenate([a[0], b[0]])
    pj = np.concatenate([a[1], b[1]])
    hits = np.concatenate([a[2], b[2]])
    return pi, pj, hits


def batch_of_pairs(pi, pj):
    """Each pair as a set of two objects (CSR), so no pair meets another."""
    m = len(pi)
    obj = np.empty((2 * m, 4), np.float32)
    obj[0::2] = pi
    obj[1::2] = pj
    off = np.arange(0, 2 * m + 1, 2, dtype=np.int64)
    return [np.ascontiguousarray(obj[:, a]) for a in range(4)], off


@pytest.mark.parametrize("planned", [False, True])
def test_batched_count_f32_pinned_pairs(pairs, planned):
    import torch
    pi, pj, hits = pairs
    arrs, off = batch_of_pairs(pi, pj)
    announce("count_f32 pinned pairs batched", planned, len(hits))
    t = dev(*arrs)
    counts = torch.empty(len(hits), dtype=torch.int64, device="cuda")
    if planned:
        plan = P.Plan(P.KIND_COUNT_F32, off)
        plan.execute(t, (counts,))
        torch.cuda.synchronize()
        plan.close()
    else:
        (toff,) = dev(off)
        P.pairs_count_f32_batched(*t, toff, counts)
    np.testing.assert_array_equal(counts.cpu().numpy(), hits.astype(np.int64))


def test_energy_count_f32_pinned_pairs(pairs):
    # the fused energy + count kernel evaluates the same pinned predicate
    import torch
    pi, pj, hits = pairs
    arrs, off = batch_of_pairs(pi, pj)
    announce("energy_count_f32 pinned pairs batched", len(hits))
    t = dev(*arrs)
    (toff,) = dev(off)
    E = torch.empty(len(hits), dtype=torch.float64, device="cuda")
    C = torch.empty(len(hits), dtype=torch.int64, device="cuda")
    P.pairs_energy_f32_batched(*t, toff, 1e-4, E, C)
    np.testing.assert_array_equal(C.cpu().numpy(), hits.astype(np.int64))


def test_single_set_count_f32_pinned_pairs(pairs):
    pi, pj, hits = pairs
    announce("count_f32 pinned pairs single-set", len(hits))
    for k in range(len(hits)):
        for a, b in ((pi[k], pj[k]), (pj[k], pi[k])):
            t = dev(*(np.array([a[c], b[c]], np.float32) for c in range(4)))
            assert P.count_f32(*t) == int(hits[k]), k
