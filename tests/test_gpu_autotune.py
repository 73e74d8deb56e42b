"""The tile-shape autotuner on the GPU: tuning a small batch and small
single sets over a few candidates, saving the cache, reloading it both
in-process and through the binding's load path in a fresh process
(PAIRS_TUNE_CACHE), with the tuned shapes' results checked against the CPU
oracle.  Shapes change only the speed, never a result."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import paper_1901_11204_amd as P
import workloads as w
from gpu_util import announce, dev
from paper_1901_11204_amd import autotune as A

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def restore_shapes():
    yield
    for kind in (P.KIND_COUNT_I32, P.KIND_COUNT_F32, P.KIND_ENERGY_F32):
        for batched in (False, True):
            P.pairs_set_shapes(kind, batched, None)


def test_tune_batched_save_and_reload(tmp_path, restore_shapes):
    import torch
    b = w.binned_sets(n_sets=600, seed=51)
    ins = tuple(dev(*b.objs.arrays()))
    out = torch.empty(b.n_sets, dtype=torch.int64, device="cuda")
    shapes = [(2, 272, P.FORM_STEPPING), (1, 288, P.FORM_STEPPING), (4, 512, P.FORM_BROADCAST)]
    announce("autotune tune_batched, 600 sets, 3 candidates")
    log = []
    table, ms = A.tune_batched(P.KIND_COUNT_I32, b.offsets, ins, (out,), shapes=shapes,
                               log=log.append)
    assert ms > 0 and len(table) == len(P.pairs_get_shapes(P.KIND_COUNT_I32, True))
    assert [tuple(e) for e in P.pairs_get_shapes(P.KIND_COUNT_I32, True)] == \
        [tuple(e) for e in table]
    # the tuned table gives the oracle's counts, planned and unplanned
    want = oracle.count_i32_batched(*b.objs.arrays(), b.offsets)
    plan = P.Plan(P.KIND_COUNT_I32, b.offsets)
    plan.execute(ins, (out,))
    torch.cuda.synchronize()
    plan.close()
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.uint64), want)
    P.pairs_count_i32_batched(*ins, *dev(b.offsets), out)
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.uint64), want)

    path = str(tmp_path / "cache.json")
    A.save_cache(path, P.KIND_COUNT_I32, True, table, "600 binned sets", ms)
    data = json.load(open(path))
    key = f"{A.arch()}/count_i32/batched"
    assert [tuple(e) for e in data["tables"][key]["table"]] == [tuple(e) for e in table]

    # in-process reload over the defaults
    P.pairs_set_shapes(P.KIND_COUNT_I32, True, None)
    A.load_cache(path, apply=True)
    assert [tuple(e) for e in P.pairs_get_shapes(P.KIND_COUNT_I32, True)] == \
        [tuple(e) for e in table]

    # a fresh process applies the cache when the library loads
    code = ("import sys, json; sys.path.insert(0, %r); import torch; "
            "import paper_1901_11204_amd as P; P.lib(); "
            "print('TABLE', json.dumps(P.pairs_get_shapes(P.KIND_COUNT_I32, True)))" % ROOT)
    env = dict(os.environ, PAIRS_TUNE_CACHE=path)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("TABLE ")][0]
    assert [tuple(e) for e in json.loads(line[6:])] == [tuple(e) for e in table]


def test_tune_single_and_boundaries(tmp_path, restore_shapes):
    sizes = [3000, 700]
    arrays = {n: w.spheres_i32(n, 60 + n, 48, 6, radius_lo=0).arrays() for n in sizes}
    t = {n: dev(*arrays[n]) for n in sizes}
    announce("autotune tune_single, 2 sizes x 4 shapes")
    table, times = A.tune_single(P.KIND_COUNT_I32, sizes, lambda n: (lambda: P.count_i32(*t[n])),
                                 rows=(1, 4), chunks=(128, 256), log=lambda *m: None)
    assert [e[0] for e in table] == [700, 0] and len(times) == 2
    for n in sizes:
        assert P.count_i32(*t[n]) == oracle.count_i32(*arrays[n])
    # boundary candidates keep the bounds strictly decreasing
    tab = [(4096, 2, 272, 1), (1024, 2, 272, 1), (256, 2, 272, 1), (0, 2, 272, 1)]
    for c in range(3):
        for lo in A.boundary_candidates(tab, c):
            cand = list(tab)
            cand[c] = (lo,) + tab[c][1:]
            bounds = [e[0] for e in cand]
            assert all(a > b for a, b in zip(bounds, bounds[1:]))
