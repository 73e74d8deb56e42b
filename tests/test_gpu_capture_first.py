"""The library's first call in a process made inside a HIP graph capture.

The unplanned batched count and the lattice count look up per-device state
(a status word in the library's own device memory and the CU count) on their
first call on a device.  That set-up allocates nothing and makes no stream
operation, so it may happen inside a capture: the captured graph is then
replayed, with eager work in between, and every replay is checked against the
CPU oracle.  The calls run in a fresh Python process so that they are really
the first ones."""
import os
import subprocess
import sys

import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import numpy as np
import torch

import oracle
import paper_1901_11204_amd as P
import workloads as w

kind = sys.argv[1]
torch.cuda.set_device(0)
if kind == "batched":
    rng = np.random.default_rng(3)
    sizes = np.concatenate([[0, 1, 2, 700], rng.integers(2, 300, 60)])
    off = w.offsets_from_sizes(sizes)
    n = int(off[-1])
    arrays = w.spheres_i32(n, 4, 64, 6, radius_lo=0).arrays()
    want = oracle.count_i32_batched(*arrays, off)
    t = [torch.from_numpy(a).cuda() for a in arrays]
    d_off = torch.from_numpy(off).cuda()
    out = torch.full((len(sizes),), -1, dtype=torch.int64, device="cuda")
    ws = torch.empty(P.pairs_batched_workspace_size(len(sizes), n), dtype=torch.uint8,
                     device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.pairs_count_i32_batched(*t, d_off, out, ws=ws)
    check = lambda: np.array_equal(out.cpu().numpy().astype(np.uint64), want.astype(np.uint64))
else:
    b = w.lattice_walks(12, 500, 5)
    arrays = b.objs.arrays()[:3]
    want = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets)
    t = [torch.from_numpy(a).cuda() for a in arrays]
    d_off = torch.from_numpy(b.offsets).cuda()
    coll = torch.full((12,), -1, dtype=torch.int64, device="cuda")
    cont = torch.full((12,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.pairs_lattice_count_batched(*t, d_off, 500, coll, cont)
    check = lambda: (np.array_equal(coll.cpu().numpy(), want[0].astype(np.int64)) and
                     np.array_equal(cont.cpu().numpy(), want[1].astype(np.int64)))
ok = []
for rep in range(3):
    g.replay()
    torch.cuda.synchronize()
    ok.append(bool(check()))
    # eager work between replays
    junk = torch.randn(1 << 20, device="cuda") * 2
    torch.cuda.synchronize()
print("REPLAYS", ok, flush=True)
sys.exit(0 if all(ok) else 1)
""".replace("ROOT", repr(ROOT))


@pytest.mark.parametrize("kind", ["batched", "lattice"])
def test_first_call_inside_a_capture(kind):
    announce("first library call inside a graph capture", kind)
    r = subprocess.run([sys.executable, "-c", SCRIPT, kind], capture_output=True, text=True,
                       timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "REPLAYS [True, True, True]" in r.stdout
