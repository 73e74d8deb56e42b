"""Write tests/golden/workload_values.json: expected results of the full-size
workloads, computed by the CPU oracle only (oracle/) on inputs from workloads/.

    python tests/golden/make_golden.py [--threads T] [--only KEY ...]

The two sets of about 2^20 spheres (5.5e11 pair tests each) take tens of
minutes on 8 cores; the others take seconds to minutes.  Existing keys are kept
unless recomputed.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as w  # noqa: E402

OUT = os.path.join(HERE, "workload_values.json")
FORCE_ROWS = [0, 1, 4096, 65535, 131072, 200000, 262142, 262143]
# the 2^18 particles' per-particle energies: both ends, around n/2, and 56 seeded rows
ENERGY_ROWS = sorted(set([0, 1, 131071, 131072, 262142, 262143] +
                         np.random.default_rng(33).integers(0, 2 ** 18, 58).tolist()))


def compute(key, threads):
    if key == "spheres_4096_count":
        return oracle.count_i32(*w.spheres_4096().arrays(), threads=threads)
    if key == "spheres_2p20_count":
        return oracle.count_i32(*w.spheres_2p24(2 ** 20).arrays(), threads=threads)
    if key == "spheres_2p20m1_count":
        return oracle.count_i32(*w.spheres_2p24(2 ** 20 - 1).arrays(), threads=threads)
    if key == "particles_2p18_energy_total":
        return oracle.energy_total(*w.particles_unit_cube().arrays(), np.float32(1e-4), threads=threads)
    if key == "binned_sets_200k_counts":
        b = w.binned_sets()
        c = oracle.count_i32_batched(*b.objs.arrays(), b.offsets, threads=threads)
        return {"total": int(c.sum()),
                "sha256_le_u64": hashlib.sha256(c.astype("<u8").tobytes()).hexdigest(),
                "first16": [int(v) for v in c[:16]]}
    if key == "particles_2p18_energy_rows":
        rows = np.array(ENERGY_ROWS, np.int64)
        E = oracle.energy_rows(*w.particles_unit_cube().arrays(), np.float32(1e-4), rows=rows,
                               threads=threads)
        return {"rows": ENERGY_ROWS, "E": E.tolist()}
    if key == "moving_sets_50k_sampled":
        # 24 seeded sets of the 50 000 moving sets, jittered by the oracle through 100 steps
        # (seed 6, sigma 1e-3); per-set energy and pinned-float32 count after
        # steps 0, 49 and 99
        b = w.moving_sets()
        x, y, z, r = b.objs.arrays()
        sets = sorted(np.random.default_rng(55).choice(b.n_sets, 24, replace=False).tolist())
        out = {"sets": sets, "steps": [0, 49, 99], "energy": [], "count": []}
        for st in sets:
            a, e = int(b.offsets[st]), int(b.offsets[st + 1])
            px, py, pz = x[a:e].copy(), y[a:e].copy(), z[a:e].copy()
            en, cn = [], []
            for k in range(100):
                px, py, pz = oracle.jitter_f32(px, py, pz, 6, k, 1e-3, first_index=a)
                if k in (0, 49, 99):
                    en.append(oracle.energy_total(px, py, pz, np.float32(1e-4), threads=threads))
                    cn.append(oracle.count_f32(px, py, pz, r[a:e], threads=threads))
            out["energy"].append(en)
            out["count"].append(cn)
        return out
    if key == "particles_2p18_force_rows":
        rows = np.array(FORCE_ROWS, np.int64)
        F, S = oracle.force_rows(*w.particles_unit_cube().arrays(), np.float32(1e-4), rows=rows,
                                 threads=threads)
        return {"rows": FORCE_ROWS, "F": F.tolist(), "S": S.tolist()}
    if key in ("lattice_paper_counts", "lattice_large_counts", "lattice_short_counts"):
        b = {"lattice_paper_counts": w.lattice_paper, "lattice_large_counts": w.lattice_large,
             "lattice_short_counts": w.lattice_short}[key]()
        coll, cont = oracle.lattice_counts_batched(*b.objs.arrays(), b.offsets, threads=threads)
        return {"collisions_total": int(coll.sum()), "contacts_total": int(cont.sum()),
                "collisions_sha256_le_u64": hashlib.sha256(coll.astype("<u8").tobytes()).hexdigest(),
                "contacts_sha256_le_u64": hashlib.sha256(cont.astype("<u8").tobytes()).hexdigest(),
                "first8": [[int(a), int(c)] for a, c in zip(coll[:8], cont[:8])]}
    raise KeyError(key)


KEYS = ["spheres_4096_count", "binned_sets_200k_counts", "particles_2p18_energy_total", "spheres_2p20m1_count",
        "spheres_2p20_count", "lattice_paper_counts", "lattice_large_counts",
        "particles_2p18_force_rows", "lattice_short_counts", "particles_2p18_energy_rows",
        "moving_sets_50k_sampled"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", nargs="*", default=None)
    a = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.setdefault("_about", "Expected values of the full-size workloads, written by "
                    "tests/golden/make_golden.py from the CPU oracle only.")
    for key in (a.only or KEYS):
        t = time.time()
        data[key] = compute(key, a.threads)
        print(f"{key}: {data[key]}  ({time.time() - t:.1f} s, "
              f"{oracle.threads(a.threads)} threads)", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
