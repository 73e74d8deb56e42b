"""Tile-shape autotuner.

The kernels tile each set into wave tasks of 64*K rows against chunks of U
virtual partners; the best (K, U) depends on the set sizes (small sets waste
lanes on the two band edges of a row block, large K amortises the partner
staging over more rows).  Shapes are chosen per size class (include/pairs.h,
pairs_shape_table_t).  This module times candidate tables on a workload, keeps
the fastest, and stores the choices in a JSON cache keyed by device
architecture, kind and mode:

    python -m paper_1901_11204_amd.autotune --workload binned-int32 --out cache.json

The binding applies a cache at load time when PAIRS_TUNE_CACHE names one, or
when tuned_shapes.json exists next to this file.  Results never depend on the
shapes, only the speed does.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import (FORM_BROADCAST, FORM_MATRIX, FORM_STEPPING, KIND_COUNT_F32, KIND_COUNT_I32,
               KIND_ENERGY_F32, SHAPES_BATCHED, SHAPES_SINGLE, SHAPES_TOTAL_ONLY, Plan,
               pairs_get_shapes, pairs_set_shapes)

ROWS = (1, 2, 4, 8)
CHUNKS = (128, 256, 512, 1024, 2048, 4096, 8192)
# (rows per lane, step chunks) of the row-stepping form (batched tables only)
STEP_SHAPES = ((1, (64, 128, 192, 288)), (2, (48, 96, 144, 208, 272)))
# chunks of the matrix-core form (single-set int32 counts only)
MATRIX_CHUNKS = (1024, 4096)


def candidates(batched: bool):
    """Every (K, U, form) the tuner tries for one size class."""
    out = [(k, u, FORM_BROADCAST) for k in ROWS for u in CHUNKS]
    if batched:
        out += [(k, u, FORM_STEPPING) for k, us in STEP_SHAPES for u in us]
    return out
KIND_NAMES = {KIND_COUNT_I32: "count_i32", KIND_COUNT_F32: "count_f32",
              KIND_ENERGY_F32: "energy_f32"}
MODE_NAMES = {SHAPES_SINGLE: "single", SHAPES_BATCHED: "batched", SHAPES_TOTAL_ONLY: "total_only"}
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")


def arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _time(fn, reps: int = 3, warmup_s: float = 0.25) -> float:
    """Mean milliseconds of `reps` back-to-back calls, after about warmup_s
    seconds of calls: the engine clock of an idle GPU takes that long to
    reach its running speed, and millisecond-scale calls timed straight
    after an idle spell read up to 15 % slow."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = time.perf_counter() - t0
    for _ in range(max(0, min(400, int(warmup_s / max(one, 1e-5))) - 1)):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def time_batched(kind, table, offsets, inputs, outputs, eps2=1e-4, reps=10) -> float:
    """Milliseconds of one plan execution of the batch under `table`."""
    pairs_set_shapes(kind, True, table)
    plan = Plan(kind, offsets)
    try:
        return _time(lambda: plan.execute(inputs, outputs, eps2), reps)
    finally:
        plan.close()


def _entry(e):
    e = tuple(int(v) for v in e)
    return e if len(e) == 4 else e + (FORM_BROADCAST,)


def boundary_candidates(table, c):
    """Lower bounds the tuner tries for class c (c >= 0 and not the last
    class): halving and doubling steps of the current bound that keep the
    bounds strictly decreasing."""
    lo = table[c][0]
    upper = table[c - 1][0] if c > 0 else None
    lower = table[c + 1][0] if c + 1 < len(table) else -1
    out = []
    for f in (0.25, 0.5, 2.0, 4.0):
        v = int(lo * f)
        if v > lower and (upper is None or v < upper) and v != lo and v > 0:
            out.append(v)
    return out


def tune_batched(kind, offsets, inputs, outputs, eps2=1e-4, start=None, rounds=1, log=print,
                 shapes=None, boundaries=True, trace=None):
    """Coordinate descent over the (K, U, form) of each size class of a batch,
    largest class first, then over the class boundaries (min_n of every class
    but the last).  shapes: the (K, U, form) candidates (default: all)."""
    table = [_entry(e) for e in (start or pairs_get_shapes(kind, True))]
    best = time_batched(kind, table, offsets, inputs, outputs, eps2)
    log(f"start {table}: {best:.3f} ms")
    shapes = list(shapes) if shapes is not None else candidates(True)
    for _ in range(rounds):
        for c in range(len(table)):
            for k, u, form in shapes:
                if (k, u, form) == table[c][1:]:
                    continue
                cand = list(table)
                cand[c] = (table[c][0], k, u, form)
                ms = time_batched(kind, cand, offsets, inputs, outputs, eps2)
                if trace:
                    trace(f"    class {c} K={k} U={u} form={form}: {ms:.3f} ms")
                if ms < best:
                    best, table = ms, cand
                    log(f"  class {c} -> K={k} U={u} form={form}: {ms:.3f} ms")
        if boundaries:
            for c in range(len(table) - 1):
                for lo in boundary_candidates(table, c):
                    cand = list(table)
                    cand[c] = (lo,) + tuple(table[c][1:])
                    ms = time_batched(kind, cand, offsets, inputs, outputs, eps2)
                    if trace:
                        trace(f"    class {c} min_n={lo}: {ms:.3f} ms")
                    if ms < best:
                        best, table = ms, cand
                        log(f"  class {c} -> min_n={lo}: {ms:.3f} ms")
    pairs_set_shapes(kind, True, table)
    return table, best


def single_candidates(kind, rows=ROWS, chunks=CHUNKS):
    """Every (K, U, form) the tuner tries for one size class of single sets."""
    out = [(k, u, FORM_BROADCAST) for k in rows for u in chunks]
    if kind == KIND_COUNT_I32:
        out += [(1, u, FORM_MATRIX) for u in MATRIX_CHUNKS]
    return out


def tune_single(kind, n_values, make_call, start=None, log=print, rows=ROWS, chunks=CHUNKS,
                trace=None, mode=SHAPES_SINGLE):
    """For each size n (largest first) pick the (K, U, form) with the fastest
    single-set call; make_call(n) returns a zero-argument callable.  mode:
    SHAPES_SINGLE, or SHAPES_TOTAL_ONLY for float32 energies without
    per-object output.  Returns the table and the best time of each size."""
    entries, times = [], []
    ns = sorted(n_values, reverse=True)
    if not 1 <= len(ns) <= 4:
        raise ValueError("tune_single takes 1 to 4 sizes, one per size class")
    for i, n in enumerate(ns):
        call = make_call(n)
        best = None
        lo = ns[i + 1] if i + 1 < len(ns) else 0
        for k, u, form in single_candidates(kind, rows, chunks):
            pairs_set_shapes(kind, mode, entries + [(lo, k, u, form)])
            ms = _time(call)
            if trace:
                trace(f"    n={n} K={k} U={u} form={form}: {ms:.3f} ms")
            if best is None or ms < best[0]:
                best = (ms, k, u, form)
        entries.append((lo,) + best[1:])
        times.append(best[0])
        log(f"n={n}: K={best[1]} U={best[2]} form={best[3]} {best[0]:.3f} ms")
    pairs_set_shapes(kind, mode, entries)
    return entries, times


def load_cache(path=None, apply=True):
    """Read a cache and apply the entries that match this device."""
    path = path or os.environ.get("PAIRS_TUNE_CACHE") or DEFAULT_CACHE
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if apply:
        try:
            a = arch()
        except Exception:
            return data
        for key, entry in data.get("tables", {}).items():
            d_arch, kind_name, mode = key.split("/")
            if d_arch != a:
                continue
            kind = {v: k for k, v in KIND_NAMES.items()}[kind_name]
            mode = {v: k for k, v in MODE_NAMES.items()}[mode]
            pairs_set_shapes(kind, mode, [_entry(e) for e in entry["table"]])
    return data


def save_cache(path, kind, batched, table, note, ms):
    """Store a table under arch/kind/mode; batched: False/True or a SHAPES_* mode."""
    data = {"tables": {}}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    mode = int(batched)
    key = f"{arch()}/{KIND_NAMES[kind]}/{MODE_NAMES[mode]}"
    data.setdefault("tables", {})[key] = {"table": [list(e) for e in table], "workload": note,
                                          "ms": ms, "when": time.strftime("%Y-%m-%d")}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


def main(argv=None):
    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as w

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["binned-int32", "particles-f32", "single-int32",
                                           "single-energy", "single-energy-total"],
                    default="binned-int32")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--rounds", type=int, default=1)
    ap.add_argument("--sizes", default="1048576,262144,16384,4096",
                    help="single-set workloads: the set sizes tuned, one per class (at most 4)")
    ap.add_argument("--verbose", action="store_true", help="print every candidate's time")
    a = ap.parse_args(argv)
    say = lambda *m: print(*m, flush=True)
    trace = say if a.verbose else None
    dev = torch.device("cuda", 0)
    if a.workload.startswith("single"):
        from . import count_i32, energy_f32
        ns = [int(v) for v in a.sizes.split(",")]
        mode = SHAPES_SINGLE
        if a.workload == "single-int32":
            kind, note = KIND_COUNT_I32, "single int32 sets, centres in [0,2^24)^3, radii [1,2^14]"

            def make_call(n):
                t = [torch.from_numpy(v).to(dev) for v in w.spheres_i32(n, 2, 2 ** 24,
                                                                          2 ** 14).arrays()]
                return lambda: count_i32(*t)
        elif a.workload == "single-energy":
            kind, note = KIND_ENERGY_F32, "single float32 particle sets in the unit cube"

            def make_call(n):
                t = [torch.from_numpy(v).to(dev) for v in w.particles_f32(n, 4).arrays()]
                return lambda: energy_f32(*t)
        else:
            kind, mode = KIND_ENERGY_F32, SHAPES_TOTAL_ONLY
            note = "single float32 particle sets in the unit cube, total only"

            def make_call(n):
                t = [torch.from_numpy(v).to(dev) for v in w.particles_f32(n, 4).arrays()]
                return lambda: energy_f32(*t, per_particle=False)
        table, times = tune_single(kind, ns, make_call, log=say, trace=trace, mode=mode)
        save_cache(a.out, kind, mode, table, note + f"; sizes {ns}", times)
        print(json.dumps({"kind": KIND_NAMES[kind], "table": table, "ms": times}), flush=True)
        return 0
    if a.workload == "binned-int32":
        b = w.binned_sets()
        ins = tuple(torch.from_numpy(v).to(dev) for v in b.objs.arrays())
        outs = (torch.empty(b.n_sets, dtype=torch.int64, device=dev),)
        kind, note = KIND_COUNT_I32, "200000 binned int32 sets, lognormal(4,1.2) sizes, seed 5"
    else:
        b = w.moving_sets()
        ins = tuple(torch.from_numpy(v).to(dev) for v in b.objs.arrays())
        outs = (torch.empty(b.n_sets, dtype=torch.float64, device=dev),
                torch.empty(b.n_sets, dtype=torch.int64, device=dev))
        kind, note = KIND_ENERGY_F32, "50000 float32 sets, lognormal(5,1) sizes, seed 6, r=0.01"
    table, ms = tune_batched(kind, b.offsets, ins, outs, rounds=a.rounds, log=say, trace=trace)
    save_cache(a.out, kind, True, table, note, ms)
    print(json.dumps({"kind": KIND_NAMES[kind], "table": table, "ms": ms}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
