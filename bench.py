"""Benchmark of the balanced all-pairs collision count on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step is one call of the hot path on the headline workload: the exact
collision count of one set of N = 2^20 int32 spheres (centres uniform in
[0, 2^24)^3, radii uniform in [1, 2^14], seed 2), 549 755 289 600 pair tests,
inputs resident in device memory.  The timed region is bracketed by stream
synchronisation; per-step durations come from HIP events recorded on the
stream the kernels run on.  Prints one JSON line.

Secondary lines of the same run (odd N, the float32 energy, the small set) are
reported under "secondary"; the CPU oracle timed on a bounded sample of the
same workload is reported under "cpu_baseline".
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs, 64 lanes per CU per cycle of VALU issue, 2.4 GHz peak engine clock
N_CU = 256
VALU_LANES_PER_CU = 64
SCLK_HZ = 2.4e9
VALU_PEAK = N_CU * VALU_LANES_PER_CU * SCLK_HZ          # lane-operations per second
# Algorithmic VALU work per pair test of each kernel (lane-operations):
#   exact int32 count, Gram form: 4 32x32->64-bit multiply-adds + 1 compare
#   float32 energy with per-object sums: 3 sub + 3 fma + 2 adds (the total
#     alone: 1 add); the reciprocal square root issues to the separate
#     transcendental pipe and takes no VALU slot (total-only energy runs
#     above the VALU bound that a slot for it would impose)
#   float32 energy with the pinned collision count: 3 sub + 1 mul + 2 fma
#     (pinned squared distance) + add, mul, compare (radius test) + add
#     (softening) + add
C_ALG = {"count_i32": 5, "energy_f32": 8, "energy_total_f32": 7, "energy_count_f32": 11,
         "force_f32": 18, "energy_f64": 13}
PLAIN_DEF_OPS = 12   # operations of the plain definition per pair (either kind)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "count_i32_n2p20_hbm.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1901_11204_amd", "csrc", f)
                  for f in ("band.h", "device.h", "tasks.h", "steps.h", "pairs.hip")]


def recorded_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a device copy), or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        fields = {}
        with open(TRAFFIC_PROFILE) as f:
            for line in f:
                k, _, v = line.partition(":")
                if k.strip() in ("traffic_bytes_per_launch", "kernel_sources_sha256"):
                    fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for p in KERNEL_SOURCES:
            with open(p, "rb") as f:
                h.update(f.read())
        if fields.get("kernel_sources_sha256") != h.hexdigest():
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


GOLDEN = os.path.join(ROOT, "tests", "golden", "workload_values.json")


def golden():
    """Expected values of the full-size workloads, written by the CPU oracle
    (tests/golden/make_golden.py)."""
    with open(GOLDEN) as f:
        return json.load(f)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class SclkSampler:
    """Engine clock (MHz) while a region runs, read every few ms from the
    amdgpu driver's sysfs table (the current level is the one marked '*');
    None where the system does not expose it."""

    def __init__(self, period_s=0.002):
        import glob
        self.paths = [q for q in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
                      if os.access(q, os.R_OK)]
        self.period = period_s
        self.samples = []

    def _read(self):
        for q in self.paths:
            try:
                for line in open(q).read().splitlines():
                    if line.strip().endswith("*"):
                        return float(line.split(":")[1].strip().rstrip("*").strip().lower()
                                     .replace("mhz", ""))
            except (OSError, ValueError, IndexError):
                continue
        return None

    def __enter__(self):
        import threading
        self.stop = threading.Event()

        def run():
            while not self.stop.is_set():
                v = self._read()
                if v is not None:
                    self.samples.append(v)
                time.sleep(self.period)
        self.thread = threading.Thread(target=run, daemon=True)
        if self.paths:
            self.thread.start()
        return self

    def __exit__(self, *exc):
        self.stop.set()
        if self.paths:
            self.thread.join()

    def mean_mhz(self):
        """The mean of samples taken at a fixed period: the time average of a
        clock that moves between levels while the region runs."""
        return sum(self.samples) / len(self.samples) if self.samples else None


def timed_steps(fn, steps, warmup, sampler=None):
    """Milliseconds of each of `steps` calls after `warmup` untimed ones; a
    SclkSampler given as `sampler` reads the clock over the timed calls only
    (the first calls after an idle spell run while the clock ramps up)."""
    import contextlib
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    with sampler if sampler is not None else contextlib.nullcontext():
        t0 = time.perf_counter()
        for k in range(steps):
            starts[k].record()
            fn()
            ends[k].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return ms, wall


def sclk_during(fn, seconds=0.25):
    """Engine clock (MHz) while fn runs back to back for about `seconds`
    (None where the clock is not exposed): the VALU fraction of a kernel at
    the clock it actually ran at.  Run before a line's timed steps, it is
    also their warm-up: a millisecond-scale call timed after two warm-up
    calls reads up to a tenth slower than in steady state."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    reps = max(1, int(seconds / max(time.perf_counter() - t0, 1e-5)))
    with SclkSampler() as sclk:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    return sclk.mean_mhz()


def at_sclk(frac, mhz):
    """A VALU fraction of the nominal 2.4 GHz peak restated at a measured clock."""
    return frac * SCLK_HZ / (mhz * 1e6) if mhz else None


def valu_probe(torch):
    """Lane-operations per second of each probe pattern, as a fraction of the
    256 CU x 64 lane x 2.4 GHz issue peak."""
    import ctypes
    from paper_1901_11204_amd import build as B
    L = ctypes.CDLL(B.PROBE_LIB)
    L.valu_probe_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
    names = ctypes.c_char_p.in_dll(L, "valu_probe_names").value.decode().split(",")
    blocks = torch.cuda.get_device_properties(0).multi_processor_count * 16
    out = {"blocks": blocks, "threads_per_block": 256}
    for k, name in enumerate(names):
        ms, ops = ctypes.c_double(), ctypes.c_double()
        rc = L.valu_probe_run(k, blocks, ctypes.byref(ms), ctypes.byref(ops))
        if rc != 0:
            raise RuntimeError(f"valu probe {name}: hipError {rc}")
        rate = ops.value / (ms.value * 1e-3)
        if name.startswith("lds_"):
            # lane reads -> wave-wide reads per clock per CU, and bytes
            per_clk = rate / 64 / N_CU / SCLK_HZ
            width = 16 if "b128" in name else 4 if "b32" in name else 8
            out[name] = {"ms": ms.value, "wave_ops_per_clk_per_cu": per_clk,
                         "bytes_per_clk_per_cu": per_clk * 64 * width}
        else:
            out[name] = {"ms": ms.value, "T_lane_ops_per_s": rate / 1e12,
                         "frac_of_peak": rate / VALU_PEAK}
    return out


def cpu_baseline(sample_n):
    import oracle
    import workloads as w
    s = w.spheres_2p24(2 ** 20)
    arrs = [a[:sample_n].copy() for a in s.arrays()]
    threads = oracle.threads(0)
    t = time.perf_counter()
    oracle.count_i32(*arrs, threads=0)
    dt = time.perf_counter() - t
    pairs = sample_n * (sample_n - 1) // 2
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pairs / dt / 1e9, "unit": "G pair tests/s", "cores": threads,
            "kind": "oracle", "seconds": dt, "nproc": os.cpu_count(), "cpu_model": model,
            "sample": f"plain i<j loop over the first {sample_n} spheres of the N=2^20 "
                      f"set ({pairs} pair tests), {threads} OpenMP threads",
            "serial": cpu_serial(oracle, w)}


def cpu_serial(oracle, w):
    """One-thread oracle rates: the whole 4096-sphere set, and row slices of
    the 2^20 count and the 2^18 energy, extrapolated to the whole set by the
    pair count (every pair costs the same)."""
    import numpy as np
    out = {}
    a1 = w.spheres_4096().arrays()
    t = time.perf_counter()
    oracle.count_i32(*a1, threads=1)
    dt = time.perf_counter() - t
    p1 = 4096 * 4095 // 2
    out["count_i32_4096"] = {"seconds": dt, "G_pairs_per_s": p1 / dt / 1e9}
    s2 = w.spheres_2p24(2 ** 20).arrays()
    rows, cols = 2 ** 12, 2 ** 17
    a = [v[:rows].copy() for v in s2]
    b = [v[rows:rows + cols].copy() for v in s2]
    t = time.perf_counter()
    oracle.cross_count_i32(a, b, threads=1)
    dt = time.perf_counter() - t
    rate = rows * cols / dt
    p2 = 2 ** 20 * (2 ** 20 - 1) // 2
    out["count_i32_2^20"] = {"sample": f"{rows} rows x {cols} partners", "seconds": dt,
                             "G_pairs_per_s": rate / 1e9, "extrapolated_full_s": p2 / rate}
    x3, y3, z3 = w.particles_unit_cube().arrays()
    rows3 = 2 ** 8
    t = time.perf_counter()
    oracle.energy_rows(x3, y3, z3, np.float32(1e-4), np.arange(rows3), threads=1)
    dt = time.perf_counter() - t
    n3 = x3.shape[0]
    rate3 = rows3 * (n3 - 1) / dt
    out["energy_2^18"] = {"sample": f"E_i of {rows3} rows over all {n3 - 1} partners",
                          "seconds": dt, "G_pairs_per_s": rate3 / 1e9,
                          "extrapolated_full_s": n3 * (n3 - 1) // 2 / rate3}
    return out


# The paper's own GPU result for this path, quoted as context next to the
# MI355X numbers (its hardware, not a target): Section 5 reports the balanced
# assignment at least 12 % faster than the straightforward triangular
# parallelisation for every N above 525 000.
PAPER_CONTEXT = {
    "claim": "balanced circular assignment >= 1.12x the straightforward (triangular) "
             "GPU parallelisation for every N > 525000 (collision counting, spheres of "
             "diameter 1, 100 vectors per run)",
    "hardware": "NVIDIA Tesla P100 (56 SMs, 3584 CUDA cores, 16 GB)",
    "absolute_numbers": "none published (timings only in a figure)",
    "source": "paper, Section 5",
}


HBM_PEAK = 8.0e12  # bytes per second
LATTICE_BYTES_PER_BEAD = 12  # three int32 coordinates, read once


def bench_lattice(P, w, torch, np, dev, steps):
    """Lattice-bead collision and contact counts (Section 3): the paper's batch of
    1000 chains of 1920 beads, 65536 such chains for throughput, and 131072
    chains of 128 beads (the common protein length of its structure
    prediction runs).  The per-vector counts are checked against the oracle's
    stored values."""
    def sha(t):
        return hashlib.sha256(t.cpu().numpy().astype("<u8").tobytes()).hexdigest()

    out = {}
    for name, make, key, nsteps, maxn in [
            ("paper_1000x1920", w.lattice_paper, "lattice_paper_counts", 50, 1920),
            ("large_65536x1920", w.lattice_large, "lattice_large_counts", max(3, steps), 1920),
            ("short_131072x128", w.lattice_short, "lattice_short_counts", max(3, steps), 128)]:
        b = make()
        log(f"[bench] lattice {name}: {b.n_sets} chains, {b.n_total} beads")
        x, y, z = (torch.from_numpy(v).to(dev) for v in b.objs.arrays())
        off = torch.from_numpy(b.offsets).to(dev)
        coll = torch.empty(b.n_sets, dtype=torch.int64, device=dev)
        cont = torch.empty_like(coll)
        ms, _ = timed_steps(lambda: P.pairs_lattice_count_batched(x, y, z, off, maxn, coll, cont),
                            nsteps, 3)
        m = float(np.median(ms))
        ms1, _ = timed_steps(lambda: P.pairs_lattice_count_batched(x, y, z, off, maxn, coll, None),
                             nsteps, 3)
        P.pairs_lattice_count_batched(x, y, z, off, maxn, coll, cont)
        g = golden()[key]
        beads = b.n_total
        gbs = beads * LATTICE_BYTES_PER_BEAD / (m * 1e-3)
        out[name] = {
            "workload": f"{b.n_sets} random chains of {maxn} beads (unit steps from the origin on Z^3)",
            "beads": beads, "ms": m, "G_beads_per_s": beads / m / 1e6,
            "ms_collisions_only": float(np.median(ms1)),
            "roofline": {"bound": "hbm", "achieved": gbs / 1e9, "peak": HBM_PEAK / 1e9,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK,
                         "bytes_per_bead": LATTICE_BYTES_PER_BEAD},
            "collisions_total": int(coll.sum().item()), "contacts_total": int(cont.sum().item()),
            "matches_oracle": sha(coll) == g["collisions_sha256_le_u64"]
                              and sha(cont) == g["contacts_sha256_le_u64"]}
        del x, y, z, off, coll, cont
    return out


def graph_per_call(torch, P, t, out, calls):
    """Per-call time of the small-set count when `calls` calls are captured in
    one HIP graph (the calls allocate nothing and synchronise nothing)."""
    import numpy as np
    want = int(out.item())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.pairs_count_i32(*t, out)  # warm-up on the capturing stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(calls):
            P.pairs_count_i32(*t, out)
    ms, _ = timed_steps(lambda: g.replay(), 3, 1)
    if int(out.item()) != want:
        raise RuntimeError("graph replay changed the count")
    return {"us_per_call": float(np.mean(ms)) * 1e3 / calls, "calls": calls}


def assignment_comparison(torch, x, y, z, r, n, want, steps):
    """The paper's Section 5 comparison on this GPU: the balanced circular
    assignment against the straightforward triangular one, both with one wave
    per row block, no partner chunking and the same task body (pairs_ab.h)."""
    import ctypes
    import numpy as np
    from paper_1901_11204_amd import build as B
    L = ctypes.CDLL(B.AB_LIB)
    f = L.pairs_ab_count_i32
    f.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int,
                                                           ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    out = torch.empty(1, dtype=torch.int64, device=x.device)
    stream = torch.cuda.current_stream().cuda_stream
    res = {"n": n, "note": "one wave per row block, whole row ranges, same task body"}
    for K in (1, 8):
        ms = {}
        for variant, name in ((0, "balanced"), (1, "straightforward")):
            def call():
                rc = f(variant, x.data_ptr(), y.data_ptr(), z.data_ptr(), r.data_ptr(), n, K,
                       out.data_ptr(), stream)
                if rc != 0:
                    raise RuntimeError(f"pairs_ab_count_i32 returned {rc}")
            t, _ = timed_steps(call, steps, 1)
            if int(out.item()) != want:
                raise RuntimeError(f"{name} K={K}: count {int(out.item())} != {want}")
            ms[name] = float(np.mean(t))
        res[f"rows_per_lane_{K}"] = {"balanced_ms": ms["balanced"],
                                     "straightforward_ms": ms["straightforward"],
                                     "speedup": ms["straightforward"] / ms["balanced"],
                                     "waves": {name: wave_timeline(L, torch, np, variant, x, y, z,
                                                                   r, n, K, out, stream)
                                               for variant, name in ((0, "balanced"),
                                                                     (1, "straightforward"))}}
    return res


def wave_timeline(L, torch, np, variant, x, y, z, r, n, K, out, stream):
    """One timed run of the comparison kernel: every wave's start and end on
    the device's wall clock, summarised as the span, the waves' durations,
    the mean number of waves running over the span against the most that ran
    at once, the time at the end with fewer than 90 % of that maximum running,
    and the rank correlation of start order with row-block order."""
    import ctypes
    t = L.pairs_ab_count_i32_timed
    t.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int,
                                                           ctypes.c_void_p, ctypes.c_void_p,
                                                           ctypes.c_void_p]
    t.restype = ctypes.c_int
    L.pairs_ab_waves.argtypes = [ctypes.c_int64, ctypes.c_int]
    L.pairs_ab_waves.restype = ctypes.c_int64
    waves = L.pairs_ab_waves(n, K)
    times = torch.zeros(2 * waves, dtype=torch.int64, device=x.device)
    if t(variant, x.data_ptr(), y.data_ptr(), z.data_ptr(), r.data_ptr(), n, K, out.data_ptr(),
         times.data_ptr(), stream) != 0:
        raise RuntimeError("pairs_ab_count_i32_timed failed")
    torch.cuda.synchronize()
    khz = ctypes.c_int64(0)
    L.pairs_ab_wall_clock_khz(ctypes.byref(khz))
    tt = times.cpu().numpy().reshape(-1, 2).astype(np.float64)
    t0 = tt[:, 0].min()
    st, en = (tt[:, 0] - t0) / khz.value, (tt[:, 1] - t0) / khz.value  # ms
    span = float(en.max())
    ev = np.concatenate([np.stack([st, np.ones_like(st)], 1), np.stack([en, -np.ones_like(en)], 1)])
    ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]
    active = np.cumsum(ev[:, 1])
    dt = np.diff(ev[:, 0], append=span)
    peak = float(active.max())
    above = np.nonzero(active >= 0.9 * peak)[0]
    last_full = float(ev[above[-1], 0] + dt[above[-1]]) if len(above) else 0.0
    order = np.argsort(np.argsort(st))
    rank_corr = float(np.corrcoef(order, np.arange(len(st)))[0, 1]) if len(st) > 1 else 1.0
    dur = en - st
    return {"span_ms": span, "wave_ms_mean": float(dur.mean()), "wave_ms_min": float(dur.min()),
            "wave_ms_max": float(dur.max()), "max_running": int(peak),
            "mean_running_over_span": float((active * dt).sum() / span),
            "tail_ms_below_90pct": span - last_full,
            "start_order_vs_block_order_rank_corr": rank_corr}


SIZE_SLICES = ((2, 16), (17, 32), (33, 64), (65, 128), (129, 256), (257, 512), (513, 1024),
               (1025, 2048), (2049, 8192))


def size_slices(P, w, torch, np, dev, steps):
    """The 200 000 binned sets split by size, each slice timed alone as its own batch
    (a plan and the unplanned call): where the batched count's time goes."""
    b = w.binned_sets()
    off, sizes = b.offsets, np.diff(b.offsets)
    arrays = b.objs.arrays()
    out = []
    for lo, hi in SIZE_SLICES:
        sel = np.nonzero((sizes >= lo) & (sizes <= hi))[0]
        idx = np.concatenate([np.arange(off[s], off[s + 1]) for s in sel])
        offs = np.concatenate([[0], np.cumsum(sizes[sel])]).astype(np.int64)
        x, y, z, r = (torch.from_numpy(np.ascontiguousarray(a[idx])).to(dev) for a in arrays)
        counts = torch.empty(len(sel), dtype=torch.int64, device=dev)
        pairs = int((sizes[sel] * (sizes[sel] - 1) // 2).sum())
        plan = P.Plan(P.KIND_COUNT_I32, offs)
        sclk_during(lambda: plan.execute((x, y, z, r), (counts,)))
        mp = float(np.mean(timed_steps(lambda: plan.execute((x, y, z, r), (counts,)),
                                       max(10, steps), 2)[0]))
        plan.close()
        toff = torch.from_numpy(offs).to(dev)
        ws = torch.empty(P.pairs_batched_workspace_size(len(sel), int(offs[-1])),
                         dtype=torch.uint8, device=dev)
        sclk_during(lambda: P.pairs_count_i32_batched(x, y, z, r, toff, counts, ws))
        mu = float(np.mean(timed_steps(lambda: P.pairs_count_i32_batched(x, y, z, r, toff,
                                                                          counts, ws),
                                       max(10, steps), 2)[0]))
        frac = lambda m: pairs / (m * 1e-3) * C_ALG["count_i32"] / VALU_PEAK
        out.append({"sizes": [lo, hi], "sets": int(len(sel)), "pair_tests": pairs,
                    "plan_ms": mp, "plan_valu_frac": frac(mp),
                    "unplanned_ms": mu, "unplanned_valu_frac": frac(mu)})
        log(f"[bench] binned sets of {lo}..{hi} objects: plan {mp:.4f} ms")
    return out


def bench_batched(P, w, torch, np, dev, steps):
    """Batched lines: the binned int32 batch (one persistent launch through a
    plan, and the unplanned call), and the float32 repeated-step loop captured
    in one HIP graph of 100 steps."""
    out = {}
    b = w.binned_sets()
    x, y, z, r = (torch.from_numpy(v).to(dev) for v in b.objs.arrays())
    sizes = np.diff(b.offsets)
    pairs = int((sizes * (sizes - 1) // 2).sum())
    counts = torch.empty(b.n_sets, dtype=torch.int64, device=dev)
    plan = P.Plan(P.KIND_COUNT_I32, b.offsets)
    log(f"[bench] batched count_i32: {b.n_sets} sets, {pairs} pair tests")
    mhz = sclk_during(lambda: plan.execute((x, y, z, r), (counts,)))
    # millisecond calls: a window of 100 calls, so that a transient slow spell
    # of the engine clock (a few calls up to a quarter slower) weighs less
    ms, _ = timed_steps(lambda: plan.execute((x, y, z, r), (counts,)), max(100, steps), 2)
    m = float(np.mean(ms))
    frac = pairs / (m * 1e-3) * C_ALG["count_i32"] / VALU_PEAK
    out["count_i32_binned_200k_sets"] = {
        "workload": "200000 sets, sizes lognormal(4,1.2) clipped to [2,8192], seed 5",
        "pair_tests": pairs, "ms": m, "G_pairs_per_s": pairs / m / 1e6,
        "valu_frac": frac, "sclk_mhz_measured": mhz, "valu_frac_at_measured_sclk": at_sclk(frac, mhz),
        "n_tasks": plan.info()["n_tasks"], "total_count": int(counts.sum().item()),
        "matches_oracle": hashlib.sha256(counts.cpu().numpy().astype("<u8").tobytes()).hexdigest()
                          == golden()["binned_sets_200k_counts"]["sha256_le_u64"]}
    toff = torch.from_numpy(b.offsets).to(dev)
    ws = torch.empty(P.pairs_batched_workspace_size(b.n_sets, b.n_total), dtype=torch.uint8,
                     device=dev)
    mhz = sclk_during(lambda: P.pairs_count_i32_batched(x, y, z, r, toff, counts, ws))
    ms, _ = timed_steps(lambda: P.pairs_count_i32_batched(x, y, z, r, toff, counts, ws),
                        max(100, steps), 2)
    m = float(np.mean(ms))
    frac = pairs / (m * 1e-3) * C_ALG["count_i32"] / VALU_PEAK
    out.update(bench_binned_sets(P, torch, np, dev, b, (x, y, z, r), toff))
    out["count_i32_binned_200k_sets_unplanned"] = {
        "ms": m, "G_pairs_per_s": pairs / m / 1e6,
        "valu_frac": frac, "sclk_mhz_measured": mhz, "valu_frac_at_measured_sclk": at_sclk(frac, mhz),
        "matches_oracle": hashlib.sha256(counts.cpu().numpy().astype("<u8").tobytes()).hexdigest()
                          == golden()["binned_sets_200k_counts"]["sha256_le_u64"]}
    plan.close()
    del x, y, z, r, ws

    b5 = w.moving_sets()
    x, y, z, r = (torch.from_numpy(v).to(dev) for v in b5.objs.arrays())
    sizes = np.diff(b5.offsets)
    pairs5 = int((sizes * (sizes - 1) // 2).sum())
    nsteps = 100
    E = torch.empty(nsteps * b5.n_sets, dtype=torch.float64, device=dev)
    C = torch.empty(nsteps * b5.n_sets, dtype=torch.int64, device=dev)
    plan5 = P.Plan(P.KIND_ENERGY_F32, b5.offsets)
    g = plan5.capture_steps(x, y, z, r, seed=6, sigma=1e-3, first_step=0, n_steps=nsteps,
                            eps2=1e-4, energy=E, counts=C)
    log(f"[bench] graph of {nsteps} steps: {b5.n_sets} sets, {pairs5} pair tests per step")
    mhz = sclk_during(lambda: g.launch())
    ms, _ = timed_steps(lambda: g.launch(), 3, 1)
    m = float(np.mean(ms)) / nsteps
    frac = pairs5 / (m * 1e-3) * C_ALG["energy_count_f32"] / VALU_PEAK
    ms_j, _ = timed_steps(lambda: P.pairs_jitter_f32(x, y, z, 6, 0, 1e-3), 20, 2)
    # one more replay from the initial positions, checked on sampled sets at
    # steps 0, 49 and 99 against the oracle's stored values
    for t, v in zip((x, y, z), b5.objs.arrays()[:3]):
        t.copy_(torch.from_numpy(v).to(dev))
    g.launch()
    torch.cuda.synchronize()
    g5 = golden()["moving_sets_50k_sampled"]
    En, Cn = E.cpu().numpy(), C.cpu().numpy()
    errs, exact = [], True
    for i, st in enumerate(g5["sets"]):
        for j, k in enumerate(g5["steps"]):
            want = g5["energy"][i][j]
            errs.append(abs(En[k * b5.n_sets + st] - want) / want)
            exact = exact and int(Cn[k * b5.n_sets + st]) == g5["count"][i][j]
    out["energy_count_f32_graph_100_steps"] = {
        "workload": "50000 sets, sizes lognormal(5,1) clipped to [2,4096], seed 6; "
                    "per step: jitter + per-set energy and pinned-fp32 count (r=0.01)",
        "pair_tests_per_step": pairs5, "ms_per_step": m, "G_pairs_per_s": pairs5 / m / 1e6,
        "valu_frac": frac, "sclk_mhz_measured": mhz, "valu_frac_at_measured_sclk": at_sclk(frac, mhz),
        "jitter_ms": float(np.mean(ms_j)),
        "max_rel_err_per_set_energy_vs_fp64_oracle": float(max(errs)),
        "counts_match_oracle": exact,
        "sampled": f"{len(g5['sets'])} sets at steps {g5['steps']}"}
    g.close()
    plan5.close()
    return out


def bench_binned_sets(P, torch, np, dev, b, xyzr, toff):
    """The 200 000 binned sets' objects through the binned path: all 22.5 M as one set in
    cells of 2^14 (the sets' own grid cells, up to 8192 objects, so big cells
    and their neighbours go through the work items) and of 1024 (about twice
    the largest radius), and the 200 000 sets binned per set as a CSR batch
    in cells of 2^14 and 4096."""
    out = {}
    n4 = b.n_total
    wsb = torch.empty(P.pairs_binned_workspace_size(n4), dtype=torch.uint8, device=dev)
    outb = torch.empty(1, dtype=torch.int64, device=dev)
    for cell in (1 << 14, 1024):
        log(f"[bench] binned count of the {n4} objects as one set, cells of {cell}")
        msb, _ = timed_steps(lambda: P.pairs_count_i32_binned(*xyzr, cell, outb, wsb), 3, 1)
        out[f"count_i32_binned_one_set_cell{cell}"] = {
            "workload": f"the 200 000 binned sets' {n4} objects as one set, cells of {cell}",
            "ms": float(np.median(msb)), "count": int(outb.item())}
    countsb = torch.empty(b.n_sets, dtype=torch.int64, device=dev)
    for cell in (1 << 14, 4096):
        log(f"[bench] binned count of the {b.n_sets} sets as a CSR batch, cells of {cell}")
        msb, _ = timed_steps(lambda: P.pairs_count_i32_binned_batched(*xyzr, toff, cell, countsb,
                                                                      wsb), 3, 1)
        out[f"count_i32_binned_batched_200k_sets_cell{cell}"] = {
            "workload": f"the {b.n_sets} sets, each binned on its own, cells of {cell}",
            "ms": float(np.median(msb)),
            "matches_oracle": hashlib.sha256(countsb.cpu().numpy().astype("<u8").tobytes())
                              .hexdigest() == golden()["binned_sets_200k_counts"]["sha256_le_u64"]}
    return out


def bench_binned(P, torch, np, dev, xyzr, steps, ms_all_pairs=None):
    """The binned count of the 2^20-sphere set with cells of 2^15."""
    n = xyzr[0].numel()
    log("[bench] binned count_i32 N=2^20, cells of 2^15")
    wsb = torch.empty(P.pairs_binned_workspace_size(n), dtype=torch.uint8, device=dev)
    outb = torch.empty(1, dtype=torch.int64, device=dev)
    msb, _ = timed_steps(lambda: P.pairs_count_i32_binned(*xyzr, 1 << 15, outb, wsb), steps, 2)
    mb = float(np.median(msb))
    # algorithmic HBM bytes per object (about one occupied cell per object
    # here, two table slots per object): clearing the slots' keys, tags and
    # sizes (26 B); the insert reads 16 B of input, probes and sets an 8 B
    # key, writes a tag byte, the 8 B (slot, rank) and the 16 B record
    # (49 B); the slot sums read 10 B; the slot prefix reads 10 B and, per
    # cell, the 8 B key, and writes 20 B (38 B); the scatter reads 16 B and
    # writes a 4 B index (20 B); the gather reads 4 + 16 B and writes the
    # 16 B record and its 8 B q (44 B); the count reads 4 B of offset, the
    # 8 B key and the 16 B record (28 B)
    bpo = 26 + 49 + 10 + 38 + 20 + 44 + 28
    res = {"ms": mb, "cell": 1 << 15, "count": int(outb.item()),
           "workspace_bytes_per_object": wsb.numel() / n,
           "matches_oracle": int(outb.item()) == golden()["spheres_2p20_count"],
           "roofline": {"bound": "hbm", "achieved": n * bpo / (mb * 1e-3) / 1e9,
                        "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": n * bpo / (mb * 1e-3) / HBM_PEAK, "bytes_per_object": bpo}}
    if ms_all_pairs:
        res["speedup_vs_all_pairs"] = ms_all_pairs / mb
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=420_000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (HBM counter scale)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only measure the VALU issue rate of the kernels' instruction patterns")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched lines (for profiling their kernels)")
    ap.add_argument("--lattice-only", action="store_true",
                    help="only the lattice-bead counts (for profiling)")
    ap.add_argument("--binned-only", action="store_true",
                    help="only the binned counts of the 2^20 set and of the 200 000 binned sets (for profiling)")
    ap.add_argument("--binned-workload", choices=["2p20", "sets200k", "all"], default="all",
                    help="with --binned-only: which binned workloads")
    ap.add_argument("--size-slices", action="store_true",
                    help="only the 200 000 binned sets split by size, each slice timed alone")
    ap.add_argument("--count-form", choices=["broadcast", "broadcast-k1", "matrix"],
                    help="only the N=2^20 count with one single-set shape (for profiling): "
                         "the default table, or 64-row tasks of 4096 partners on the VALU "
                         "or on the matrix cores")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_11204_amd as P
    import workloads as w

    P.lib()
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    if a.valu_probe:
        print(json.dumps(valu_probe(torch)), flush=True)
        return

    if a.calibrate_copy:
        nbytes = a.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        ms, _ = timed_steps(lambda: dst.copy_(src), a.steps, a.warmup)
        print(json.dumps({"calibrate_copy_bytes": nbytes, "ms": float(np.mean(ms)),
                          "GB_per_s": 2 * nbytes / (float(np.mean(ms)) * 1e-3) / 1e9}), flush=True)
        return

    if a.batched_only:
        print(json.dumps({"batched": bench_batched(P, w, torch, np, dev, a.steps)}), flush=True)
        return
    if a.count_form:
        t = tuple(torch.from_numpy(v).to(dev) for v in w.spheres_2p24(2 ** 20).arrays())
        out = torch.empty(1, dtype=torch.int64, device=dev)
        shapes = {"broadcast-k1": [(0, 1, 4096, P.FORM_BROADCAST)],
                  "matrix": [(0, 1, 4096, P.FORM_MATRIX)]}.get(a.count_form)
        if shapes:
            P.pairs_set_shapes(P.KIND_COUNT_I32, False, shapes)
        ms, _ = timed_steps(lambda: P.pairs_count_i32(*t, out), a.steps, a.warmup)
        P.pairs_set_shapes(P.KIND_COUNT_I32, False, None)
        pairs = 2 ** 20 * (2 ** 20 - 1) // 2
        print(json.dumps({"count_form": a.count_form, "ms": float(np.mean(ms)),
                          "G_pairs_per_s": pairs / float(np.mean(ms)) / 1e6,
                          "count": int(out.item())}), flush=True)
        return
    if a.size_slices:
        print(json.dumps({"size_slices": size_slices(P, w, torch, np, dev,
                                                                      a.steps)}), flush=True)
        return
    if a.lattice_only:
        print(json.dumps({"lattice": bench_lattice(P, w, torch, np, dev, a.steps)}), flush=True)
        return
    if a.binned_only:
        res = {}
        if a.binned_workload in ("2p20", "all"):
            xyzr = tuple(torch.from_numpy(v).to(dev) for v in w.spheres_2p24(2 ** 20).arrays())
            res["count_i32_binned_2^20"] = bench_binned(P, torch, np, dev, xyzr, a.steps)
            del xyzr
        if a.binned_workload in ("sets200k", "all"):
            b4 = w.binned_sets()
            xyzr = tuple(torch.from_numpy(v).to(dev) for v in b4.objs.arrays())
            res.update(bench_binned_sets(P, torch, np, dev, b4, xyzr,
                                            torch.from_numpy(b4.offsets).to(dev)))
        print(json.dumps({"binned": res}), flush=True)
        return

    # headline workload
    n = 2 ** 20
    s = w.spheres_2p24(n)
    x, y, z, r = (torch.from_numpy(v).to(dev) for v in s.arrays())
    out = torch.empty(1, dtype=torch.int64, device=dev)
    pairs = n * (n - 1) // 2
    log(f"[bench] count_i32 N={n}: {a.warmup} warmup + {a.steps} timed steps")
    sclk = SclkSampler()
    ms, wall = timed_steps(lambda: P.pairs_count_i32(x, y, z, r, out), a.steps, a.warmup, sclk)
    ms_step = float(np.mean(ms))
    sclk_mhz = sclk.mean_mhz()
    value = pairs / (ms_step * 1e-3) / 1e9
    achieved = pairs / (ms_step * 1e-3) * C_ALG["count_i32"]
    count = int(out.item())

    rec = {
        "metric": "pair tests/sec (G pairs/s) and % of VALU peak; batched vs single-set on 1 GPU",
        "value": value,
        "unit": "G pair tests/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 in; exact Gram predicate in fp64 (int64 for 1-2 rows per lane); u64 count",
        "data": "synthetic (seeded uniform spheres)",
        "config": {"workload": "single set, N=2^20 int32 spheres, centres in [0,2^24)^3, "
                               "radii in [1,2^14], seed 2; exact collision count",
                   "n": n, "pair_tests": pairs, "parallelism": "single GPU"},
        "result": {"count": count, "matches_oracle": count == golden()["spheres_2p20_count"]},
        "paper_context": PAPER_CONTEXT,
        "timing": {"ms_min": float(np.min(ms)), "ms_median": float(np.median(ms)),
                   "ms_iqr": float(np.percentile(ms, 75) - np.percentile(ms, 25)),
                   "ms_max": float(np.max(ms)), "wall_s": wall},
        "c_pair": {"per_pair_ops": C_ALG["count_i32"],
                   "inner_loop": "per partner and row slice: 4 v_fma_f64 + 1 v_cmp_ge_f64 "
                                 "(exact Gram form, 8 rows per lane); ballot into "
                                 "s_bcnt1/s_add on the scalar unit",
                   "measured_valu_lane_instr_per_pair": "5.16 (rocprofv3 SQ_INSTS_VALU)"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "T VALU lane-op/s", "frac": achieved / VALU_PEAK,
                     "traffic": recorded_traffic(),
                     "per_pair_ops": C_ALG["count_i32"],
                     "plain_definition_frac": pairs / (ms_step * 1e-3) * PLAIN_DEF_OPS / VALU_PEAK,
                     "sclk_mhz_measured": sclk_mhz,
                     "frac_at_measured_sclk": (achieved / (N_CU * VALU_LANES_PER_CU *
                                                           sclk_mhz * 1e6)
                                               if sclk_mhz else None),
                     "sclk_source": ("amdgpu sysfs pp_dpm_sclk, mean of samples every 2 ms "
                                     "during the timed steps"
                                     if sclk_mhz else "not exposed by the system")},
    }

    if not a.no_secondary:
        sec = {}
        n2 = 2 ** 20 - 1
        s2 = w.spheres_2p24(n2)
        t2 = [torch.from_numpy(v).to(dev) for v in s2.arrays()]
        p2 = n2 * (n2 - 1) // 2
        log(f"[bench] count_i32 N={n2}")
        ms2, _ = timed_steps(lambda: P.pairs_count_i32(*t2, out), max(3, a.steps // 2), 1)
        m2 = float(np.mean(ms2))
        sec["count_i32_odd_2^20-1"] = {"ms": m2, "G_pairs_per_s": p2 / m2 / 1e6,
                                       "valu_frac": p2 / (m2 * 1e-3) * C_ALG["count_i32"] / VALU_PEAK,
                                       "count": int(out.item())}
        del t2
        s1 = w.spheres_4096()
        t1 = [torch.from_numpy(v).to(dev) for v in s1.arrays()]
        p1 = 4096 * 4095 // 2
        log("[bench] count_i32 N=4096")
        ms1, _ = timed_steps(lambda: P.pairs_count_i32(*t1, out), 50, 5)
        m1 = float(np.median(ms1))
        sec["count_i32_4096"] = {"ms": m1, "G_pairs_per_s": p1 / m1 / 1e6, "count": int(out.item())}
        sec["count_i32_4096"]["graph_of_1000_calls"] = graph_per_call(torch, P, t1, out, 1000)
        p3 = w.particles_unit_cube()
        t3 = [torch.from_numpy(v).to(dev) for v in p3.arrays()]
        n3 = p3.n
        E = torch.empty(n3, dtype=torch.float64, device=dev)
        tot = torch.empty(1, dtype=torch.float64, device=dev)
        pp3 = n3 * (n3 - 1) // 2
        log(f"[bench] energy_f32 N={n3}")
        mhz3 = sclk_during(lambda: P.pairs_energy_f32(*t3, 1e-4, E, tot))
        ms3, _ = timed_steps(lambda: P.pairs_energy_f32(*t3, 1e-4, E, tot), max(3, a.steps // 2), 1)
        m3 = float(np.mean(ms3))
        frac3 = pp3 / (m3 * 1e-3) * C_ALG["energy_f32"] / VALU_PEAK
        ge = golden()["particles_2p18_energy_rows"]
        got_rows = E[torch.tensor(ge["rows"], device=dev)].cpu().numpy()
        want_rows = np.array(ge["E"])
        sec["energy_f32_2^18"] = {"ms": m3, "G_pairs_per_s": pp3 / m3 / 1e6,
                                  "valu_frac": frac3, "sclk_mhz_measured": mhz3,
                                  "valu_frac_at_measured_sclk": at_sclk(frac3, mhz3),
                                  "total": float(tot.item()),
                                  "rel_err_total_vs_fp64_oracle":
                                      abs(float(tot.item()) - golden()["particles_2p18_energy_total"])
                                      / golden()["particles_2p18_energy_total"],
                                  "max_rel_err_per_particle_vs_fp64_oracle":
                                      float(np.max(np.abs(got_rows - want_rows) / want_rows)),
                                  "sampled_particles": len(ge["rows"])}
        mhz3b = sclk_during(lambda: P.pairs_energy_f32(*t3, 1e-4, None, tot))
        ms3b, _ = timed_steps(lambda: P.pairs_energy_f32(*t3, 1e-4, None, tot), max(3, a.steps // 2), 1)
        m3b = float(np.mean(ms3b))
        frac3b = pp3 / (m3b * 1e-3) * C_ALG["energy_total_f32"] / VALU_PEAK
        sec["energy_f32_2^18_total_only"] = {
            "ms": m3b, "G_pairs_per_s": pp3 / m3b / 1e6, "valu_frac": frac3b,
            "per_pair_ops": C_ALG["energy_total_f32"], "sclk_mhz_measured": mhz3b,
            "valu_frac_at_measured_sclk": at_sclk(frac3b, mhz3b),
            "rel_err_total_vs_fp64_oracle": abs(float(tot.item()) - golden()["particles_2p18_energy_total"])
                                            / golden()["particles_2p18_energy_total"]}
        log(f"[bench] energy_f64 N={n3}")
        t3d = [v.to(torch.float64) for v in t3]
        ms5, _ = timed_steps(lambda: P.pairs_energy_f64(*t3d, float(np.float32(1e-4)), E, tot),
                             max(3, a.steps // 2), 1)
        m5 = float(np.mean(ms5))
        sec["energy_f64_2^18"] = {"ms": m5, "G_pairs_per_s": pp3 / m5 / 1e6,
                                  "valu_frac": pp3 / (m5 * 1e-3) * C_ALG["energy_f64"] / VALU_PEAK,
                                  "per_pair_ops": C_ALG["energy_f64"],
                                  "rel_err_total_vs_fp64_oracle":
                                      abs(float(tot.item()) - golden()["particles_2p18_energy_total"])
                                      / golden()["particles_2p18_energy_total"],
                                  "inputs": "the 2^18 float32 particles promoted to double"}
        del t3d
        log(f"[bench] force_f32 N={n3}")
        Fxyz = [torch.empty(n3, dtype=torch.float64, device=dev) for _ in range(3)]
        mhz4 = sclk_during(lambda: P.pairs_force_f32(*t3, 1e-4, *Fxyz))
        ms4, _ = timed_steps(lambda: P.pairs_force_f32(*t3, 1e-4, *Fxyz), max(3, a.steps // 2), 1)
        m4 = float(np.mean(ms4))
        frac4 = pp3 / (m4 * 1e-3) * C_ALG["force_f32"] / VALU_PEAK
        gf = golden()["particles_2p18_force_rows"]
        got = np.stack([f[torch.tensor(gf["rows"], device=dev)].cpu().numpy() for f in Fxyz], 1)
        err = float((np.abs(got - np.array(gf["F"])).max(axis=1) / np.array(gf["S"])).max())
        sec["force_f32_2^18"] = {"ms": m4, "G_pairs_per_s": pp3 / m4 / 1e6,
                                 "valu_frac": frac4, "sclk_mhz_measured": mhz4,
                                 "valu_frac_at_measured_sclk": at_sclk(frac4, mhz4),
                                 "per_pair_ops": C_ALG["force_f32"],
                                 "max_err_over_norm_sum_vs_fp64_oracle": err,
                                 "sampled_rows": len(gf["rows"])}
        del Fxyz
        sec["count_i32_binned_2^20"] = bench_binned(P, torch, np, dev, (x, y, z, r),
                                                    max(5, a.steps), ms_step)
        log("[bench] assignment comparison: balanced vs straightforward, N=2^20")
        sec["assignment_comparison_n2p20"] = assignment_comparison(torch, x, y, z, r, n, count,
                                                                   max(2, a.steps // 2))
        rec["secondary"] = sec
        rec["batched"] = bench_batched(P, w, torch, np, dev, a.steps)
        rec["lattice"] = bench_lattice(P, w, torch, np, dev, a.steps)

    if not a.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on {a.cpu_sample} spheres")
        rec["cpu_baseline"] = cpu_baseline(a.cpu_sample)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
