"""The C ABI library on the CPU: it loads, exports every function that
include/pairs.h declares, and rejects bad arguments before touching a device.
No computation runs here (there is no GPU in this environment)."""
import ctypes
import os
import re

import pytest

import paper_1901_11204_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pairs.h")

OK, INVALID, DOMAIN, HIP, NOMEM, WORKSPACE, NODEV = 0, -1, -2, -3, -4, -5, -6


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pairs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["pairs_count_i32", "pairs_count_f32", "pairs_energy_f32"]:
        assert must in names


def test_library_exports_every_declared_function():
    L = ctypes.CDLL(P.lib_path())
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    L = P.lib()
    for code in [OK, INVALID, DOMAIN, HIP, NOMEM, WORKSPACE, NODEV]:
        s = L.pairs_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.pairs_status_string(12345).decode() == "unknown status"


def fake(k):
    # non-null host addresses that are never dereferenced: every call below
    # fails its argument check or finds no device before any device access
    return ctypes.c_void_p(0x1000 * (k + 1))


def test_invalid_arguments_are_rejected_on_the_host():
    L = P.lib()
    x, y, z, r, out = (fake(k) for k in range(5))
    assert L.pairs_count_i32(x, y, z, r, -1, out, 0, None) == INVALID
    assert L.pairs_count_i32(x, y, z, r, 10, None, 0, None) == INVALID
    assert L.pairs_count_i32(None, y, z, r, 10, out, 0, None) == INVALID
    assert L.pairs_count_i32(x, y, z, r, 10, out, 0x80, None) == INVALID
    assert L.pairs_count_i32(x, y, z, r, (1 << 30) + 1, out, 0, None) == INVALID
    assert L.pairs_count_f32(x, y, z, None, 10, out, 0, None) == INVALID
    assert L.pairs_energy_f32(x, y, z, 10, 0.0, None, out, 0, None) == INVALID
    assert L.pairs_energy_f32(x, y, z, 10, float("nan"), None, out, 0, None) == INVALID
    assert L.pairs_energy_f32(x, y, z, 10, 1e-4, None, None, 0, None) == INVALID


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES", None) is None and
                    os.path.exists("/dev/kfd"), reason="a device may be present")
def test_no_device_is_reported():
    L = P.lib()
    x, y, z, r, out = (fake(k) for k in range(5))
    assert L.pairs_count_i32(x, y, z, r, 10, out, 0, None) == NODEV
    assert L.pairs_energy_f32(x, y, z, 10, 1e-4, None, out, 0, None) == NODEV


def test_batched_argument_errors_on_the_host():
    L = P.lib()
    x, y, z, r, off, out, ws = (fake(k) for k in range(7))
    need = P.pairs_batched_workspace_size(10, 100)
    assert need > 0
    assert L.pairs_count_i32_batched(x, y, z, r, off, 10, 100, out, ws, need - 1, 0,
                                     None) == WORKSPACE
    assert L.pairs_count_i32_batched(x, y, z, r, off, 10, 100, out, None, need, 0,
                                     None) == WORKSPACE
    assert L.pairs_count_i32_batched(x, y, z, r, None, 10, 100, out, ws, need, 0,
                                     None) == INVALID
    assert L.pairs_count_i32_batched(x, y, z, r, off, -1, 100, out, ws, need, 0, None) == INVALID
    # the no-allocation variant: its static scratch holds at most
    # NOALLOC_MAX_SETS sets; more is refused on the host
    lim = P.NOALLOC_MAX_SETS
    assert L.pairs_count_i32_batched_noalloc(x, y, z, r, off, lim + 1, 100, out, 0,
                                             None) == WORKSPACE
    assert L.pairs_count_i32_batched_noalloc(x, y, z, r, None, 10, 100, out, 0,
                                             None) == INVALID
    assert L.pairs_count_i32_batched_noalloc(x, y, z, None, off, 10, 100, out, 0,
                                             None) == INVALID
    assert L.pairs_count_i32_batched_noalloc(x, y, z, r, off, 10, 100, None, 0,
                                             None) == INVALID
    # batched forces and double-precision energies
    assert L.pairs_force_f32_batched(x, y, z, off, 10, 100, 1e-4, out, out, out, ws, need - 1, 0,
                                     None) == WORKSPACE
    assert L.pairs_force_f32_batched(x, y, z, off, 10, 100, 0.0, out, out, out, ws, need, 0,
                                     None) == INVALID
    assert L.pairs_force_f32_batched(x, y, z, off, 10, 100, 1e-4, None, out, out, ws, need, 0,
                                     None) == INVALID
    assert L.pairs_energy_f64_batched(x, y, z, off, 10, 100, 1e-4, None, None, ws, need, 0,
                                      None) == INVALID
    assert L.pairs_energy_f64_batched(x, y, z, off, 10, 100, -1.0, out, None, ws, need, 0,
                                      None) == INVALID
    assert L.pairs_energy_f64_batched(x, y, z, off, 10, 100, 1e-4, out, None, ws, need, 0x80,
                                      None) == INVALID
    # energies: r and counts must be both given or both absent
    assert L.pairs_energy_f32_batched(x, y, z, r, off, 10, 100, 1e-4, out, None, ws, need, 0,
                                      None) == INVALID
    assert L.pairs_energy_f32_batched(x, y, z, None, off, 10, 100, 0.0, out, None, ws, need, 0,
                                      None) == INVALID


def test_plan_argument_errors_on_the_host():
    import numpy as np
    L = P.lib()
    h = ctypes.c_void_p()
    bad = np.array([0, 5, 3], np.int64)
    assert L.pairs_plan_create(1, bad.ctypes.data_as(ctypes.c_void_p), 2,
                               ctypes.byref(h)) == INVALID
    assert L.pairs_plan_create(9, bad.ctypes.data_as(ctypes.c_void_p), 2,
                               ctypes.byref(h)) == INVALID
    start = np.array([1, 5], np.int64)
    assert L.pairs_plan_create(1, start.ctypes.data_as(ctypes.c_void_p), 1,
                               ctypes.byref(h)) == INVALID
    assert L.pairs_plan_execute(None, None, None, 0.0, None) == INVALID
    assert L.pairs_graph_launch(None, None) == INVALID
    assert L.pairs_plan_destroy(None) == OK
    assert L.pairs_jitter_f32(x_ := fake(0), fake(1), fake(2), 10, 1, 0, -1.0, 0,
                              None) == INVALID


def test_comparison_library_exports_and_checks_arguments():
    """include/pairs_ab.h: the benchmark's assignment comparison."""
    from paper_1901_11204_amd import build as B
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "pairs_ab.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(pairs_[a-z0-9_]+)\s*\(", text)))
    assert names == ["pairs_ab_count_i32", "pairs_ab_count_i32_timed", "pairs_ab_wall_clock_khz",
                     "pairs_ab_waves"]
    L = ctypes.CDLL(B.AB_LIB)
    for name in names:
        assert hasattr(L, name), name
    f = L.pairs_ab_count_i32
    f.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int,
                                                           ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    x, y, z, r, out = (fake(k) for k in range(5))
    assert f(2, x, y, z, r, 10, 1, out, None) == -1      # no such variant
    assert f(0, x, y, z, r, 10, 4, out, None) == -1      # rows per lane 1 or 8
    assert f(0, None, y, z, r, 10, 1, out, None) == -1   # missing input
    assert f(1, x, y, z, r, 10, 1, None, None) == -1     # missing output
    assert f(1, x, y, z, r, -1, 1, out, None) == -1
    t = L.pairs_ab_count_i32_timed
    t.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int,
                                                           ctypes.c_void_p, ctypes.c_void_p,
                                                           ctypes.c_void_p]
    t.restype = ctypes.c_int
    assert t(0, x, y, z, r, 10, 1, out, None, None) == -1   # no timestamp buffer
    assert t(2, x, y, z, r, 10, 1, out, fake(5), None) == -1
    wv = L.pairs_ab_waves
    wv.argtypes = [ctypes.c_int64, ctypes.c_int]
    wv.restype = ctypes.c_int64
    assert wv(1 << 20, 1) == 16384 and wv(1 << 20, 8) == 2048 and wv(65, 1) == 2
    assert wv(1, 1) == 0 and wv(100, 4) == 0


def test_lattice_arguments_are_rejected_on_the_host():
    L = P.lib()
    x, y, z, c, k, ws, off = (fake(k) for k in range(7))
    n_sz = ctypes.c_size_t(0)
    assert L.pairs_lattice_workspace_size(1, 100, -1, ctypes.byref(n_sz)) == INVALID
    assert L.pairs_lattice_workspace_size(1, 100, 100, ctypes.byref(n_sz)) == OK
    assert n_sz.value == 0
    assert L.pairs_lattice_workspace_size(1, 5000, 5000, ctypes.byref(n_sz)) == OK
    assert n_sz.value >= 32 * 5000
    # single vector: bad length, no outputs, bad flags, missing workspace
    assert L.pairs_lattice_count(x, y, z, -1, c, k, None, 0, 0, None) == INVALID
    assert L.pairs_lattice_count(x, y, z, 10, None, None, None, 0, 0, None) == INVALID
    assert L.pairs_lattice_count(None, y, z, 10, c, k, None, 0, 0, None) == INVALID
    assert L.pairs_lattice_count(x, y, z, 10, c, k, None, 0, 0x10, None) == INVALID
    assert L.pairs_lattice_count(x, y, z, 1 << 24, c, k, ws, 1 << 40, 0, None) == INVALID
    assert L.pairs_lattice_count(x, y, z, 5000, c, k, None, 0, 0, None) == WORKSPACE
    assert L.pairs_lattice_count(x, y, z, 5000, c, k, ws, 1000, 0, None) == WORKSPACE
    # batches: negative bound, missing offsets, unknown bound without workspace
    assert L.pairs_lattice_count_batched(x, y, z, off, 2, 10, -1, c, k, None, 0, 0,
                                         None) == INVALID
    assert L.pairs_lattice_count_batched(x, y, z, None, 2, 10, 5, c, k, None, 0, 0,
                                         None) == INVALID
    assert L.pairs_lattice_count_batched(x, y, z, off, 2, 10, 5, None, None, None, 0, 0,
                                         None) == INVALID
    assert L.pairs_lattice_count_batched(x, y, z, off, 2, 10, 0, c, k, None, 0, 0,
                                         None) == WORKSPACE
    assert L.pairs_lattice_count_batched(x, y, z, off, 2, 10, 5000, c, k, ws, 64, 0,
                                         None) == WORKSPACE


def test_force_arguments_are_rejected_on_the_host():
    L = P.lib()
    x, y, z, a, b, c = (fake(k) for k in range(6))
    assert L.pairs_force_f32(x, y, z, -1, 1e-4, a, b, c, 0, None) == INVALID
    assert L.pairs_force_f32(x, y, z, 10, 0.0, a, b, c, 0, None) == INVALID
    assert L.pairs_force_f32(x, y, z, 10, float("inf"), a, b, c, 0, None) == INVALID
    assert L.pairs_force_f32(x, y, z, 10, 1e-4, a, None, c, 0, None) == INVALID
    assert L.pairs_force_f32(None, y, z, 10, 1e-4, a, b, c, 0, None) == INVALID
    assert L.pairs_force_f32(x, y, z, 10, 1e-4, a, b, c, 0x40, None) == INVALID


def test_energy64_arguments_are_rejected_on_the_host():
    L = P.lib()
    x, y, z, e, t = (fake(k) for k in range(5))
    assert L.pairs_energy_f64(x, y, z, 10, 1e-4, e, None, 0, None) == INVALID
    assert L.pairs_energy_f64(x, y, z, -1, 1e-4, e, t, 0, None) == INVALID
    assert L.pairs_energy_f64(x, y, z, 10, 0.0, e, t, 0, None) == INVALID
    assert L.pairs_energy_f64(x, y, z, 10, float("nan"), e, t, 0, None) == INVALID
    assert L.pairs_energy_f64(None, y, z, 10, 1e-4, e, t, 0, None) == INVALID


def test_binned_arguments_are_rejected_on_the_host():
    L = P.lib()
    x, y, z, r, out, ws = (fake(k) for k in range(6))
    n_sz = ctypes.c_size_t(0)
    assert L.pairs_binned_workspace_size(-1, ctypes.byref(n_sz)) == INVALID
    assert L.pairs_binned_workspace_size(0, ctypes.byref(n_sz)) == OK
    # the size query needs no device: 48 bytes per object plus the table of
    # at least 2n slots of 21 bytes and the work-item list
    assert L.pairs_binned_workspace_size(1000, ctypes.byref(n_sz)) == OK
    assert n_sz.value >= 1000 * (48 + 42)
    assert L.pairs_binned_workspace_size(1 << 30, ctypes.byref(n_sz)) == OK
    assert L.pairs_binned_workspace_size((1 << 30) + 1, ctypes.byref(n_sz)) == INVALID
    assert L.pairs_count_i32_binned(x, y, z, r, -1, 64, out, ws, 0, 0, None) == INVALID
    assert L.pairs_count_i32_binned(x, y, z, r, 10, 16, out, ws, 0, 0, None) == INVALID
    assert L.pairs_count_i32_binned(x, y, z, r, 10, 1 << 26, out, ws, 0, 0, None) == INVALID
    assert L.pairs_count_i32_binned(x, y, z, r, 10, 64, None, ws, 0, 0, None) == INVALID
    assert L.pairs_count_i32_binned(None, y, z, r, 10, 64, out, ws, 0, 0, None) == INVALID
    assert L.pairs_count_i32_binned(x, y, z, r, 10, 64, out, ws, 0, 0x10, None) == INVALID
    off = fake(7)
    B = L.pairs_count_i32_binned_batched
    assert B(x, y, z, r, off, -1, 10, 64, out, ws, 0, 0, None) == INVALID
    assert B(x, y, z, r, None, 2, 10, 64, out, ws, 0, 0, None) == INVALID
    assert B(x, y, z, r, off, 2, 10, 64, None, ws, 0, 0, None) == INVALID
    assert B(x, y, z, r, off, 2, 10, 16, out, ws, 0, 0, None) == INVALID
    assert B(None, y, z, r, off, 2, 10, 64, out, ws, 0, 0, None) == INVALID
    assert B(x, y, z, r, off, 2, 10, 64, out, ws, 0, 0x10, None) == INVALID
    assert B(x, y, z, r, off, 0, 10, 64, out, ws, 0, 0, None) == INVALID
    assert B(x, y, z, r, off, 0, 0, 64, out, ws, 0, 0, None) == OK
    # cells of 32 take 3 x 21 key bits, so a batch of two sets needs 64 bits
    # and one of three sets 65
    assert B(x, y, z, r, off, 3, 10, 32, out, ws, 1 << 20, 0, None) == INVALID
