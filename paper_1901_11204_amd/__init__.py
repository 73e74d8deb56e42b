"""Python binding of libpairs (include/pairs.h): argument marshalling only.

Every function below has the name of the C entry point it calls, takes torch
tensors on the current HIP device, passes their device pointers and the
current torch stream to the library, and raises on a non-OK status.  All the
computation runs in the library's HIP kernels; if the library is not built the
binding raises instead of computing anything itself.

Counts are written to a one-element int64 tensor that the library treats as
uint64 (every count here is below 2^63).
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "PairsError", "lib", "lib_path", "FLAG_VALIDATE", "FLAG_DETERMINISTIC", "PLAN_DETERMINISTIC",
    "KIND_COUNT_I32", "KIND_COUNT_F32", "KIND_ENERGY_F32",
    "pairs_count_i32", "pairs_count_f32", "pairs_energy_f32", "pairs_energy_f64",
    "pairs_force_f32",
    "pairs_batched_workspace_size", "pairs_count_i32_batched", "pairs_count_f32_batched",
    "pairs_energy_f32_batched", "pairs_count_i32_batched_noalloc", "NOALLOC_MAX_SETS",
    "pairs_force_f32_batched", "pairs_energy_f64_batched",
    "pairs_jitter_f32", "pairs_debug_task_ranges",
    "pairs_debug_step_ranges", "pairs_debug_single_launch", "pairs_debug_task_at", "FORM_BROADCAST", "FORM_STEPPING", "FORM_MATRIX",
    "SHAPES_SINGLE", "SHAPES_BATCHED", "SHAPES_TOTAL_ONLY",
    "KIND_ENERGY_F64", "KIND_FORCE_F32",
    "Plan", "Graph", "ShapeTable", "pairs_get_shapes", "pairs_set_shapes",
    "count_i32", "count_f32", "energy_f32",
    "pairs_lattice_workspace_size", "pairs_lattice_count", "pairs_lattice_count_batched",
    "pairs_binned_workspace_size", "pairs_count_i32_binned", "pairs_count_i32_binned_batched",
    "LATTICE_LDS_BEADS", "LATTICE_MAX_BEADS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpairs.so")
_lib = None

FLAG_VALIDATE = 1
FLAG_DETERMINISTIC = 2
PLAN_DETERMINISTIC = 0x100  # or'ed into a plan's kind (KIND_ENERGY_F32)
LATTICE_LDS_BEADS = 4096
LATTICE_MAX_BEADS = (1 << 24) - 1
KIND_COUNT_I32, KIND_COUNT_F32, KIND_ENERGY_F32 = 1, 2, 3
KIND_ENERGY_F64, KIND_FORCE_F32 = 4, 5  # pairs_debug_single_launch only
NOALLOC_MAX_SETS = 250000

_STATUS = {
    0: "ok", -1: "invalid argument", -2: "input outside the exact domain",
    -3: "HIP runtime error", -4: "out of memory", -5: "workspace missing or too small",
    -6: "no usable HIP device",
}


class PairsError(RuntimeError):
    def __init__(self, status: int, where: str, hip_error: int = 0):
        self.status = status
        self.hip_error = hip_error
        msg = f"{where}: {_STATUS.get(status, 'unknown status')} (status {status}"
        if status == -3:
            msg += f", hipError {hip_error}"
        super().__init__(msg + ")")


def lib_path() -> str:
    return _LIB_PATH


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_f32 = ctypes.c_float


_sz = ctypes.c_size_t
_u64 = ctypes.c_uint64
_int = ctypes.c_int


FORM_BROADCAST = 0
FORM_STEPPING = 1
FORM_MATRIX = 2
SHAPES_SINGLE, SHAPES_BATCHED, SHAPES_TOTAL_ONLY = 0, 1, 2


class ShapeTable(ctypes.Structure):
    """pairs_shape_table_t: up to 4 (min_n, rows_per_lane, chunk, form) entries."""
    _fields_ = [("count", ctypes.c_int32), ("min_n", ctypes.c_int32 * 4),
                ("rows_per_lane", ctypes.c_int32 * 4), ("chunk", ctypes.c_int32 * 4),
                ("form", ctypes.c_int32 * 4)]


def _declare(L):
    sig = {
        "pairs_count_i32": [_vp, _vp, _vp, _vp, _i64, _vp, _u32, _vp],
        "pairs_count_f32": [_vp, _vp, _vp, _vp, _i64, _vp, _u32, _vp],
        "pairs_energy_f32": [_vp, _vp, _vp, _i64, _f32, _vp, _vp, _u32, _vp],
        "pairs_force_f32": [_vp, _vp, _vp, _i64, _f32, _vp, _vp, _vp, _u32, _vp],
        "pairs_energy_f64": [_vp, _vp, _vp, _i64, ctypes.c_double, _vp, _vp, _u32, _vp],
        "pairs_batched_workspace_size": [_i64, _i64, ctypes.POINTER(_sz)],
        "pairs_count_i32_batched": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _sz, _u32,
                                    _vp],
        "pairs_count_f32_batched": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _sz, _u32,
                                    _vp],
        "pairs_count_i32_batched_noalloc": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _u32, _vp],
        "pairs_force_f32_batched": [_vp, _vp, _vp, _vp, _i64, _i64, _f32, _vp, _vp, _vp, _vp, _sz,
                                    _u32, _vp],
        "pairs_energy_f64_batched": [_vp, _vp, _vp, _vp, _i64, _i64, ctypes.c_double, _vp, _vp,
                                     _vp, _sz, _u32, _vp],
        "pairs_energy_f32_batched": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _f32, _vp, _vp, _vp,
                                     _sz, _u32, _vp],
        "pairs_plan_create": [_int, _vp, _i64, ctypes.POINTER(_vp)],
        "pairs_plan_execute": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _f32, _vp],
        "pairs_plan_info": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                            ctypes.POINTER(_i64)],
        "pairs_plan_destroy": [_vp],
        "pairs_jitter_f32": [_vp, _vp, _vp, _i64, _u64, _u32, _f32, _i64, _vp],
        "pairs_plan_capture_steps": [_vp, _vp, _vp, _vp, _vp, _u64, _f32, _u32, _int, _f32, _vp,
                                     _vp, ctypes.POINTER(_vp)],
        "pairs_graph_launch": [_vp, _vp],
        "pairs_graph_destroy": [_vp],
        "pairs_debug_task_ranges": [_int, _int, _int, _vp, _i64, ctypes.POINTER(_i64)],
        "pairs_debug_step_ranges": [_int, _int, _int, _vp, _i64, ctypes.POINTER(_i64)],
        "pairs_debug_task_at": [_i64, _int, _int, _vp, _i64, _vp],
        "pairs_debug_single_launch": [_int, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                      ctypes.POINTER(ctypes.c_int32)],
        "pairs_get_shapes": [_int, _int, ctypes.POINTER(ShapeTable)],
        "pairs_lattice_workspace_size": [_i64, _i64, _i64, ctypes.POINTER(_sz)],
        "pairs_binned_workspace_size": [_i64, ctypes.POINTER(_sz)],
        "pairs_count_i32_binned": [_vp, _vp, _vp, _vp, _i64, ctypes.c_int32, _vp, _vp, _sz, _u32,
                                   _vp],
        "pairs_count_i32_binned_batched": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, ctypes.c_int32,
                                           _vp, _vp, _sz, _u32, _vp],
        "pairs_lattice_count": [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _u32, _vp],
        "pairs_lattice_count_batched": [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp, _sz,
                                        _u32, _vp],
        "pairs_set_shapes": [_int, _int, ctypes.POINTER(ShapeTable)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.pairs_status_string.argtypes = [ctypes.c_int]
    L.pairs_status_string.restype = ctypes.c_char_p
    L.pairs_last_hip_error.argtypes = []
    L.pairs_last_hip_error.restype = ctypes.c_int


def lib():
    """Load libpairs.so (built in-tree by build.py).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run "
                               "`python -m paper_1901_11204_amd.build` first")
        # torch first: its HIP runtime is then the one libpairs.so binds to
        # (same soname).  Loaded the other way round, the process would hold
        # two HIP runtimes, and the library's would find no device once
        # torch's has opened it.
        import torch  # noqa: F401
        L = ctypes.CDLL(_LIB_PATH)
        _declare(L)
        _lib = L
        _apply_tuned_shapes()
    return _lib


def _apply_tuned_shapes():
    """Apply the tile shapes of a tuning cache (PAIRS_TUNE_CACHE, else
    tuned_shapes.json beside this file) when one exists for this device."""
    path = os.environ.get("PAIRS_TUNE_CACHE") or os.path.join(_HERE, "tuned_shapes.json")
    if not os.path.exists(path):
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
        from . import autotune
        autotune.load_cache(path, apply=True)
    except Exception as e:  # a bad cache only costs speed
        import warnings
        warnings.warn(f"tile-shape cache {path} not applied: {e}")


def _check(status: int, where: str):
    if status != 0:
        raise PairsError(status, where, lib().pairs_last_hip_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require(tensors, dtype, n, what):
    import torch
    for t in tensors:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what}: expected torch tensors")
        if t.device.type != "cuda":
            raise ValueError(f"{what}: tensors must be on the HIP device")
        if t.dtype != dtype:
            raise ValueError(f"{what}: expected {dtype}, got {t.dtype}")
        if not t.is_contiguous() or t.dim() != 1 or t.shape[0] != n:
            raise ValueError(f"{what}: expected contiguous 1-D tensors of length {n}")


def pairs_count_i32(x, y, z, r, out, flags: int = 0, stream=None) -> None:
    """Exact collision count of one int32 sphere set into out (int64[1], read as uint64)."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z, r), torch.int32, n, "pairs_count_i32")
    _require((out,), torch.int64, 1, "pairs_count_i32 out")
    _check(lib().pairs_count_i32(_ptr(x), _ptr(y), _ptr(z), _ptr(r), n, _ptr(out), flags,
                                 _stream(stream)), "pairs_count_i32")


def pairs_count_f32(x, y, z, r, out, flags: int = 0, stream=None) -> None:
    """Collision count of one float32 sphere set (pinned binary32 predicate)."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z, r), torch.float32, n, "pairs_count_f32")
    _require((out,), torch.int64, 1, "pairs_count_f32 out")
    _check(lib().pairs_count_f32(_ptr(x), _ptr(y), _ptr(z), _ptr(r), n, _ptr(out), flags,
                                 _stream(stream)), "pairs_count_f32")


def pairs_energy_f32(x, y, z, eps2: float, energy, total, flags: int = 0, stream=None) -> None:
    """Softened potential of one float32 particle set: total (float64[1]) and, if
    energy is not None, the per-particle sums (float64[n])."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z), torch.float32, n, "pairs_energy_f32")
    _require((total,), torch.float64, 1, "pairs_energy_f32 total")
    if energy is not None:
        _require((energy,), torch.float64, n, "pairs_energy_f32 energy")
    _check(lib().pairs_energy_f32(_ptr(x), _ptr(y), _ptr(z), n, float(eps2), _ptr(energy),
                                  _ptr(total), flags, _stream(stream)), "pairs_energy_f32")


def pairs_energy_f64(x, y, z, eps2: float, energy, total, flags: int = 0, stream=None) -> None:
    """Softened potential of one float64 particle set in double arithmetic: total
    (float64[1]) and, if energy is not None, the per-particle sums (float64[n])."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z), torch.float64, n, "pairs_energy_f64")
    _require((total,), torch.float64, 1, "pairs_energy_f64 total")
    if energy is not None:
        _require((energy,), torch.float64, n, "pairs_energy_f64 energy")
    _check(lib().pairs_energy_f64(_ptr(x), _ptr(y), _ptr(z), n, float(eps2), _ptr(energy),
                                  _ptr(total), flags, _stream(stream)), "pairs_energy_f64")


def pairs_force_f32(x, y, z, eps2: float, fx, fy, fz, flags: int = 0, stream=None) -> None:
    """Forces of the softened potential on one float32 particle set: the three
    components into float64[n] tensors fx, fy, fz."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z), torch.float32, n, "pairs_force_f32")
    _require((fx, fy, fz), torch.float64, n, "pairs_force_f32 forces")
    _check(lib().pairs_force_f32(_ptr(x), _ptr(y), _ptr(z), n, float(eps2), _ptr(fx), _ptr(fy),
                                 _ptr(fz), flags, _stream(stream)), "pairs_force_f32")


def pairs_batched_workspace_size(n_sets: int, n_total: int) -> int:
    """Bytes of device workspace an unplanned batched call needs."""
    b = _sz(0)
    _check(lib().pairs_batched_workspace_size(n_sets, n_total, ctypes.byref(b)),
           "pairs_batched_workspace_size")
    return int(b.value)


def _batch_checks(x, tensors, dtype, offsets, what):
    import torch
    n_total = int(x.shape[0])
    _require(tensors, dtype, n_total, what)
    if offsets.dtype != torch.int64 or offsets.device.type != "cuda" or offsets.dim() != 1 \
            or not offsets.is_contiguous():
        raise ValueError(f"{what}: offsets must be a contiguous int64 device tensor")
    return n_total, int(offsets.shape[0]) - 1


def _workspace(ws, n_sets, n_total, device):
    import torch
    need = pairs_batched_workspace_size(n_sets, n_total)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    return ws, int(ws.numel() * ws.element_size())


def pairs_count_i32_batched(x, y, z, r, offsets, counts, ws=None, flags: int = 0,
                            stream=None) -> None:
    """Per-set exact collision counts of a CSR batch into counts (int64[n_sets],
    read as uint64).  ws: device workspace (allocated here if None)."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z, r), torch.int32, offsets,
                                    "pairs_count_i32_batched")
    _require((counts,), torch.int64, n_sets, "pairs_count_i32_batched counts")
    ws, nbytes = _workspace(ws, n_sets, n_total, x.device)
    _check(lib().pairs_count_i32_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(r), _ptr(offsets),
                                         n_sets, n_total, _ptr(counts), _ptr(ws), nbytes, flags,
                                         _stream(stream)), "pairs_count_i32_batched")


def pairs_count_i32_batched_noalloc(x, y, z, r, offsets, counts, flags: int = 0,
                                    stream=None) -> None:
    """pairs_count_i32_batched with the library's static scratch as workspace:
    allocates nothing (at most NOALLOC_MAX_SETS sets; calls overlapping on one
    device race)."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z, r), torch.int32, offsets,
                                    "pairs_count_i32_batched_noalloc")
    _require((counts,), torch.int64, n_sets, "pairs_count_i32_batched_noalloc counts")
    _check(lib().pairs_count_i32_batched_noalloc(_ptr(x), _ptr(y), _ptr(z), _ptr(r),
                                                 _ptr(offsets), n_sets, n_total, _ptr(counts),
                                                 flags, _stream(stream)),
           "pairs_count_i32_batched_noalloc")


def pairs_count_f32_batched(x, y, z, r, offsets, counts, ws=None, flags: int = 0,
                            stream=None) -> None:
    """Per-set pinned-binary32 collision counts of a CSR batch."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z, r), torch.float32, offsets,
                                    "pairs_count_f32_batched")
    _require((counts,), torch.int64, n_sets, "pairs_count_f32_batched counts")
    ws, nbytes = _workspace(ws, n_sets, n_total, x.device)
    _check(lib().pairs_count_f32_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(r), _ptr(offsets),
                                         n_sets, n_total, _ptr(counts), _ptr(ws), nbytes, flags,
                                         _stream(stream)), "pairs_count_f32_batched")


def pairs_energy_f32_batched(x, y, z, r, offsets, eps2, energy, counts=None, ws=None,
                             flags: int = 0, stream=None) -> None:
    """Per-set potential totals (float64[n_sets]) and, if r is given, per-set
    pinned-binary32 collision counts (int64[n_sets])."""
    import torch
    tens = (x, y, z) if r is None else (x, y, z, r)
    n_total, n_sets = _batch_checks(x, tens, torch.float32, offsets, "pairs_energy_f32_batched")
    _require((energy,), torch.float64, n_sets, "pairs_energy_f32_batched energy")
    if counts is not None:
        _require((counts,), torch.int64, n_sets, "pairs_energy_f32_batched counts")
    ws, nbytes = _workspace(ws, n_sets, n_total, x.device)
    _check(lib().pairs_energy_f32_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(r), _ptr(offsets),
                                          n_sets, n_total, float(eps2), _ptr(energy),
                                          _ptr(counts), _ptr(ws), nbytes, flags,
                                          _stream(stream)), "pairs_energy_f32_batched")


def pairs_force_f32_batched(x, y, z, offsets, eps2, fx, fy, fz, ws=None, flags: int = 0,
                            stream=None) -> None:
    """Forces within every set of a CSR batch into float64[n_total] tensors."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z), torch.float32, offsets,
                                    "pairs_force_f32_batched")
    _require((fx, fy, fz), torch.float64, n_total, "pairs_force_f32_batched forces")
    ws, nbytes = _workspace(ws, n_sets, n_total, x.device)
    _check(lib().pairs_force_f32_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(offsets), n_sets,
                                         n_total, float(eps2), _ptr(fx), _ptr(fy), _ptr(fz),
                                         _ptr(ws), nbytes, flags, _stream(stream)),
           "pairs_force_f32_batched")


def pairs_energy_f64_batched(x, y, z, offsets, eps2, set_energy, energy=None, ws=None,
                             flags: int = 0, stream=None) -> None:
    """Double-precision potential per set (float64[n_sets]) and, if energy is
    given, per object (float64[n_total]), for float64 inputs."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z), torch.float64, offsets,
                                    "pairs_energy_f64_batched")
    _require((set_energy,), torch.float64, n_sets, "pairs_energy_f64_batched set_energy")
    if energy is not None:
        _require((energy,), torch.float64, n_total, "pairs_energy_f64_batched energy")
    ws, nbytes = _workspace(ws, n_sets, n_total, x.device)
    _check(lib().pairs_energy_f64_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(offsets), n_sets,
                                          n_total, float(eps2), _ptr(set_energy),
                                          _ptr(energy), _ptr(ws), nbytes, flags,
                                          _stream(stream)), "pairs_energy_f64_batched")


def pairs_binned_workspace_size(n: int) -> int:
    """Bytes of device workspace a binned count of n objects needs."""
    b = _sz(0)
    _check(lib().pairs_binned_workspace_size(n, ctypes.byref(b)), "pairs_binned_workspace_size")
    return int(b.value)


def pairs_count_i32_binned(x, y, z, r, cell: int, out, ws=None, flags: int = 0,
                           stream=None) -> None:
    """Exact collision count of one int32 sphere set through a uniform grid of
    cells of side `cell` (every radius at most cell/2) into out (int64[1])."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z, r), torch.int32, n, "pairs_count_i32_binned")
    _require((out,), torch.int64, 1, "pairs_count_i32_binned out")
    need = pairs_binned_workspace_size(n)
    if ws is None and need > 0:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
    _check(lib().pairs_count_i32_binned(_ptr(x), _ptr(y), _ptr(z), _ptr(r), n, int(cell),
                                        _ptr(out), _ptr(ws), nbytes, flags, _stream(stream)),
           "pairs_count_i32_binned")


def pairs_count_i32_binned_batched(x, y, z, r, offsets, cell: int, counts, ws=None,
                                   flags: int = 0, stream=None) -> None:
    """Binned collision count of every set of a CSR batch into counts
    (int64[n_sets], read as uint64); pairs across sets are never counted."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z, r), torch.int32, offsets,
                                    "pairs_count_i32_binned_batched")
    _require((counts,), torch.int64, n_sets, "pairs_count_i32_binned_batched counts")
    need = pairs_binned_workspace_size(n_total)
    if ws is None and need > 0:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
    _check(lib().pairs_count_i32_binned_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(r),
                                                _ptr(offsets), n_sets, n_total, int(cell),
                                                _ptr(counts), _ptr(ws), nbytes, flags,
                                                _stream(stream)),
           "pairs_count_i32_binned_batched")


def pairs_lattice_workspace_size(n_sets: int, n_total: int, max_n: int) -> int:
    """Bytes of device workspace a lattice call needs (max_n = 0: unknown)."""
    b = _sz(0)
    _check(lib().pairs_lattice_workspace_size(n_sets, n_total, max_n, ctypes.byref(b)),
           "pairs_lattice_workspace_size")
    return int(b.value)


def _lattice_ws(ws, n_sets, n_total, max_n, device):
    import torch
    need = pairs_lattice_workspace_size(n_sets, n_total, max_n)
    if ws is None and need > 0:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    return ws, 0 if ws is None else int(ws.numel() * ws.element_size())


def pairs_lattice_count(x, y, z, collisions, contacts, ws=None, flags: int = 0,
                        stream=None) -> None:
    """Collisions and contacts of one vector of int32 lattice beads into
    int64[1] tensors (read as uint64); either output may be None."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z), torch.int32, n, "pairs_lattice_count")
    for t in (collisions, contacts):
        if t is not None:
            _require((t,), torch.int64, 1, "pairs_lattice_count outputs")
    ws, nbytes = _lattice_ws(ws, 1, n, n, x.device)
    _check(lib().pairs_lattice_count(_ptr(x), _ptr(y), _ptr(z), n, _ptr(collisions),
                                     _ptr(contacts), _ptr(ws), nbytes, flags, _stream(stream)),
           "pairs_lattice_count")


def pairs_lattice_count_batched(x, y, z, offsets, max_n: int, collisions, contacts, ws=None,
                                flags: int = 0, stream=None) -> None:
    """Per-vector collisions and contacts of a CSR batch of lattice bead vectors
    into int64[n_sets] tensors (read as uint64); either output may be None.
    max_n bounds every vector's length (0: unknown)."""
    import torch
    n_total, n_sets = _batch_checks(x, (x, y, z), torch.int32, offsets,
                                    "pairs_lattice_count_batched")
    for t in (collisions, contacts):
        if t is not None:
            _require((t,), torch.int64, n_sets, "pairs_lattice_count_batched outputs")
    ws, nbytes = _lattice_ws(ws, n_sets, n_total, max_n, x.device)
    _check(lib().pairs_lattice_count_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(offsets), n_sets,
                                             n_total, max_n, _ptr(collisions), _ptr(contacts),
                                             _ptr(ws), nbytes, flags, _stream(stream)),
           "pairs_lattice_count_batched")


def pairs_jitter_f32(x, y, z, seed: int, step: int, sigma: float, first_index: int = 0,
                     stream=None) -> None:
    """One in-place perturbation step of float32 positions (see include/pairs.h)."""
    import torch
    n = int(x.shape[0])
    _require((x, y, z), torch.float32, n, "pairs_jitter_f32")
    _check(lib().pairs_jitter_f32(_ptr(x), _ptr(y), _ptr(z), n, seed, step, float(sigma),
                                  first_index, _stream(stream)), "pairs_jitter_f32")


def pairs_debug_task_ranges(n: int, rows_per_lane: int, chunk: int):
    """Host-only: the (first row, u0, u1) of every wave task of a set of n objects."""
    import numpy as np
    cnt = _i64(0)
    _check(lib().pairs_debug_task_ranges(n, rows_per_lane, chunk, None, 0, ctypes.byref(cnt)),
           "pairs_debug_task_ranges")
    out = np.zeros((int(cnt.value), 3), dtype=np.int32)
    _check(lib().pairs_debug_task_ranges(n, rows_per_lane, chunk, out.ctypes.data_as(_vp),
                                         int(cnt.value), ctypes.byref(cnt)),
           "pairs_debug_task_ranges")
    return out


def pairs_debug_step_ranges(n: int, rows_per_lane: int, chunk: int):
    """Host-only: the (first row, s0, T, x) of every stepping-form task of a
    set of n objects."""
    import numpy as np
    cnt = _i64(0)
    _check(lib().pairs_debug_step_ranges(n, rows_per_lane, chunk, None, 0, ctypes.byref(cnt)),
           "pairs_debug_step_ranges")
    out = np.zeros((int(cnt.value), 4), dtype=np.int32)
    _check(lib().pairs_debug_step_ranges(n, rows_per_lane, chunk, out.ctypes.data_as(_vp),
                                         int(cnt.value), ctypes.byref(cnt)),
           "pairs_debug_step_ranges")
    return out


def pairs_debug_task_at(n: int, rows_per_lane: int, chunk: int, tasks):
    """Host-only: (first row, u0, u1) of the given task indices of a set of n
    objects, decoded as the single-set kernels decode them."""
    import numpy as np
    t = np.ascontiguousarray(tasks, dtype=np.int64)
    out = np.zeros((t.shape[0], 3), dtype=np.int64)
    _check(lib().pairs_debug_task_at(n, rows_per_lane, chunk, t.ctypes.data_as(_vp),
                                     int(t.shape[0]), out.ctypes.data_as(_vp)),
           "pairs_debug_task_at")
    return out


def pairs_debug_single_launch(kind: int, n: int):
    """Host-only: (tasks, blocks, threads per block) of the launch a single-set
    call of `kind` makes for n objects."""
    t, b, w = _i64(0), _i64(0), ctypes.c_int32(0)
    _check(lib().pairs_debug_single_launch(kind, n, ctypes.byref(t), ctypes.byref(b),
                                           ctypes.byref(w)), "pairs_debug_single_launch")
    return int(t.value), int(b.value), int(w.value)


def _shape_mode(batched) -> int:
    """False/True (single-set or batched calls) or a SHAPES_* mode (any
    integral type)."""
    import numbers
    if isinstance(batched, numbers.Integral):   # bool is integral too: 0 or 1
        return int(batched)
    return int(bool(batched))


def pairs_get_shapes(kind: int, batched):
    """The tile-shape table as a list of (min_n, rows_per_lane, chunk, form);
    batched: False/True or SHAPES_SINGLE, SHAPES_BATCHED, SHAPES_TOTAL_ONLY."""
    t = ShapeTable()
    _check(lib().pairs_get_shapes(kind, _shape_mode(batched), ctypes.byref(t)),
           "pairs_get_shapes")
    return [(t.min_n[c], t.rows_per_lane[c], t.chunk[c], t.form[c]) for c in range(t.count)]


def pairs_set_shapes(kind: int, batched, entries) -> None:
    """Set the tile-shape table from (min_n, rows_per_lane, chunk[, form])
    entries, largest sets first (form defaults to FORM_BROADCAST); None
    restores the defaults.  batched as for pairs_get_shapes."""
    if entries is None:
        _check(lib().pairs_set_shapes(kind, _shape_mode(batched), None), "pairs_set_shapes")
        return
    t = ShapeTable()
    t.count = len(entries)
    for c, e in enumerate(entries):
        lo, k, u = e[:3]
        form = e[3] if len(e) > 3 else FORM_BROADCAST
        t.min_n[c], t.rows_per_lane[c], t.chunk[c], t.form[c] = int(lo), int(k), int(u), int(form)
    _check(lib().pairs_set_shapes(kind, _shape_mode(batched), ctypes.byref(t)), "pairs_set_shapes")


class Plan:
    """A precomputed batched schedule (pairs_plan_create); h_offsets is a host
    int64 array of n_sets + 1 offsets."""

    def __init__(self, kind: int, h_offsets):
        import numpy as np
        off = np.ascontiguousarray(h_offsets, dtype=np.int64)
        self.kind = kind
        self.n_sets = int(off.shape[0]) - 1
        self.n_total = int(off[-1]) if off.shape[0] else 0
        h = _vp()
        _check(lib().pairs_plan_create(kind, off.ctypes.data_as(_vp), self.n_sets,
                                       ctypes.byref(h)), "pairs_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self):
        a, b, c = _i64(0), _i64(0), _i64(0)
        _check(lib().pairs_plan_info(self._h, ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(c)), "pairs_plan_info")
        return {"n_sets": a.value, "n_total": b.value, "n_tasks": c.value}

    def execute(self, inputs, outputs, eps2: float = 0.0, stream=None) -> None:
        """inputs = (x, y, z, r or None); outputs = (counts,) or (energy, counts or None)."""
        ins = (_vp * 4)(*[None if t is None else t.data_ptr() for t in inputs])
        outs = (_vp * 2)(*[None if t is None else t.data_ptr() for t in outputs] +
                         [None] * (2 - len(outputs)))
        _check(lib().pairs_plan_execute(self._h, ins, outs, float(eps2), _stream(stream)),
               "pairs_plan_execute")

    def capture_steps(self, x, y, z, r, seed: int, sigma: float, first_step: int,
                      n_steps: int, eps2: float, energy, counts=None):
        """Graph of n_steps (jitter, execute) steps; energy is float64[n_steps * n_sets]."""
        import torch
        _require((x, y, z) if r is None else (x, y, z, r), torch.float32, self.n_total,
                 "Plan.capture_steps")
        need = n_steps * self.n_sets
        if energy.dtype != torch.float64 or energy.numel() < need or not energy.is_contiguous():
            raise ValueError(f"Plan.capture_steps: energy must hold {need} float64 values")
        if (counts is None) != (r is None):
            raise ValueError("Plan.capture_steps: give both r and counts or neither")
        if counts is not None and (counts.dtype != torch.int64 or counts.numel() < need
                                   or not counts.is_contiguous()):
            raise ValueError(f"Plan.capture_steps: counts must hold {need} int64 values")
        g = _vp()
        _check(lib().pairs_plan_capture_steps(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(r), seed,
                                              float(sigma), first_step, n_steps, float(eps2),
                                              _ptr(energy), _ptr(counts), ctypes.byref(g)),
               "pairs_plan_capture_steps")
        return Graph(g)

    def close(self):
        if getattr(self, "_h", None):
            lib().pairs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured HIP graph of repeated steps (pairs_plan_capture_steps)."""

    def __init__(self, handle):
        self._h = handle

    def launch(self, stream=None) -> None:
        _check(lib().pairs_graph_launch(self._h, _stream(stream)), "pairs_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            lib().pairs_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Convenience forms that allocate their outputs.

def count_i32(x, y, z, r, validate: bool = False) -> int:
    import torch
    out = torch.empty(1, dtype=torch.int64, device=x.device)
    pairs_count_i32(x, y, z, r, out, FLAG_VALIDATE if validate else 0)
    return int(out.item())


def count_f32(x, y, z, r, validate: bool = False) -> int:
    import torch
    out = torch.empty(1, dtype=torch.int64, device=x.device)
    pairs_count_f32(x, y, z, r, out, FLAG_VALIDATE if validate else 0)
    return int(out.item())


def energy_f32(x, y, z, eps2: float = 1e-4, per_particle: bool = True,
               deterministic: bool = False):
    """Returns (per-particle float64 tensor or None, total as a Python float);
    deterministic selects the run-to-run reproducible fixed-point reduction."""
    import torch
    n = int(x.shape[0])
    total = torch.empty(1, dtype=torch.float64, device=x.device)
    energy = torch.empty(n, dtype=torch.float64, device=x.device) if per_particle else None
    pairs_energy_f32(x, y, z, eps2, energy, total,
                     FLAG_DETERMINISTIC if deterministic else 0)
    return energy, float(total.item())
