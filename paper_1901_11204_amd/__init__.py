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
    "PairsError", "lib", "lib_path", "FLAG_VALIDATE",
    "pairs_count_i32", "pairs_count_f32", "pairs_energy_f32",
    "count_i32", "count_f32", "energy_f32",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpairs.so")
_lib = None

FLAG_VALIDATE = 1

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


def _declare(L):
    sig = {
        "pairs_count_i32": [_vp, _vp, _vp, _vp, _i64, _vp, _u32, _vp],
        "pairs_count_f32": [_vp, _vp, _vp, _vp, _i64, _vp, _u32, _vp],
        "pairs_energy_f32": [_vp, _vp, _vp, _i64, _f32, _vp, _vp, _u32, _vp],
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
        L = ctypes.CDLL(_LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


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


def energy_f32(x, y, z, eps2: float = 1e-4, per_particle: bool = True):
    """Returns (per-particle float64 tensor or None, total as a Python float)."""
    import torch
    n = int(x.shape[0])
    total = torch.empty(1, dtype=torch.float64, device=x.device)
    energy = torch.empty(n, dtype=torch.float64, device=x.device) if per_particle else None
    pairs_energy_f32(x, y, z, eps2, energy, total)
    return energy, float(total.item())
