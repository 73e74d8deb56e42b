"""CPU oracle for the all-pairs interaction path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library does not import, link or call it.

The functions are thin ctypes wrappers over ``pairs_oracle.c``, the plain
definition of what the path computes (the standard i < j pairwise loop of the
paper, Section 4).  Arrays are numpy, converted to contiguous arrays of the
stated dtype.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_I64 = ctypes.c_int64
_INT = ctypes.c_int


def lib():
    """Load liboracle.so, building it first only if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    L = ctypes.CDLL(_build.LIB)
    L.oracle_threads.argtypes = [_INT]
    L.oracle_threads.restype = _INT
    L.oracle_count_i32.argtypes = [_i32p] * 4 + [_I64, _INT]
    L.oracle_count_i32.restype = ctypes.c_uint64
    L.oracle_count_f32.argtypes = [_f32p] * 4 + [_I64, _INT]
    L.oracle_count_f32.restype = ctypes.c_uint64
    L.oracle_cross_count_i32.argtypes = [_i32p] * 4 + [_I64] + [_i32p] * 4 + [_I64, _INT]
    L.oracle_cross_count_i32.restype = ctypes.c_uint64
    L.oracle_energy_total.argtypes = [_f32p] * 3 + [_I64, ctypes.c_float, _INT]
    L.oracle_energy_total.restype = ctypes.c_double
    L.oracle_energy_rows.argtypes = [_f32p] * 3 + [_I64, ctypes.c_float, ctypes.c_void_p,
                                                   _I64, _f64p, _INT]
    L.oracle_energy_rows.restype = None
    L.oracle_count_i32_batched.argtypes = [_i32p] * 4 + [_i64p, _I64, _u64p, _INT]
    L.oracle_count_i32_batched.restype = None
    L.oracle_energy_count_f32_batched.argtypes = [_f32p] * 4 + [_i64p, _I64, ctypes.c_float,
                                                               ctypes.c_void_p, ctypes.c_void_p,
                                                               _INT]
    L.oracle_energy_count_f32_batched.restype = None
    L.oracle_energy_f64_total.argtypes = [_f64p] * 3 + [_I64, ctypes.c_double, _INT]
    L.oracle_energy_f64_total.restype = ctypes.c_double
    L.oracle_energy_f64_rows.argtypes = [_f64p] * 3 + [_I64, ctypes.c_double, ctypes.c_void_p,
                                                       _I64, _f64p, _INT]
    L.oracle_energy_f64_rows.restype = None
    L.oracle_force_rows.argtypes = [_f32p] * 3 + [_I64, ctypes.c_float, ctypes.c_void_p, _I64,
                                             _f64p, _f64p, _f64p, _f64p, _INT]
    L.oracle_force_rows.restype = None
    L.oracle_lattice_batched.argtypes = [_i32p] * 3 + [_i64p, _I64, _u64p, _u64p, _INT]
    L.oracle_lattice_batched.restype = None
    L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.oracle_philox4x32_10.restype = None
    L.oracle_jitter_scale.argtypes = [ctypes.c_float]
    L.oracle_jitter_scale.restype = ctypes.c_float
    L.oracle_jitter_f32.argtypes = [_f32p] * 3 + [_I64, ctypes.c_uint64, ctypes.c_uint32,
                                                  ctypes.c_float, _I64]
    L.oracle_jitter_f32.restype = None
    _lib = L
    return L


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def threads(threads: int = 0) -> int:
    """Threads an oracle call with this ``threads`` argument uses (0 = all)."""
    return int(lib().oracle_threads(threads))


def count_i32(x, y, z, r, threads: int = 0) -> int:
    """Exact collision count of one int32 sphere set (i < j loop, 128-bit arithmetic)."""
    x, y, z, r = (_c(a, np.int32) for a in (x, y, z, r))
    return int(lib().oracle_count_i32(x, y, z, r, x.shape[0], threads))


def count_f32(x, y, z, r, threads: int = 0) -> int:
    """Collision count of one float32 sphere set under the pinned binary32 predicate."""
    x, y, z, r = (_c(a, np.float32) for a in (x, y, z, r))
    return int(lib().oracle_count_f32(x, y, z, r, x.shape[0], threads))


def cross_count_i32(a, b, threads: int = 0) -> int:
    """Colliding pairs with one sphere in set a and one in set b; a, b = (x, y, z, r)."""
    a = [_c(v, np.int32) for v in a]
    b = [_c(v, np.int32) for v in b]
    return int(lib().oracle_cross_count_i32(*a, a[0].shape[0], *b, b[0].shape[0], threads))


def energy_total(x, y, z, eps2=np.float32(1e-4), threads: int = 0) -> float:
    """sum_{i<j} 1/sqrt(|p_i - p_j|^2 + eps2) in double, Neumaier-compensated."""
    x, y, z = (_c(a, np.float32) for a in (x, y, z))
    return float(lib().oracle_energy_total(x, y, z, x.shape[0], np.float32(eps2), threads))


def energy_rows(x, y, z, eps2=np.float32(1e-4), rows=None, threads: int = 0) -> np.ndarray:
    """E_i = sum_{j != i} e_ij for the given rows (all rows if None), double."""
    x, y, z = (_c(a, np.float32) for a in (x, y, z))
    n = x.shape[0]
    if rows is None:
        out = np.zeros(n, np.float64)
        lib().oracle_energy_rows(x, y, z, n, np.float32(eps2), None, 0, out, threads)
    else:
        rows = _c(rows, np.int64)
        out = np.zeros(rows.shape[0], np.float64)
        lib().oracle_energy_rows(x, y, z, n, np.float32(eps2),
                                 rows.ctypes.data_as(ctypes.c_void_p), rows.shape[0], out,
                                 threads)
    return out


def energy_f64_total(x, y, z, eps2=1e-4, threads: int = 0) -> float:
    """sum_{i<j} 1/sqrt(|p_i - p_j|^2 + eps2) for float64 inputs, Neumaier-compensated."""
    x, y, z = (_c(a, np.float64) for a in (x, y, z))
    return float(lib().oracle_energy_f64_total(x, y, z, x.shape[0], float(eps2), threads))


def energy_f64_rows(x, y, z, eps2=1e-4, rows=None, threads: int = 0) -> np.ndarray:
    """E_i = sum_{j != i} e_ij for float64 inputs, for the given rows (all if None)."""
    x, y, z = (_c(a, np.float64) for a in (x, y, z))
    n = x.shape[0]
    if rows is None:
        out = np.zeros(n, np.float64)
        lib().oracle_energy_f64_rows(x, y, z, n, float(eps2), None, 0, out, threads)
    else:
        rows = _c(rows, np.int64)
        out = np.zeros(rows.shape[0], np.float64)
        lib().oracle_energy_f64_rows(x, y, z, n, float(eps2),
                                     rows.ctypes.data_as(ctypes.c_void_p), rows.shape[0], out,
                                     threads)
    return out


def force_rows(x, y, z, eps2=np.float32(1e-4), rows=None, threads: int = 0):
    """Forces of the softened potential on the given rows (all if None):
    (F, S) with F float64[m, 3], F_i = sum_{j != i} (p_i - p_j)/(d^2 + eps2)^1.5,
    and S float64[m] the sum of the terms' norms."""
    x, y, z = (_c(a, np.float32) for a in (x, y, z))
    n = x.shape[0]
    if rows is None:
        m, rp = n, None
    else:
        rows = _c(rows, np.int64)
        m, rp = rows.shape[0], rows.ctypes.data_as(ctypes.c_void_p)
    F = [np.zeros(m, np.float64) for _ in range(3)]
    S = np.zeros(m, np.float64)
    lib().oracle_force_rows(x, y, z, n, np.float32(eps2), rp, m, F[0], F[1], F[2], S, threads)
    return np.stack(F, axis=1), S


def count_i32_batched(x, y, z, r, offsets, threads: int = 0) -> np.ndarray:
    """Per-set exact collision counts of a CSR batch of int32 sphere sets."""
    x, y, z, r = (_c(a, np.int32) for a in (x, y, z, r))
    off = _c(offsets, np.int64)
    out = np.zeros(off.shape[0] - 1, np.uint64)
    lib().oracle_count_i32_batched(x, y, z, r, off, off.shape[0] - 1, out, threads)
    return out


def energy_count_f32_batched(x, y, z, r, offsets, eps2=np.float32(1e-4), threads: int = 0):
    """Per-set (energy total, pinned-fp32 collision count) of a CSR batch."""
    x, y, z, r = (_c(a, np.float32) for a in (x, y, z, r))
    off = _c(offsets, np.int64)
    m = off.shape[0] - 1
    e = np.zeros(m, np.float64)
    c = np.zeros(m, np.uint64)
    lib().oracle_energy_count_f32_batched(x, y, z, r, off, m, np.float32(eps2),
                                          e.ctypes.data_as(ctypes.c_void_p),
                                          c.ctypes.data_as(ctypes.c_void_p), threads)
    return e, c


def lattice_counts_batched(x, y, z, offsets, threads: int = 0):
    """Per bead vector (CSR), the number of bead pairs on one lattice site
    (collisions) and on neighbouring sites (contacts), as two uint64 arrays;
    the plain pairwise definition of the paper's Section 3 counts."""
    x, y, z = (_c(a, np.int32) for a in (x, y, z))
    off = _c(offsets, np.int64)
    n_sets = off.shape[0] - 1
    coll = np.zeros(n_sets, np.uint64)
    cont = np.zeros(n_sets, np.uint64)
    lib().oracle_lattice_batched(x, y, z, off, n_sets, coll, cont, threads)
    return coll, cont


def lattice_counts(x, y, z, threads: int = 0):
    """(collisions, contacts) of one bead vector."""
    n = np.asarray(x).shape[0]
    c, t = lattice_counts_batched(x, y, z, np.array([0, n], np.int64), threads)
    return int(c[0]), int(t[0])


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al., SC 2011)."""
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_c(ctr, np.uint32), _c(key, np.uint32), out)
    return out


def jitter_scale(sigma: float) -> np.float32:
    return np.float32(lib().oracle_jitter_scale(np.float32(sigma)))


def jitter_f32(x, y, z, seed: int, step: int, sigma: float, first_index: int = 0):
    """Return perturbed copies of (x, y, z) after one jitter step."""
    x, y, z = (np.array(a, dtype=np.float32, copy=True) for a in (x, y, z))
    lib().oracle_jitter_f32(x, y, z, x.shape[0], seed, step, np.float32(sigma), first_index)
    return x, y, z
