"""Seeded synthetic inputs for the all-pairs interaction path.

This module only draws random inputs; it holds none of the method's arithmetic.
Both the CPU oracle tests and the GPU path (tests, bench) take their inputs from
here, so they see identical arrays for a given recipe and seed.

Every generator uses ``numpy.random.default_rng(seed)`` and draws in the order
written.  The object sets are returned as structure-of-arrays (one contiguous
array per coordinate), the layout the GPU kernels read.

The paper's own GPU workload is "random vectors of floating point spheres of
diameter 1" with an unstated distribution (Section 5, experiments on the GPU).
The recipes below stand in for it with uniform boxes, as fixed in the
measurement plan of this library.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Spheres", "Particles", "Batch",
    "spheres_i32", "particles_f32",
    "config1", "config2", "config3", "config4", "config5",
    "lognormal_sizes", "offsets_from_sizes",
]


class Spheres:
    """int32 or float32 sphere centres and radii, SoA."""

    def __init__(self, x, y, z, r):
        self.x, self.y, self.z, self.r = x, y, z, r

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return self.x, self.y, self.z, self.r


class Particles:
    """float32 particle positions, SoA."""

    def __init__(self, x, y, z):
        self.x, self.y, self.z = x, y, z

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return self.x, self.y, self.z


class Batch:
    """A CSR batch: set s owns objects [offsets[s], offsets[s+1])."""

    def __init__(self, offsets, objs):
        self.offsets = offsets
        self.objs = objs

    @property
    def n_sets(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_total(self) -> int:
        return int(self.offsets[-1])


def _soa(a: np.ndarray):
    return tuple(np.ascontiguousarray(a[:, k]) for k in range(a.shape[1]))


def spheres_i32(n: int, seed: int, coord_hi: int, radius_hi: int, coord_lo: int = 0,
                radius_lo: int = 1) -> Spheres:
    """Centres uniform in [coord_lo, coord_hi)^3, radii uniform in [radius_lo, radius_hi]."""
    rng = np.random.default_rng(seed)
    xyz = rng.integers(coord_lo, coord_hi, (n, 3), dtype=np.int32)
    r = rng.integers(radius_lo, radius_hi, n, dtype=np.int32, endpoint=True)
    x, y, z = _soa(xyz)
    return Spheres(x, y, z, r)


def particles_f32(n: int, seed: int) -> Particles:
    """Positions uniform in the unit cube [0, 1)^3, float32."""
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3), dtype=np.float32)
    return Particles(*_soa(xyz))


def config1(seed: int = 1) -> Spheres:
    """N=4096 int32 spheres: centres in [0, 2^16)^3, radii in [1, 2^9]."""
    return spheres_i32(4096, seed, 2 ** 16, 2 ** 9)


def config2(n: int = 2 ** 20, seed: int | None = None) -> Spheres:
    """N=2^20 (seed 2) or N=2^20-1 (seed 3) int32 spheres: centres in [0, 2^24)^3,
    radii in [1, 2^14]."""
    if seed is None:
        seed = 2 if n % 2 == 0 else 3
    return spheres_i32(n, seed, 2 ** 24, 2 ** 14)


def config3(n: int = 2 ** 18, seed: int = 4) -> Particles:
    """N=2^18 float32 particles uniform in the unit cube."""
    return particles_f32(n, seed)


def lognormal_sizes(rng: np.random.Generator, n_sets: int, mu: float, sigma: float,
                    lo: int, hi: int) -> np.ndarray:
    """Set sizes clip(rint(lognormal(mu, sigma)), lo, hi) as int64."""
    s = rng.lognormal(mu, sigma, n_sets)
    return np.clip(np.rint(s), lo, hi).astype(np.int64)


def offsets_from_sizes(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def config4(n_sets: int = 200_000, seed: int = 5, size_hi: int = 8192) -> Batch:
    """Binned int32 spheres: set s is the content of one 2^14-sided cell of a 64^3 grid
    over [0, 2^20)^3.  Sizes lognormal(4, 1.2) clipped to [2, size_hi]; radii in [1, 2^8]."""
    rng = np.random.default_rng(seed)
    sizes = lognormal_sizes(rng, n_sets, 4.0, 1.2, 2, size_hi)
    cells = rng.choice(64 ** 3, n_sets, replace=False).astype(np.int64)
    off = offsets_from_sizes(sizes)
    total = int(off[-1])
    set_of = np.repeat(np.arange(n_sets, dtype=np.int64), sizes)
    c = cells[set_of]
    origin = np.stack([c % 64, (c // 64) % 64, c // 4096], axis=1) * (2 ** 14)
    xyz = (origin + rng.integers(0, 2 ** 14, (total, 3))).astype(np.int32)
    r = rng.integers(1, 2 ** 8, total, dtype=np.int32, endpoint=True)
    x, y, z = _soa(xyz)
    return Batch(off, Spheres(x, y, z, r))


def config5(n_sets: int = 50_000, seed: int = 6, size_hi: int = 4096,
            radius: float = 0.01) -> Batch:
    """float32 particle sets, each in its own unit cube; sizes lognormal(5, 1) clipped to
    [2, size_hi]; a common collision radius (0.01) stored per object."""
    rng = np.random.default_rng(seed)
    sizes = lognormal_sizes(rng, n_sets, 5.0, 1.0, 2, size_hi)
    off = offsets_from_sizes(sizes)
    total = int(off[-1])
    xyz = rng.random((total, 3), dtype=np.float32)
    x, y, z = _soa(xyz)
    r = np.full(total, np.float32(radius), dtype=np.float32)
    return Batch(off, Spheres(x, y, z, r))
