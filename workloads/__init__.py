"""Seeded synthetic inputs for the all-pairs interaction path.

This module only draws random inputs; it holds none of the method's arithmetic.
Both the CPU oracle tests and the GPU path (tests, bench) take their inputs from
here, so they see identical arrays for a given recipe and seed.

Every generator uses ``numpy.random.default_rng(seed)`` and draws in the order
written.  The object sets are returned as structure-of-arrays (one contiguous
array per coordinate), the layout the GPU kernels read.

The paper's own GPU workload is randomly generated vectors of spheres with
floating-point coordinates and unit diameter, distribution unstated (Section
5).  The sphere recipes below stand in for it with uniform boxes.  The lattice
recipes follow the bead vectors of the paper's linear-time counting
experiments (Section 5): chains grown from the origin by random unit steps, or
coordinates drawn from a rounded normal distribution.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Spheres", "Particles", "Batch",
    "spheres_i32", "particles_f32",
    "spheres_4096", "spheres_2p24", "particles_unit_cube", "binned_sets", "moving_sets",
    "lognormal_sizes", "offsets_from_sizes",
    "Beads", "lattice_walks", "lattice_normal", "lattice_paper", "lattice_large",
    "lattice_short",
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


def spheres_4096(seed: int = 1) -> Spheres:
    """N=4096 int32 spheres: centres in [0, 2^16)^3, radii in [1, 2^9]."""
    return spheres_i32(4096, seed, 2 ** 16, 2 ** 9)


def spheres_2p24(n: int = 2 ** 20, seed: int | None = None) -> Spheres:
    """N=2^20 (seed 2) or N=2^20-1 (seed 3) int32 spheres: centres in [0, 2^24)^3,
    radii in [1, 2^14]."""
    if seed is None:
        seed = 2 if n % 2 == 0 else 3
    return spheres_i32(n, seed, 2 ** 24, 2 ** 14)


def particles_unit_cube(n: int = 2 ** 18, seed: int = 4) -> Particles:
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


def binned_sets(n_sets: int = 200_000, seed: int = 5, size_hi: int = 8192) -> Batch:
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


def moving_sets(n_sets: int = 50_000, seed: int = 6, size_hi: int = 4096,
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


class Beads:
    """int32 lattice points, SoA."""

    def __init__(self, x, y, z):
        self.x, self.y, self.z = x, y, z

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return self.x, self.y, self.z


_STEPS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                  dtype=np.int32)


def lattice_walks(n_vectors: int, n_beads, seed: int) -> Batch:
    """Bead vectors grown as chains: bead 0 of every vector at the origin, each
    later bead one unit from the previous one along one of the six axis
    directions, drawn uniformly.  n_beads is one length for all vectors or an
    array of lengths (each >= 1)."""
    rng = np.random.default_rng(seed)
    sizes = np.broadcast_to(np.asarray(n_beads, dtype=np.int64), (n_vectors,)).copy()
    off = offsets_from_sizes(sizes)
    total = int(off[-1])
    d = rng.integers(0, 6, total, dtype=np.int8)
    first = off[:-1][sizes > 0]
    out = []
    for axis in range(3):
        step = _STEPS[:, axis][d]
        step[first] = 0  # the first bead of each vector sits at the origin
        c = np.cumsum(step, dtype=np.int64)
        # restart the running sum at every vector
        base = np.repeat(c[first] - step[first], sizes[sizes > 0])
        out.append((c - base).astype(np.int32))
    return Batch(off, Beads(*out))


def lattice_normal(n_vectors: int, n_beads: int, sigma: float, seed: int) -> Batch:
    """Bead vectors with every coordinate rint(normal(0, sigma)), as int32."""
    rng = np.random.default_rng(seed)
    sizes = np.full(n_vectors, n_beads, dtype=np.int64)
    off = offsets_from_sizes(sizes)
    xyz = np.rint(rng.normal(0.0, sigma, (int(off[-1]), 3))).astype(np.int32)
    return Batch(off, Beads(*_soa(xyz)))


def lattice_paper(seed: int = 7) -> Batch:
    """1000 chains of 1920 beads: the batch size and the largest chain length of
    the paper's linear-time counting experiments."""
    return lattice_walks(1000, 1920, seed)


def lattice_large(seed: int = 8) -> Batch:
    """65536 chains of 1920 beads (126 M beads, 1.5 GB of int32 coordinates): the
    throughput workload of the lattice counts."""
    return lattice_walks(65536, 1920, seed)


def lattice_short(seed: int = 9) -> Batch:
    """131072 chains of 128 beads, the common protein length of the paper's
    structure-prediction experiments (16.8 M beads)."""
    return lattice_walks(131072, 128, seed)
