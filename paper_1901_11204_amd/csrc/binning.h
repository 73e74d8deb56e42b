// Collision count of one set of int32 spheres through a uniform grid of
// cells: the pruning step the paper places before the pairwise count (pruned
// sets, Sections 1 and 6), with the pairwise count itself done on the
// balanced assignment inside each cell.
//
// With every radius at most half the cell side L, two spheres that touch
// are at most L apart along each axis, so their cells differ by at most one
// along each axis.  The count is then the sum, over occupied cells c, of the
// pairs inside c and the pairs between c and each occupied cell among its 13
// forward neighbours (offsets (dx, dy, dz) after (0, 0, 0) in lexicographic
// order), which meets every pair of neighbouring cells once.
//
// Pipeline (all on the device, no host synchronisation):
//   1. k_bin_keys: cell coordinates (x + 2^24) / L + 1 per axis (the +1 keeps
//      the -1 neighbours of cell 0 in range), packed 21 bits per axis into a
//      64-bit key, and the object index;
//   2. radix sort of (key, index) (rocPRIM);
//   3. k_bin_gather: the objects in key order, structure of arrays;
//   4. run-length encoding of the sorted keys (rocPRIM) into the occupied
//      cells' keys and sizes, and an exclusive scan of the sizes into cell
//      offsets;
//   5. k_bin_hash_build: a hash table from occupied cell keys to their
//      indices;
//   6. k_bin_count: 16 lanes per occupied cell (cells of more than 64
//      objects go to a list that k_bin_count_big counts, one wave per cell).
//      Lanes 0..12 of a group look up the 13 forward neighbours in the
//      table; the pairs inside
//      the cell run on the balanced circular assignment (each lane takes rows
//      and their steps s = 1 .. floor((n-1)/2), rows i < n/2 also s = n/2
//      when n is even); the pairs with each neighbour run with the lanes
//      taking the cell's objects against all of the neighbour's.  Wave sums
//      go to the count with one atomic per wave.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace pairs_binning {

using pairs_dev::kWave;

constexpr int kBlock = 256;
constexpr int kCellBits = 21;  // per axis
constexpr uint64_t kAxisMask = (uint64_t(1) << kCellBits) - 1;
constexpr int kOffsetBias = 1 << 24;  // coordinates in [-2^24, 2^24]

// Cell coordinate of a coordinate, offset by one.
__device__ __forceinline__ uint32_t cell_of(int v, int L) {
    return (uint32_t)(v + kOffsetBias) / (uint32_t)L + 1;
}

__device__ __forceinline__ uint64_t cell_key(uint32_t cx, uint32_t cy, uint32_t cz) {
    return ((uint64_t)cx << (2 * kCellBits)) | ((uint64_t)cy << kCellBits) | (uint64_t)cz;
}

// Domain check of the binned count: coordinates in [-2^24, 2^24] and radii
// in [0, L/2].
__global__ void k_bin_validate(const int32_t *x, const int32_t *y, const int32_t *z,
                               const int32_t *r, int64_t n, int L, int *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int B = kOffsetBias;
    const bool ok = x[i] >= -B && x[i] <= B && y[i] >= -B && y[i] <= B && z[i] >= -B &&
                    z[i] <= B && r[i] >= 0 && 2 * (int64_t)r[i] <= L;
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_bin_keys(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                           const int32_t *__restrict__ z, int64_t n, int L,
                           uint64_t *__restrict__ keys, uint32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = cell_key(cell_of(x[i], L), cell_of(y[i], L), cell_of(z[i], L));
    idx[i] = (uint32_t)i;
}

__global__ void k_bin_gather(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                             const int32_t *__restrict__ z, const int32_t *__restrict__ r,
                             const uint32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ sx,
                             int32_t *__restrict__ sy, int32_t *__restrict__ sz,
                             int32_t *__restrict__ sr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = perm[i];
    sx[i] = x[p];
    sy[i] = y[p];
    sz[i] = z[p];
    sr[i] = r[p];
}

// Touch test in 64-bit integers: coordinates lie in [-2^24, 2^24] and radii
// in [0, 2^24], so every square and sum stays below 2^53.
__device__ __forceinline__ bool touch(int xi, int yi, int zi, int ri, int xj, int yj, int zj,
                                      int rj) {
    const int64_t dx = (int64_t)xi - xj, dy = (int64_t)yi - yj, dz = (int64_t)zi - zj;
    const int64_t R = (int64_t)ri + rj;
    return dx * dx + dy * dy + dz * dz <= R * R;
}

// Cell index by key: an open-addressing table of 2^hlog slots (at least
// twice the objects, so at most half full), keys in hkeys (0 = empty; no
// cell key is 0, its fields being at least 1) and cell indices in hvals.
// A neighbour lookup is then one or two dependent loads, not the twenty of a
// binary search over a million keys.
__device__ __forceinline__ uint32_t cell_slot(uint64_t key, int hlog) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - hlog));
}

__global__ void k_bin_hash_build(const uint64_t *__restrict__ ukeys,
                                 const uint32_t *__restrict__ m_ptr, uint64_t *hkeys,
                                 uint32_t *hvals, int hlog) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)*m_ptr) return;
    const uint64_t key = ukeys[c];
    const uint32_t mask = (1u << hlog) - 1;
    uint32_t sl = cell_slot(key, hlog);
    for (uint32_t p = 0; p <= mask; ++p, sl = (sl + 1) & mask) {
        // keys are distinct, so a claim either succeeds or meets another key
        if (atomicCAS((unsigned long long *)&hkeys[sl], 0ull, (unsigned long long)key) == 0) {
            hvals[sl] = (uint32_t)c;
            return;
        }
    }
}

// Index of the occupied cell with `key`, or -1.
__device__ __forceinline__ int64_t find_cell(const uint64_t *__restrict__ hkeys,
                                             const uint32_t *__restrict__ hvals, int hlog,
                                             uint64_t key) {
    const uint32_t mask = (1u << hlog) - 1;
    uint32_t sl = cell_slot(key, hlog);
    for (uint32_t p = 0; p <= mask; ++p, sl = (sl + 1) & mask) {
        const uint64_t k = hkeys[sl];
        if (k == key) return hvals[sl];
        if (k == 0) return -1;
    }
    return -1;
}

// Key of forward neighbour d of a cell.  Cell coordinates are at least 1
// (the +1 offset) and at most 2^20 + 1, so every neighbour's coordinates stay
// inside their 21-bit fields.
__device__ __forceinline__ uint64_t neighbour_key(uint64_t key, int d) {
    // d = 0..12 enumerates (dx, dy, dz) > (0, 0, 0) lexicographically
    const int e = d + 14;  // index in the 3x3x3 cube, 13 being the centre
    const int dx = e / 9 - 1, dy = (e / 3) % 3 - 1, dz = e % 3 - 1;
    const uint64_t cx = (key >> (2 * kCellBits)) & kAxisMask;
    const uint64_t cy = (key >> kCellBits) & kAxisMask;
    const uint64_t cz = key & kAxisMask;
    return cell_key((uint32_t)(cx + dx), (uint32_t)(cy + dy), (uint32_t)(cz + dz));
}

// Pairs of one occupied cell c, counted by the G lanes of a group (gl = lane
// in the group, g0 = the group's first lane in the wave): its 13 forward
// neighbours are looked up by lanes 0..12 of the group, the pairs inside the
// cell run on the balanced circular assignment, and the pairs with each
// occupied neighbour with the lanes taking the cell's objects against all of
// the neighbour's.
template <int G>
__device__ __forceinline__ uint64_t count_cell(int64_t c, int gl, int g0,
                                               const int32_t *__restrict__ sx,
                                               const int32_t *__restrict__ sy,
                                               const int32_t *__restrict__ sz,
                                               const int32_t *__restrict__ sr,
                                               const uint64_t *__restrict__ ukeys,
                                               const uint32_t *__restrict__ off,
                                               const uint64_t *__restrict__ hkeys,
                                               const uint32_t *__restrict__ hvals, int hlog) {
    static_assert(G >= 13 && kWave % G == 0, "13 neighbour lookups per group");
    uint64_t cnt = 0;
    const int64_t a0 = off[c], n = (int64_t)off[c + 1] - a0;
    int64_t nb = -1;
    if (gl < 13) nb = find_cell(hkeys, hvals, hlog, neighbour_key(ukeys[c], gl));
    const int64_t h = (n - 1) / 2;
    for (int64_t i = gl; i < n; i += G) {
        const int xi = sx[a0 + i], yi = sy[a0 + i], zi = sz[a0 + i], ri = sr[a0 + i];
        const int64_t steps = h + ((n % 2 == 0 && i < n / 2) ? 1 : 0);
        for (int64_t s = 1; s <= steps; ++s) {
            int64_t j = i + s;
            j = j >= n ? j - n : j;
            cnt += touch(xi, yi, zi, ri, sx[a0 + j], sy[a0 + j], sz[a0 + j], sr[a0 + j]);
        }
    }
    for (int d = 0; d < 13; ++d) {
        const int64_t b = __shfl(nb, g0 + d, kWave);
        if (b < 0) continue;
        const int64_t b0 = off[b], nbn = (int64_t)off[b + 1] - b0;
        for (int64_t i = gl; i < n; i += G) {
            const int xi = sx[a0 + i], yi = sy[a0 + i], zi = sz[a0 + i], ri = sr[a0 + i];
            for (int64_t j = 0; j < nbn; ++j)
                cnt += touch(xi, yi, zi, ri, sx[b0 + j], sy[b0 + j], sz[b0 + j], sr[b0 + j]);
        }
    }
    return cnt;
}

__device__ __forceinline__ void wave_count_to(uint64_t *count, uint64_t cnt) {
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && cnt)
        atomicAdd((unsigned long long *)count, (unsigned long long)cnt);
}

// Small cells: 16 lanes per occupied cell, four cells per wave in flight,
// which hides the latency of a cell's dependent loads.  Cells of more than
// kBigCell objects are appended to `big` (their number in big_n) for
// k_bin_count_big.  m_ptr: number of occupied cells (device); ukeys: their
// keys; off: their first object in the sorted arrays, off[m] = n; hkeys,
// hvals, hlog: the table from keys to cell indices.
constexpr int kGroup = 16;
constexpr int64_t kBigCell = 64;

__global__ __launch_bounds__(kBlock) void k_bin_count(const int32_t *__restrict__ sx,
                                                      const int32_t *__restrict__ sy,
                                                      const int32_t *__restrict__ sz,
                                                      const int32_t *__restrict__ sr,
                                                      const uint64_t *__restrict__ ukeys,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ m_ptr,
                                                      const uint64_t *__restrict__ hkeys,
                                                      const uint32_t *__restrict__ hvals,
                                                      int hlog, uint32_t *big, uint32_t *big_n,
                                                      uint64_t *count) {
    const int lane = threadIdx.x & (kWave - 1);
    const int gl = lane % kGroup, g0 = lane - gl;
    const int64_t m = *m_ptr;
    const int64_t groups = (int64_t)gridDim.x * (kBlock / kGroup);
    uint64_t cnt = 0;
    for (int64_t c = (int64_t)blockIdx.x * (kBlock / kGroup) + threadIdx.x / kGroup; c < m;
         c += groups) {
        if ((int64_t)off[c + 1] - off[c] > kBigCell) {
            if (gl == 0) big[atomicAdd(big_n, 1u)] = (uint32_t)c;
            continue;
        }
        cnt += count_cell<kGroup>(c, gl, g0, sx, sy, sz, sr, ukeys, off, hkeys, hvals, hlog);
    }
    wave_count_to(count, cnt);
}

// Big cells: one wave per cell of the list.
__global__ __launch_bounds__(kBlock) void k_bin_count_big(const int32_t *__restrict__ sx,
                                                          const int32_t *__restrict__ sy,
                                                          const int32_t *__restrict__ sz,
                                                          const int32_t *__restrict__ sr,
                                                          const uint64_t *__restrict__ ukeys,
                                                          const uint32_t *__restrict__ off,
                                                          const uint64_t *__restrict__ hkeys,
                                                          const uint32_t *__restrict__ hvals,
                                                          int hlog, const uint32_t *big,
                                                          const uint32_t *big_n,
                                                          uint64_t *count) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nbig = *big_n;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    uint64_t cnt = 0;
    for (int64_t q = (int64_t)blockIdx.x * (kBlock / kWave) + pairs_dev::wave_id(); q < nbig;
         q += waves)
        cnt += count_cell<kWave>(big[q], lane, 0, sx, sy, sz, sr, ukeys, off, hkeys, hvals, hlog);
    wave_count_to(count, cnt);
}

// Clears the cell sizes before the run-length encoding: the scan then runs
// over n + 1 sizes, zero past the m occupied cells, so that off[m] = n.
__global__ void k_bin_clear_u32(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace pairs_binning
