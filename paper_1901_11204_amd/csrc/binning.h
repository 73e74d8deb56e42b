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
//   0. k_bin_clear: every buffer that has to start at zero, in one launch;
//   1. k_bin_keys: cell coordinates (x + 2^24) / L + 1 per axis (the +1 keeps
//      the -1 neighbours of cell 0 in range), packed fb bits per axis into a
//      64-bit key, and the object index.  fb is the fewest bits that hold
//      2^25 / L + 2, the largest neighbour coordinate: 21 for L = 32, 11 for
//      L = 2^15.  Each object is also written as one 16-byte record;
//   2. radix sort of (key, index) over the key's 3 fb bits (rocPRIM);
//   3. k_bin_gather: the records in key order;
//   4. run-length encoding of the sorted keys (rocPRIM) into the occupied
//      cells' keys and sizes, and an exclusive scan of the sizes into cell
//      offsets;
//   5. k_bin_hash_build: a hash table of 8-slot buckets from occupied cell
//      keys to each cell's first object and size;
//   6. k_bin_count: 16 lanes per occupied cell (cells of more than 64
//      objects go to a list that k_bin_count_big counts, one wave per cell).
//      Lanes 0..12 of a group look up the 13 forward neighbours in the
//      table; the pairs inside the cell run on the balanced circular
//      assignment (each lane takes rows and their steps s = 1 ..
//      floor((n-1)/2), rows i < n/2 also s = n/2 when n is even); the pairs
//      with each occupied neighbour run with the lanes taking the cell's
//      objects against all of the neighbour's.  Wave sums go to the count
//      with one atomic per wave.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace pairs_binning {

using pairs_dev::kWave;

constexpr int kBlock = 256;
constexpr int kMaxCellBits = 21;  // per axis, for the smallest cell of 32
constexpr int kOffsetBias = 1 << 24;  // coordinates in [-2^24, 2^24]

// Cell coordinate of a coordinate, offset by one.
__device__ __forceinline__ uint32_t cell_of(int v, int L) {
    return (uint32_t)(v + kOffsetBias) / (uint32_t)L + 1;
}

// Key of a cell: fb bits per axis, x in the high field.  Sorting by key sorts
// the cells in (x, y, z) lexicographic order.
__device__ __forceinline__ uint64_t cell_key(uint32_t cx, uint32_t cy, uint32_t cz, int fb) {
    return ((uint64_t)cx << (2 * fb)) | ((uint64_t)cy << fb) | (uint64_t)cz;
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

// Keys and indices for the sort, and each object as one 16-byte record
// (x, y, z, r), so that the gather after the sort reads one record per
// object rather than four scattered words.
__global__ void k_bin_keys(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                           const int32_t *__restrict__ z, const int32_t *__restrict__ r,
                           int64_t n, int L, int fb, uint64_t *__restrict__ keys,
                           uint32_t *__restrict__ idx, int4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int xi = x[i], yi = y[i], zi = z[i];
    keys[i] = cell_key(cell_of(xi, L), cell_of(yi, L), cell_of(zi, L), fb);
    idx[i] = (uint32_t)i;
    rec[i] = make_int4(xi, yi, zi, r[i]);
}

// The records in key order.
__global__ void k_bin_gather(const int4 *__restrict__ rec, const uint32_t *__restrict__ perm,
                             int64_t n, int4 *__restrict__ so) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    so[i] = rec[perm[i]];
}

// Touch test: coordinates lie in [-2^24, 2^24] and radii in [0, 2^24], so
// the differences and the radius sum fit 32 bits (at most 2^25 in size) and
// the squares and their sum fit 64 bits exactly.
__device__ __forceinline__ bool touch(int4 a, int4 b) {
    const int dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, R = a.w + b.w;
    return (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz <= (int64_t)R * R;
}

// Cells by key: a table of 2^blog buckets of kSlots slots (at least twice as
// many slots as objects).  Per slot: a tag byte in htags (0 = empty, else 8
// bits of the key's hash), the key in hkeys and the cell's first object and
// size in hvals; per bucket, the number of claims in hcnt.  A key goes to the
// first bucket, from its home bucket on, whose claim count is below kSlots,
// so a bucket's slots fill in order and a key can be further on only if its
// home bucket is full.
//
// A lookup reads the bucket's eight tags as one 8-byte word, from a tag array
// of one byte per slot that the L2 cache holds, and reads a key only where
// its tag matches.  In a sparse grid most neighbours are empty, and most
// lookups end at the tag word.
constexpr int kSlots = 8;

__device__ __forceinline__ uint64_t cell_hash(uint64_t key) {
    return key * 0x9E3779B97F4A7C15ull;
}

__device__ __forceinline__ uint32_t home_bucket(uint64_t h, int blog) {
    return (uint32_t)(h >> (64 - blog));
}

// The 8 hash bits below the bucket bits, never 0.
__device__ __forceinline__ uint32_t cell_tag(uint64_t h, int blog) {
    const uint32_t t = (uint32_t)(h >> (56 - blog)) & 0xFFu;
    return t ? t : 1u;
}

__global__ void k_bin_hash_build(const uint64_t *__restrict__ ukeys,
                                 const uint32_t *__restrict__ off,
                                 const uint32_t *__restrict__ m_ptr, uint8_t *htags,
                                 uint64_t *hkeys, uint2 *hvals, uint32_t *hcnt, int blog) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)*m_ptr) return;
    const uint64_t key = ukeys[c], h = cell_hash(key);
    const uint2 val = make_uint2(off[c], off[c + 1] - off[c]);
    const uint32_t mask = (1u << blog) - 1;
    uint32_t b = home_bucket(h, blog);
    // the slots outnumber the cells, so some bucket has room
    for (uint32_t p = 0; p <= mask; ++p, b = (b + 1) & mask) {
        const uint32_t at = atomicAdd(&hcnt[b], 1u);
        if (at < (uint32_t)kSlots) {
            const size_t slot = (size_t)b * kSlots + at;
            htags[slot] = (uint8_t)cell_tag(h, blog);
            hkeys[slot] = key;
            hvals[slot] = val;
            return;
        }
    }
}

// 0x80 in each byte of x that is zero, 0 elsewhere (exact: no carry crosses
// a byte, since (b & 0x7F) + 0x7F <= 0xFE).
__device__ __forceinline__ uint64_t zero_bytes(uint64_t x) {
    constexpr uint64_t lo7 = 0x7F7F7F7F7F7F7F7Full;
    return ~(((x & lo7) + lo7) | x | lo7);
}

// First object and size of the occupied cell with `key`, or size 0.  The
// tag word is matched with whole-word arithmetic, so the common case (no
// matching tag) takes no per-slot branch.
__device__ __forceinline__ uint2 find_cell(const uint64_t *__restrict__ htags,
                                           const uint64_t *__restrict__ hkeys,
                                           const uint2 *__restrict__ hvals, int blog,
                                           uint64_t key) {
    const uint64_t h = cell_hash(key);
    const uint32_t mask = (1u << blog) - 1;
    const uint64_t tags = 0x0101010101010101ull * cell_tag(h, blog);
    uint32_t b = home_bucket(h, blog);
    for (uint32_t p = 0; p <= mask; ++p, b = (b + 1) & mask) {
        const uint64_t tw = htags[b];
        uint64_t hit = zero_bytes(tw ^ tags);
        while (hit) {
            const size_t slot = (size_t)b * kSlots + (__builtin_ctzll(hit) >> 3);
            hit &= hit - 1;
            if (hkeys[slot] == key) return hvals[slot];
        }
        if (zero_bytes(tw)) break;  // the bucket has room: the key is nowhere further
    }
    return make_uint2(0, 0);
}

// Key of forward neighbour d of a cell.  Cell coordinates are at least 1
// (the +1 offset) and at most 2^25 / L + 1, so every neighbour's coordinates
// stay inside their fb-bit fields.
__device__ __forceinline__ uint64_t neighbour_key(uint64_t key, int d, int fb) {
    // d = 0..12 enumerates (dx, dy, dz) > (0, 0, 0) lexicographically
    const int e = d + 14;  // index in the 3x3x3 cube, 13 being the centre
    const int dx = e / 9 - 1, dy = (e / 3) % 3 - 1, dz = e % 3 - 1;
    const uint64_t mask = (uint64_t(1) << fb) - 1;
    const uint64_t cx = (key >> (2 * fb)) & mask;
    const uint64_t cy = (key >> fb) & mask;
    const uint64_t cz = key & mask;
    return cell_key((uint32_t)(cx + dx), (uint32_t)(cy + dy), (uint32_t)(cz + dz), fb);
}

// Pairs of one occupied cell (first object a0, n objects, key `key`),
// counted by the G lanes of a group (gl = lane in the group, g0 = the group's
// first lane in the wave): its 13 forward neighbours are looked up by lanes
// 0..12 of the group, the pairs inside the cell run on the balanced circular
// assignment, and the pairs with each occupied neighbour with the lanes
// taking the cell's objects against all of the neighbour's.
template <int G>
__device__ __forceinline__ uint64_t count_cell(int64_t a0, int64_t n, uint64_t key, int gl, int g0,
                                               const int4 *__restrict__ so,
                                               const uint64_t *__restrict__ htags,
                                               const uint64_t *__restrict__ hkeys,
                                               const uint2 *__restrict__ hvals, int blog,
                                               int fb) {
    static_assert(G >= 13 && kWave % G == 0, "13 neighbour lookups per group");
    uint64_t cnt = 0;
    uint2 nb = make_uint2(0, 0);
    if (gl < 13) nb = find_cell(htags, hkeys, hvals, blog, neighbour_key(key, gl, fb));
    const int64_t h = (n - 1) / 2;
    for (int64_t i = gl; n >= 2 && i < n; i += G) {
        const int4 oi = so[a0 + i];
        const int64_t steps = h + ((n % 2 == 0 && i < n / 2) ? 1 : 0);
        for (int64_t s = 1; s <= steps; ++s) {
            int64_t j = i + s;
            j = j >= n ? j - n : j;
            cnt += touch(oi, so[a0 + j]);
        }
    }
    // only the occupied neighbours, usually none in a sparse grid
    uint32_t occ = (uint32_t)(__ballot(nb.y != 0) >> g0) & ((1u << 13) - 1);
    while (occ) {
        const int d = __builtin_ctz(occ);
        occ &= occ - 1;
        int nbn32 = __shfl((int)nb.y, g0 + d, kWave), b032 = __shfl((int)nb.x, g0 + d, kWave);
        if constexpr (G == kWave) {
            // one cell per wave: the neighbour's records are wave-uniform
            // reads, which go through the scalar unit
            nbn32 = __builtin_amdgcn_readfirstlane(nbn32);
            b032 = __builtin_amdgcn_readfirstlane(b032);
        }
        const int64_t nbn = (uint32_t)nbn32, b0 = (uint32_t)b032;
        for (int64_t i = gl; i < n; i += G) {
            const int4 oi = so[a0 + i];
#pragma unroll 4
            for (int64_t j = 0; j < nbn; ++j) cnt += touch(oi, so[b0 + j]);
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
// keys; off: their first object in the sorted arrays, off[m] = n; htags,
// hkeys, hvals, blog: the table from keys to cell ranges; fb: bits per axis
// of a key; so: the object records in key order.
constexpr int kGroup = 16;
constexpr int64_t kBigCell = 64;

// Eight waves per SIMD: the loop waits on loads, so occupancy pays.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_bin_count(
    const int4 *__restrict__ so, const uint64_t *__restrict__ ukeys,
    const uint32_t *__restrict__ off, const uint32_t *__restrict__ m_ptr,
    const uint64_t *__restrict__ htags, const uint64_t *__restrict__ hkeys,
    const uint2 *__restrict__ hvals, int blog, int fb, uint32_t *big, uint32_t *big_n,
    uint64_t *count) {
    const int lane = threadIdx.x & (kWave - 1);
    const int gl = lane % kGroup, g0 = lane - gl;
    const int64_t m = *m_ptr;
    const int64_t groups = (int64_t)gridDim.x * (kBlock / kGroup);
    uint64_t cnt = 0;
    int64_t c = (int64_t)blockIdx.x * (kBlock / kGroup) + threadIdx.x / kGroup;
    // the next cell's offsets and key are loaded one iteration ahead, so that
    // they are in flight together with the current cell's lookups
    uint32_t o0 = 0, o1 = 0;
    uint64_t key = 0;
    if (c < m) o0 = off[c], o1 = off[c + 1], key = ukeys[c];
    for (; c < m; c += groups) {
        const int64_t cn = c + groups;
        uint32_t p0 = 0, p1 = 0;
        uint64_t pk = 0;
        if (cn < m) p0 = off[cn], p1 = off[cn + 1], pk = ukeys[cn];
        const int64_t n = (int64_t)o1 - o0;
        if (n > kBigCell) {
            if (gl == 0) big[atomicAdd(big_n, 1u)] = (uint32_t)c;
        } else {
            cnt += count_cell<kGroup>(o0, n, key, gl, g0, so, htags, hkeys, hvals, blog, fb);
        }
        o0 = p0, o1 = p1, key = pk;
    }
    wave_count_to(count, cnt);
}

// Big cells: one wave per cell of the list.
__global__ __launch_bounds__(kBlock) void k_bin_count_big(const int4 *__restrict__ so,
                                                          const uint64_t *__restrict__ ukeys,
                                                          const uint32_t *__restrict__ off,
                                                          const uint64_t *__restrict__ htags,
                                                          const uint64_t *__restrict__ hkeys,
                                                          const uint2 *__restrict__ hvals,
                                                          int blog, int fb, const uint32_t *big,
                                                          const uint32_t *big_n,
                                                          uint64_t *count) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nbig = *big_n;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    uint64_t cnt = 0;
    for (int64_t q = (int64_t)blockIdx.x * (kBlock / kWave) + pairs_dev::wave_id(); q < nbig;
         q += waves) {
        const uint32_t c = big[q];
        cnt += count_cell<kWave>(off[c], (int64_t)off[c + 1] - off[c], ukeys[c], lane, 0, so,
                                 htags, hkeys, hvals, blog, fb);
    }
    wave_count_to(count, cnt);
}

// Ranges of 32-bit words that the pipeline needs zeroed, cleared by one
// launch (blockIdx.y picks the range): the count, the cell sizes (the scan
// runs over n + 1 sizes, zero past the m occupied cells, so that off[m] = n),
// the table's tags and claim counts, and the number of big cells.
constexpr int kClearRanges = 5;
struct ClearRanges {
    uint32_t *p[kClearRanges];
    int64_t n[kClearRanges];
};

__global__ void k_bin_clear(ClearRanges r) {
    uint32_t *p = r.p[blockIdx.y];
    const int64_t n = r.n[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace pairs_binning
