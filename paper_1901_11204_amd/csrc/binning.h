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
//   3. k_bin_gather: the records in key order, with each one's q = |p|^2 - r^2;
//   4. run-length encoding of the sorted keys (rocPRIM) into the occupied
//      cells' keys and sizes, and an exclusive scan of the sizes into cell
//      offsets;
//   5. k_bin_hash_build: a hash table of 8-slot buckets from occupied cell
//      keys to each cell's first object and size;
//   6. k_bin_count: 16 lanes per occupied cell.  Lanes 0..12 of a group
//      look up the 13 forward neighbours in the table; the pairs inside a
//      cell of at most kBigCell objects run on the balanced circular
//      assignment (each lane takes rows and their steps s = 1 ..
//      floor((n-1)/2), rows i < n/2 also s = n/2 when n is even); the pairs
//      with each occupied neighbour of at most kBigCell objects run with the
//      lanes taking the cell's objects against all of the neighbour's.  Wave
//      sums go to the count with one atomic per wave.  Every pair of ranges
//      with more than kBigCell objects on one side -- a big cell's own pairs,
//      and the pairs between a cell and a neighbour when either is big -- is
//      appended instead to a list of work items;
//   7. k_bin_item_scan and k_bin_count_items: each item is tiled into wave
//      tasks of at most 64 K rows against kItemChunk partners (the balanced
//      assignment's row blocks and chunks for a cell's own pairs, a
//      rectangle of rows and partners between two cells), and all waves
//      share the tasks, so no wave's work grows with a cell's size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "band.h"
#include "device.h"
#include "tasks.h"

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

// The records in key order, and each record's q = |p|^2 - r^2 (the partner
// term of the Gram test, read by the work items' tasks).
__global__ void k_bin_gather(const int4 *__restrict__ rec, const uint32_t *__restrict__ perm,
                             int64_t n, int4 *__restrict__ so, int64_t *__restrict__ sq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 o = rec[perm[i]];
    so[i] = o;
    sq[i] = pairs_dev::gram_q(o.x, o.y, o.z, o.w);
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
// A work item: the pairs between objects [a0, a0 + na) and [b0, b0 + nb) of
// the sorted records, or the pairs within [a0, a0 + na) when b0 == a0.
struct Item {
    uint32_t a0, na, b0, nb;
};
constexpr int64_t kBigCell = 64;

// Capacity of the item list for n objects: at most n / (kBigCell + 1) cells
// are big, and each takes part in at most 27 items (its own pairs and one
// per neighbour in either direction).  Pushes beyond it (possible only for
// inputs outside the domain, whose keys can wrap) are dropped, never
// written.
__host__ __device__ inline int64_t item_capacity(int64_t n) {
    return 27 * (n / (kBigCell + 1)) + 1;
}

struct ItemList {
    Item *items;
    uint32_t *n;   // pushes so far (may pass cap)
    uint32_t cap;
};

// Appends the calling lanes' items (a lane may push none, one or two) with
// one atomic per wave: a lane's slots follow the items of the lanes below it.
// Called by every active lane of the wave together.
__device__ __forceinline__ void push_items(const ItemList &L, bool p0, const Item &i0, bool p1,
                                           const Item &i1) {
    const uint64_t b0 = __ballot(p0), b1 = __ballot(p1);
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (1ull << lane) - 1;
    const uint32_t total = __popcll(b0) + __popcll(b1);
    if (total == 0) return;
    const int first = __builtin_ctzll(__ballot(true));
    uint32_t base = 0;
    if (lane == first) base = atomicAdd(L.n, total);
    base = (uint32_t)__shfl((int)base, first, kWave);
    uint32_t k = base + __popcll(b0 & below) + __popcll(b1 & below);
    if (p0) {
        if (k < L.cap) L.items[k] = i0;
        ++k;
    }
    if (p1 && k < L.cap) L.items[k] = i1;
}

__device__ __forceinline__ int64_t item_count(const ItemList &L) {
    const uint32_t n = *L.n;
    return n < L.cap ? n : L.cap;
}

template <int G>
__device__ __forceinline__ uint64_t count_cell(int64_t a0, int64_t n, uint64_t key, int gl, int g0,
                                               const int4 *__restrict__ so,
                                               const uint64_t *__restrict__ htags,
                                               const uint64_t *__restrict__ hkeys,
                                               const uint2 *__restrict__ hvals, int blog,
                                               int fb, const ItemList &items) {
    static_assert(G >= 13 && kWave % G == 0, "13 neighbour lookups per group");
    uint64_t cnt = 0;
    uint2 nb = make_uint2(0, 0);
    if (gl < 13) nb = find_cell(htags, hkeys, hvals, blog, neighbour_key(key, gl, fb));
    const bool big = n > kBigCell;
    // ranges with a big side go to the item list: the cell's own pairs, and
    // those with each big (or, for a big cell, every) occupied neighbour
    push_items(items, big && gl == 0, Item{(uint32_t)a0, (uint32_t)n, (uint32_t)a0, (uint32_t)n},
               gl < 13 && nb.y != 0 && (big || nb.y > (uint32_t)kBigCell),
               Item{(uint32_t)a0, (uint32_t)n, nb.x, nb.y});
    if (big) return 0;
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
    // only the occupied neighbours of at most kBigCell objects, usually none
    // in a sparse grid
    uint32_t occ =
        (uint32_t)(__ballot(nb.y != 0 && nb.y <= (uint32_t)kBigCell) >> g0) & ((1u << 13) - 1);
    while (occ) {
        const int d = __builtin_ctz(occ);
        occ &= occ - 1;
        const int nbn32 = __shfl((int)nb.y, g0 + d, kWave),
                  b032 = __shfl((int)nb.x, g0 + d, kWave);
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

// 16 lanes per occupied cell, four cells per wave in flight, which hides the
// latency of a cell's dependent loads.  Ranges with a big side go to `items`
// (their number in item_n).  m_ptr: number of occupied cells (device); ukeys:
// their keys; off: their first object in the sorted arrays, off[m] = n;
// htags, hkeys, hvals, blog: the table from keys to cell ranges; fb: bits per
// axis of a key; so: the object records in key order.
constexpr int kGroup = 16;

// Eight waves per SIMD: the loop waits on loads, so occupancy pays.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_bin_count(
    const int4 *__restrict__ so, const uint64_t *__restrict__ ukeys,
    const uint32_t *__restrict__ off, const uint32_t *__restrict__ m_ptr,
    const uint64_t *__restrict__ htags, const uint64_t *__restrict__ hkeys,
    const uint2 *__restrict__ hvals, int blog, int fb, ItemList items, uint64_t *count) {
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
        cnt += count_cell<kGroup>(o0, n, key, gl, g0, so, htags, hkeys, hvals, blog, fb, items);
        o0 = p0, o1 = p1, key = pk;
    }
    wave_count_to(count, cnt);
}

// ------------------------------------------------------------- work items --
//
// Tasks of an item: a cell's own pairs are the balanced assignment of its na
// objects (band.h) tiled into row blocks of 64 K rows and chunks of
// kItemChunk virtual partners; the pairs between two ranges are a rectangle
// of row blocks of A against chunks of kItemChunk objects of B.  K (rows per
// lane, 1, 2 or 4) follows the item's na, so that a row block of a
// 100-object cell does not leave half of 256 lanes' rows empty.
constexpr int kItemChunk = 512;

__host__ __device__ inline int item_rows(uint32_t na) { return na <= 64 ? 1 : na <= 128 ? 2 : 4; }

__device__ __forceinline__ int64_t item_tasks(const Item &it) {
    const int K = item_rows(it.na);
    if (it.a0 == it.b0) return Tiling::of(Band::of((int)it.na), K, kItemChunk).tasks();
    return (int64_t)((it.na + 64 * K - 1) / (64 * K)) * ((it.nb + kItemChunk - 1) / kItemChunk);
}

// The items' task range, as the unplanned batched schedule lays out sets: pre[k]
// is the first task of item k (pre[m] = T), and a bucket table tab[q] names
// the item holding task q B, with B = ceil(T / m), so a wave finds a task's
// item with one table read and a search over at most B + 1 entries of pre.
struct ItemSched {
    int64_t m;         // items
    int64_t T;         // tasks in all
    int64_t B;         // tasks per bucket
    int64_t nbuckets;  // ceil(T / B)
};

// The exclusive prefix of the items' task counts in three steps over blocks
// of kScanBlock items (the item count is known on the device only, so the
// grids cover the list's capacity and blocks past the items return):
// per-block sums, one block scanning them and writing the header, and the
// block-local prefixes.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_bin_item_sums(ItemList L,
                                                             int64_t *__restrict__ bsum) {
    const int64_t m = item_count(L), k0 = (int64_t)blockIdx.x * kScanBlock;
    if (k0 >= m) return;
    __shared__ int64_t wave_tot[kScanBlock / kWave + 1];
    const int64_t k = k0 + threadIdx.x;
    int64_t sum;
    pairs_dev::block_exclusive_scan<kScanBlock>(k < m ? item_tasks(L.items[k]) : 0, wave_tot,
                                                &sum);
    if (threadIdx.x == 0) bsum[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kScanBlock) void k_bin_item_scan(ItemList L,
                                                             int64_t *__restrict__ bsum,
                                                             ItemSched *__restrict__ hdr) {
    __shared__ int64_t wave_tot[kScanBlock / kWave + 1];
    const int tid = threadIdx.x;
    const int64_t m = item_count(L), nb = (m + kScanBlock - 1) / kScanBlock;
    const int64_t chunk = (nb + kScanBlock - 1) / kScanBlock;
    const int64_t b0 = min((int64_t)tid * chunk, nb), b1 = min(b0 + chunk, nb);
    int64_t part = 0;
    for (int64_t b = b0; b < b1; ++b) part += bsum[b];
    int64_t T;
    int64_t run = pairs_dev::block_exclusive_scan<kScanBlock>(part, wave_tot, &T);
    if (tid == 0) {
        const int64_t B = m > 0 ? max((int64_t)1, (T + m - 1) / m) : 1;
        hdr->m = m;
        hdr->T = T;
        hdr->B = B;
        hdr->nbuckets = (T + B - 1) / B;
    }
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = bsum[b];
        bsum[b] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_bin_item_prefix(ItemList L,
                                                               const int64_t *__restrict__ bsum,
                                                               const ItemSched *__restrict__ hdr,
                                                               int64_t *__restrict__ pre) {
    const int64_t m = item_count(L), k0 = (int64_t)blockIdx.x * kScanBlock;
    if (k0 >= m) {
        if (blockIdx.x == 0 && threadIdx.x == 0) pre[0] = 0;  // no items
        return;
    }
    __shared__ int64_t wave_tot[kScanBlock / kWave + 1];
    const int64_t k = k0 + threadIdx.x;
    int64_t sum;
    const int64_t r = pairs_dev::block_exclusive_scan<kScanBlock>(
        k < m ? item_tasks(L.items[k]) : 0, wave_tot, &sum);
    if (k < m) pre[k] = bsum[blockIdx.x] + r;
    if (k == m - 1) pre[m] = hdr->T;
}

// The bucket table: tab[q] = the item holding task q B; tab[nbuckets] = m - 1.
__global__ void k_bin_item_tab(const int64_t *__restrict__ pre,
                               const ItemSched *__restrict__ hdr, int32_t *__restrict__ tab) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nbk = hdr->nbuckets, m = hdr->m;
    if (q > nbk) return;
    if (q == nbk) {
        tab[q] = (int32_t)max((int64_t)0, m - 1);
        return;
    }
    const int64_t t = q * hdr->B;
    int64_t lo = 0, hi = m;  // pre[lo] <= t < pre[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    tab[q] = (int32_t)lo;
}

// One task of an item with K rows per lane: rows [ra, ra + 64 K) of A held as
// in the pairs_count_i32 kernels (RowI32), partners u in [u0, u1) staged 64
// at a time in LDS (the next group's records in flight while a group is
// counted) and read back as broadcasts, PU = 8 / K partners at a time for 8
// independent multiply-add chains.  (Wave-uniform scalar reads of the
// partners measured twice as slow: their latency exceeds the 40 VALU
// operations each group of PU feeds.)  The binned domain (coordinates within
// 2^24) lies inside the box of the plain 64-bit Gram test.  Padding rows
// (nq = -2^62) and padding partners (q = INT64_MAX) never hit.
template <int K>
__device__ __forceinline__ uint32_t item_task(const int4 *__restrict__ so,
                                              const int64_t *__restrict__ sq, const Item &it,
                                              int64_t local, pairs_dev::PartnerI32 *wp,
                                              int64_t *wq) {
    using namespace pairs_dev;
    const int lane = lane_id();
    const bool self = it.a0 == it.b0;
    const Band band = Band::of((int)it.na);
    int ra, u0, u1;
    if (self) {
        task_at(band, Tiling::of(band, K, kItemChunk), local, &ra, &u0, &u1);
    } else {
        const int64_t nch = (it.nb + kItemChunk - 1) / kItemChunk;
        ra = (int)(local / nch) * 64 * K;
        u0 = (int)(local % nch) * kItemChunk;
        u1 = min(u0 + kItemChunk, (int)it.nb);
    }
    RowI32 rows[K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ra + kWave * k + lane;
        row[k] = i;
        nsteps[k] = 0;
        rows[k].ax = rows[k].ay = rows[k].az = rows[k].ar = 0;
        rows[k].nq = -((int64_t)1 << 62);
        if (i < (int)it.na) {
            const int4 o = so[it.a0 + i];
            rows[k] = gram_row(o.x, o.y, o.z, o.w);
            nsteps[k] = self ? band.steps(i) : 0;
        }
    }
    // the partner record and q of virtual partner u (padding past u1)
    auto fetch = [&](int u, int4 &o, int64_t &q) {
        if (u >= u1) {
            o = make_int4(0, 0, 0, 0);
            q = INT64_MAX;
            return;
        }
        const uint32_t j = self ? it.a0 + (uint32_t)(u >= (int)it.na ? u - (int)it.na : u)
                                : it.b0 + (uint32_t)u;
        o = so[j];
        q = sq[j];
    };
    constexpr int PU = 8 / K;
    uint32_t cnt = 0;
    int4 no;
    int64_t nq;
    fetch(u0 + lane, no, nq);
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        wp[lane] = PartnerI32{no.x, no.y, no.z, no.w};
        wq[lane] = nq;
        fetch(g0 + kWave + lane, no, nq);  // in flight while this group is counted
        wave_sync();
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (self) {
            for (int q = 0; q < gn; ++q) {
                const PartnerI32 b = wp[q];
                const int64_t qb = wq[q];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cnt += count_bits_both(gram_hit(rows[k], b, qb),
                                           owns(g0 + q, row[k], nsteps[k]));
            }
        } else {
            // entries past gn are padding and never hit
            for (int q = 0; q < gn; q += PU) {
                PartnerI32 b[PU];
                int64_t qb[PU];
#pragma unroll
                for (int d = 0; d < PU; ++d) {
                    b[d] = wp[q + d];
                    qb[d] = wq[q + d];
                }
#pragma unroll
                for (int d = 0; d < PU; ++d)
#pragma unroll
                    for (int k = 0; k < K; ++k) cnt += count_bits(gram_hit(rows[k], b[d], qb[d]));
            }
        }
        wave_sync();
    }
    return cnt;
}

// The tasks of all items, taken by the waves with a grid stride.
__global__ __launch_bounds__(kBlock) void k_bin_count_items(const int4 *__restrict__ so,
                                                            const int64_t *__restrict__ sq,
                                                            ItemList L,
                                                            const int64_t *__restrict__ pre,
                                                            const int32_t *__restrict__ tab,
                                                            const ItemSched *__restrict__ hdr,
                                                            uint64_t *count) {
    using namespace pairs_dev;
    __shared__ PartnerI32 wp_all[kBlock / kWave][kWave];
    __shared__ int64_t wq_all[kBlock / kWave][kWave];
    const int wave = wave_id();
    PartnerI32 *wp = wp_all[wave];
    int64_t *wq = wq_all[wave];
    const int64_t total = hdr->T, B = hdr->B;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / kWave);
    uint64_t cnt = 0;
    for (int64_t t = (int64_t)blockIdx.x * (kBlock / kWave) + wave; t < total; t += stride) {
        const int64_t b = t / B;
        int64_t lo = tab[b], hi = (int64_t)tab[b + 1] + 1;  // pre[lo] <= t < pre[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (pre[mid] <= t) lo = mid; else hi = mid;
        }
        const Item it = L.items[lo];
        const int64_t local = t - pre[lo];
        const int K = item_rows(it.na);
        if (K == 1)
            cnt += item_task<1>(so, sq, it, local, wp, wq);
        else if (K == 2)
            cnt += item_task<2>(so, sq, it, local, wp, wq);
        else
            cnt += item_task<4>(so, sq, it, local, wp, wq);
    }
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)count, (unsigned long long)cnt);
}

// Ranges of 32-bit words that the pipeline needs zeroed, cleared by one
// launch (blockIdx.y picks the range): the count, the cell sizes (the scan
// runs over n + 1 sizes, zero past the m occupied cells, so that off[m] = n),
// the table's tags and claim counts, and the number of work items.
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
