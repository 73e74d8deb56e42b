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
// Pipeline (all on the device, no host synchronisation, no library call, so
// a call can be captured into a HIP graph):
//   0. k_bin_clear: every buffer that has to start at zero, in one launch;
//   1. k_bin_insert: cell coordinates (x + 2^24) / L + 1 per axis (the +1
//      keeps the -1 neighbours of cell 0 in range), packed fb bits per axis
//      into a 64-bit key above which sits the object's set (batched calls).
//      fb is the fewest bits that hold 2^25 / L + 2, the largest neighbour
//      coordinate: 21 for L = 32, 11 for L = 2^15.  Each object finds or
//      inserts its cell's key in a hash table of 8-slot buckets and takes a
//      rank in the cell;
//   2. k_bin_slot_sums, k_bin_slot_scan, k_bin_slot_prefix: a prefix over
//      the table's slots numbers the cells in slot order and gives each its
//      first object, stored with the size in the table and, with the key,
//      in per-cell arrays;
//   3. k_bin_scatter, k_bin_gather: each object's record (x, y, z, r) and
//      its q = |p|^2 - r^2 at its cell's first object plus its rank;
//   4. k_bin_count: 16 lanes per occupied cell.  Lanes 0..12 of a group
//      look up the 13 forward neighbours in the table; the pairs inside a
//      cell of at most kBigCell objects run on the balanced circular
//      assignment (each lane takes rows and their steps s = 1 ..
//      floor((n-1)/2), rows i < n/2 also s = n/2 when n is even); the pairs
//      with each occupied neighbour of at most kBigCell objects run with the
//      lanes taking the cell's objects against all of the neighbour's.
//      Every pair of ranges with more than kBigCell objects on one side -- a
//      big cell's own pairs, and the pairs between a cell and a neighbour
//      when either is big -- is appended instead to a list of work items;
//   5. k_bin_item_sums, k_bin_item_scan, k_bin_item_prefix, k_bin_item_tab
//      and k_bin_count_items: each item is tiled into wave tasks of at most
//      64 K rows against kItemChunk partners (the balanced assignment's row
//      blocks and chunks for a cell's own pairs, a rectangle of rows and
//      partners between two cells), and all waves share the tasks, so no
//      wave's work grows with a cell's size.
// The cells follow the table's slot order; the order of the objects in a
// cell follows the order of the atomic operations, which varies from run to
// run; the count does not.
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

// Key of a cell: fb bits per axis, x in the high field; a batched call puts
// the object's set above the 3 fb cell bits, so cells of different sets
// never meet.  Occupied cells have z >= 1, so no occupied cell's key is 0,
// the key of an empty table slot.
__device__ __forceinline__ uint64_t cell_key(uint32_t cx, uint32_t cy, uint32_t cz, int fb) {
    return ((uint64_t)cx << (2 * fb)) | ((uint64_t)cy << fb) | (uint64_t)cz;
}
constexpr uint64_t kEmptyKey = 0;

// Set of object i of a CSR batch: the largest s with off[s] <= i (empty
// sets share their offset with the next set, which is then the larger s).
__device__ __forceinline__ uint32_t set_of(const int64_t *__restrict__ off, int64_t n_sets,
                                           int64_t i) {
    int64_t lo = 0, hi = n_sets;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return (uint32_t)lo;
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

// Touch test: coordinates lie in [-2^24, 2^24] and radii in [0, 2^24], so
// the differences and the radius sum fit 32 bits (at most 2^25 in size) and
// the squares and their sum fit 64 bits exactly.
__device__ __forceinline__ bool touch(int4 a, int4 b) {
    const int dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, R = a.w + b.w;
    return (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz <= (int64_t)R * R;
}

// Cells by key: a table of 2^blog buckets of kSlots slots (at least twice as
// many slots as objects, so at most half full).  Per slot: the key in hkeys
// (kEmptyKey = free), a tag byte in htags (0 = free, else 8 bits of the
// key's hash), the cell's size minus one in hsize and its first object and
// size in hvals.  A key
// takes the first free slot from its home bucket's first slot on (one
// compare-and-swap per free slot probed), so a bucket's slots fill in order
// and a key lies past its home bucket only if every bucket in between is
// full.
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

// Slot of `key`, inserted if absent; *won tells whether this call inserted
// it.  Keys only ever go from free to set during the insert pass, so a
// plain load that sees a key is final, and one that sees a free slot is
// settled by the compare-and-swap.  The slots outnumber the keys, so the
// probe ends.
__device__ __forceinline__ uint32_t find_or_insert(uint64_t *hkeys, uint8_t *htags, int blog,
                                                   uint64_t key, bool *won) {
    const uint64_t h = cell_hash(key);
    const uint32_t last = ((uint32_t)kSlots << blog) - 1;
    uint32_t slot = home_bucket(h, blog) * (uint32_t)kSlots;
    for (;;) {
        uint64_t cur = __atomic_load_n(&hkeys[slot], __ATOMIC_RELAXED);
        if (cur == kEmptyKey)
            cur = atomicCAS((unsigned long long *)&hkeys[slot], (unsigned long long)kEmptyKey,
                            (unsigned long long)key);
        if (cur == kEmptyKey) {
            htags[slot] = (uint8_t)cell_tag(h, blog);
            *won = true;
            return slot;
        }
        if (cur == key) {
            *won = false;
            return slot;
        }
        slot = slot == last ? 0 : slot + 1;
    }
}

// Ranks in a cell: the object that inserts the cell's key takes rank 0 with
// no further atomic (in a sparse grid, nearly every object), every other
// object 1 + the value it adds 1 to in the slot's counter hsize, which so
// ends at the cell's size minus one.  Lanes that share a key are served by
// one probe and one counter update while the first pending lane's key is
// shared by at least kPeelMin lanes, for at most kPeelMax keys per wave
// (objects listed by cell or by set come in such runs); the other lanes
// probe and count one by one.
constexpr int kPeelMax = 4, kPeelMin = 4;

// Step 1: the cell of every object: obj[i] = (slot, rank in the cell), and
// the object as one 16-byte record rec[i] = (x, y, z, r).  off: the batch's
// set offsets (null for one set).
__global__ __launch_bounds__(kBlock) void k_bin_insert(
    const int32_t *__restrict__ x, const int32_t *__restrict__ y, const int32_t *__restrict__ z,
    const int32_t *__restrict__ r, const int64_t *__restrict__ off, int64_t n_sets, int64_t n,
    int L, int fb, int blog, uint64_t *hkeys, uint8_t *htags, uint32_t *hsize,
    uint2 *__restrict__ obj, int4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (1ull << lane) - 1;
    const bool active = i < n;
    uint64_t key = 0;
    if (active) {
        const int xi = x[i], yi = y[i], zi = z[i];
        rec[i] = make_int4(xi, yi, zi, r[i]);
        key = cell_key(cell_of(xi, L), cell_of(yi, L), cell_of(zi, L), fb);
        if (off) key |= (uint64_t)set_of(off, n_sets, i) << (3 * fb);
    }
    bool pending = active;
    uint32_t slot = 0, rank = 0;
    for (int it = 0; it < kPeelMax; ++it) {
        const uint64_t pend = __ballot(pending);
        if (!pend) break;
        const int leader = __builtin_ctzll(pend);
        const uint64_t lk = __shfl((unsigned long long)key, leader, kWave);
        const bool mine = pending && key == lk;
        const uint64_t grp = __ballot(mine);
        const uint32_t g = (uint32_t)__popcll(grp);
        if (g < (uint32_t)kPeelMin) break;
        uint32_t s = 0, base = 0, won = 0;
        if (lane == leader) {
            bool w;
            s = find_or_insert(hkeys, htags, blog, lk, &w);
            won = w;
            // the group's j-th lane takes rank base + j, except an inserting
            // leader (j = 0), which takes rank 0
            base = w ? atomicAdd(&hsize[s], g - 1) : atomicAdd(&hsize[s], g) + 1;
        }
        s = (uint32_t)__shfl((int)s, leader, kWave);
        base = (uint32_t)__shfl((int)base, leader, kWave);
        won = (uint32_t)__shfl((int)won, leader, kWave);
        if (mine) {
            const uint32_t j = (uint32_t)__popcll(grp & below);
            slot = s;
            rank = (won && j == 0) ? 0u : base + j;
            pending = false;
        }
    }
    if (pending) {
        bool won;
        slot = find_or_insert(hkeys, htags, blog, key, &won);
        rank = won ? 0u : atomicAdd(&hsize[slot], 1u) + 1;
    }
    if (active) obj[i] = make_uint2(slot, rank);
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

// Key of forward neighbour d of a cell, in the cell's set.  Cell
// coordinates are at least 1 (the +1 offset) and at most 2^25 / L + 1, so
// every neighbour's coordinates stay inside their fb-bit fields.
__device__ __forceinline__ uint64_t neighbour_key(uint64_t key, int d, int fb) {
    // d = 0..12 enumerates (dx, dy, dz) > (0, 0, 0) lexicographically
    const int e = d + 14;  // index in the 3x3x3 cube, 13 being the centre
    const int dx = e / 9 - 1, dy = (e / 3) % 3 - 1, dz = e % 3 - 1;
    const uint64_t mask = (uint64_t(1) << fb) - 1;
    const uint64_t cx = (key >> (2 * fb)) & mask;
    const uint64_t cy = (key >> fb) & mask;
    const uint64_t cz = key & mask;
    const uint64_t set_bits = key & ~((uint64_t(1) << (3 * fb)) - 1);
    return set_bits |
           cell_key((uint32_t)(cx + dx), (uint32_t)(cy + dy), (uint32_t)(cz + dz), fb);
}

// Prefix sums over lists whose length is known on the device only run over
// blocks of kScanBlock entries: per-block sums, one block scanning them, and
// the block-local prefixes.
constexpr int kScanBlock = 1024;

// Exclusive scan, in place, of the nb block sums in bsum, by one block of
// kScanBlock threads; returns the total to every thread.
__device__ __forceinline__ int64_t scan_block_sums(int64_t nb, int64_t *__restrict__ bsum,
                                                   int64_t *wave_tot) {
    const int tid = threadIdx.x;
    const int64_t chunk = (nb + kScanBlock - 1) / kScanBlock;
    const int64_t b0 = min((int64_t)tid * chunk, nb), b1 = min(b0 + chunk, nb);
    int64_t part = 0;
    for (int64_t b = b0; b < b1; ++b) part += bsum[b];
    int64_t T;
    int64_t run = pairs_dev::block_exclusive_scan<kScanBlock>(part, wave_tot, &T);
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = bsum[b];
        bsum[b] = run;
        run += v;
    }
    return T;
}

// Step 2: the first object of every cell and the cells' order, by an
// exclusive prefix over the table's slots in slot order of the pair (objects,
// cells) packed in one 64-bit word (objects in the high half, 1 per
// occupied slot in the low half; both stay below 2^31), in three launches:
// per-block sums over blocks of kSlotBlock slots (4 per thread, read as one
// word of tags and one 16-byte load of sizes), one block scanning them (and
// setting *ncell, the number of cells), and the block-local prefixes.
constexpr int kSlotsPerThread = 4, kSlotBlock = kScanBlock * kSlotsPerThread;

struct SlotPairs {
    uint64_t v[kSlotsPerThread];
    uint64_t sum;
};

// The pairs of slots [k, k + 4) (k a multiple of 4; the slot count is a
// multiple of 8, so a group starting below it ends within it).
__device__ __forceinline__ SlotPairs slot_pairs(const uint8_t *__restrict__ htags,
                                                const uint32_t *__restrict__ hsize, int64_t k,
                                                int64_t slots) {
    SlotPairs p;
    p.sum = 0;
    uint32_t tw = 0;
    uint4 sz = make_uint4(0, 0, 0, 0);
    if (k < slots) {
        tw = *(const uint32_t *)(htags + k);
        sz = *(const uint4 *)(hsize + k);
    }
    const uint32_t szs[kSlotsPerThread] = {sz.x, sz.y, sz.z, sz.w};
#pragma unroll
    for (int j = 0; j < kSlotsPerThread; ++j) {
        const bool occ = (tw >> (8 * j)) & 0xFFu;
        p.v[j] = occ ? ((uint64_t)(szs[j] + 1) << 32) | 1u : 0;
        p.sum += p.v[j];
    }
    return p;
}

__global__ __launch_bounds__(kScanBlock) void k_bin_slot_sums(const uint8_t *__restrict__ htags,
                                                             const uint32_t *__restrict__ hsize,
                                                             int64_t slots,
                                                             int64_t *__restrict__ bsum) {
    __shared__ int64_t wave_tot[kScanBlock / kWave + 1];
    const int64_t k = ((int64_t)blockIdx.x * kScanBlock + threadIdx.x) * kSlotsPerThread;
    const SlotPairs p = slot_pairs(htags, hsize, k, slots);
    int64_t sum;
    pairs_dev::block_exclusive_scan<kScanBlock>((int64_t)p.sum, wave_tot, &sum);
    if (threadIdx.x == 0) bsum[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kScanBlock) void k_bin_slot_scan(int64_t nb,
                                                             int64_t *__restrict__ bsum,
                                                             uint32_t *__restrict__ ncell) {
    __shared__ int64_t wave_tot[kScanBlock / kWave + 1];
    const int64_t T = scan_block_sums(nb, bsum, wave_tot);
    if (threadIdx.x == 0) *ncell = (uint32_t)(T & 0xFFFFFFFFu);
}

// Per occupied slot sl, the cell c it holds in slot order: off[c] its first
// object, ukeys[c] its key, hvals[sl] = (first object, size) for the
// lookups; off[m] = n.
__global__ __launch_bounds__(kScanBlock) void k_bin_slot_prefix(
    const uint8_t *__restrict__ htags, const uint32_t *__restrict__ hsize,
    const uint64_t *__restrict__ hkeys, int64_t slots, const int64_t *__restrict__ bsum,
    const uint32_t *__restrict__ ncell, int64_t n, uint32_t *__restrict__ off,
    uint64_t *__restrict__ ukeys, uint2 *__restrict__ hvals) {
    __shared__ int64_t wave_tot[kScanBlock / kWave + 1];
    const int64_t k = ((int64_t)blockIdx.x * kScanBlock + threadIdx.x) * kSlotsPerThread;
    const SlotPairs p = slot_pairs(htags, hsize, k, slots);
    int64_t sum;
    uint64_t at = (uint64_t)bsum[blockIdx.x] +
                  (uint64_t)pairs_dev::block_exclusive_scan<kScanBlock>((int64_t)p.sum, wave_tot,
                                                                         &sum);
#pragma unroll
    for (int j = 0; j < kSlotsPerThread; ++j) {
        if (p.v[j]) {
            const uint32_t c = (uint32_t)(at & 0xFFFFFFFFu), first = (uint32_t)(at >> 32);
            off[c] = first;
            ukeys[c] = hkeys[k + j];
            hvals[k + j] = make_uint2(first, (uint32_t)(p.v[j] >> 32));
        }
        at += p.v[j];
    }
    if (k == 0) off[*ncell] = (uint32_t)n;
}

// Step 3: the records grouped by cell, in two passes: each object's index
// at its cell's first object plus its rank (a 4-byte scattered write), then
// the records and each one's q = |p|^2 - r^2 (the partner term of the Gram
// test, read by the work items' tasks) gathered in that order (scattered
// 16-byte reads, written in order).
__global__ void k_bin_scatter(int64_t n, const uint2 *__restrict__ obj,
                              const uint2 *__restrict__ hvals, uint32_t *__restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint2 o = obj[i];
    perm[hvals[o.x].x + o.y] = (uint32_t)i;
}

__global__ void k_bin_gather(const int4 *__restrict__ rec, const uint32_t *__restrict__ perm,
                             int64_t n, int4 *__restrict__ so, int64_t *__restrict__ sq) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const int4 o = rec[perm[d]];
    so[d] = o;
    sq[d] = pairs_dev::gram_q(o.x, o.y, o.z, o.w);
}

// Pairs of one occupied cell (first object a0, n objects, key `key`),
// counted by the G lanes of a group (gl = lane in the group, g0 = the group's
// first lane in the wave): its 13 forward neighbours are looked up by lanes
// 0..12 of the group, the pairs inside the cell run on the balanced circular
// assignment, and the pairs with each occupied neighbour with the lanes
// taking the cell's objects against all of the neighbour's.
// A work item: the pairs between objects [a0, a0 + na) and [b0, b0 + nb) of
// the grouped records, or the pairs within [a0, a0 + na) when b0 == a0, all
// in set `set`.
struct Item {
    uint32_t a0, na, b0, nb, set;
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
__device__ __forceinline__ uint64_t count_cell(int64_t a0, int64_t n, uint64_t key, uint32_t set,
                                               int gl, int g0, const int4 *__restrict__ so,
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
    // those with each big (or, for a big cell, every) occupied neighbour,
    // with the larger range as the rows (more rows per lane, so each staged
    // partner feeds more tests)
    const bool swap = nb.y > (uint32_t)n;
    push_items(items, big && gl == 0,
               Item{(uint32_t)a0, (uint32_t)n, (uint32_t)a0, (uint32_t)n, set},
               gl < 13 && nb.y != 0 && (big || nb.y > (uint32_t)kBigCell),
               Item{swap ? nb.x : (uint32_t)a0, swap ? nb.y : (uint32_t)n,
                    swap ? (uint32_t)a0 : nb.x, swap ? (uint32_t)n : nb.y, set});
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
    const bool small_nb = nb.y != 0 && nb.y <= (uint32_t)kBigCell;
    uint32_t occ = (uint32_t)(__ballot(small_nb) >> g0) & ((1u << 13) - 1);
    if (n < __popc(occ)) {
        // fewer objects in the cell than occupied neighbours: each of lanes
        // 0..12 takes its own neighbour's pairs with the whole cell, in
        // place of the lanes sharing the cell's objects one neighbour after
        // the other
        if (small_nb)
            for (int64_t i = 0; i < n; ++i) {
                const int4 oi = so[a0 + i];
                for (uint32_t j = 0; j < nb.y; ++j) cnt += touch(oi, so[nb.x + j]);
            }
        return cnt;
    }
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
// their keys; off: their first object in the grouped records, off[m] = n;
// htags, hkeys, hvals, blog: the table from keys to cell ranges; fb: bits per
// axis of a key; so: the object records grouped by cell.  counts: one count
// per set; with one set, each wave adds its cells' pairs once at the end,
// otherwise each group adds each cell's pairs (when any) to its set's count.
constexpr int kGroup = 16;

// Eight waves per SIMD: the loop waits on loads, so occupancy pays.
template <bool Batched>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_bin_count(
    const int4 *__restrict__ so, const uint64_t *__restrict__ ukeys,
    const uint32_t *__restrict__ off, const uint32_t *__restrict__ m_ptr,
    const uint64_t *__restrict__ htags, const uint64_t *__restrict__ hkeys,
    const uint2 *__restrict__ hvals, int blog, int fb, ItemList items, uint64_t *counts) {
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
        const uint32_t set = Batched ? (uint32_t)(key >> (3 * fb)) : 0u;
        uint64_t cc = count_cell<kGroup>(o0, n, key, set, gl, g0, so, htags, hkeys, hvals, blog,
                                         fb, items);
        if (Batched) {
            // the 16 lanes of a group run the same cells, so the xor partners
            // stay inside the group and are active together
            for (int o = kGroup / 2; o >= 1; o >>= 1) cc += __shfl_xor(cc, o, kWave);
            if (gl == 0 && cc) atomicAdd((unsigned long long *)&counts[set], (unsigned long long)cc);
        } else {
            cnt += cc;
        }
        o0 = p0, o1 = p1, key = pk;
    }
    if (!Batched) wave_count_to(counts, cnt);
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
    const int64_t m = item_count(L);
    const int64_t T = scan_block_sums((m + kScanBlock - 1) / kScanBlock, bsum, wave_tot);
    if (threadIdx.x == 0) {
        const int64_t B = m > 0 ? max((int64_t)1, (T + m - 1) / m) : 1;
        hdr->m = m;
        hdr->T = T;
        hdr->B = B;
        hdr->nbuckets = (T + B - 1) / B;
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
    const int rlast = min(ra + kWave * K, (int)it.na) - 1;
    const int core_lo = rlast + 1, core_hi = self ? ra + band.steps(ra) : INT32_MAX;
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
        // a cell's own pairs need the ownership mask only at the band's edges:
        // every row of the block owns the partners in [core_lo, core_hi]
        if (self && !(g0 >= core_lo && g0 + gn - 1 <= core_hi)) {
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

// The tasks of all items, taken by the waves with a grid stride; each task
// adds its pairs (when any) to its item's set's count.
__global__ __launch_bounds__(kBlock) void k_bin_count_items(const int4 *__restrict__ so,
                                                            const int64_t *__restrict__ sq,
                                                            ItemList L,
                                                            const int64_t *__restrict__ pre,
                                                            const int32_t *__restrict__ tab,
                                                            const ItemSched *__restrict__ hdr,
                                                            uint64_t *counts) {
    using namespace pairs_dev;
    __shared__ PartnerI32 wp_all[kBlock / kWave][kWave];
    __shared__ int64_t wq_all[kBlock / kWave][kWave];
    const int wave = wave_id();
    PartnerI32 *wp = wp_all[wave];
    int64_t *wq = wq_all[wave];
    const int64_t total = hdr->T, B = hdr->B;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / kWave);
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
        uint32_t cnt;
        if (K == 1)
            cnt = item_task<1>(so, sq, it, local, wp, wq);
        else if (K == 2)
            cnt = item_task<2>(so, sq, it, local, wp, wq);
        else
            cnt = item_task<4>(so, sq, it, local, wp, wq);
        if (lane_id() == 0 && cnt)
            atomicAdd((unsigned long long *)&counts[it.set], (unsigned long long)cnt);
    }
}

// Ranges of 32-bit words that the pipeline needs zeroed, cleared by one
// launch (blockIdx.y picks the range): the counts, the table's keys, tags
// and per-slot object counts, and the numbers of cells and work items.
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
