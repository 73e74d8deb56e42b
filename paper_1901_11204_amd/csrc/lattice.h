// Collision and contact counts of bead vectors on the integer lattice Z^3
// (Section 3, algorithms countColls and countContacts).
//
// The paper keeps an occupancy array `space` over the whole bounded lattice
// S^3 and walks the beads once: each bead adds the site's current occupancy
// to the collision count and then increments it; a second pass sums the
// occupancy of the six neighbouring sites of every bead and halves the total
// to count contacts.  Both results are order independent: collisions are the
// pairs of beads on one site, contacts the pairs on sites one unit apart
// along one axis.
//
// On gfx950 the occupancy array becomes a hash table in LDS, one per bead
// vector, sized from the vector's length rather than from the lattice: the
// dense (2a+1)^3 array of the paper would not fit a workgroup, and the sites a
// vector touches are at most its length.  One workgroup handles one vector at
// a time:
//   1. its beads (at most kBlock * BPT) are loaded into registers, coalesced,
//      and reduced to the vector's bounding box;
//   2. each bead's site becomes a key in the box padded by one site on every
//      side, key = ((x - x0 + 1) * Y + (y - y0 + 1)) * Z + (z - z0 + 1) with
//      Y, Z the padded extents, so that the neighbour at +z, +y, +x is key + 1,
//      key + Z, key + Y*Z, and no neighbour key aliases another site;
//   3. the insertion pass is countColls with LDS atomics: a compare-and-swap
//      claims an empty slot for a new site, an atomic add on an existing site
//      returns the occupancy before this bead, and the returned values summed
//      over all beads are the number of colliding pairs whatever the order;
//   4. after a barrier, the lookup pass is countContacts over the three
//      positive neighbours only: each unordered pair of neighbouring sites is
//      met once, from its lower site, so no halving is needed.
// A slot is one 64-bit word: the key in the upper 40 bits and the occupancy
// in the lower 24 bits, so a claim and an increment are single LDS atomics.
// Tables use linear probing at load at most 1/2 (2^tlog slots for at most
// 2^(tlog-1) beads); every probe sequence ends at the key or an empty slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace pairs_lattice {

using pairs_dev::kWave;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kMinLog = 6;   // smallest table: 64 slots
constexpr int kMaxLog = 13;  // largest table: 8192 slots, 64 KiB of LDS
constexpr int kMaxBpt = 16;  // beads per thread held in registers
constexpr int64_t kMaxLdsBeads = int64_t(1) << (kMaxLog - 1);
static_assert(kMaxLdsBeads == int64_t(kBlock) * kMaxBpt, "largest table matches the registers");
static_assert(3 * kMaxBpt <= 64 && kMaxBpt <= 32, "pending-lookup and pending-bead masks fit their words");

constexpr int kCountBits = 24;
constexpr uint64_t kCountMask = (uint64_t(1) << kCountBits) - 1;
constexpr uint64_t kKeyLimit = uint64_t(1) << (64 - kCountBits);  // keys below 2^40
constexpr uint64_t kBad = ~uint64_t(0);

// Bits of the device status word.
constexpr int kFlagDomain = 1;  // a vector's padded box holds 2^40 sites or more
constexpr int kFlagSize = 2;    // a vector longer than the launch's capacity
constexpr int kFlagTable = 4;   // a probe sequence ran through the whole table

struct IO {
    const int32_t *x, *y, *z;
    const int64_t *off;  // CSR offsets [n_sets + 1]; null: one vector [0, n_total)
    int64_t n_sets, n_total;
    uint64_t *coll, *cont;  // [n_sets] each, either may be null
    int *flag;
};

__device__ __forceinline__ void vector_range(const IO &io, int64_t s, int64_t &b, int64_t &n) {
    if (io.off) {
        b = io.off[s];
        n = io.off[s + 1] - b;
    } else {
        b = 0;
        n = io.n_total;
    }
}

// Fibonacci hashing of a key onto 2^tlog slots.
__device__ __forceinline__ uint32_t home_slot(uint64_t key, int tlog) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - tlog));
}

// Wave reductions with DPP: inclusive scans inside each row of 16 lanes,
// then row broadcasts carry them across rows, so lane 63 ends with the
// result, which is then read into a scalar.  Lanes without a DPP source keep
// their own value (`old` = v), which leaves min, max and (with 0) sums intact.
template <int Ctrl, int RowMask>
__device__ __forceinline__ int dpp_keep(int v) {
    return __builtin_amdgcn_update_dpp(v, v, Ctrl, RowMask, 0xf, false);
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ int dpp_zero(int v) {
    return __builtin_amdgcn_update_dpp(0, v, Ctrl, RowMask, 0xf, false);
}

__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp_keep<0x111, 0xf>(v));
    v = min(v, dpp_keep<0x112, 0xf>(v));
    v = min(v, dpp_keep<0x114, 0xf>(v));
    v = min(v, dpp_keep<0x118, 0xf>(v));
    v = min(v, dpp_keep<0x142, 0xa>(v));
    v = min(v, dpp_keep<0x143, 0xc>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_max(int v) {
    v = max(v, dpp_keep<0x111, 0xf>(v));
    v = max(v, dpp_keep<0x112, 0xf>(v));
    v = max(v, dpp_keep<0x114, 0xf>(v));
    v = max(v, dpp_keep<0x118, 0xf>(v));
    v = max(v, dpp_keep<0x142, 0xa>(v));
    v = max(v, dpp_keep<0x143, 0xc>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Sum of a count below 2^32 over the wave.
__device__ __forceinline__ uint32_t wave_add(uint32_t u) {
    int v = (int)u;
    v += dpp_zero<0x111, 0xf>(v);
    v += dpp_zero<0x112, 0xf>(v);
    v += dpp_zero<0x114, 0xf>(v);
    v += dpp_zero<0x118, 0xf>(v);
    v += dpp_zero<0x142, 0xa>(v);
    v += dpp_zero<0x143, 0xc>(v);
    return (uint32_t)__builtin_amdgcn_readlane(v, 63);
}

typedef unsigned long long ull;

// Continues the insertion of `key` after its home slot held another key:
// linear probing from the slot after `slot`.  Returns the occupancy before
// this bead, or kCountMask + 1 if every slot was taken by other keys.
__device__ __noinline__ uint32_t insert_probe(uint64_t *table, uint32_t mask, uint64_t key,
                                              uint32_t slot) {
    const uint64_t fresh = (key << kCountBits) | 1;
    for (uint32_t p = 0; p < mask; ++p) {
        slot = (slot + 1) & mask;
        const uint64_t v = atomicCAS((ull *)&table[slot], 0ull, (ull)fresh);
        if (v == 0) return 0;
        if ((v >> kCountBits) == key)
            return (uint32_t)(atomicAdd((ull *)&table[slot], 1ull) & kCountMask);
    }
    return (uint32_t)kCountMask + 1;
}

// Reads a slot after the insertion phase.  An LDS table is read directly; a
// table in global memory is read at device scope, past the L1 cache, which
// the atomics of other waves bypass.
template <bool Global>
__device__ __forceinline__ uint64_t read_slot(const uint64_t *p) {
    if (Global) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

// Occupancy of `key` once its home slot held another key.
template <bool Global>
__device__ __noinline__ uint32_t lookup_probe(const uint64_t *table, uint32_t mask, uint64_t key,
                                              uint32_t slot) {
    for (uint32_t p = 0; p < mask; ++p) {
        slot = (slot + 1) & mask;
        const uint64_t v = read_slot<Global>(&table[slot]);
        if (v == 0) return 0;
        if ((v >> kCountBits) == key) return (uint32_t)(v & kCountMask);
    }
    return 0;
}

template <bool Global>
__device__ __forceinline__ uint32_t occupancy(const uint64_t *table, uint32_t mask, int tlog,
                                              uint64_t key) {
    const uint32_t h = home_slot(key, tlog);
    const uint64_t v = read_slot<Global>(&table[h]);
    if (v == 0) return 0;
    if ((v >> kCountBits) == key) return (uint32_t)(v & kCountMask);
    return lookup_probe<Global>(table, mask, key, h);
}

// Adds one bead at `key` to a table; returns the occupancy before it, or
// kCountMask + 1 if the table had no room.
__device__ __forceinline__ uint32_t insert(uint64_t *table, uint32_t mask, int tlog, uint64_t key) {
    const uint32_t h = home_slot(key, tlog);
    const uint64_t v = atomicCAS((ull *)&table[h], 0ull, (ull)((key << kCountBits) | 1));
    if (v == 0) return 0;
    if ((v >> kCountBits) == key) return (uint32_t)(atomicAdd((ull *)&table[h], 1ull) & kCountMask);
    return insert_probe(table, mask, key, h);
}

// Site key of a bead in the padded box with corner (x0, y0, z0) - 1.
__device__ __forceinline__ uint64_t site_key(int x, int y, int z, int x0, int y0, int z0,
                                             uint64_t Y, uint64_t Z) {
    return (((uint64_t)((uint32_t)x - (uint32_t)x0) + 1) * Y +
            ((uint64_t)((uint32_t)y - (uint32_t)y0) + 1)) * Z +
           ((uint64_t)((uint32_t)z - (uint32_t)z0) + 1);
}

// Padded extents of a box; false if it holds 2^40 sites or more.  Each
// extent is below 2^33, so the product is formed in double: every partial
// product below 2^53 is exact, and one at or above 2^53 stays above 2^40
// after rounding, so the comparison is exact.
__device__ __forceinline__ bool padded_box(const int (&mn)[3], const int (&mx)[3], uint64_t &Y,
                                           uint64_t &Z, uint64_t &YZ) {
    const uint64_t X = (uint64_t)((uint32_t)mx[0] - (uint32_t)mn[0]) + 3;
    Y = (uint64_t)((uint32_t)mx[1] - (uint32_t)mn[1]) + 3;
    Z = (uint64_t)((uint32_t)mx[2] - (uint32_t)mn[2]) + 3;
    if ((double)X * (double)Y * (double)Z >= (double)kKeyLimit) return false;
    YZ = Y * Z;
    return true;
}

// Block-wide bounding box: every thread ends with the box of the values it
// and the other threads passed in.  `red` holds 6 * kWaves ints and is free
// again after the call.
__device__ __forceinline__ void block_box(int (&mn)[3], int (&mx)[3], int *red) {
    const int lane = threadIdx.x & (kWave - 1), w = pairs_dev::wave_id();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min(mn[a]);
        mx[a] = wave_max(mx[a]);
    }
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            red[a * kWaves + w] = mn[a];
            red[(3 + a) * kWaves + w] = mx[a];
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            mn[a] = min(mn[a], red[a * kWaves + q]);
            mx[a] = max(mx[a], red[(3 + a) * kWaves + q]);
        }
    }
    __syncthreads();
}

// Block sums of two per-thread counts below 2^32 each per wave, in thread 0.
// `red` holds 2 * kWaves 64-bit words; its reads and writes start after the
// call's first barrier, so a table it shares memory with may be read until
// then.
__device__ __forceinline__ void block_sums32(uint32_t a, uint32_t b, uint64_t &sa, uint64_t &sb,
                                             uint64_t *red) {
    const int lane = threadIdx.x & (kWave - 1), w = pairs_dev::wave_id();
    a = wave_add(a);
    b = wave_add(b);
    __syncthreads();
    if (lane == 0) {
        red[w] = a;
        red[kWaves + w] = b;
    }
    __syncthreads();
    sa = sb = 0;
    if (threadIdx.x == 0) {
        for (int q = 0; q < kWaves; ++q) {
            sa += red[q];
            sb += red[kWaves + q];
        }
    }
    __syncthreads();
}

// Block sums of two per-thread counts, in thread 0.  `red` holds 2 * kWaves
// 64-bit words and may be reused after the call.
__device__ __forceinline__ void block_sums(uint64_t &a, uint64_t &b, uint64_t *red) {
    const int lane = threadIdx.x & (kWave - 1), w = pairs_dev::wave_id();
    for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o, kWave);
        b += __shfl_xor(b, o, kWave);
    }
    __syncthreads();
    if (lane == 0) {
        red[w] = a;
        red[kWaves + w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kWaves; ++q) {
            a += red[q];
            b += red[kWaves + q];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void write_both(const IO &io, int64_t s, uint64_t c, uint64_t k) {
    if (io.coll) io.coll[s] = c;
    if (io.cont) io.cont[s] = k;
}

// Slot layout of an LDS table for 32- or 64-bit site keys: the key in the
// upper bits of the 64-bit slot, the occupancy in the rest.  32-bit keys
// serve boxes of fewer than 2^32 sites (any chain of up to about 4800 beads)
// and make the key arithmetic, the hash and the comparisons single 32-bit
// instructions; 64-bit keys serve boxes up to the 2^40 limit.
template <typename K>
struct Slots {
    static constexpr int kBits = 8 * sizeof(K);
    static constexpr int kShift = sizeof(K) == 4 ? 32 : kCountBits;
    static constexpr uint64_t kCnt = (uint64_t(1) << kShift) - 1;
    static constexpr K kMul = sizeof(K) == 4 ? (K)0x9E3779B1u : (K)0x9E3779B97F4A7C15ull;
    // Fibonacci hashing: slot = top tlog bits of key * kMul.  The product is
    // kept, so a neighbour's hash is (key + d) * kMul = h + d * kMul, one add.
    __device__ static __forceinline__ uint32_t slot(K h, int tlog) {
        return (uint32_t)(h >> (kBits - tlog));
    }
    __device__ static __forceinline__ K key_of(uint64_t v) { return (K)(v >> kShift); }
};

// Counts one vector whose beads (BPT per thread) are in registers, in the
// LDS table of 2^tlog slots: insertion (countColls) then lookups
// (countContacts over the positive neighbours).  Returns this thread's
// shares; ends with the barrier after the insertion, so the caller must
// synchronise before the table is reused.
//
// Insertion: the home-slot claims of all beads go out together; then the
// increments, again together, one per bead (adding 0 where the claim found
// an empty slot or another key: a branch around each would make the wave
// wait for every returned value in turn); beads whose home slot held another
// key then probe the next slots, all pending beads of a lane at once.
// Lookups: G beads at a time, their 3G home-slot reads go out together and
// only the reads that met another key probe further.
template <typename K, int BPT, bool Contacts>
__device__ __forceinline__ void count_vector(uint64_t *table, int tlog, int64_t n,
                                             const int (&px)[BPT], const int (&py)[BPT],
                                             const int (&pz)[BPT], const int (&mn)[3],
                                             uint64_t Y64, uint64_t Z64, int *flag,
                                             uint32_t &coll, uint32_t &cont) {
    using S = Slots<K>;
    // A compare-and-swap expecting kNever never succeeds: no slot holds it
    // (keys stay below the box volume, so the key bits are never all ones).
    // Beads a lane does not hold, or does not need to move, issue their
    // atomics with it, so that every atomic and read is unconditional: the
    // conditional forms make the compiler build whole-array copies.
    constexpr uint64_t kNever = ~uint64_t(0);
    const int t = threadIdx.x;
    const uint32_t mask = (1u << tlog) - 1;
    const K Y = (K)Y64, Z = (K)Z64, YZ = Y * Z;
    K key[BPT], hk[BPT];
    uint32_t slot[BPT];
    uint64_t got[BPT];
    bool valid[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        valid[k] = t + (int64_t)k * kBlock < n;
        key[k] = ((K)((uint32_t)px[k] - (uint32_t)mn[0]) + 1) * Y;
        key[k] = (key[k] + (K)((uint32_t)py[k] - (uint32_t)mn[1]) + 1) * Z;
        key[k] = key[k] + (K)((uint32_t)pz[k] - (uint32_t)mn[2]) + 1;
        hk[k] = key[k] * S::kMul;
        slot[k] = S::slot(hk[k], tlog);
        got[k] = atomicCAS((ull *)&table[slot[k]], (ull)(valid[k] ? 0 : kNever),
                           (ull)(((uint64_t)key[k] << S::kShift) | 1));
        if (!valid[k]) got[k] = 0;
    }
    uint64_t before[BPT];
    bool inc[BPT];
    uint32_t pend = 0;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        inc[k] = got[k] != 0 && S::key_of(got[k]) == key[k];
        pend |= (got[k] != 0 && !inc[k]) ? 1u << k : 0u;
        before[k] = atomicAdd((ull *)&table[slot[k]], inc[k] ? 1ull : 0ull);
    }
    coll = 0;
#pragma unroll
    for (int k = 0; k < BPT; ++k) coll += inc[k] ? (uint32_t)(before[k] & S::kCnt) : 0u;
    // probing rounds: a bead index k takes part only if some lane of the
    // wave still has bead k pending (a wave-uniform test)
    for (uint32_t round = 0; __builtin_amdgcn_ballot_w64(pend != 0) && round <= mask; ++round) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const bool p = pend & (1u << k);
            got[k] = 0;
            if (__builtin_amdgcn_ballot_w64(p)) {
                slot[k] = p ? (slot[k] + 1) & mask : slot[k];
                got[k] = atomicCAS((ull *)&table[slot[k]], (ull)(p ? 0 : kNever),
                                   (ull)(((uint64_t)key[k] << S::kShift) | 1));
            }
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const bool p = pend & (1u << k);
            inc[k] = p && got[k] != 0 && S::key_of(got[k]) == key[k];
            pend &= (p && (got[k] == 0 || inc[k])) ? ~(1u << k) : ~0u;
            before[k] = 0;
            if (__builtin_amdgcn_ballot_w64(inc[k]))
                before[k] = atomicAdd((ull *)&table[slot[k]], inc[k] ? 1ull : 0ull);
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k) coll += inc[k] ? (uint32_t)(before[k] & S::kCnt) : 0u;
    }
    if (pend) atomicOr(flag, kFlagTable);
    __syncthreads();

    cont = 0;
    if (!Contacts) return;
    const K dK[3] = {(K)1, Z, YZ};
    const K dH[3] = {S::kMul, Z * S::kMul, YZ * S::kMul};
    constexpr int G = BPT < 4 ? BPT : 4;
#pragma unroll
    for (int g = 0; g < BPT; g += G) {
        uint64_t v[3 * G];
        uint32_t sl[3 * G];
        uint32_t lp = 0;
#pragma unroll
        for (int j = 0; j < 3 * G; ++j) {
            sl[j] = S::slot(hk[g + j / 3] + dH[j % 3], tlog);
            v[j] = table[sl[j]];
            v[j] = valid[g + j / 3] ? v[j] : 0;
        }
#pragma unroll
        for (int j = 0; j < 3 * G; ++j) {
            const K nk = key[g + j / 3] + dK[j % 3];
            const bool hit = S::key_of(v[j]) == nk;
            cont += hit ? (uint32_t)(v[j] & S::kCnt) : 0u;
            lp |= (v[j] != 0 && !hit) ? 1u << j : 0u;
        }
        for (uint32_t round = 0; __builtin_amdgcn_ballot_w64(lp != 0) && round <= mask;
             ++round) {
#pragma unroll
            for (int j = 0; j < 3 * G; ++j) {
                if (__builtin_amdgcn_ballot_w64(lp & (1u << j))) {
                    sl[j] = (lp & (1u << j)) ? (sl[j] + 1) & mask : sl[j];
                    v[j] = table[sl[j]];
                }
            }
#pragma unroll
            for (int j = 0; j < 3 * G; ++j) {
                const bool p = lp & (1u << j);
                const K nk = key[g + j / 3] + dK[j % 3];
                const bool hit = p && S::key_of(v[j]) == nk;
                cont += hit ? (uint32_t)(v[j] & S::kCnt) : 0u;
                lp &= (p && (v[j] == 0 || hit)) ? ~(1u << j) : ~0u;
            }
        }
    }
}

// --- near path: 32-bit keys relative to the vector's first bead ------------
//
// A chain of unit steps stays near its first bead: a random chain of 1920
// beads strays some tens of sites along each axis.  Offsets from the first
// bead up to 1022 sites along x and y and 510 along z are packed, biased,
// into one 32-bit key, x in 11 bits, y in 11 and z in 10, so that the
// neighbours at +z, +y, +x are key + 1, key + 2^10, key + 2^21 and no field
// overflows into the next.  A vector with a bead outside that range is left
// to the box-based pass (k_lattice with 64-bit keys).
//
// Table: 2^tlog 32-bit keys followed by 2^tlog 32-bit occupancies in LDS
// (the same 8 bytes per slot as the 64-bit slots of the box-based pass).
// Keys are read four at a time (one 16-byte LDS read): a key's probe
// sequence starts at its home bucket of four slots and moves by whole
// buckets.  Slots of a bucket fill in order and a bucket is passed only when
// full, so a search stops at the bucket holding the key or an empty slot.
//
// Counting: a bead finds its site's key or claims an empty slot for it
// (compare-and-swap on the key), then increments the slot's occupancy; the
// value before the increment is its countColls term.  After the barrier the
// contact lookups read the three positive neighbours' buckets and, for the
// neighbours present, their occupancies.  Beads whose home bucket is full of
// other keys (or whose claim another key won) are few; they and the
// matching lookups are finished one at a time per lane after a batched round
// over all beads.  Wave sums go to the outputs with device atomics (the
// outputs are cleared before the launch).

constexpr int kNearXBits = 11, kNearYBits = 11, kNearZBits = 10;
constexpr uint32_t kNearDy = 1u << kNearZBits;                // key step of +y
constexpr uint32_t kNearDx = 1u << (kNearZBits + kNearYBits);  // key step of +x
constexpr uint32_t kNearMul = 0x9E3779B1u;

// Biased field of an offset d from the first bead; in range when 1 <= f and
// f + 1 < 2^bits, so that the +1 neighbour stays in the field.
template <int Bits>
__device__ __forceinline__ bool near_field(int v, int v0, uint32_t &f) {
    int d;
    const bool wrapped = __builtin_sub_overflow(v, v0, &d);  // 32-bit, overflow detected
    f = (uint32_t)d + (1u << (Bits - 1));
    return !wrapped & (f - 1u <= (1u << Bits) - 3u);  // 1 <= f <= 2^Bits - 2
}

// Where `key` stands in a bucket of four keys: j < 4 if slot j holds it,
// 4 + j if it is absent and slot j is the first empty one, 8 if the bucket
// is full of other keys.
// Every comparison is made and combined with bitwise operators, so the
// result is a few selects on the comparison masks: chains of conditional
// operators become branches that wait out each LDS read in turn.
__device__ __forceinline__ uint32_t bucket_pick(const uint4 &v, uint32_t key) {
    const bool k0 = v.x == key, k1 = v.y == key, k2 = v.z == key, k3 = v.w == key;
    const bool z0 = v.x == 0, z1 = v.y == 0, z2 = v.z == 0, z3 = v.w == 0;
    const uint32_t f = k0 ? 0u : k1 ? 1u : k2 ? 2u : 3u;
    const uint32_t e = z0 ? 4u : z1 ? 5u : z2 ? 6u : 7u;
    const bool any_k = k0 | k1 | k2 | k3, any_z = z0 | z1 | z2 | z3;
    return any_k ? f : any_z ? e : 8u;
}

// Lookup of `key` in a bucket once insertion is over: j < 4 if slot j holds
// it, 4 if it is absent (the bucket has an empty slot; slots fill in order,
// so the last one tells), 8 if the bucket is full of other keys.
__device__ __forceinline__ uint32_t bucket_find(const uint4 &v, uint32_t key) {
    const bool k0 = v.x == key, k1 = v.y == key, k2 = v.z == key, k3 = v.w == key;
    const uint32_t f = k0 ? 0u : k1 ? 1u : k2 ? 2u : 3u;
    return (k0 | k1 | k2 | k3) ? f : v.w == 0 ? 4u : 8u;
}

// Sum of the lanes' values into *out with one device atomic per wave.
__device__ __forceinline__ void wave_add_to(uint64_t *out, uint32_t v) {
    const uint32_t s = wave_add(v);
    if ((threadIdx.x & (kWave - 1)) == 0 && s) atomicAdd((ull *)out, (ull)s);
}

// Bit 63 of a vector's collision output (its contact output when collisions
// are not asked for) marks a vector that the near pass leaves to the
// box-based pass.  Counts never reach it, so the atomic sums of the other
// waves leave it intact.
constexpr uint64_t kFarBit = uint64_t(1) << 63;

__device__ __forceinline__ uint64_t *marker(const IO &io) { return io.coll ? io.coll : io.cont; }

// Barrier of the threads that count one vector together.
template <int Waves>
__device__ __forceinline__ void group_sync() {
    if (Waves == 1)
        pairs_dev::wave_sync();
    else
        __syncthreads();
}

// Waves = 4: the workgroup counts one vector at a time (kBlock threads, one
// table, workgroup barriers).  Waves = 1: each wave counts its own vectors
// with its own table (2^tlog slots per wave) and orders its LDS accesses
// with wave-local fences instead of barriers; for short vectors, which
// would leave most of a workgroup idle.
template <int BPT, bool Contacts, int Waves>
__global__ __launch_bounds__(kBlock) void k_lattice_near(IO io, int tlog, int defer) {
    static_assert(Waves == 1 || Waves == kWaves, "a wave or the whole workgroup per vector");
    constexpr int G = kWave * Waves;  // threads per vector
    extern __shared__ uint64_t lds_tables[];
    constexpr uint32_t kNever32 = ~0u;  // no key equals it: keys are below 2^32 - 1
    const int t = threadIdx.x % G;
    const uint32_t T = 1u << tlog, qmask = (T >> 2) - 1;
    const int qshift = 32 - (tlog - 2);  // home bucket = top tlog - 2 bits of the hash
    const int64_t cap = min((int64_t)(T / 2), (int64_t)BPT * G);
    const int group = Waves == 1 ? pairs_dev::wave_id() : 0;
    uint64_t *table = lds_tables + (size_t)group * T;
    const int64_t first = (int64_t)blockIdx.x * (kWaves / Waves) + group;
    const int64_t stride = (int64_t)gridDim.x * (kWaves / Waves);

    for (int64_t s = first; s < io.n_sets; s += stride) {
        int64_t b, n;
        vector_range(io, s, b, n);
        if (n < 2 || n > cap) {
            if (t == 0 && !(defer && n > kMaxLdsBeads)) {
                write_both(io, s, n < 2 ? 0 : kBad, n < 2 ? 0 : kBad);
                if (n >= 2) atomicOr(io.flag, kFlagSize);
            }
            continue;
        }
        // the vector's arrays from its first bead; n <= 4096, so 32-bit indices
        const int32_t *xb = io.x + b, *yb = io.y + b, *zb = io.z + b;
        const int x0 = xb[0], y0 = yb[0], z0 = zb[0];
        uint32_t key[BPT], hk[BPT];
        bool valid[BPT], far = false;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = t + k * G;
            const int ii = i < n ? i : 0;
            uint32_t fx, fy, fz;
            const bool ok = near_field<kNearXBits>(xb[ii], x0, fx) &
                            near_field<kNearYBits>(yb[ii], y0, fy) &
                            near_field<kNearZBits>(zb[ii], z0, fz);
            far |= (i < n) & !ok;
            valid[k] = (i < n) & ok;
            key[k] = (fx << (kNearZBits + kNearYBits)) | (fy << kNearZBits) | fz;
            hk[k] = key[k] * kNearMul;
        }
        if (__builtin_amdgcn_ballot_w64(far) && (t & (kWave - 1)) == 0)
            atomicOr((ull *)marker(io) + s, (ull)kFarBit);
        group_sync<Waves>();  // the previous vector's lookups are done
        for (uint32_t e = t; e < T; e += G) table[e] = 0;
        group_sync<Waves>();

        uint32_t *keys = (uint32_t *)table, *occ = keys + T;

        // Insertion, batched round: every bead reads its home bucket; those
        // that found an empty slot claim it, all at once; those whose key is
        // there or whose claim held take their occupancy increment.
        uint32_t slot[BPT], pend = 0, coll = 0, cont = 0;
        {
            uint32_t want = 0;
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const uint32_t h4 = 4 * (hk[k] >> qshift);
                const uint4 v = *(const uint4 *)&keys[h4];
                const uint32_t j = bucket_pick(v, key[k]);
                slot[k] = h4 + (j & 3);
                want |= (valid[k] && j == 4 + (j & 3)) ? 1u << k : 0u;  // an empty slot
                pend |= (valid[k] && j >= 4) ? 1u << k : 0u;            // not found
            }
            // A claim lost to another key (distinct sites sharing a home
            // bucket race for its first empty slot) moves on to the bucket's
            // next slot, so that slots still fill in order; only a bead that
            // loses the bucket's last slot is left to the per-lane probes.
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                bool w = want & (1u << k);
                uint32_t sl = slot[k];
                for (int a = 0; a < 4 && __builtin_amdgcn_ballot_w64(w); ++a) {
                    const uint32_t g = atomicCAS(&keys[sl], w ? 0u : kNever32, key[k]);
                    const bool mine = w && (g == 0 || g == key[k]);
                    pend &= mine ? ~(1u << k) : ~0u;
                    w = w && !mine && (sl & 3u) != 3u;
                    sl += w ? 1u : 0u;
                }
                slot[k] = sl;
            }
            uint32_t before[BPT];
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const bool done = valid[k] && !(pend & (1u << k));
                before[k] = atomicAdd(&occ[slot[k]], done ? 1u : 0u);
                coll += done ? before[k] : 0u;
            }
        }
        // The rest: a lane takes its lowest pending bead and follows it
        // bucket by bucket from its home bucket until it is placed.
        {
            uint32_t ck = 0, cq = 0;
            bool busy = false;
            for (uint32_t round = 0;
                 __builtin_amdgcn_ballot_w64(pend != 0 || busy) && round < 4 * T; ++round) {
                if (!busy && pend) {
                    const int k0 = __builtin_ctz(pend);
                    uint32_t h = 0;
#pragma unroll
                    for (int k = 0; k < BPT; ++k) {
                        ck = k == k0 ? key[k] : ck;
                        h = k == k0 ? hk[k] : h;
                    }
                    cq = h >> qshift;
                    pend &= pend - 1;
                    busy = true;
                }
                if (busy) {
                    const uint4 v = *(const uint4 *)&keys[4 * cq];
                    const uint32_t j = bucket_pick(v, ck);
                    const uint32_t sl = 4 * cq + (j & 3);
                    bool placed = j < 4;
                    if (j >= 4 && j < 8) {
                        const uint32_t g = atomicCAS(&keys[sl], 0u, ck);
                        placed = g == 0 || g == ck;
                    } else if (j >= 8) {
                        cq = (cq + 1) & qmask;
                    }
                    if (placed) {
                        coll += atomicAdd(&occ[sl], 1u);
                        busy = false;
                    }
                }
            }
            if (pend || busy) atomicOr(io.flag, kFlagTable);
        }
        group_sync<Waves>();

        // Contacts: the three positive neighbours of every bead, one batched
        // round over their home buckets (two beads at a time), then the
        // lookups that met a full bucket of other keys, one at a time per lane.
        if (Contacts) {
            const uint32_t dK[3] = {1u, kNearDy, kNearDx};
            uint64_t lp = 0;  // pending lookups, bit 3k + d (up to 48 of them)
            constexpr int G = BPT < 2 ? BPT : 2;
#pragma unroll
            for (int g = 0; g < BPT; g += G) {
                uint32_t cs[3 * G];
                bool hit[3 * G];
#pragma unroll
                for (int j = 0; j < 3 * G; ++j) {
                    const int k = g + j / 3, d = j % 3;
                    const uint32_t h4 = 4 * ((hk[k] + dK[d] * kNearMul) >> qshift);
                    const uint4 v = *(const uint4 *)&keys[h4];
                    const uint32_t p = bucket_find(v, key[k] + dK[d]);
                    hit[j] = valid[k] & (p < 4);
                    cs[j] = h4 + (p & 3);
                    lp |= (valid[k] & (p >= 8)) ? uint64_t(1) << (3 * k + d) : uint64_t(0);
                }
#pragma unroll
                for (int j = 0; j < 3 * G; ++j) {
                    const uint32_t c = occ[cs[j]];
                    cont += hit[j] ? c : 0u;
                }
            }
            uint32_t ck = 0, cq = 0;
            bool busy = false;
            for (uint32_t round = 0;
                 __builtin_amdgcn_ballot_w64(lp != 0 || busy) && round < 4 * T; ++round) {
                if (!busy && lp) {
                    const int j0 = __builtin_ctzll(lp);
                    const int k0 = j0 / 3, d0 = j0 - 3 * k0;
                    uint32_t kk = 0, h = 0;
#pragma unroll
                    for (int k = 0; k < BPT; ++k) {
                        kk = k == k0 ? key[k] : kk;
                        h = k == k0 ? hk[k] : h;
                    }
                    const uint32_t dd = d0 == 0 ? 1u : d0 == 1 ? kNearDy : kNearDx;
                    ck = kk + dd;
                    cq = (((h + dd * kNearMul) >> qshift) + 1) & qmask;
                    lp &= lp - 1;
                    busy = true;
                }
                if (busy) {
                    const uint4 v = *(const uint4 *)&keys[4 * cq];
                    const uint32_t p = bucket_find(v, ck);
                    if (p < 4) cont += occ[4 * cq + p];
                    busy = p >= 8;
                    cq = (cq + 1) & qmask;
                }
            }
        }
        if (io.coll) wave_add_to(&io.coll[s], coll);
        if (Contacts) wave_add_to(&io.cont[s], cont);
    }
}

// Box-based LDS pass for the vectors the near pass marked with kFarBit (and
// only those): one workgroup per vector, grid-stride over the vectors.  The
// keys are positions in the vector's bounding box padded by one site, so
// any box of fewer than 2^40 sites fits.  BPT beads per thread bound the
// vector length to kBlock * BPT; the table has 2^tlog slots of dynamic LDS
// and takes at most 2^(tlog-1) beads.  Vectors longer than that get kBad and
// raise kFlagSize, except those longer than kMaxLdsBeads when `defer` is
// set: k_lattice_global takes them.
template <int BPT, bool Contacts, typename K>
__global__ __launch_bounds__(kBlock) void k_lattice(IO io, int tlog, int defer) {
    constexpr bool kWide = sizeof(K) == 8;
    extern __shared__ uint64_t table[];
    const int t = threadIdx.x;
    const uint32_t T = 1u << tlog;
    const int64_t cap = min((int64_t)(T / 2), (int64_t)BPT * kBlock);
    int *red = (int *)table;  // the reductions borrow the table's first words

    for (int64_t s = blockIdx.x; s < io.n_sets; s += gridDim.x) {
        if (kWide && !(marker(io)[s] & kFarBit)) continue;
        int64_t b, n;
        vector_range(io, s, b, n);
        if (n < 2 || n > cap) {
            if (t == 0 && !(defer && n > kMaxLdsBeads)) {
                write_both(io, s, n < 2 ? 0 : kBad, n < 2 ? 0 : kBad);
                if (n >= 2) atomicOr(io.flag, kFlagSize);
            }
            continue;
        }

        // beads into registers, bounding box
        int px[BPT], py[BPT], pz[BPT];
        int mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int64_t i = t + (int64_t)k * kBlock;
            px[k] = py[k] = pz[k] = 0;
            if (i < n) {
                px[k] = io.x[b + i];
                py[k] = io.y[b + i];
                pz[k] = io.z[b + i];
                mn[0] = min(mn[0], px[k]);
                mn[1] = min(mn[1], py[k]);
                mn[2] = min(mn[2], pz[k]);
                mx[0] = max(mx[0], px[k]);
                mx[1] = max(mx[1], py[k]);
                mx[2] = max(mx[2], pz[k]);
            }
        }
        block_box(mn, mx, red);
        uint64_t Y, Z, YZ;
        if (!padded_box(mn, mx, Y, Z, YZ)) {
            if (t == 0) {
                write_both(io, s, kBad, kBad);
                atomicOr(io.flag, kFlagDomain);
            }
            continue;
        }
        const uint64_t X = (uint64_t)((uint32_t)mx[0] - (uint32_t)mn[0]) + 3;
        if (!kWide && (double)X * (double)YZ >= 4294967296.0) {
            if (t == 0) marker(io)[s] = kFarBit;
            continue;
        }

        for (uint32_t e = t; e < T; e += kBlock) table[e] = 0;
        __syncthreads();

        uint32_t coll, cont;
        count_vector<K, BPT, Contacts>(table, tlog, n, px, py, pz, mn, Y, Z, io.flag, coll,
                                       cont);

        // block sums; the table is free once every thread has passed the
        // first barrier inside, after its lookups
        uint64_t c0, c1;
        block_sums32(coll, cont, c0, c1, table);
        if (t == 0) write_both(io, s, c0, Contacts ? c1 : 0);
    }
}

// Global path of a batch: one workgroup per vector longer than kMaxLdsBeads,
// with its table in global memory at 4 * (its first bead) slots from `ws`:
// 2^tlog slots with 2n <= 2^tlog < 4n, so the tables of different vectors do
// not overlap.  The beads are read once per pass (box, insertion, lookups).
template <bool Contacts>
__global__ __launch_bounds__(kBlock) void k_lattice_global(IO io, uint64_t *ws) {
    __shared__ uint64_t red[6 * kWaves];
    const int t = threadIdx.x;
    for (int64_t s = blockIdx.x; s < io.n_sets; s += gridDim.x) {
        int64_t b, n;
        vector_range(io, s, b, n);
        if (n <= kMaxLdsBeads) continue;
        if (n > (int64_t)kCountMask) {
            if (t == 0) {
                write_both(io, s, kBad, kBad);
                atomicOr(io.flag, kFlagSize);
            }
            continue;
        }
        int mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
        for (int64_t i = t; i < n; i += kBlock) {
            const int v[3] = {io.x[b + i], io.y[b + i], io.z[b + i]};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = min(mn[a], v[a]);
                mx[a] = max(mx[a], v[a]);
            }
        }
        block_box(mn, mx, (int *)red);
        uint64_t Y, Z, YZ;
        if (!padded_box(mn, mx, Y, Z, YZ)) {
            if (t == 0) {
                write_both(io, s, kBad, kBad);
                atomicOr(io.flag, kFlagDomain);
            }
            continue;
        }
        int tlog = 1;
        while ((int64_t(1) << tlog) < 2 * n) ++tlog;
        const uint32_t mask = (1u << tlog) - 1;
        uint64_t *table = ws + 4 * b;
        for (int64_t e = t; e <= mask; e += kBlock) table[e] = 0;
        __threadfence();
        __syncthreads();

        uint64_t coll = 0, cont = 0;
        bool lost = false;
        for (int64_t i = t; i < n; i += kBlock) {
            const uint64_t key = site_key(io.x[b + i], io.y[b + i], io.z[b + i], mn[0], mn[1],
                                          mn[2], Y, Z);
            const uint32_t before = insert(table, mask, tlog, key);
            lost |= before > kCountMask;
            coll += before > kCountMask ? 0 : before;
        }
        if (lost) atomicOr(io.flag, kFlagTable);
        __threadfence();
        __syncthreads();
        if (Contacts) {
            for (int64_t i = t; i < n; i += kBlock) {
                const uint64_t key = site_key(io.x[b + i], io.y[b + i], io.z[b + i], mn[0],
                                              mn[1], mn[2], Y, Z);
                cont += occupancy<true>(table, mask, tlog, key + 1) +
                        occupancy<true>(table, mask, tlog, key + Z) +
                        occupancy<true>(table, mask, tlog, key + YZ);
            }
        }
        block_sums(coll, cont, red);
        if (t == 0) write_both(io, s, coll, Contacts ? cont : 0);
    }
}

// --- one long vector over the whole grid: box, clear, insert, look up -------
// `g` is the vector's working state in global memory: the box (6 ints) and
// the output sums, set up by k_lattice_single_init.

struct SingleState {
    int mn[3], mx[3];
};

__global__ void k_lattice_single_init(SingleState *g, uint64_t *coll, uint64_t *cont) {
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            g->mn[a] = INT32_MAX;
            g->mx[a] = INT32_MIN;
        }
        if (coll) *coll = 0;
        if (cont) *cont = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_lattice_single_box(IO io, SingleState *g) {
    __shared__ int red[6 * kWaves];
    int mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < io.n_total;
         i += (int64_t)gridDim.x * kBlock) {
        const int v[3] = {io.x[i], io.y[i], io.z[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(mn[a], v[a]);
            mx[a] = max(mx[a], v[a]);
        }
    }
    block_box(mn, mx, red);
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            atomicMin(&g->mn[a], mn[a]);
            atomicMax(&g->mx[a], mx[a]);
        }
    }
}

// Clears the table and, from block 0, marks a vector outside the domain.
__global__ __launch_bounds__(kBlock) void k_lattice_single_clear(IO io, const SingleState *g,
                                                                 uint64_t *table, int tlog) {
    const int64_t T = int64_t(1) << tlog;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < T;
         e += (int64_t)gridDim.x * kBlock)
        table[e] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint64_t Y, Z, YZ;
        if (!padded_box(g->mn, g->mx, Y, Z, YZ)) {
            write_both(io, 0, kBad, kBad);
            atomicOr(io.flag, kFlagDomain);
        }
    }
}

template <bool Lookup>
__global__ __launch_bounds__(kBlock) void k_lattice_single_pass(IO io, const SingleState *g,
                                                                uint64_t *table, int tlog) {
    __shared__ uint64_t red[2 * kWaves];
    uint64_t Y, Z, YZ;
    if (!padded_box(g->mn, g->mx, Y, Z, YZ)) return;  // uniform over the grid
    const uint32_t mask = (1u << tlog) - 1;
    uint64_t sum = 0, unused = 0;
    bool lost = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < io.n_total;
         i += (int64_t)gridDim.x * kBlock) {
        const uint64_t key = site_key(io.x[i], io.y[i], io.z[i], g->mn[0], g->mn[1], g->mn[2],
                                      Y, Z);
        if (Lookup) {
            sum += occupancy<false>(table, mask, tlog, key + 1) +
                   occupancy<false>(table, mask, tlog, key + Z) +
                   occupancy<false>(table, mask, tlog, key + YZ);
        } else {
            const uint32_t before = insert(table, mask, tlog, key);
            lost |= before > kCountMask;
            sum += before > kCountMask ? 0 : before;
        }
    }
    if (!Lookup && lost) atomicOr(io.flag, kFlagTable);
    block_sums(sum, unused, red);
    uint64_t *target = Lookup ? io.cont : io.coll;
    if (threadIdx.x == 0 && sum && target) atomicAdd((ull *)target, (ull)sum);
}

}  // namespace pairs_lattice
