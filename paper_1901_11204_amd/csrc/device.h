// Wave-level helpers for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pairs_dev {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Index of the calling wave within its block, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Lanes lo..hi (clipped to 0..63) as a bit mask; 0 if the range is empty.
__device__ __forceinline__ uint64_t lane_range(int lo, int hi) {
    lo = lo < 0 ? 0 : lo;
    hi = hi > 63 ? 63 : hi;
    if (lo > hi) return 0ull;
    return (~0ull >> (63 - (hi - lo))) << lo;
}

__device__ __forceinline__ uint32_t count_bits(bool pred) {
    return (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(pred));
}

__device__ __forceinline__ uint32_t count_bits_masked(bool pred, uint64_t mask) {
    return (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(pred) & mask);
}

// Wave-local ordering point between the LDS writes of one lane and the
// broadcast reads of another lane of the same wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP controls (GFX9 encoding).
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int Ctrl, int RowMask, int BankMask>
__device__ __forceinline__ float dpp_plus(float v) {
    int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, RowMask, BankMask, true);
    return v + __int_as_float(s);
}

// Partial sums of v over the 64 lanes after which lane 63 holds the total:
// inclusive scans inside each row of 16 lanes, then the row totals are
// carried across rows with row broadcasts.
__device__ __forceinline__ float wave_total_in_lane63(float v) {
    v = dpp_plus<kDppRowShr1, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowShr2, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowShr4, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowShr8, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowBcast15, 0xa, 0xf>(v);
    v = dpp_plus<kDppRowBcast31, 0xc, 0xf>(v);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace pairs_dev
