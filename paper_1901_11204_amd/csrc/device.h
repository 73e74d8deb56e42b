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

// Lanes where both a and b hold; the two ballots are combined with a scalar and.
__device__ __forceinline__ uint32_t count_bits_both(bool a, bool b) {
    return (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(a) &
                                          __builtin_amdgcn_ballot_w64(b));
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

// Exclusive scan of v over a block of BLOCK threads (a multiple of 64);
// *sum gets the block's total.  wave_tot: BLOCK / 64 + 1 words of LDS.
// Every thread of the block calls it.
template <int BLOCK>
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *wave_tot,
                                                        int64_t *sum) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wave_tot[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < BLOCK / kWave; ++w) {
            const int64_t t = wave_tot[w];
            wave_tot[w] = run;
            run += t;
        }
        wave_tot[BLOCK / kWave] = run;
    }
    __syncthreads();
    const int64_t r = wave_tot[wave] + x - v;
    *sum = wave_tot[BLOCK / kWave];
    __syncthreads();  // wave_tot is reused by the next scan
    return r;
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

// DPP controls for the reduce-scatter below.
constexpr int kDppRowRor8 = 0x128, kDppRowHalfMirror = 0x141;
constexpr int kDppQuadSwap1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;  // quad_perm [2,3,0,1]

template <int Ctrl>
__device__ __forceinline__ float dpp_full(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xf, 0xf, true));
}

// Sums of 16 per-lane values over the 64 lanes, scattered: on return, the
// four lanes 4g..4g+3 all hold the total of v[partner_of_group(g)].
// Levels: v_permlane32_swap folds lane halves (16 values -> 8 registers),
// v_permlane16_swap folds rows (-> 4), a row rotate by 8 and a half-row
// mirror fold within rows (-> 2, -> 1, selecting by lane bit), and two quad
// permutes finish each group of four lanes.
__device__ __forceinline__ float reduce_scatter16(const float (&v)[16]) {
    const int lane = lane_id();
    float r1[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * p]),
                                                   __float_as_uint(v[2 * p + 1]), false, false);
        r1[p] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    }
    float r2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(r1[2 * q]),
                                                   __float_as_uint(r1[2 * q + 1]), false, false);
        r2[q] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    }
    const bool hi8 = (lane & 8) != 0, hi4 = (lane & 4) != 0;
    float r3[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float e = r2[2 * h] + dpp_full<kDppRowRor8>(r2[2 * h]);
        const float f = r2[2 * h + 1] + dpp_full<kDppRowRor8>(r2[2 * h + 1]);
        r3[h] = hi8 ? f : e;
    }
    const float g0 = r3[0] + dpp_full<kDppRowHalfMirror>(r3[0]);
    const float g1 = r3[1] + dpp_full<kDppRowHalfMirror>(r3[1]);
    float r = hi4 ? g1 : g0;
    r += dpp_full<kDppQuadSwap1>(r);
    r += dpp_full<kDppQuadSwap2>(r);
    return r;
}

// Which of the 16 values reduce_scatter16 leaves in the calling lane's group,
// found by reducing the values k held by lane 0 only (exact in float32).
__device__ __forceinline__ int reduce_scatter16_slot() {
    float probe[16];
    const bool first = lane_id() == 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) probe[k] = first ? (float)k : 0.0f;
    return (int)reduce_scatter16(probe);
}

// reduce_scatter16 on doubles: every data movement of the float version is
// applied to the low and the high 32-bit words alike, so it moves whole
// doubles; the additions are in double.
__device__ __forceinline__ double dbl_of(uint32_t lo, uint32_t hi) {
    return __hiloint2double((int)hi, (int)lo);
}

template <int Ctrl>
__device__ __forceinline__ double dpp_full_f64(double v) {
    const uint32_t lo = (uint32_t)__double2loint(v), hi = (uint32_t)__double2hiint(v);
    return dbl_of((uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, Ctrl, 0xf, 0xf, true),
                  (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, Ctrl, 0xf, 0xf, true));
}

__device__ __forceinline__ double reduce_scatter16_f64(const double (&v)[16]) {
    const int lane = lane_id();
    double r1[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)__double2loint(v[2 * p]),
                                                   (uint32_t)__double2loint(v[2 * p + 1]), false,
                                                   false);
        auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)__double2hiint(v[2 * p]),
                                                   (uint32_t)__double2hiint(v[2 * p + 1]), false,
                                                   false);
        r1[p] = dbl_of(lo[0], hi[0]) + dbl_of(lo[1], hi[1]);
    }
    double r2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)__double2loint(r1[2 * q]),
                                                   (uint32_t)__double2loint(r1[2 * q + 1]), false,
                                                   false);
        auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)__double2hiint(r1[2 * q]),
                                                   (uint32_t)__double2hiint(r1[2 * q + 1]), false,
                                                   false);
        r2[q] = dbl_of(lo[0], hi[0]) + dbl_of(lo[1], hi[1]);
    }
    const bool hi8 = (lane & 8) != 0, hi4 = (lane & 4) != 0;
    double r3[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double e = r2[2 * h] + dpp_full_f64<kDppRowRor8>(r2[2 * h]);
        const double f = r2[2 * h + 1] + dpp_full_f64<kDppRowRor8>(r2[2 * h + 1]);
        r3[h] = hi8 ? f : e;
    }
    const double g0 = r3[0] + dpp_full_f64<kDppRowHalfMirror>(r3[0]);
    const double g1 = r3[1] + dpp_full_f64<kDppRowHalfMirror>(r3[1]);
    double r = hi4 ? g1 : g0;
    r += dpp_full_f64<kDppQuadSwap1>(r);
    r += dpp_full_f64<kDppQuadSwap2>(r);
    return r;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace pairs_dev
