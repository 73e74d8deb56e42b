// Wave-task bodies shared by the single-set and the batched kernels.
//
// One wave (64 lanes) runs one task: a block of 64*K consecutive rows of the
// balanced assignment of one set (band.h) held in registers, K rows per lane
// in lane-major order (row ra + 64k + lane), swept against a chunk [u0, u1)
// of virtual partners that are staged 64 at a time into a wave-private LDS
// window and read back as wave-uniform broadcasts.  Row i evaluates the
// virtual partner u iff i < u <= i + steps(i) (band.h).  Inside a row block's
// core that holds for every lane; at the two band edges each lane tests it.
// Padding rows and padding partners carry values (infinities) for which the
// predicate is false or the potential exactly zero.
//
// Objects of the set are x[base + k], k in [0, n).
#pragma once

#include <math.h>
#include <stdint.h>

#include "band.h"
#include "device.h"

namespace pairs_dev {

// ------------------------------------------------------------ int32 count --
//
// Exact predicate in double precision (Gram form).  With h = (|p|^2 - r^2)/2,
//   |p_i - p_j|^2 <= (r_i + r_j)^2  <=>  p_i.p_j + r_i r_j - h_i >= h_j.
// Inside the exact domain (|coordinate| <= 2^24, 0 <= r <= 2^24) every
// product is an integer of magnitude at most 2^48 and every partial sum a
// multiple of 1/2 below 2^51 in magnitude, so every fused multiply-add is
// exact and the comparison decides the integer predicate.

__device__ __forceinline__ void gram_features(int32_t xi, int32_t yi, int32_t zi, int32_t ri,
                                              double &X, double &Y, double &Z, double &R,
                                              double &H) {
    X = (double)xi;
    Y = (double)yi;
    Z = (double)zi;
    R = (double)ri;
    double a = X * X;
    a = __builtin_fma(Y, Y, a);
    a = __builtin_fma(Z, Z, a);
    a = __builtin_fma(-R, R, a);
    H = 0.5 * a;
}

// LDS window of one wave: 5 arrays of 64 doubles.
constexpr int kCountI32Lds = 5 * kWave;

// Row i evaluates the virtual partner u iff i < u <= i + steps(i).
__device__ __forceinline__ bool owns(int u, int i, int steps) {
    return (unsigned)(u - 1 - i) < (unsigned)steps;
}

__device__ __forceinline__ int64_t partner_index(int64_t base, const Band &band, int u) {
    return base + (u >= band.n ? u - band.n : u);
}

template <int K>
__device__ uint32_t count_i32_task(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                                   const int32_t *__restrict__ pz, const int32_t *__restrict__ pr,
                                   int64_t base, const Band band, int ra, int u0, int u1,
                                   double *__restrict__ win) {
    const int lane = lane_id();
    double xr[K], yr[K], zr[K], rr[K], nh[K];
    int row[K], nsteps[K];  // row index and its step count (0 for padding rows)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            int64_t g = base + i;
            double h;
            gram_features(px[g], py[g], pz[g], pr[g], xr[k], yr[k], zr[k], rr[k], h);
            nh[k] = -h;
            nsteps[k] = band.steps(i);
        } else {
            xr[k] = yr[k] = zr[k] = rr[k] = 0.0;
            nh[k] = -INFINITY;  // never hits
            nsteps[k] = 0;
        }
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1;            // every row has u - 1 >= row
    const int core_hi = ra + band.steps(ra);  // every row has u <= row + steps(row)

    uint32_t cnt = 0;
    int32_t qx = 0, qy = 0, qz = 0, qr = 0;  // next group's raw partner values
    {
        int u = u0 + lane;
        if (u < u1) {
            int64_t g = partner_index(base, band, u);
            qx = px[g]; qy = py[g]; qz = pz[g]; qr = pr[g];
        }
    }
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        {
            double X, Y, Z, R, H;
            gram_features(qx, qy, qz, qr, X, Y, Z, R, H);
            if (g0 + lane >= u1) H = INFINITY;  // padding partner: never hits
            win[0 * kWave + lane] = X;
            win[1 * kWave + lane] = Y;
            win[2 * kWave + lane] = Z;
            win[3 * kWave + lane] = R;
            win[4 * kWave + lane] = H;
        }
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g]; qr = pr[g];
            }
        }
        wave_sync();
        const int gn = min(kWave, u1 - g0);
        if (g0 >= core_lo && g0 + gn - 1 <= core_hi) {
#pragma unroll 2
            for (int t = 0; t < kWave; ++t) {
                const double jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                             jr = win[3 * kWave + t], jh = win[4 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    double v = __builtin_fma(xr[k], jx, nh[k]);
                    v = __builtin_fma(yr[k], jy, v);
                    v = __builtin_fma(zr[k], jz, v);
                    v = __builtin_fma(rr[k], jr, v);
                    cnt += count_bits(v >= jh);
                }
            }
        } else {
            for (int t = 0; t < gn; ++t) {
                const int u = g0 + t;
                const double jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                             jr = win[3 * kWave + t], jh = win[4 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    double v = __builtin_fma(xr[k], jx, nh[k]);
                    v = __builtin_fma(yr[k], jy, v);
                    v = __builtin_fma(zr[k], jz, v);
                    v = __builtin_fma(rr[k], jr, v);
                    cnt += count_bits(v >= jh && owns(u, row[k], nsteps[k]));
                }
            }
        }
        wave_sync();
    }
    return cnt;
}

// --------------------------------------------------------- float32 count --
//
// The pinned binary32 sequence; explicit round-to-nearest intrinsics keep the
// compiler from contracting or reordering it.

__device__ __forceinline__ float sq_dist_f32(float dx, float dy, float dz) {
    float d2 = __fmul_rn(dx, dx);
    d2 = __fmaf_rn(dy, dy, d2);
    return __fmaf_rn(dz, dz, d2);
}

__device__ __forceinline__ bool hit_f32(float xi, float yi, float zi, float ri, float xj,
                                        float yj, float zj, float rj) {
    float d2 = sq_dist_f32(__fsub_rn(xi, xj), __fsub_rn(yi, yj), __fsub_rn(zi, zj));
    float R = __fadd_rn(ri, rj);
    return d2 <= __fmul_rn(R, R);
}

constexpr int kCountF32Lds = 4 * kWave;

template <int K>
__device__ uint32_t count_f32_task(const float *__restrict__ px, const float *__restrict__ py,
                                   const float *__restrict__ pz, const float *__restrict__ pr,
                                   int64_t base, const Band band, int ra, int u0, int u1,
                                   float *__restrict__ win) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], rr[K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            int64_t g = base + i;
            xr[k] = px[g]; yr[k] = py[g]; zr[k] = pz[g]; rr[k] = pr[g];
            nsteps[k] = band.steps(i);
        } else {
            xr[k] = INFINITY;  // distance infinite: never hits
            yr[k] = zr[k] = rr[k] = 0.0f;
            nsteps[k] = 0;
        }
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
    uint32_t cnt = 0;
    float qx = 0, qy = 0, qz = 0, qr = 0;
    {
        int u = u0 + lane;
        if (u < u1) {
            int64_t g = partner_index(base, band, u);
            qx = px[g]; qy = py[g]; qz = pz[g]; qr = pr[g];
        }
    }
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        const bool pad = g0 + lane >= u1;
        win[0 * kWave + lane] = pad ? -INFINITY : qx;
        win[1 * kWave + lane] = pad ? 0.0f : qy;
        win[2 * kWave + lane] = pad ? 0.0f : qz;
        win[3 * kWave + lane] = pad ? 0.0f : qr;
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g]; qr = pr[g];
            }
        }
        wave_sync();
        const int gn = min(kWave, u1 - g0);
        if (g0 >= core_lo && g0 + gn - 1 <= core_hi) {
#pragma unroll 2
            for (int t = 0; t < kWave; ++t) {
                const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                            jr = win[3 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cnt += count_bits(hit_f32(xr[k], yr[k], zr[k], rr[k], jx, jy, jz, jr));
            }
        } else {
            for (int t = 0; t < gn; ++t) {
                const int u = g0 + t;
                const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                            jr = win[3 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cnt += count_bits(hit_f32(xr[k], yr[k], zr[k], rr[k], jx, jy, jz, jr) &&
                                      owns(u, row[k], nsteps[k]));
            }
        }
        wave_sync();
    }
    return cnt;
}

// ---------------------------------------------------------------- energy --
//
// e = 1/sqrt(d2 + eps2) in float32 with the hardware reciprocal square root.
// Row sums are float32 partials of at most kFoldEvery terms folded into
// double accumulators.  With PerObject the partner side of each pair is
// summed across the wave (DPP) and added once per partner and task.  With
// WithCount the pinned binary32 collision predicate is evaluated on the same
// differences and counted, and e uses d2 + eps2 with that squared distance.

// LDS window of one wave: x, y, z, r of 64 partners and their partner-side sums.
constexpr int kEnergyLds = 5 * kWave;
constexpr int kFoldEvery = 16;

struct EnergyResult {
    double energy;   // sum of e over the task's pairs (row side, each pair once)
    uint32_t count;  // collisions among the task's pairs (WithCount)
};

template <int K, bool PerObject, bool WithCount, bool Masked>
__device__ __forceinline__ void energy_group(const float (&xr)[K], const float (&yr)[K],
                                             const float (&zr)[K], const float (&rr)[K],
                                             const int (&row)[K], const int (&nsteps)[K],
                                             float (&part)[K], double (&acc)[K], uint32_t &cnt,
                                             float *__restrict__ win, int g0, int gn,
                                             float eps2) {
    const int lane = lane_id();
    for (int t0 = 0; t0 < gn; t0 += kFoldEvery) {
#pragma unroll 2
        for (int t = t0; t < t0 + kFoldEvery; ++t) {
            const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t];
            float jr = 0.0f;
            if (WithCount) jr = win[3 * kWave + t];
            const int u = g0 + t;
            float js = 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float dx = xr[k] - jx, dy = yr[k] - jy, dz = zr[k] - jz;
                float e;
                bool valid = true;
                if (Masked) valid = owns(u, row[k], nsteps[k]);
                if (WithCount) {
                    const float d2 = sq_dist_f32(dx, dy, dz);
                    const float R = __fadd_rn(rr[k], jr);
                    const bool hit = d2 <= __fmul_rn(R, R);
                    if (Masked)
                        cnt += count_bits(hit && valid);
                    else
                        cnt += count_bits(hit);
                    e = __builtin_amdgcn_rsqf(d2 + eps2);
                } else {
                    float d2 = __builtin_fmaf(dx, dx, eps2);
                    d2 = __builtin_fmaf(dy, dy, d2);
                    d2 = __builtin_fmaf(dz, dz, d2);
                    e = __builtin_amdgcn_rsqf(d2);
                }
                if (Masked) e = valid ? e : 0.0f;
                part[k] += e;
                if (PerObject) js += e;
            }
            if (PerObject) {
                const float s = wave_total_in_lane63(js);
                if (lane == kWave - 1) win[4 * kWave + t] = s;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            acc[k] += (double)part[k];
            part[k] = 0.0f;
        }
    }
}

template <int K, bool PerObject, bool WithCount>
__device__ EnergyResult energy_task(const float *__restrict__ px, const float *__restrict__ py,
                                    const float *__restrict__ pz, const float *__restrict__ pr,
                                    int64_t base, const Band band, int ra, int u0, int u1,
                                    float eps2, float *__restrict__ win, double *__restrict__ E) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], rr[K], part[K];
    double acc[K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            int64_t g = base + i;
            xr[k] = px[g]; yr[k] = py[g]; zr[k] = pz[g];
            rr[k] = WithCount ? pr[g] : 0.0f;
            nsteps[k] = band.steps(i);
        } else {
            xr[k] = INFINITY;  // infinite distance: e is exactly 0, never hits
            yr[k] = zr[k] = rr[k] = 0.0f;
            nsteps[k] = 0;
        }
        part[k] = 0.0f;
        acc[k] = 0.0;
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
    uint32_t cnt = 0;
    float qx = 0, qy = 0, qz = 0, qr = 0;
    {
        int u = u0 + lane;
        if (u < u1) {
            int64_t g = partner_index(base, band, u);
            qx = px[g]; qy = py[g]; qz = pz[g];
            if (WithCount) qr = pr[g];
        }
    }
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        const bool pad = g0 + lane >= u1;
        win[0 * kWave + lane] = pad ? -INFINITY : qx;
        win[1 * kWave + lane] = pad ? 0.0f : qy;
        win[2 * kWave + lane] = pad ? 0.0f : qz;
        if (WithCount) win[3 * kWave + lane] = pad ? 0.0f : qr;
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g];
                if (WithCount) qr = pr[g];
            }
        }
        wave_sync();
        const int gn = min(kWave, u1 - g0);
        if (g0 >= core_lo && g0 + gn - 1 <= core_hi)
            energy_group<K, PerObject, WithCount, false>(xr, yr, zr, rr, row, nsteps, part, acc,
                                                         cnt, win, g0, gn, eps2);
        else
            energy_group<K, PerObject, WithCount, true>(xr, yr, zr, rr, row, nsteps, part, acc,
                                                        cnt, win, g0, gn, eps2);
        if (PerObject) {
            wave_sync();
            if (lane < gn)
                atomicAdd(&E[partner_index(base, band, g0 + lane)], (double)win[4 * kWave + lane]);
        }
        wave_sync();
    }
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            if (PerObject) atomicAdd(&E[base + i], acc[k]);
            tot += acc[k];
        }
    }
    EnergyResult res;
    res.energy = wave_sum(tot);
    res.count = cnt;
    return res;
}

}  // namespace pairs_dev
