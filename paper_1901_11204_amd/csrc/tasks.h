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
// Exact predicate in 64-bit integers (Gram form).  With q = |p|^2 - r^2,
//   |p_i - p_j|^2 <= (r_i + r_j)^2  <=>  q_i + q_j <= 2 (p_i.p_j + r_i r_j),
// which is evaluated as v = -q_i + sum over the four coordinates of
// (2 c_i) c_j with 32x32->64-bit multiply-adds, and the test v >= q_j.
// For coordinates in [-2^29, 2^29) and radii in [0, 2^30) every 2 c_i fits
// in 32 bits, every product is below 2^61 in magnitude and every partial sum
// below 2^62, so nothing overflows and the test is exact.
//
// The library's domain is wider: coordinates in [-2^30, 2^30), radii in
// [0, 2^30].  There the same sum, taken modulo 2^64, still identifies the
// exact value T = v - q_j = (r_i + r_j)^2 - |p_i - p_j|^2, because T lies in
// (-3 * 2^62, 2^62], an interval of length 2^64: T >= 0 exactly when
// (v - q_j) mod 2^64 <= 2^62.  That "wide" test costs two more operations per
// pair, so a wave takes it only for a task whose rows, or a partner group
// whose objects, leave the box of the plain test (a wave-uniform ballot).

struct RowI32 {
    int32_t ax, ay, az, ar;  // 2x, 2y, 2z, 2r (2r as the low 32 bits: 2^31 at r = 2^30)
    int64_t nq;              // -q
};

struct PartnerI32 {
    int32_t x, y, z, r;
};

__device__ __forceinline__ int64_t gram_q(int32_t x, int32_t y, int32_t z, int32_t r) {
    uint64_t q = (uint64_t)((int64_t)x * x);
    q += (uint64_t)((int64_t)y * y);
    q += (uint64_t)((int64_t)z * z);
    q -= (uint64_t)((int64_t)r * r);
    return (int64_t)q;  // in [-2^60, 3 * 2^60] inside the domain
}

__device__ __forceinline__ int32_t twice(int32_t v) { return (int32_t)((uint32_t)v << 1); }

__device__ __forceinline__ RowI32 gram_row(int32_t x, int32_t y, int32_t z, int32_t r) {
    RowI32 a;
    a.ax = twice(x);
    a.ay = twice(y);
    a.az = twice(z);
    a.ar = twice(r);
    a.nq = (int64_t)(0 - (uint64_t)gram_q(x, y, z, r));
    return a;
}

__device__ __forceinline__ bool gram_hit(const RowI32 &a, const PartnerI32 &b, int64_t qb) {
    int64_t v = a.nq + (int64_t)a.ax * b.x;
    v += (int64_t)a.ay * b.y;
    v += (int64_t)a.az * b.z;
    v += (int64_t)a.ar * b.r;
    return v >= qb;
}

// The wide test, exact on the whole domain (modulo-2^64 sum; the radius
// product unsigned, as 2r may be 2^31).
__device__ __forceinline__ bool gram_hit_wide(const RowI32 &a, const PartnerI32 &b, int64_t qb) {
    uint64_t v = (uint64_t)a.nq;
    v += (uint64_t)((int64_t)a.ax * b.x);
    v += (uint64_t)((int64_t)a.ay * b.y);
    v += (uint64_t)((int64_t)a.az * b.z);
    v += (uint64_t)(uint32_t)a.ar * (uint32_t)b.r;
    return v - (uint64_t)qb <= ((uint64_t)1 << 62);
}

// Whether an object lies in the box [-B, B)^3 x [0, 2B) of a plain test,
// B = 2^bits: one unsigned comparison of the or of the shifted values.
template <int bits>
__device__ __forceinline__ bool in_box(int32_t x, int32_t y, int32_t z, int32_t r) {
    constexpr uint32_t B = 1u << bits;
    return (((uint32_t)x + B) | ((uint32_t)y + B) | ((uint32_t)z + B) | (uint32_t)r) < 2 * B;
}
constexpr int kBoxBitsI64 = 29;  // plain 64-bit integer Gram test
constexpr int kBoxBitsF64 = 24;  // double-precision Gram test

// True on every lane when no lane's flag is false.
__device__ __forceinline__ bool wave_all(bool v) { return __builtin_amdgcn_ballot_w64(!v) == 0; }

// LDS window of one wave, in 8-byte words: large enough for both forms (the
// integer form uses 64 partner records of 16 bytes and 64 q values, the
// double form five arrays of 64 doubles).
constexpr int kCountI32Lds = 5 * kWave;

// Row i evaluates the virtual partner u iff i < u <= i + steps(i).
__device__ __forceinline__ bool owns(int u, int i, int steps) {
    return (unsigned)(u - 1 - i) < (unsigned)steps;
}

__device__ __forceinline__ int64_t partner_index(int64_t base, const Band &band, int u) {
    return base + (u >= band.n ? u - band.n : u);
}

__device__ __forceinline__ int64_t partner_index(int64_t base, const TriBand &, int u) {
    return base + u;
}

// The raw inputs a task starts from: the K row objects of the lane and the
// lane's partner of the first group.  Loading them is separated from running
// the task so that a persistent wave can fetch the next task's inputs while
// the current task computes.  KM >= K is the array size (the largest shape a
// kernel serves); only the first K slices are used.
template <typename T, int KM>
struct TaskInputs {
    T x[KM], y[KM], z[KM], r[KM];
    T px, py, pz, pr;
};

template <typename T, int K, int KM, bool WithR, typename BandT = Band>
__device__ __forceinline__ void load_task_inputs(const T *__restrict__ X, const T *__restrict__ Y,
                                                 const T *__restrict__ Z, const T *__restrict__ R,
                                                 int64_t base, const BandT &band, int ra, int u0,
                                                 int u1, TaskInputs<T, KM> &in) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ra + kWave * k + lane;
        in.x[k] = in.y[k] = in.z[k] = in.r[k] = T(0);
        if (i < band.n) {
            const int64_t g = base + i;
            in.x[k] = X[g];
            in.y[k] = Y[g];
            in.z[k] = Z[g];
            if (WithR) in.r[k] = R[g];
        }
    }
    in.px = in.py = in.pz = in.pr = T(0);
    const int u = u0 + lane;
    if (u < u1) {
        const int64_t g = partner_index(base, band, u);
        in.px = X[g];
        in.py = Y[g];
        in.pz = Z[g];
        if (WithR) in.pr = R[g];
    }
}

template <int K, int KM, typename BandT = Band>
__device__ __forceinline__ uint32_t count_i32_task_i64(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                                   const int32_t *__restrict__ pz, const int32_t *__restrict__ pr,
                                   int64_t base, const BandT band, int ra, int u0, int u1,
                                   void *__restrict__ lds, const TaskInputs<int32_t, KM> &in) {
    PartnerI32 *wp = (PartnerI32 *)lds;
    int64_t *wq = (int64_t *)lds + 2 * kWave;
    const int lane = lane_id();
    RowI32 rows[K];
    int row[K], nsteps[K];  // row index and its step count (0 for padding rows)
    bool rows_in = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            const int32_t x = in.x[k], y = in.y[k], z = in.z[k], r = in.r[k];
            rows[k] = gram_row(x, y, z, r);
            rows_in = rows_in && in_box<kBoxBitsI64>(x, y, z, r);
            nsteps[k] = band.steps(i);
        } else {
            rows[k].ax = rows[k].ay = rows[k].az = rows[k].ar = 0;
            rows[k].nq = -((int64_t)1 << 62);  // never hits
            nsteps[k] = 0;
        }
    }
    const bool rows_plain = wave_all(rows_in);
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1;            // every row has u - 1 >= row
    const int core_hi = ra + band.steps(ra);  // every row has u <= row + steps(row)

    uint32_t cnt = 0;
    int32_t qx = in.px, qy = in.py, qz = in.pz, qr = in.pr;  // this group's partner values
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        bool plain;
        {
            PartnerI32 p;
            p.x = qx; p.y = qy; p.z = qz; p.r = qr;
            wp[lane] = p;
            const bool pad = g0 + lane >= u1;
            // padding partner: q above any reachable v, never hits
            wq[lane] = pad ? INT64_MAX : gram_q(qx, qy, qz, qr);
            plain = rows_plain && wave_all(pad || in_box<kBoxBitsI64>(qx, qy, qz, qr));
        }
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g]; qr = pr[g];
            }
        }
        wave_sync();
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (plain && g0 >= core_lo && g0 + gn - 1 <= core_hi) {
#pragma unroll 2
            for (int t = 0; t < kWave; ++t) {
                const PartnerI32 b = wp[t];
                const int64_t qb = wq[t];
#pragma unroll
                for (int k = 0; k < K; ++k) cnt += count_bits(gram_hit(rows[k], b, qb));
            }
        } else if (plain) {
            for (int t = 0; t < gn; ++t) {
                const int u = g0 + t;
                const PartnerI32 b = wp[t];
                const int64_t qb = wq[t];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cnt += count_bits_both(gram_hit(rows[k], b, qb), owns(u, row[k], nsteps[k]));
            }
        } else {
            for (int t = 0; t < gn; ++t) {
                const int u = g0 + t;
                const PartnerI32 b = wp[t];
                const int64_t qb = wq[t];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cnt += count_bits_both(gram_hit_wide(rows[k], b, qb),
                                           owns(u, row[k], nsteps[k]));
            }
        }
        wave_sync();
    }
    return cnt;
}

// The same predicate in double precision, for tall row blocks.  With
// h = q/2 = (|p|^2 - r^2)/2 it reads p_i.p_j + r_i r_j - h_i >= h_j; for
// coordinates in [-2^24, 2^24) and radii in [0, 2^25) every product is an
// integer below 2^50 in magnitude and every partial sum a multiple of 1/2
// below 2^52, so each fused multiply-add and the comparison are exact.
// Outside that box a group takes the wide test from the same double records
// (wide_hit_f64).  Its partner records are 40
// bytes instead of 24, but gfx950 issues its FP64 fused multiply-adds and
// compares slightly faster than the 64-bit integer ones, so it wins where
// one partner feeds many rows (K >= 4) and LDS traffic is no limit.

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

// The difference-and-square test, exact on the library's whole domain, from
// doubles that hold int32 values exactly: each difference is exact in double
// and below 2^31 in magnitude, so it converts to int32; the squares and their
// sum (below 3 * 2^62) are exact in unsigned 64-bit integers, as is
// (r_i + r_j)^2 <= 2^62.
__device__ __forceinline__ bool wide_hit_f64(double xi, double yi, double zi, double ri,
                                             double xj, double yj, double zj, double rj) {
    const int32_t dx = __double2int_rz(xi - xj), dy = __double2int_rz(yi - yj),
                  dz = __double2int_rz(zi - zj);
    const uint32_t R = __double2uint_rz(ri + rj);
    uint64_t d2 = (uint64_t)((int64_t)dx * dx);
    d2 += (uint64_t)((int64_t)dy * dy);
    d2 += (uint64_t)((int64_t)dz * dz);
    return d2 <= (uint64_t)R * R;
}

template <int K, int KM, typename BandT = Band>
__device__ __forceinline__ uint32_t count_i32_task_f64(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                                   const int32_t *__restrict__ pz, const int32_t *__restrict__ pr,
                                   int64_t base, const BandT band, int ra, int u0, int u1,
                                   void *__restrict__ lds, const TaskInputs<int32_t, KM> &in) {
    double *win = (double *)lds;
    const int lane = lane_id();
    double xr[K], yr[K], zr[K], rr[K], nh[K];
    int row[K], nsteps[K];  // row index and its step count (0 for padding rows)
    bool rows_in = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            double h;
            gram_features(in.x[k], in.y[k], in.z[k], in.r[k], xr[k], yr[k], zr[k], rr[k], h);
            rows_in = rows_in && in_box<kBoxBitsF64>(in.x[k], in.y[k], in.z[k], in.r[k]);
            nh[k] = -h;
            nsteps[k] = band.steps(i);
        } else {
            xr[k] = yr[k] = zr[k] = rr[k] = 0.0;
            nh[k] = -INFINITY;  // never hits
            nsteps[k] = 0;
        }
    }
    const bool rows_plain = wave_all(rows_in);
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1;            // every row has u - 1 >= row
    const int core_hi = ra + band.steps(ra);  // every row has u <= row + steps(row)

    uint32_t cnt = 0;
    int32_t qx = in.px, qy = in.py, qz = in.pz, qr = in.pr;  // this group's raw partner values
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        bool plain;
        {
            double X, Y, Z, R, H;
            gram_features(qx, qy, qz, qr, X, Y, Z, R, H);
            const bool pad = g0 + lane >= u1;
            plain = rows_plain && wave_all(pad || in_box<kBoxBitsF64>(qx, qy, qz, qr));
            if (pad) H = INFINITY;  // padding partner: never hits
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
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (plain && g0 >= core_lo && g0 + gn - 1 <= core_hi) {
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
        } else if (!plain) {
            for (int t = 0; t < gn; ++t) {
                const int u = g0 + t;
                const double jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                             jr = win[3 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cnt += count_bits_both(wide_hit_f64(xr[k], yr[k], zr[k], rr[k], jx, jy, jz, jr),
                                           owns(u, row[k], nsteps[k]));
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
                    cnt += count_bits_both(v >= jh, owns(u, row[k], nsteps[k]));
                }
            }
        }
        wave_sync();
    }
    return cnt;
}


// The exact int32 count task: 64-bit integer form for short row blocks
// (K <= 2, where the broadcast of each partner limits), double form for tall
// ones.  Both decide the same integer predicate inside the exact domain.
// The balanced assignment (Band) on the library's path; the comparison
// kernels of the benchmark also run the straightforward one (TriBand).
template <int K, int KM, typename BandT = Band>
__device__ __forceinline__ uint32_t count_i32_task(const int32_t *__restrict__ px,
                                                   const int32_t *__restrict__ py,
                                                   const int32_t *__restrict__ pz,
                                                   const int32_t *__restrict__ pr, int64_t base,
                                                   const BandT band, int ra, int u0, int u1,
                                                   void *__restrict__ lds,
                                                   const TaskInputs<int32_t, KM> &in) {
    if (K >= 4)
        return count_i32_task_f64<K, KM, BandT>(px, py, pz, pr, base, band, ra, u0, u1, lds, in);
    return count_i32_task_i64<K, KM, BandT>(px, py, pz, pr, base, band, ra, u0, u1, lds, in);
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

template <int K, int KM>
__device__ __forceinline__ uint32_t count_f32_task(const float *__restrict__ px, const float *__restrict__ py,
                                   const float *__restrict__ pz, const float *__restrict__ pr,
                                   int64_t base, const Band band, int ra, int u0, int u1,
                                   float *__restrict__ win, const TaskInputs<float, KM> &in) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], rr[K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            xr[k] = in.x[k]; yr[k] = in.y[k]; zr[k] = in.z[k]; rr[k] = in.r[k];
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
    float qx = in.px, qy = in.py, qz = in.pz, qr = in.pr;
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
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
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
                    cnt += count_bits_both(hit_f32(xr[k], yr[k], zr[k], rr[k], jx, jy, jz, jr),
                                           owns(u, row[k], nsteps[k]));
            }
        }
        wave_sync();
    }
    return cnt;
}

// ------------------------------------------------------ sums of doubles --
//
// The kernels add partial sums of each output (a per-object or per-set sum,
// a total) with atomics.  By default these are double atomics, whose order
// varies from run to run and with it the last bits of a result.  With a
// positive scale 2^S (PAIRS_FLAG_DETERMINISTIC) each partial is rounded once
// to a multiple of 2^-S and added as a 64-bit integer into the same 8 bytes;
// integer additions are exact and commute, so the result is the same in
// every run, and a finishing pass turns the integer back into a double.
// fixed_scale() chooses 2^S from a bound on every partial sum's magnitude:
// the largest power of two with bound * 2^S < 2^61, which leaves room for
// the rounding of each added value.  The absolute error is at most half a
// unit per added value.

PAIRS_HD double fixed_scale(double bound) {
    int e;
    frexp(bound, &e);  // bound < 2^e
    return ldexp(1.0, 61 - e);
}

struct SumSink {
    double *p;
    double scale;  // 0: double atomics; else fixed point in units of 1/scale

    __device__ __forceinline__ void add(int64_t i, double v) const {
        if (scale > 0.0)
            atomicAdd((unsigned long long *)(p + i),
                      (unsigned long long)__double2ll_rn(v * scale));
        else
            atomicAdd(p + i, v);
    }
};

// ---------------------------------------------------------------- energy --
//
// e = 1/sqrt(d2 + eps2) in float32 with the hardware reciprocal square root.
// Row sums are float32 partials of at most kFoldEvery terms folded into
// double accumulators.  With PerObject the partner side of each pair is
// summed across the wave, 16 partners at a time (reduce_scatter16), and added
// once per partner and task.  With
// WithCount the pinned binary32 collision predicate is evaluated on the same
// differences and counted, and e uses d2 + eps2 with that squared distance.

// LDS window of one wave: x, y, z, r of 64 partners and their partner-side sums.
constexpr int kEnergyLds = 5 * kWave;
constexpr int kFoldEvery = 16;

struct EnergyResult {
    double energy;   // sum of e over the task's pairs (row side, each pair once)
    uint32_t count;  // collisions among the task's pairs (WithCount)
};

// Sum of v[0..K) as a pairwise tree.  The partner side of a pair sums one
// term per row of the lane; a tree keeps each add waiting on two results
// that are already some instructions old, where a running sum would chain
// every add to the reciprocal square root just issued.
template <typename T, int K>
__device__ __forceinline__ T tree_sum(T (&v)[K]) {
#pragma unroll
    for (int w = 1; w < K; w *= 2)
#pragma unroll
        for (int k = 0; k + w < K; k += 2 * w) v[k] = v[k] + v[k + w];
    return v[0];
}

template <int K, bool PerObject, bool WithCount, bool Masked>
__device__ __forceinline__ void energy_group(const float (&xr)[K], const float (&yr)[K],
                                             const float (&zr)[K], const float (&rr)[K],
                                             const int (&row)[K], const int (&nsteps)[K],
                                             float (&part)[K], double (&acc)[K], uint32_t &cnt,
                                             float *__restrict__ win, int g0, int gn,
                                             float eps2, int slot) {
    const int lane = lane_id();
    for (int t0 = 0; t0 < gn; t0 += kFoldEvery) {
        float js_all[kFoldEvery];
#pragma unroll
        for (int tt = 0; tt < kFoldEvery; ++tt) {
            const int t = t0 + tt;
            const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t];
            float jr = 0.0f;
            if (WithCount) jr = win[3 * kWave + t];
            const int u = g0 + t;
            float es[K];
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
                        cnt += count_bits_both(hit, valid);
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
                // the first term of a fold and of a partner sum is stored,
                // not added to zero (an add of 0 is no IEEE identity, so the
                // compiler keeps it)
                part[k] = tt == 0 ? e : part[k] + e;
                es[k] = e;
            }
            if (PerObject) js_all[tt] = tree_sum(es);
        }
        if (PerObject) {
            // all 4 lanes of a group store the same value to the same slot
            const float s = reduce_scatter16(js_all);
            win[4 * kWave + t0 + slot] = s;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += (double)part[k];
    }
}

template <int K, int KM, bool PerObject, bool WithCount>
__device__ __forceinline__ EnergyResult energy_task(const float *__restrict__ px, const float *__restrict__ py,
                                    const float *__restrict__ pz, const float *__restrict__ pr,
                                    int64_t base, const Band band, int ra, int u0, int u1,
                                    float eps2, float *__restrict__ win, const SumSink E,
                                    const TaskInputs<float, KM> &in) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], rr[K], part[K];
    double acc[K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            xr[k] = in.x[k]; yr[k] = in.y[k]; zr[k] = in.z[k];
            rr[k] = WithCount ? in.r[k] : 0.0f;
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
    const int slot = PerObject ? reduce_scatter16_slot() : 0;
    uint32_t cnt = 0;
    float qx = in.px, qy = in.py, qz = in.pz, qr = WithCount ? in.pr : 0.0f;
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
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (g0 >= core_lo && g0 + gn - 1 <= core_hi)
            energy_group<K, PerObject, WithCount, false>(xr, yr, zr, rr, row, nsteps, part, acc,
                                                         cnt, win, g0, gn, eps2, slot);
        else
            energy_group<K, PerObject, WithCount, true>(xr, yr, zr, rr, row, nsteps, part, acc,
                                                        cnt, win, g0, gn, eps2, slot);
        if (PerObject) {
            wave_sync();
            if (lane < gn)
                E.add(partner_index(base, band, g0 + lane), (double)win[4 * kWave + lane]);
        }
        wave_sync();
    }
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            if (PerObject) E.add(base + i, acc[k]);
            tot += acc[k];
        }
    }
    EnergyResult res;
    res.energy = wave_sum(tot);
    res.count = cnt;
    return res;
}

// ---------------------------------------------------------------- forces --
//
// Forces of the softened potential, a symmetric interaction with a vector
// value: f = (p_i - p_j) * e^3 with e = 1/sqrt(d2 + eps2) in float32 (the
// hardware reciprocal square root), added to row i and subtracted from
// partner j, so each unordered pair is evaluated once (Newton's third law on
// the balanced assignment).  Row sums are float32 partials of at most
// kFoldEvery terms per component folded into double accumulators; partner
// sums are summed across the wave, 16 partners at a time per component
// (reduce_scatter16), and added once per partner and task.
//
// Window entries past the task's partners hold a huge finite coordinate
// (kForcePad), not an infinity: e is then exactly 0 and dx * e^3 is 0, where
// an infinite dx would make it NaN.  Rows past the set use it too.

// LDS window of one wave: x, y, z of 64 partners and their three partner sums.
constexpr int kForceLds = 6 * kWave;
constexpr float kForcePad = 1e30f;

template <int K, bool Masked>
__device__ __forceinline__ void force_group(const float (&xr)[K], const float (&yr)[K],
                                            const float (&zr)[K], const int (&row)[K],
                                            const int (&nsteps)[K], float (&part)[3][K],
                                            double (&acc)[3][K], float *__restrict__ win,
                                            int g0, int gn, float eps2, int slot) {
    for (int t0 = 0; t0 < gn; t0 += kFoldEvery) {
        float sx_all[kFoldEvery], sy_all[kFoldEvery], sz_all[kFoldEvery];
#pragma unroll
        for (int tt = 0; tt < kFoldEvery; ++tt) {
            const int t = t0 + tt;
            const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t];
            const int u = g0 + t;
            float sx[K], sy[K], sz[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float dx = xr[k] - jx, dy = yr[k] - jy, dz = zr[k] - jz;
                float d2 = __builtin_fmaf(dx, dx, eps2);
                d2 = __builtin_fmaf(dy, dy, d2);
                d2 = __builtin_fmaf(dz, dz, d2);
                const float e = __builtin_amdgcn_rsqf(d2);
                float e3 = e * e * e;
                if (Masked) e3 = owns(u, row[k], nsteps[k]) ? e3 : 0.0f;
                const float fx = dx * e3, fy = dy * e3, fz = dz * e3;
                // first terms stored, not added to zero
                part[0][k] = tt == 0 ? fx : part[0][k] + fx;
                part[1][k] = tt == 0 ? fy : part[1][k] + fy;
                part[2][k] = tt == 0 ? fz : part[2][k] + fz;
                sx[k] = fx;
                sy[k] = fy;
                sz[k] = fz;
            }
            sx_all[tt] = tree_sum(sx);
            sy_all[tt] = tree_sum(sy);
            sz_all[tt] = tree_sum(sz);
        }
        // all 4 lanes of a group store the same value to the same slot
        win[3 * kWave + t0 + slot] = reduce_scatter16(sx_all);
        win[4 * kWave + t0 + slot] = reduce_scatter16(sy_all);
        win[5 * kWave + t0 + slot] = reduce_scatter16(sz_all);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < K; ++k) acc[c][k] += (double)part[c][k];
        }
    }
}

// One wave task of the force kernel: rows [ra, ra + 64K) against partners
// [u0, u1) of the band; F (three arrays of n doubles) receives the row sums
// and, negated, the partner sums.
template <int K>
__device__ __forceinline__ void force_task(const float *__restrict__ px, const float *__restrict__ py,
                                           const float *__restrict__ pz, int64_t base,
                                           const Band band, int ra, int u0, int u1, float eps2,
                                           float *__restrict__ win, const SumSink Fx,
                                           const SumSink Fy, const SumSink Fz,
                                           const TaskInputs<float, K> &in) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], part[3][K];
    double acc[3][K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            xr[k] = in.x[k]; yr[k] = in.y[k]; zr[k] = in.z[k];
            nsteps[k] = band.steps(i);
        } else {
            xr[k] = kForcePad;
            yr[k] = zr[k] = 0.0f;
            nsteps[k] = 0;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            part[c][k] = 0.0f;
            acc[c][k] = 0.0;
        }
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
    const int slot = reduce_scatter16_slot();
    float qx = in.px, qy = in.py, qz = in.pz;
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        const bool pad = g0 + lane >= u1;
        win[0 * kWave + lane] = pad ? kForcePad : qx;
        win[1 * kWave + lane] = pad ? 0.0f : qy;
        win[2 * kWave + lane] = pad ? 0.0f : qz;
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g];
            }
        }
        wave_sync();
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (g0 >= core_lo && g0 + gn - 1 <= core_hi)
            force_group<K, false>(xr, yr, zr, row, nsteps, part, acc, win, g0, gn, eps2, slot);
        else
            force_group<K, true>(xr, yr, zr, row, nsteps, part, acc, win, g0, gn, eps2, slot);
        wave_sync();
        if (lane < gn) {
            const int64_t g = partner_index(base, band, g0 + lane);
            Fx.add(g, -(double)win[3 * kWave + lane]);
            Fy.add(g, -(double)win[4 * kWave + lane]);
            Fz.add(g, -(double)win[5 * kWave + lane]);
        }
        wave_sync();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            Fx.add(base + i, acc[0][k]);
            Fy.add(base + i, acc[1][k]);
            Fz.add(base + i, acc[2][k]);
        }
    }
}

// --------------------------------------------------------- energy, fp64 --
//
// The softened potential with double inputs and double arithmetic:
// e = 1/sqrt(d2 + eps2) from the hardware double reciprocal square root and
// one Newton step, y <- y (3/2 - (d2 + eps2) y^2 / 2), which takes its
// relative error to the order of the double rounding.  Row sums accumulate
// in double; with PerObject the partner side of each pair is summed across
// the wave, 16 partners at a time (reduce_scatter16_f64), and added once per
// partner and task, as in the float32 kernel.

// Window entries past the task's partners and rows past the set hold a huge
// finite coordinate: an infinity would give rsq(inf) = 0 and then 0 * inf =
// NaN in the Newton step.  A pair with one such coordinate has d2 near
// 1e300 and e near 1e-150, which masked groups replace by 0 and unmasked
// ones add to partner sums (at most 256 such terms per partner and task,
// some 1e-148 against sums of order 1).
//
// LDS window of one wave: x, y, z of 64 partners and their partner sums.
constexpr int kEnergy64Lds = 4 * kWave;
constexpr double kEnergy64Pad = 1e150;

__device__ __forceinline__ double rsq_f64(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a * y;
    return y * __builtin_fma(-h, y, 1.5);
}

template <int K, bool PerObject, bool Masked>
__device__ __forceinline__ void energy64_group(const double (&xr)[K], const double (&yr)[K],
                                               const double (&zr)[K], const int (&row)[K],
                                               const int (&nsteps)[K], double (&acc)[K],
                                               double *__restrict__ win, int g0, int gn,
                                               double eps2, int slot) {
    for (int t0 = 0; t0 < gn; t0 += 16) {
        double js_all[16];
#pragma unroll
        for (int tt = 0; tt < 16; ++tt) {
            const int t = t0 + tt;
            const double jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t];
            const int u = g0 + t;
            double es[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double dx = xr[k] - jx, dy = yr[k] - jy, dz = zr[k] - jz;
                double d2 = __builtin_fma(dx, dx, eps2);
                d2 = __builtin_fma(dy, dy, d2);
                d2 = __builtin_fma(dz, dz, d2);
                double e = rsq_f64(d2);
                if (Masked) e = owns(u, row[k], nsteps[k]) ? e : 0.0;
                acc[k] += e;
                es[k] = e;
            }
            if (PerObject) js_all[tt] = tree_sum(es);
        }
        if (PerObject) win[3 * kWave + t0 + slot] = reduce_scatter16_f64(js_all);
    }
}

template <int K, bool PerObject>
__device__ __forceinline__ double energy64_task(const double *__restrict__ px,
                                                const double *__restrict__ py,
                                                const double *__restrict__ pz, int64_t base,
                                                const Band band, int ra, int u0, int u1,
                                                double eps2, double *__restrict__ win,
                                                const SumSink E,
                                                const TaskInputs<double, K> &in) {
    const int lane = lane_id();
    double xr[K], yr[K], zr[K], acc[K];
    int row[K], nsteps[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        row[k] = i;
        if (i < band.n) {
            xr[k] = in.x[k]; yr[k] = in.y[k]; zr[k] = in.z[k];
            nsteps[k] = band.steps(i);
        } else {
            xr[k] = kEnergy64Pad;
            yr[k] = zr[k] = 0.0;
            nsteps[k] = 0;
        }
        acc[k] = 0.0;
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
    const int slot = PerObject ? reduce_scatter16_slot() : 0;
    double qx = in.px, qy = in.py, qz = in.pz;
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        const bool pad = g0 + lane >= u1;
        win[0 * kWave + lane] = pad ? -kEnergy64Pad : qx;
        win[1 * kWave + lane] = pad ? 0.0 : qy;
        win[2 * kWave + lane] = pad ? 0.0 : qz;
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g];
            }
        }
        wave_sync();
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (g0 >= core_lo && g0 + gn - 1 <= core_hi)
            energy64_group<K, PerObject, false>(xr, yr, zr, row, nsteps, acc, win, g0, gn, eps2,
                                                slot);
        else
            energy64_group<K, PerObject, true>(xr, yr, zr, row, nsteps, acc, win, g0, gn, eps2,
                                               slot);
        if (PerObject) {
            wave_sync();
            if (lane < gn) E.add(partner_index(base, band, g0 + lane), win[3 * kWave + lane]);
        }
        wave_sync();
    }
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            if (PerObject) E.add(base + i, acc[k]);
            tot += acc[k];
        }
    }
    return wave_sum(tot);
}

}  // namespace pairs_dev
