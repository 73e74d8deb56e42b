// libpairs: all-pairs interactions within sets of objects, for gfx950.
//
// One wave (64 lanes) runs one task: a block of 64*K consecutive rows of the
// balanced assignment (band.h) held in registers, K rows per lane in
// lane-major order (row ra + 64k + lane), swept against a chunk of virtual
// partners u that are staged 64 at a time into a wave-private LDS window and
// read back as wave-uniform broadcasts.  For a fixed u the rows that own the
// pair (row, u mod n) are the contiguous range [first_row(u), u-1]
// (band.h), so inside a row block's core every lane is valid and at the two
// band edges a scalar lane-range mask selects them.  Padding rows and padding
// partners carry values (infinities) for which the predicate is false or the
// potential is exactly zero, so they need no mask.
//
// Counts: the wave's predicate mask is counted with a scalar popcount and the
// wave adds its total to the output with one 64-bit atomic.
// Energies: float32 pair arithmetic; per-row float32 partials of at most 16
// terms are folded into double accumulators; the partner side of each pair
// is reduced across the wave with DPP and added once per partner and task.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "band.h"
#include "pairs.h"

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

thread_local hipError_t g_last_hip_error = hipSuccess;

// --------------------------------------------------------------- helpers --

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

// DPP row/bank controls (GFX9 encoding).
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int Ctrl, int RowMask, int BankMask>
__device__ __forceinline__ float dpp_plus(float v) {
    int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, RowMask, BankMask, true);
    return v + __int_as_float(s);
}

// Sum of v over the 64 lanes, returned as a wave-uniform value.
__device__ __forceinline__ float wave_sum(float v) {
    v = dpp_plus<kDppRowShr1, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowShr2, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowShr4, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowShr8, 0xf, 0xf>(v);
    v = dpp_plus<kDppRowBcast15, 0xa, 0xf>(v);
    v = dpp_plus<kDppRowBcast31, 0xc, 0xf>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ validation --

__global__ void k_validate_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                               const int32_t *r, int64_t n, int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t L = PAIRS_I32_COORD_LIMIT, RL = PAIRS_I32_RADIUS_LIMIT;
    bool ok = x[i] >= -L && x[i] <= L && y[i] >= -L && y[i] <= L && z[i] >= -L && z[i] <= L &&
              r[i] >= 0 && r[i] <= RL;
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_validate_f32(const float *x, const float *y, const float *z, const float *r,
                               int64_t n, int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool ok = isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]) && (r == nullptr || isfinite(r[i]));
    if (!ok) atomicOr(bad, 1);
}

// ---------------------------------------------------------- int32 count --
//
// Exact predicate in double precision (Gram form).  With h = (|p|^2 - r^2)/2,
//   |p_i - p_j|^2 <= (r_i + r_j)^2  <=>  p_i.p_j + r_i r_j - h_i >= h_j.
// Inside the exact domain (|coordinate| <= 2^24, 0 <= r <= 2^24) every
// product is an integer below 2^48 in magnitude and every partial sum a
// multiple of 1/2 below 2^51, so all fused multiply-adds are exact and the
// comparison decides the integer predicate.

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

// LDS window of one wave for the int32 count: 5 arrays of 64 doubles.
constexpr int kCountLds = 5 * kWave;

template <int K>
__device__ uint32_t count_i32_task(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                                   const int32_t *__restrict__ pz, const int32_t *__restrict__ pr,
                                   int64_t base, const Band band, int ra, int u0, int u1,
                                   double *__restrict__ win) {
    const int lane = lane_id();
    double xr[K], yr[K], zr[K], rr[K], nh[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            int64_t g = base + i;
            double h;
            gram_features(px[g], py[g], pz[g], pr[g], xr[k], yr[k], zr[k], rr[k], h);
            nh[k] = -h;
        } else {
            xr[k] = yr[k] = zr[k] = rr[k] = 0.0;
            nh[k] = -INFINITY;  // never hits
        }
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1;                 // every row has u - 1 >= row
    const int core_hi = ra + band.steps(ra);       // every row has u <= row + steps(row)

    uint32_t cnt = 0;
    // raw partner values for the next group (register prefetch)
    int32_t qx = 0, qy = 0, qz = 0, qr = 0;
    {
        int u = u0 + lane;
        if (u < u1) {
            int64_t g = base + (u >= band.n ? u - band.n : u);
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
                int64_t g = base + (u >= band.n ? u - band.n : u);
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
                const int first = max(band.first_row(u), ra);
                const double jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                             jr = win[3 * kWave + t], jh = win[4 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int b = ra + kWave * k;
                    const uint64_t m = lane_range(first - b, u - 1 - b);
                    if (m == 0) continue;
                    double v = __builtin_fma(xr[k], jx, nh[k]);
                    v = __builtin_fma(yr[k], jy, v);
                    v = __builtin_fma(zr[k], jz, v);
                    v = __builtin_fma(rr[k], jr, v);
                    cnt += count_bits_masked(v >= jh, m);
                }
            }
        }
        wave_sync();
    }
    return cnt;
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_count_i32(const int32_t *__restrict__ x,
                                                      const int32_t *__restrict__ y,
                                                      const int32_t *__restrict__ z,
                                                      const int32_t *__restrict__ r, int n,
                                                      int U, uint64_t *out) {
    __shared__ double lds[kWavesPerBlock * kCountLds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (task >= til.tasks()) return;
    const int blk = (int)(task / til.nchunks), c = (int)(task % til.nchunks);
    int ra, u0, u1;
    task_range(band, til, blk, c, &ra, &u0, &u1);
    if (u0 >= u1) return;
    uint32_t cnt = count_i32_task<K>(x, y, z, r, 0, band, ra, u0, u1, lds + wave * kCountLds);
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
}

// -------------------------------------------------------- float32 count --
//
// The pinned binary32 sequence; explicit round-to-nearest intrinsics keep the
// compiler from contracting or reordering it.

__device__ __forceinline__ bool hit_f32(float xi, float yi, float zi, float ri, float xj,
                                        float yj, float zj, float rj) {
    float dx = __fsub_rn(xi, xj), dy = __fsub_rn(yi, yj), dz = __fsub_rn(zi, zj);
    float d2 = __fmul_rn(dx, dx);
    d2 = __fmaf_rn(dy, dy, d2);
    d2 = __fmaf_rn(dz, dz, d2);
    float R = __fadd_rn(ri, rj);
    return d2 <= __fmul_rn(R, R);
}

constexpr int kF32Lds = 4 * kWave;

template <int K>
__device__ uint32_t count_f32_task(const float *__restrict__ px, const float *__restrict__ py,
                                   const float *__restrict__ pz, const float *__restrict__ pr,
                                   int64_t base, const Band band, int ra, int u0, int u1,
                                   float *__restrict__ win) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], rr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            int64_t g = base + i;
            xr[k] = px[g]; yr[k] = py[g]; zr[k] = pz[g]; rr[k] = pr[g];
        } else {
            xr[k] = INFINITY;  // distance infinite: never hits
            yr[k] = zr[k] = rr[k] = 0.0f;
        }
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
    uint32_t cnt = 0;
    float qx = 0, qy = 0, qz = 0, qr = 0;
    {
        int u = u0 + lane;
        if (u < u1) {
            int64_t g = base + (u >= band.n ? u - band.n : u);
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
                int64_t g = base + (u >= band.n ? u - band.n : u);
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
                const int first = max(band.first_row(u), ra);
                const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                            jr = win[3 * kWave + t];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int b = ra + kWave * k;
                    const uint64_t m = lane_range(first - b, u - 1 - b);
                    if (m == 0) continue;
                    cnt += count_bits_masked(hit_f32(xr[k], yr[k], zr[k], rr[k], jx, jy, jz, jr), m);
                }
            }
        }
        wave_sync();
    }
    return cnt;
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_count_f32(const float *__restrict__ x,
                                                      const float *__restrict__ y,
                                                      const float *__restrict__ z,
                                                      const float *__restrict__ r, int n, int U,
                                                      uint64_t *out) {
    __shared__ float lds[kWavesPerBlock * kF32Lds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (task >= til.tasks()) return;
    const int blk = (int)(task / til.nchunks), c = (int)(task % til.nchunks);
    int ra, u0, u1;
    task_range(band, til, blk, c, &ra, &u0, &u1);
    if (u0 >= u1) return;
    uint32_t cnt = count_f32_task<K>(x, y, z, r, 0, band, ra, u0, u1, lds + wave * kF32Lds);
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
}

// ---------------------------------------------------------------- energy --

constexpr int kEnergyLds = 3 * kWave;
constexpr int kFoldEvery = 16;  // float32 partials hold at most this many terms

// Returns the sum of e over the task's pairs (each pair once, on the row side).
// With PerObject, adds each row's and each partner's share to E.
template <int K, bool PerObject>
__device__ double energy_task(const float *__restrict__ px, const float *__restrict__ py,
                              const float *__restrict__ pz, int64_t base, const Band band,
                              int ra, int u0, int u1, float eps2, float *__restrict__ win,
                              double *__restrict__ E) {
    const int lane = lane_id();
    float xr[K], yr[K], zr[K], part[K];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = ra + kWave * k + lane;
        if (i < band.n) {
            int64_t g = base + i;
            xr[k] = px[g]; yr[k] = py[g]; zr[k] = pz[g];
        } else {
            xr[k] = INFINITY;  // infinite distance: e is exactly 0
            yr[k] = zr[k] = 0.0f;
        }
        part[k] = 0.0f;
        acc[k] = 0.0;
    }
    const int rlast = min(ra + kWave * K, band.n) - 1;
    const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
    float qx = 0, qy = 0, qz = 0;
    {
        int u = u0 + lane;
        if (u < u1) {
            int64_t g = base + (u >= band.n ? u - band.n : u);
            qx = px[g]; qy = py[g]; qz = pz[g];
        }
    }
    for (int g0 = u0; g0 < u1; g0 += kWave) {
        const bool pad = g0 + lane >= u1;
        win[0 * kWave + lane] = pad ? -INFINITY : qx;
        win[1 * kWave + lane] = pad ? 0.0f : qy;
        win[2 * kWave + lane] = pad ? 0.0f : qz;
        {
            int u = g0 + kWave + lane;
            if (u < u1) {
                int64_t g = base + (u >= band.n ? u - band.n : u);
                qx = px[g]; qy = py[g]; qz = pz[g];
            }
        }
        wave_sync();
        const int gn = min(kWave, u1 - g0);
        const bool full = g0 >= core_lo && g0 + gn - 1 <= core_hi;
        float jsum = 0.0f;  // lane t: partner share of virtual partner g0 + t
        for (int t0 = 0; t0 < kWave; t0 += kFoldEvery) {
            if (t0 >= gn) break;
#pragma unroll 2
            for (int t = t0; t < t0 + kFoldEvery; ++t) {
                const float jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t];
                const int u = g0 + t;
                const int first = max(band.first_row(u), ra);
                float js = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float dx = xr[k] - jx, dy = yr[k] - jy, dz = zr[k] - jz;
                    float d2 = __builtin_fmaf(dx, dx, eps2);
                    d2 = __builtin_fmaf(dy, dy, d2);
                    d2 = __builtin_fmaf(dz, dz, d2);
                    float e = __builtin_amdgcn_rsqf(d2);
                    if (!full) {
                        const int b = ra + kWave * k;
                        const uint64_t m = lane_range(first - b, u - 1 - b);
                        e = ((m >> lane) & 1ull) ? e : 0.0f;
                    }
                    part[k] += e;
                    if (PerObject) js += e;
                }
                if (PerObject) {
                    const float s = wave_sum(js);
                    jsum = (lane == t) ? s : jsum;
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                acc[k] += (double)part[k];
                part[k] = 0.0f;
            }
        }
        if (PerObject && lane < gn) {
            const int u = g0 + lane;
            atomicAdd(&E[base + (u >= band.n ? u - band.n : u)], (double)jsum);
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
    return wave_sum(tot);
}

template <int K, bool PerObject>
__global__ __launch_bounds__(kBlock) void k_energy(const float *__restrict__ x,
                                                   const float *__restrict__ y,
                                                   const float *__restrict__ z, int n, int U,
                                                   float eps2, double *E, double *total) {
    __shared__ float lds[kWavesPerBlock * kEnergyLds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (task >= til.tasks()) return;
    const int blk = (int)(task / til.nchunks), c = (int)(task % til.nchunks);
    int ra, u0, u1;
    task_range(band, til, blk, c, &ra, &u0, &u1);
    if (u0 >= u1) return;
    double s = energy_task<K, PerObject>(x, y, z, 0, band, ra, u0, u1, eps2,
                                         lds + wave * kEnergyLds, E);
    if (lane_id() == 0) atomicAdd(total, s);
}

// ------------------------------------------------------------------ host --

pairs_status_t hip_fail(hipError_t e) {
    g_last_hip_error = e;
    return PAIRS_ERR_HIP;
}

#define PAIRS_HIP_CHECK(expr)                          \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_);     \
    } while (0)

// Per-device state: a small device word for validation results.
struct DeviceState {
    int *d_flag = nullptr;
};

constexpr int kMaxDevices = 64;
DeviceState g_dev[kMaxDevices];

pairs_status_t current_device(int *dev) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        g_last_hip_error = e;
        return PAIRS_ERR_NO_DEVICE;
    }
    PAIRS_HIP_CHECK(hipGetDevice(dev));
    if (*dev < 0 || *dev >= kMaxDevices) return PAIRS_ERR_NO_DEVICE;
    return PAIRS_OK;
}

pairs_status_t device_flag(int **flag) {
    int dev;
    pairs_status_t st = current_device(&dev);
    if (st != PAIRS_OK) return st;
    if (!g_dev[dev].d_flag) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, 256);
        if (e != hipSuccess) {
            g_last_hip_error = e;
            return PAIRS_ERR_NO_MEMORY;
        }
        g_dev[dev].d_flag = (int *)p;
    }
    *flag = g_dev[dev].d_flag;
    return PAIRS_OK;
}

int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

pairs_status_t fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return PAIRS_OK;
    k_fill_u64<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return PAIRS_OK;
    k_fill_f64<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

// Reads the validation word after the stream has run the check.
pairs_status_t finish_validation(int *d_flag, hipStream_t s) {
    int bad = 0;
    PAIRS_HIP_CHECK(hipMemcpyAsync(&bad, d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PAIRS_HIP_CHECK(hipStreamSynchronize(s));
    return bad ? PAIRS_ERR_DOMAIN : PAIRS_OK;
}

template <typename T>
pairs_status_t validate(const T *x, const T *y, const T *z, const T *r, int64_t n, hipStream_t s);

template <>
pairs_status_t validate<int32_t>(const int32_t *x, const int32_t *y, const int32_t *z,
                                 const int32_t *r, int64_t n, hipStream_t s) {
    int *flag;
    pairs_status_t st = device_flag(&flag);
    if (st != PAIRS_OK) return st;
    PAIRS_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), s));
    if (n > 0) k_validate_i32<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, r, n, flag);
    PAIRS_HIP_CHECK(hipGetLastError());
    return finish_validation(flag, s);
}

template <>
pairs_status_t validate<float>(const float *x, const float *y, const float *z, const float *r,
                               int64_t n, hipStream_t s) {
    int *flag;
    pairs_status_t st = device_flag(&flag);
    if (st != PAIRS_OK) return st;
    PAIRS_HIP_CHECK(hipMemsetAsync(flag, 0, sizeof(int), s));
    if (n > 0) k_validate_f32<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, r, n, flag);
    PAIRS_HIP_CHECK(hipGetLastError());
    return finish_validation(flag, s);
}

// Tile shape of a single-set call: rows per lane K and partner chunk U.
struct Shape {
    int K;
    int U;
};

Shape single_set_shape(int64_t n) {
    if (n <= 8192) return {1, 256};
    if (n <= 65536) return {4, 1024};
    return {8, 8192};
}

template <int K>
void launch_count_i32(const int32_t *x, const int32_t *y, const int32_t *z, const int32_t *r,
                      int n, int U, uint64_t *out, hipStream_t s) {
    Tiling t = Tiling::of(Band::of(n), K, U);
    int64_t blocks = (t.tasks() + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0) k_count_i32<K><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, r, n, U, out);
}

template <int K>
void launch_count_f32(const float *x, const float *y, const float *z, const float *r, int n,
                      int U, uint64_t *out, hipStream_t s) {
    Tiling t = Tiling::of(Band::of(n), K, U);
    int64_t blocks = (t.tasks() + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0) k_count_f32<K><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, r, n, U, out);
}

template <int K>
void launch_energy(const float *x, const float *y, const float *z, int n, int U, float eps2,
                   double *E, double *total, hipStream_t s) {
    Tiling t = Tiling::of(Band::of(n), K, U);
    int64_t blocks = (t.tasks() + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks <= 0) return;
    if (E)
        k_energy<K, true><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
    else
        k_energy<K, false><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
}

}  // namespace

// ------------------------------------------------------------ public ABI --

extern "C" {

pairs_status_t pairs_count_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                               const int32_t *r, int64_t n, uint64_t *d_count, unsigned flags,
                               pairs_stream_t stream) {
    if (!d_count || n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z || !r)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    pairs_status_t st = current_device(&dev);
    if (st != PAIRS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        st = validate<int32_t>(x, y, z, r, n, s);
        if (st != PAIRS_OK) return st;
    }
    st = fill_u64(d_count, 1, 0, s);
    if (st != PAIRS_OK) return st;
    if (n < 2) return PAIRS_OK;
    Shape sh = single_set_shape(n);
    switch (sh.K) {
        case 1: launch_count_i32<1>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        case 4: launch_count_i32<4>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        default: launch_count_i32<8>(x, y, z, r, (int)n, sh.U, d_count, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t pairs_count_f32(const float *x, const float *y, const float *z, const float *r,
                               int64_t n, uint64_t *d_count, unsigned flags,
                               pairs_stream_t stream) {
    if (!d_count || n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z || !r)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    pairs_status_t st = current_device(&dev);
    if (st != PAIRS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        st = validate<float>(x, y, z, r, n, s);
        if (st != PAIRS_OK) return st;
    }
    st = fill_u64(d_count, 1, 0, s);
    if (st != PAIRS_OK) return st;
    if (n < 2) return PAIRS_OK;
    Shape sh = single_set_shape(n);
    switch (sh.K) {
        case 1: launch_count_f32<1>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        case 4: launch_count_f32<4>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        default: launch_count_f32<8>(x, y, z, r, (int)n, sh.U, d_count, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t pairs_energy_f32(const float *x, const float *y, const float *z, int64_t n,
                                float eps2, double *d_energy, double *d_total, unsigned flags,
                                pairs_stream_t stream) {
    if (!d_total || n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (!(eps2 > 0.0f) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    pairs_status_t st = current_device(&dev);
    if (st != PAIRS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        st = validate<float>(x, y, z, nullptr, n, s);
        if (st != PAIRS_OK) return st;
    }
    st = fill_f64(d_total, 1, 0.0, s);
    if (st != PAIRS_OK) return st;
    if (d_energy) {
        st = fill_f64(d_energy, n, 0.0, s);
        if (st != PAIRS_OK) return st;
    }
    if (n < 2) return PAIRS_OK;
    Shape sh = single_set_shape(n);
    switch (sh.K) {
        case 1: launch_energy<1>(x, y, z, (int)n, sh.U, eps2, d_energy, d_total, s); break;
        case 4: launch_energy<4>(x, y, z, (int)n, sh.U, eps2, d_energy, d_total, s); break;
        default: launch_energy<8>(x, y, z, (int)n, sh.U, eps2, d_energy, d_total, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

const char *pairs_status_string(pairs_status_t s) {
    switch (s) {
        case PAIRS_OK: return "ok";
        case PAIRS_ERR_INVALID_ARG: return "invalid argument";
        case PAIRS_ERR_DOMAIN: return "input outside the exact domain";
        case PAIRS_ERR_HIP: return "HIP runtime error";
        case PAIRS_ERR_NO_MEMORY: return "out of memory";
        case PAIRS_ERR_WORKSPACE: return "workspace missing or too small";
        case PAIRS_ERR_NO_DEVICE: return "no usable HIP device";
    }
    return "unknown status";
}

int pairs_last_hip_error(void) { return (int)g_last_hip_error; }

}  // extern "C"
