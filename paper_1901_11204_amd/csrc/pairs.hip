// libpairs: all-pairs interactions within sets of objects, for gfx950.
//
// Kernels (the wave-task bodies are in tasks.h):
//   single set : one wave per task, tasks enumerated row block by chunk;
//   batched    : one persistent grid; each wave walks the task list with a
//                grid stride.  The task list is either a table built on the
//                host by a plan (set, local task) sorted so that the tasks of
//                the largest size class come first, or, for unplanned calls,
//                per-class prefix sums built on the device by one scheduling
//                kernel, searched by each wave;
//   jitter     : the per-step perturbation of the repeated-step workload;
//   helpers    : fills (in place of memsets, so every launch can be
//                captured into a graph), validation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "band.h"
#include "device.h"
#include "pairs.h"
#include "tasks.h"

using namespace pairs_dev;

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

thread_local hipError_t g_last_hip_error = hipSuccess;

// ------------------------------------------------------------ size classes --
//
// A batch mixes set sizes over orders of magnitude.  Each set is tiled with
// the shape (K rows per lane, U partners per chunk) of its size class; the
// classes are listed from the largest sets down, and class c holds the sets
// with n > lo[c] that no earlier class holds.

constexpr int kMaxClasses = 4;

struct ClassTable {
    int count;
    int lo[kMaxClasses];
    int K[kMaxClasses];
    int U[kMaxClasses];

    __host__ __device__ int class_of(int n) const {
        for (int c = 0; c < count - 1; ++c)
            if (n > lo[c]) return c;
        return count - 1;
    }
    __host__ __device__ int64_t tasks(int n, int c) const {
        return Tiling::of(Band::of(n), K[c], U[c]).tasks();
    }
};

ClassTable default_classes() {
    ClassTable t;
    t.count = 4;
    const int lo[4] = {4096, 1024, 256, 0};
    const int K[4] = {8, 4, 2, 1};
    const int U[4] = {2048, 1024, 512, 256};
    for (int c = 0; c < 4; ++c) {
        t.lo[c] = lo[c];
        t.K[c] = K[c];
        t.U[c] = U[c];
    }
    return t;
}

// Set s of a CSR batch, clipped to [0, n_total) so that malformed offsets can
// never index outside the object arrays.
__device__ __forceinline__ void set_range(const int64_t *__restrict__ off, int64_t s,
                                          int64_t n_total, int64_t *base, int *n) {
    int64_t a = off[s], b = off[s + 1];
    a = a < 0 ? 0 : (a > n_total ? n_total : a);
    b = b < a ? a : (b > n_total ? n_total : b);
    int64_t m = b - a;
    *base = a;
    *n = (int)(m > PAIRS_MAX_BATCH_SET_SIZE ? PAIRS_MAX_BATCH_SET_SIZE : m);
}

// --------------------------------------------------------------- helpers --

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

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
    bool ok = isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]) &&
              (r == nullptr || isfinite(r[i]));
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_validate_offsets(const int64_t *off, int64_t n_sets, int64_t n_total, int *bad) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_sets) return;
    bool ok = true;
    if (s == 0) ok = off[0] == 0;
    if (s == n_sets) ok = ok && off[n_sets] == n_total;
    if (s < n_sets)
        ok = ok && off[s + 1] >= off[s] && off[s + 1] - off[s] <= PAIRS_MAX_BATCH_SET_SIZE;
    if (!ok) atomicOr(bad, 2);
}

// ------------------------------------------------------- single-set kernels --

template <int K>
__global__ __launch_bounds__(kBlock) void k_count_i32(const int32_t *__restrict__ x,
                                                      const int32_t *__restrict__ y,
                                                      const int32_t *__restrict__ z,
                                                      const int32_t *__restrict__ r, int n,
                                                      int U, uint64_t *out) {
    __shared__ double lds[kWavesPerBlock * kCountI32Lds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (task >= til.tasks()) return;
    const int blk = (int)(task / til.nchunks), c = (int)(task % til.nchunks);
    int ra, u0, u1;
    task_range(band, til, blk, c, &ra, &u0, &u1);
    if (u0 >= u1) return;
    uint32_t cnt = count_i32_task<K>(x, y, z, r, 0, band, ra, u0, u1, lds + wave * kCountI32Lds);
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_count_f32(const float *__restrict__ x,
                                                      const float *__restrict__ y,
                                                      const float *__restrict__ z,
                                                      const float *__restrict__ r, int n, int U,
                                                      uint64_t *out) {
    __shared__ float lds[kWavesPerBlock * kCountF32Lds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (task >= til.tasks()) return;
    const int blk = (int)(task / til.nchunks), c = (int)(task % til.nchunks);
    int ra, u0, u1;
    task_range(band, til, blk, c, &ra, &u0, &u1);
    if (u0 >= u1) return;
    uint32_t cnt = count_f32_task<K>(x, y, z, r, 0, band, ra, u0, u1, lds + wave * kCountF32Lds);
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
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
    EnergyResult res = energy_task<K, PerObject, false>(x, y, z, nullptr, 0, band, ra, u0, u1,
                                                        eps2, lds + wave * kEnergyLds, E);
    if (lane_id() == 0) atomicAdd(total, res.energy);
}

// ---------------------------------------------------------- batched kernels --

// Task source of a plan: a host-built table of (set, local task index).
struct TableSource {
    const int2 *tasks;
    int64_t ntasks;
    __device__ int64_t total() const { return ntasks; }
    __device__ void decode(int64_t t, int64_t *set, int *local) const {
        int2 e = tasks[t];
        *set = e.x;
        *local = e.y;
    }
};

// Task source of an unplanned call: per-class exclusive prefix sums of the
// per-set task counts (coff[c][s], s = 0..n_sets) and the class bases.
struct ScanSource {
    const int64_t *bases;  // [kMaxClasses + 1]
    const int64_t *coff;   // [kMaxClasses][n_sets + 1]
    int64_t n_sets;
    int classes;
    __device__ int64_t total() const { return bases[classes]; }
    __device__ void decode(int64_t t, int64_t *set, int *local) const {
        int c = 0;
        while (c + 1 < classes && t >= bases[c + 1]) ++c;
        const int64_t tl = t - bases[c];
        const int64_t *o = coff + (int64_t)c * (n_sets + 1);
        // last s with o[s] <= tl; sets of other classes have empty ranges
        int64_t lo = 0, hi = n_sets;  // o[lo] <= tl < o[hi]
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if (o[mid] <= tl) lo = mid; else hi = mid;
        }
        *set = lo;
        *local = (int)(tl - o[lo]);
    }
};

// The single-block scheduler of unplanned calls.
constexpr int kSchedThreads = 1024;

__global__ __launch_bounds__(kSchedThreads) void k_batch_schedule(
    const int64_t *__restrict__ off, int64_t n_sets, int64_t n_total, ClassTable ct,
    int64_t *__restrict__ coff, int64_t *__restrict__ bases) {
    __shared__ int64_t part[kMaxClasses][kSchedThreads];
    __shared__ int64_t class_total[kMaxClasses];
    const int tid = threadIdx.x;
    const int64_t chunk = (n_sets + kSchedThreads - 1) / kSchedThreads;
    const int64_t s0 = min((int64_t)tid * chunk, n_sets), s1 = min(s0 + chunk, n_sets);
    int64_t sum[kMaxClasses] = {0, 0, 0, 0};
    for (int64_t s = s0; s < s1; ++s) {
        int64_t b;
        int n;
        set_range(off, s, n_total, &b, &n);
        int c = ct.class_of(n);
        sum[c] += ct.tasks(n, c);
    }
    for (int c = 0; c < kMaxClasses; ++c) part[c][tid] = sum[c];
    __syncthreads();
    if (tid < ct.count) {  // exclusive scan of class tid over the threads
        int64_t run = 0;
        for (int k = 0; k < kSchedThreads; ++k) {
            int64_t v = part[tid][k];
            part[tid][k] = run;
            run += v;
        }
        class_total[tid] = run;
        coff[(int64_t)tid * (n_sets + 1) + n_sets] = run;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t acc = 0;
        for (int c = 0; c < ct.count; ++c) {
            bases[c] = acc;
            acc += class_total[c];
        }
        bases[ct.count] = acc;
    }
    int64_t run[kMaxClasses];
    for (int c = 0; c < kMaxClasses; ++c) run[c] = part[c][tid];
    for (int64_t s = s0; s < s1; ++s) {
        int64_t b;
        int n;
        set_range(off, s, n_total, &b, &n);
        int cs = ct.class_of(n);
        for (int c = 0; c < ct.count; ++c)
            coff[(int64_t)c * (n_sets + 1) + s] = run[c];
        run[cs] += ct.tasks(n, cs);
    }
}

enum Kind { kCountI32 = 1, kCountF32 = 2, kEnergyF32 = 3 };

// LDS of one wave, in bytes, for every kind.
constexpr int kLdsBytes = (kCountI32Lds * 8 > kEnergyLds * 4 ? kCountI32Lds * 8 : kEnergyLds * 4);

struct BatchIO {
    const void *x, *y, *z, *r;  // object arrays (r may be null for energies)
    const int64_t *off;
    int64_t n_total;
    uint64_t *counts;  // [n_sets] or null
    double *energy;    // [n_sets] (energies)
    float eps2;
};

template <int K, int KindV>
__device__ __forceinline__ void batched_task(const BatchIO &io, int64_t base, const Band &band,
                                             int ra, int u0, int u1, int64_t set, void *win) {
    if (KindV == kCountI32) {
        uint32_t c = count_i32_task<K>((const int32_t *)io.x, (const int32_t *)io.y,
                                       (const int32_t *)io.z, (const int32_t *)io.r, base, band,
                                       ra, u0, u1, (double *)win);
        if (lane_id() == 0 && c)
            atomicAdd((unsigned long long *)&io.counts[set], (unsigned long long)c);
    } else if (KindV == kCountF32) {
        uint32_t c = count_f32_task<K>((const float *)io.x, (const float *)io.y,
                                       (const float *)io.z, (const float *)io.r, base, band, ra,
                                       u0, u1, (float *)win);
        if (lane_id() == 0 && c)
            atomicAdd((unsigned long long *)&io.counts[set], (unsigned long long)c);
    } else {
        EnergyResult res;
        if (io.r)
            res = energy_task<K, false, true>((const float *)io.x, (const float *)io.y,
                                              (const float *)io.z, (const float *)io.r, base,
                                              band, ra, u0, u1, io.eps2, (float *)win, nullptr);
        else
            res = energy_task<K, false, false>((const float *)io.x, (const float *)io.y,
                                               (const float *)io.z, nullptr, base, band, ra, u0,
                                               u1, io.eps2, (float *)win, nullptr);
        if (lane_id() == 0) {
            atomicAdd(&io.energy[set], res.energy);
            if (io.r && res.count)
                atomicAdd((unsigned long long *)&io.counts[set], (unsigned long long)res.count);
        }
    }
}

template <int KindV, typename Source>
__global__ __launch_bounds__(kBlock) void k_batched(BatchIO io, Source src, ClassTable ct) {
    __shared__ __align__(16) unsigned char lds[kWavesPerBlock * kLdsBytes];
    const int wave = wave_id();
    void *win = lds + wave * kLdsBytes;
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t ntasks = src.total();
    for (int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave; t < ntasks; t += stride) {
        int64_t set;
        int local;
        src.decode(t, &set, &local);
        int64_t base;
        int n;
        set_range(io.off, set, io.n_total, &base, &n);
        if (n < 2) continue;
        const int c = ct.class_of(n);
        const Band band = Band::of(n);
        const Tiling til = Tiling::of(band, ct.K[c], ct.U[c]);
        if (local < 0 || (int64_t)local >= til.tasks()) continue;
        int ra, u0, u1;
        task_range(band, til, local / til.nchunks, local % til.nchunks, &ra, &u0, &u1);
        if (u0 >= u1) continue;
        switch (ct.K[c]) {
            case 8: batched_task<8, KindV>(io, base, band, ra, u0, u1, set, win); break;
            case 4: batched_task<4, KindV>(io, base, band, ra, u0, u1, set, win); break;
            case 2: batched_task<2, KindV>(io, base, band, ra, u0, u1, set, win); break;
            default: batched_task<1, KindV>(io, base, band, ra, u0, u1, set, win); break;
        }
    }
}

// ------------------------------------------------------------------ jitter --
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32->64-bit multiplications by 0xD2511F53 and 0xCD9E8D57, a word exchange
// and a key xor, with the key advanced by 0x9E3779B9 and 0xBB67AE85 between
// rounds.  Counter (global index, step, axis, 0), key (seed low, seed high).
// The four words give an Irwin-Hall(4) variate S = 2 sum(w_k >> 8) - 4(2^24-1)
// (zero mean, variance (4/3)(2^48-1)), scaled by c = sigma / sqrt of that
// variance: delta = fl32(fl32(S) * c), x = fl32(x + delta).

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__global__ void k_jitter(float *x, float *y, float *z, int64_t n, uint32_t k0, uint32_t k1,
                         uint32_t step, float scale, int64_t first_index) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *coord[3] = {x, y, z};
#pragma unroll
    for (uint32_t axis = 0; axis < 3; ++axis) {
        uint32_t w[4];
        philox4x32_10((uint32_t)(first_index + i), step, axis, 0u, k0, k1, w);
        int32_t sum = (int32_t)(w[0] >> 8) + (int32_t)(w[1] >> 8) + (int32_t)(w[2] >> 8) +
                      (int32_t)(w[3] >> 8);
        int32_t S = 2 * sum - 4 * ((1 << 24) - 1);
        float delta = __fmul_rn((float)S, scale);
        coord[axis][i] = __fadd_rn(coord[axis][i], delta);
    }
}

// ------------------------------------------------------------------ host --

pairs_status_t hip_fail(hipError_t e) {
    g_last_hip_error = e;
    return PAIRS_ERR_HIP;
}

#define PAIRS_HIP_CHECK(expr)                      \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

#define PAIRS_TRY(expr)                \
    do {                               \
        pairs_status_t s_ = (expr);    \
        if (s_ != PAIRS_OK) return s_; \
    } while (0)

// Per-device state: a device word for validation results and the CU count.
struct DeviceState {
    int *d_flag = nullptr;
    int n_cu = 0;
};

constexpr int kMaxDevices = 64;
DeviceState g_dev[kMaxDevices];
std::mutex g_dev_mutex;

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

pairs_status_t device_state(DeviceState **st) {
    int dev;
    PAIRS_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    DeviceState &d = g_dev[dev];
    if (!d.d_flag) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, 256);
        if (e != hipSuccess) {
            g_last_hip_error = e;
            return PAIRS_ERR_NO_MEMORY;
        }
        int ncu = 0;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) {
            hipFree(p);
            return hip_fail(e);
        }
        d.n_cu = ncu;
        d.d_flag = (int *)p;
    }
    *st = &d;
    return PAIRS_OK;
}

int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

pairs_status_t fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0 || !p) return PAIRS_OK;
    k_fill_u64<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0 || !p) return PAIRS_OK;
    k_fill_f64<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

// Runs the checks that `launch` enqueues against a cleared device word and
// waits for the answer (the synchronous PAIRS_FLAG_VALIDATE path).
template <typename F>
pairs_status_t run_validation(hipStream_t s, F launch) {
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    k_fill_u64<<<1, 1, 0, s>>>((uint64_t *)st->d_flag, 1, 0);
    launch(st->d_flag);
    PAIRS_HIP_CHECK(hipGetLastError());
    int bad = 0;
    PAIRS_HIP_CHECK(hipMemcpyAsync(&bad, st->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PAIRS_HIP_CHECK(hipStreamSynchronize(s));
    if (bad & 2) return PAIRS_ERR_INVALID_ARG;
    return bad ? PAIRS_ERR_DOMAIN : PAIRS_OK;
}

pairs_status_t validate_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                            const int32_t *r, int64_t n, hipStream_t s) {
    return run_validation(s, [&](int *flag) {
        if (n > 0) k_validate_i32<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, r, n, flag);
    });
}

pairs_status_t validate_f32(const float *x, const float *y, const float *z, const float *r,
                            int64_t n, hipStream_t s) {
    return run_validation(s, [&](int *flag) {
        if (n > 0) k_validate_f32<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, r, n, flag);
    });
}

pairs_status_t validate_offsets(const int64_t *off, int64_t n_sets, int64_t n_total,
                                hipStream_t s) {
    return run_validation(s, [&](int *flag) {
        k_validate_offsets<<<blocks_for(n_sets + 1, 256), 256, 0, s>>>(off, n_sets, n_total, flag);
    });
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

int64_t single_blocks(int n, int K, int U) {
    Tiling t = Tiling::of(Band::of(n), K, U);
    return (t.tasks() + kWavesPerBlock - 1) / kWavesPerBlock;
}

template <int K>
void launch_count_i32(const int32_t *x, const int32_t *y, const int32_t *z, const int32_t *r,
                      int n, int U, uint64_t *out, hipStream_t s) {
    int64_t blocks = single_blocks(n, K, U);
    if (blocks > 0) k_count_i32<K><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, r, n, U, out);
}

template <int K>
void launch_count_f32(const float *x, const float *y, const float *z, const float *r, int n,
                      int U, uint64_t *out, hipStream_t s) {
    int64_t blocks = single_blocks(n, K, U);
    if (blocks > 0) k_count_f32<K><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, r, n, U, out);
}

template <int K>
void launch_energy(const float *x, const float *y, const float *z, int n, int U, float eps2,
                   double *E, double *total, hipStream_t s) {
    int64_t blocks = single_blocks(n, K, U);
    if (blocks <= 0) return;
    if (E)
        k_energy<K, true><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
    else
        k_energy<K, false><<<(unsigned)blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
}

// Resident blocks of one persistent batched kernel on the current device.
template <int KindV, typename Source>
int64_t persistent_blocks(const DeviceState *st) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<KindV, Source>, kBlock,
                                                     0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    return (int64_t)per_cu * (st->n_cu > 0 ? st->n_cu : 1);
}

template <typename Source>
pairs_status_t launch_batched(int kind, const BatchIO &io, const Source &src,
                              const ClassTable &ct, int64_t max_tasks, hipStream_t s) {
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    int64_t blocks;
    switch (kind) {
        case kCountI32: blocks = persistent_blocks<kCountI32, Source>(st); break;
        case kCountF32: blocks = persistent_blocks<kCountF32, Source>(st); break;
        default: blocks = persistent_blocks<kEnergyF32, Source>(st); break;
    }
    if (max_tasks >= 0)
        blocks = std::min(blocks, (max_tasks + kWavesPerBlock - 1) / kWavesPerBlock);
    if (blocks <= 0) return PAIRS_OK;
    switch (kind) {
        case kCountI32:
            k_batched<kCountI32, Source><<<(unsigned)blocks, kBlock, 0, s>>>(io, src, ct);
            break;
        case kCountF32:
            k_batched<kCountF32, Source><<<(unsigned)blocks, kBlock, 0, s>>>(io, src, ct);
            break;
        default:
            k_batched<kEnergyF32, Source><<<(unsigned)blocks, kBlock, 0, s>>>(io, src, ct);
            break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t batched_ws_bytes(int64_t n_sets) {
    return align256(sizeof(int64_t) * (kMaxClasses + 1)) +
           align256(sizeof(int64_t) * (size_t)kMaxClasses * (size_t)(n_sets + 1));
}

pairs_status_t batched_common(int kind, const BatchIO &io, int64_t n_sets, void *ws,
                              size_t ws_bytes, hipStream_t s) {
    if (!ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    unsigned char *p = (unsigned char *)ws;
    int64_t *bases = (int64_t *)p;
    p += align256(sizeof(int64_t) * (kMaxClasses + 1));
    int64_t *coff = (int64_t *)p;
    const ClassTable ct = default_classes();
    k_batch_schedule<<<1, kSchedThreads, 0, s>>>(io.off, n_sets, io.n_total, ct, coff, bases);
    PAIRS_HIP_CHECK(hipGetLastError());
    ScanSource src{bases, coff, n_sets, ct.count};
    return launch_batched(kind, io, src, ct, -1, s);
}

pairs_status_t batched_args(const void *x, const void *y, const void *z,
                            const int64_t *d_offsets, int64_t n_sets, int64_t n_total,
                            unsigned flags) {
    if (n_sets < 0 || n_total < 0 || !d_offsets || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (n_sets >= INT32_MAX) return PAIRS_ERR_INVALID_ARG;
    if (n_total > 0 && (!x || !y || !z)) return PAIRS_ERR_INVALID_ARG;
    return PAIRS_OK;
}

}  // namespace

// ------------------------------------------------------------------- plans --

struct pairs_plan_s {
    int kind;
    int device;
    int64_t n_sets;
    int64_t n_total;
    int64_t ntasks;
    ClassTable classes;
    int64_t *d_offsets;
    int2 *d_tasks;
};

struct pairs_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int device;
};

// ------------------------------------------------------------ public ABI --

extern "C" {

pairs_status_t pairs_count_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                               const int32_t *r, int64_t n, uint64_t *d_count, unsigned flags,
                               pairs_stream_t stream) {
    if (!d_count || n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z || !r)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) PAIRS_TRY(validate_i32(x, y, z, r, n, s));
    PAIRS_TRY(fill_u64(d_count, 1, 0, s));
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
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) PAIRS_TRY(validate_f32(x, y, z, r, n, s));
    PAIRS_TRY(fill_u64(d_count, 1, 0, s));
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
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) PAIRS_TRY(validate_f32(x, y, z, nullptr, n, s));
    PAIRS_TRY(fill_f64(d_total, 1, 0.0, s));
    PAIRS_TRY(fill_f64(d_energy, n, 0.0, s));
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

pairs_status_t pairs_batched_workspace_size(int64_t n_sets, int64_t n_total, size_t *bytes) {
    if (!bytes || n_sets < 0 || n_total < 0 || n_sets >= INT32_MAX) return PAIRS_ERR_INVALID_ARG;
    *bytes = batched_ws_bytes(n_sets);
    return PAIRS_OK;
}

pairs_status_t pairs_count_i32_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                                       const int32_t *r, const int64_t *d_offsets, int64_t n_sets,
                                       int64_t n_total, uint64_t *d_counts, void *d_ws,
                                       size_t ws_bytes, unsigned flags, pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags));
    if ((n_sets > 0 && !d_counts) || (n_total > 0 && !r)) return PAIRS_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
        PAIRS_TRY(validate_i32(x, y, z, r, n_total, s));
    }
    PAIRS_TRY(fill_u64(d_counts, n_sets, 0, s));
    if (n_sets == 0) return PAIRS_OK;
    BatchIO io{x, y, z, r, d_offsets, n_total, d_counts, nullptr, 0.0f};
    return batched_common(kCountI32, io, n_sets, d_ws, ws_bytes, s);
}

pairs_status_t pairs_count_f32_batched(const float *x, const float *y, const float *z,
                                       const float *r, const int64_t *d_offsets, int64_t n_sets,
                                       int64_t n_total, uint64_t *d_counts, void *d_ws,
                                       size_t ws_bytes, unsigned flags, pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags));
    if ((n_sets > 0 && !d_counts) || (n_total > 0 && !r)) return PAIRS_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
        PAIRS_TRY(validate_f32(x, y, z, r, n_total, s));
    }
    PAIRS_TRY(fill_u64(d_counts, n_sets, 0, s));
    if (n_sets == 0) return PAIRS_OK;
    BatchIO io{x, y, z, r, d_offsets, n_total, d_counts, nullptr, 0.0f};
    return batched_common(kCountF32, io, n_sets, d_ws, ws_bytes, s);
}

pairs_status_t pairs_energy_f32_batched(const float *x, const float *y, const float *z,
                                        const float *r, const int64_t *d_offsets, int64_t n_sets,
                                        int64_t n_total, float eps2, double *d_set_energy,
                                        uint64_t *d_set_counts, void *d_ws, size_t ws_bytes,
                                        unsigned flags, pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags));
    if (!(eps2 > 0.0f) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
    if (n_sets > 0 && !d_set_energy) return PAIRS_ERR_INVALID_ARG;
    if ((r == nullptr) != (d_set_counts == nullptr)) return PAIRS_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
        PAIRS_TRY(validate_f32(x, y, z, r, n_total, s));
    }
    PAIRS_TRY(fill_f64(d_set_energy, n_sets, 0.0, s));
    PAIRS_TRY(fill_u64(d_set_counts, n_sets, 0, s));
    if (n_sets == 0) return PAIRS_OK;
    BatchIO io{x, y, z, r, d_offsets, n_total, d_set_counts, d_set_energy, eps2};
    return batched_common(kEnergyF32, io, n_sets, d_ws, ws_bytes, s);
}

pairs_status_t pairs_plan_create(int kind, const int64_t *h_offsets, int64_t n_sets,
                                 pairs_plan_t *out) {
    if (!out) return PAIRS_ERR_INVALID_ARG;
    *out = nullptr;
    if (kind != PAIRS_KIND_COUNT_I32 && kind != PAIRS_KIND_COUNT_F32 &&
        kind != PAIRS_KIND_ENERGY_F32)
        return PAIRS_ERR_INVALID_ARG;
    if (n_sets < 0 || n_sets >= INT32_MAX || !h_offsets) return PAIRS_ERR_INVALID_ARG;
    if (h_offsets[0] != 0) return PAIRS_ERR_INVALID_ARG;
    for (int64_t s = 0; s < n_sets; ++s) {
        int64_t m = h_offsets[s + 1] - h_offsets[s];
        if (m < 0 || m > PAIRS_MAX_BATCH_SET_SIZE) return PAIRS_ERR_INVALID_ARG;
    }
    int dev;
    PAIRS_TRY(current_device(&dev));
    const ClassTable ct = default_classes();
    // tasks of class 0 (largest sets) first, then class 1, ...
    std::vector<int64_t> per_class(ct.count, 0);
    for (int64_t s = 0; s < n_sets; ++s) {
        int n = (int)(h_offsets[s + 1] - h_offsets[s]);
        if (n < 2) continue;
        int c = ct.class_of(n);
        per_class[c] += ct.tasks(n, c);
    }
    int64_t ntasks = 0;
    std::vector<int64_t> cursor(ct.count, 0);
    for (int c = 0; c < ct.count; ++c) {
        cursor[c] = ntasks;
        ntasks += per_class[c];
    }
    if (ntasks >= INT32_MAX) return PAIRS_ERR_INVALID_ARG;
    std::vector<int2> table;
    try {
        table.resize((size_t)ntasks);
    } catch (const std::bad_alloc &) {
        return PAIRS_ERR_NO_MEMORY;
    }
    for (int64_t s = 0; s < n_sets; ++s) {
        int n = (int)(h_offsets[s + 1] - h_offsets[s]);
        if (n < 2) continue;
        int c = ct.class_of(n);
        int64_t m = ct.tasks(n, c);
        for (int64_t l = 0; l < m; ++l) table[(size_t)cursor[c]++] = make_int2((int)s, (int)l);
    }
    pairs_plan_s *p = new (std::nothrow) pairs_plan_s();
    if (!p) return PAIRS_ERR_NO_MEMORY;
    p->kind = kind;
    p->device = dev;
    p->n_sets = n_sets;
    p->n_total = h_offsets[n_sets];
    p->ntasks = ntasks;
    p->classes = ct;
    p->d_offsets = nullptr;
    p->d_tasks = nullptr;
    hipError_t e = hipMalloc(&p->d_offsets, sizeof(int64_t) * (size_t)(n_sets + 1));
    if (e == hipSuccess && ntasks > 0) e = hipMalloc(&p->d_tasks, sizeof(int2) * (size_t)ntasks);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_offsets, h_offsets, sizeof(int64_t) * (size_t)(n_sets + 1),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && ntasks > 0)
        e = hipMemcpy(p->d_tasks, table.data(), sizeof(int2) * (size_t)ntasks,
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_offsets) hipFree(p->d_offsets);
        if (p->d_tasks) hipFree(p->d_tasks);
        delete p;
        g_last_hip_error = e;
        return e == hipErrorOutOfMemory ? PAIRS_ERR_NO_MEMORY : PAIRS_ERR_HIP;
    }
    *out = p;
    return PAIRS_OK;
}

pairs_status_t pairs_plan_info(pairs_plan_t plan, int64_t *n_sets, int64_t *n_total,
                               int64_t *n_tasks) {
    if (!plan) return PAIRS_ERR_INVALID_ARG;
    if (n_sets) *n_sets = plan->n_sets;
    if (n_total) *n_total = plan->n_total;
    if (n_tasks) *n_tasks = plan->ntasks;
    return PAIRS_OK;
}

pairs_status_t pairs_plan_execute(pairs_plan_t plan, const void *const *in, void *const *out,
                                  float eps2, pairs_stream_t stream) {
    if (!plan || !in || !out) return PAIRS_ERR_INVALID_ARG;
    int dev;
    PAIRS_TRY(current_device(&dev));
    if (dev != plan->device) return PAIRS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    BatchIO io{};
    io.x = in[0];
    io.y = in[1];
    io.z = in[2];
    io.r = in[3];
    io.off = plan->d_offsets;
    io.n_total = plan->n_total;
    if (plan->n_total > 0 && (!io.x || !io.y || !io.z)) return PAIRS_ERR_INVALID_ARG;
    if (plan->kind == PAIRS_KIND_ENERGY_F32) {
        if (!(eps2 > 0.0f) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
        io.energy = (double *)out[0];
        io.counts = (uint64_t *)out[1];
        io.eps2 = eps2;
        if (plan->n_sets > 0 && !io.energy) return PAIRS_ERR_INVALID_ARG;
        if ((io.r == nullptr) != (io.counts == nullptr)) return PAIRS_ERR_INVALID_ARG;
        PAIRS_TRY(fill_f64(io.energy, plan->n_sets, 0.0, s));
        PAIRS_TRY(fill_u64(io.counts, plan->n_sets, 0, s));
    } else {
        io.counts = (uint64_t *)out[0];
        if (plan->n_sets > 0 && !io.counts) return PAIRS_ERR_INVALID_ARG;
        if (plan->n_total > 0 && !io.r) return PAIRS_ERR_INVALID_ARG;
        PAIRS_TRY(fill_u64(io.counts, plan->n_sets, 0, s));
    }
    if (plan->ntasks == 0) return PAIRS_OK;
    TableSource src{plan->d_tasks, plan->ntasks};
    int kind = plan->kind == PAIRS_KIND_COUNT_I32   ? kCountI32
               : plan->kind == PAIRS_KIND_COUNT_F32 ? kCountF32
                                                    : kEnergyF32;
    return launch_batched(kind, io, src, plan->classes, plan->ntasks, s);
}

pairs_status_t pairs_plan_destroy(pairs_plan_t plan) {
    if (!plan) return PAIRS_OK;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(plan->device);
    if (plan->d_offsets) hipFree(plan->d_offsets);
    if (plan->d_tasks) hipFree(plan->d_tasks);
    hipSetDevice(cur);
    delete plan;
    return PAIRS_OK;
}

pairs_status_t pairs_jitter_f32(float *x, float *y, float *z, int64_t n, uint64_t seed,
                                uint32_t step, float sigma, int64_t first_index,
                                pairs_stream_t stream) {
    if (n < 0 || (n > 0 && (!x || !y || !z)) || !(sigma >= 0.0f) || !isfinite(sigma) ||
        first_index < 0 || first_index + n > ((int64_t)1 << 32))
        return PAIRS_ERR_INVALID_ARG;
    int dev;
    PAIRS_TRY(current_device(&dev));
    if (n == 0) return PAIRS_OK;
    hipStream_t s = (hipStream_t)stream;
    const float scale = (float)((double)sigma / sqrt(4.0 / 3.0 * (ldexp(1.0, 48) - 1.0)));
    k_jitter<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, n, (uint32_t)seed,
                                                (uint32_t)(seed >> 32), step, scale, first_index);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t pairs_plan_capture_steps(pairs_plan_t plan, float *x, float *y, float *z,
                                        const float *r, uint64_t seed, float sigma,
                                        uint32_t first_step, int n_steps, float eps2,
                                        double *d_energy, uint64_t *d_counts,
                                        pairs_graph_t *out) {
    if (!out) return PAIRS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!plan || plan->kind != PAIRS_KIND_ENERGY_F32 || n_steps <= 0 || !d_energy)
        return PAIRS_ERR_INVALID_ARG;
    if ((r == nullptr) != (d_counts == nullptr)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    PAIRS_TRY(current_device(&dev));
    if (dev != plan->device) return PAIRS_ERR_INVALID_ARG;
    DeviceState *dst;
    PAIRS_TRY(device_state(&dst));  // any one-time set-up happens outside the capture
    hipStream_t cs;
    PAIRS_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    pairs_status_t st = PAIRS_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        hipStreamDestroy(cs);
        return hip_fail(e);
    }
    for (int k = 0; k < n_steps && st == PAIRS_OK; ++k) {
        st = pairs_jitter_f32(x, y, z, plan->n_total, seed, first_step + (uint32_t)k, sigma, 0,
                              cs);
        if (st != PAIRS_OK) break;
        const void *in[4] = {x, y, z, r};
        void *o[2] = {d_energy + (int64_t)k * plan->n_sets,
                      d_counts ? d_counts + (int64_t)k * plan->n_sets : nullptr};
        st = pairs_plan_execute(plan, in, o, eps2, cs);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    hipStreamDestroy(cs);
    if (st != PAIRS_OK) {
        if (g) hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e);
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return hip_fail(e);
    }
    pairs_graph_s *pg = new (std::nothrow) pairs_graph_s{g, ex, dev};
    if (!pg) {
        hipGraphExecDestroy(ex);
        hipGraphDestroy(g);
        return PAIRS_ERR_NO_MEMORY;
    }
    *out = pg;
    return PAIRS_OK;
}

pairs_status_t pairs_graph_launch(pairs_graph_t graph, pairs_stream_t stream) {
    if (!graph) return PAIRS_ERR_INVALID_ARG;
    PAIRS_HIP_CHECK(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return PAIRS_OK;
}

pairs_status_t pairs_graph_destroy(pairs_graph_t graph) {
    if (!graph) return PAIRS_OK;
    hipGraphExecDestroy(graph->exec);
    hipGraphDestroy(graph->graph);
    delete graph;
    return PAIRS_OK;
}

pairs_status_t pairs_debug_task_ranges(int n, int rows_per_lane, int chunk, int32_t *out,
                                       int64_t capacity, int64_t *n_tasks) {
    if (n < 0 || !n_tasks ||
        (rows_per_lane != 1 && rows_per_lane != 2 && rows_per_lane != 4 && rows_per_lane != 8) ||
        chunk <= 0 || chunk % 64 != 0)
        return PAIRS_ERR_INVALID_ARG;
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, rows_per_lane, chunk);
    *n_tasks = til.tasks();
    if (!out) return PAIRS_OK;
    if (capacity < til.tasks()) return PAIRS_ERR_WORKSPACE;
    int64_t k = 0;
    for (int b = 0; b < til.nblocks; ++b)
        for (int c = 0; c < til.nchunks; ++c, ++k) {
            int ra, u0, u1;
            task_range(band, til, b, c, &ra, &u0, &u1);
            out[3 * k] = ra;
            out[3 * k + 1] = u0;
            out[3 * k + 2] = u1;
        }
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
