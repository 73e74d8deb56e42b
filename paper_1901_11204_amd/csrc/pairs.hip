// libpairs: all-pairs interactions within sets of objects, for gfx950.
//
// Kernels (the wave-task bodies are in tasks.h and steps.h):
//   single set : tasks (row block x partner chunk) enumerated row block by
//                chunk; each wave takes tasks with a grid stride over the
//                64-bit task index;
//   batched    : persistent grids.  A plan gives each wave a task list
//                balanced on the host (longest processing time first); an
//                unplanned call builds a class-major task prefix and a
//                bucket table on the device (four small kernels) and the
//                waves take tasks with a grid stride;
//   jitter     : the per-step perturbation of the repeated-step workload;
//   lattice    : collision and contact counts of lattice beads (lattice.h);
//   binned     : counts through a uniform grid of cells, objects grouped by
//                cell through a hash table (binning.h);
//   helpers    : fills (in place of memsets, so every launch can be
//                captured into a graph), validation, fixed-point finishes.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <type_traits>
#include <utility>
#include <mutex>
#include <new>
#include <vector>


#include "band.h"
#include "binning.h"
#include "device.h"
#include "lattice.h"
#include "mfma.h"
#include "pairs.h"
#include "steps.h"
#include "tasks.h"

using namespace pairs_dev;

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
// The batched kernels run one wave per workgroup: a wave's LDS window is its
// workgroup's, so a wave that finishes early frees its slot at once rather
// than when the slowest wave of a four-wave workgroup is done (the unplanned
// count of 200 000 binned sets of lognormal sizes: 1.49 -> 1.43 ms).
constexpr int kBatchWaves = 1;
constexpr int kBatchBlock = kWave * kBatchWaves;
// The wave's index in a batched kernel's workgroup.  With one wave per
// workgroup it is the constant 0, which keeps the wave's LDS window at a
// fixed address: the sweeps' LDS reads then take their addresses with no
// per-iteration add of a window base.
__device__ __forceinline__ int batch_wave() { return kBatchWaves == 1 ? 0 : wave_id(); }

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
    int form[kMaxClasses];  // PAIRS_FORM_*

    __host__ __device__ int class_of(int n) const {
        for (int c = 0; c < count - 1; ++c)
            if (n > lo[c]) return c;
        return count - 1;
    }
    __host__ __device__ int64_t tasks(int n, int c) const {
        if (form[c] == PAIRS_FORM_STEPPING)
            return StepTiling::of(Band::of(n), K[c], U[c]).tasks();
        return Tiling::of(Band::of(n), K[c], U[c]).tasks();
    }
};

ClassTable make_table(int count, const int *lo, const int *K, const int *U, const int *form) {
    ClassTable t;
    t.count = count;
    for (int c = 0; c < kMaxClasses; ++c) {
        t.lo[c] = c < count ? lo[c] : 0;
        t.K[c] = c < count ? K[c] : 1;
        t.U[c] = c < count ? U[c] : 64;
        t.form[c] = c < count && form ? form[c] : PAIRS_FORM_BROADCAST;
    }
    return t;
}

// Shape-table modes: single-set calls, batched calls and plans, and
// single-set float32 energies without per-object output.
constexpr int kModeSingle = 0, kModeBatched = 1, kModeTotalOnly = 2, kShapeModes = 3;

// Default tile shapes by kind (index kind - 1) and mode.
ClassTable default_table(int kind, int mode) {
    if (mode == kModeTotalOnly) {
        // a total alone has no partner-side sums to amortise over the rows
        // of a lane, so large sets run one row per lane (measured by
        // autotune.tune_single at n = 4096, 16384, 262144 and 2^20); long
        // chunks keep the per-task atomics on the total few
        const int lo[4] = {65536, 16384, 4096, 0}, K[4] = {1, 1, 2, 4},
                  U[4] = {2048, 2048, 512, 128};
        return make_table(4, lo, K, U, nullptr);
    }
    const bool batched = mode == kModeBatched;
    if (batched) {
        const int lo[4] = {4096, 1024, 256, 0}, K[4] = {2, 2, 2, 2},
                  U[4] = {272, 272, 272, 272},
                  form[4] = {PAIRS_FORM_STEPPING, PAIRS_FORM_STEPPING, PAIRS_FORM_STEPPING,
                             PAIRS_FORM_STEPPING};
        return make_table(4, lo, K, U, form);
    }
    // single sets: measured on MI355X by autotune.tune_single at n = 4096,
    // 16384, 65536 and 262144 (the largest class is the N = 2^20 optimum);
    // with tasks in row-block groups (task_at_grouped) the largest classes
    // gain a little from longer chunks
    if (kind == PAIRS_KIND_ENERGY_F32) {
        const int lo[4] = {65536, 16384, 4096, 0}, K[4] = {8, 8, 4, 4},
                  U[4] = {1024, 128, 128, 64};
        return make_table(4, lo, K, U, nullptr);
    }
    const int lo[4] = {524288, 65536, 8192, 0}, K[4] = {8, 4, 4, 1},
              U[4] = {2048, 512, 128, 64};
    return make_table(4, lo, K, U, nullptr);
}

// Largest step chunk of a stepping task with K rows per lane: a row block's
// window (64 K + chunk + K records) must fit the wave's window capacity.
__host__ __device__ constexpr int step_max_chunk(int K) { return K == 1 ? 288 : 272; }
// (a chunk of U steps has T + x <= U: the extra step only joins a short chunk)
static_assert(1 * step_window_entries(1, 64, 287, 1) <= kStepCap, "K=1 window fits");
static_assert(2 * step_window_entries(2, 64, 271, 1) <= kStepCap, "K=2 window fits");
static_assert(step_window_entries(1, 64, 287, 1) <= 64 * step_iters<1>(), "K=1 staging slots");
static_assert(step_window_entries(2, 64, 271, 1) <= 64 * step_iters<2>(), "K=2 staging slots");

std::mutex g_shape_mutex;
ClassTable g_shapes[3][kShapeModes];
bool g_shapes_set[3][kShapeModes];

ClassTable shapes(int kind, int mode) {
    std::lock_guard<std::mutex> lock(g_shape_mutex);
    return g_shapes_set[kind - 1][mode] ? g_shapes[kind - 1][mode] : default_table(kind, mode);
}

bool valid_table(const ClassTable &t, bool batched, int kind) {
    if (t.count < 1 || t.count > kMaxClasses) return false;
    for (int c = 0; c < t.count; ++c) {
        if (t.lo[c] < 0 || (c > 0 && t.lo[c] >= t.lo[c - 1])) return false;
        if (t.form[c] == PAIRS_FORM_MATRIX) {
            // single-set exact int32 counts only: 64-row tasks
            if (batched || kind != PAIRS_KIND_COUNT_I32 || t.K[c] != 1) return false;
            if (t.U[c] < 64 || t.U[c] % 64 != 0 || t.U[c] > (1 << 22)) return false;
        } else if (t.form[c] == PAIRS_FORM_STEPPING) {
            if (!batched || (t.K[c] != 1 && t.K[c] != 2)) return false;
            if (t.U[c] < 16 || t.U[c] % 16 != 0 || t.U[c] > step_max_chunk(t.K[c])) return false;
        } else if (t.form[c] == PAIRS_FORM_BROADCAST) {
            if (t.K[c] != 1 && t.K[c] != 2 && t.K[c] != 4 && t.K[c] != 8) return false;
            // a task's count (at most 64 K U pairs) stays below 2^32
            if (t.U[c] < 64 || t.U[c] % 64 != 0 || t.U[c] > (1 << 22)) return false;
        } else {
            return false;
        }
    }
    return true;
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

// Finishing passes of the fixed-point sums: the integer held in each 8-byte
// word back to a double (one rounding; the scale is a power of two).
__global__ void k_fixed_finish(double *p, int64_t n, double inv_scale) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (double)__double_as_longlong(p[i]) * inv_scale;
}

__global__ void k_validate_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                               const int32_t *r, int64_t n, int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t lo = PAIRS_I32_COORD_MIN, hi = PAIRS_I32_COORD_MAX;
    bool ok = x[i] >= lo && x[i] <= hi && y[i] >= lo && y[i] <= hi && z[i] >= lo && z[i] <= hi &&
              r[i] >= 0 && r[i] <= PAIRS_I32_RADIUS_MAX;
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

__global__ void k_validate_f64(const double *x, const double *y, const double *z, int64_t n,
                               int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) atomicOr(bad, 1);
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
//
// A single-set launch enumerates the tiling's tasks row block by chunk.  Up to
// kMaxSingleBlocks blocks each wave runs one task; a larger tiling keeps that
// grid and its waves take tasks with a grid stride over the 64-bit task
// index, so every set size up to PAIRS_MAX_SET_SIZE launches within the
// dispatch limit of 2^32 work-items.

constexpr int64_t kMaxSingleBlocks = (int64_t)1 << 22;

// The dispatcher deals workgroups to gfx950's eight XCDs in turn (workgroup w
// to XCD w % 8), and each XCD has an L2 cache of its own.  Numbering the
// workgroups XCD by XCD gives each XCD one contiguous range of the task
// order, so tasks that share partners share an L2.  A bijection on
// [0, blocks): XCDs x < blocks % 8 hold one workgroup more than the others.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_major_block(int64_t w, int64_t blocks) {
    const int64_t q = blocks / kXcds, r = blocks % kXcds, x = w % kXcds, i = w / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Runs f(ra, u0, u1) for every non-empty task of the tiling owned by the
// calling wave, in the grouped order of task_at_grouped.
template <typename F>
__device__ __forceinline__ void for_each_task(const Band &band, const Tiling &til, F &&f) {
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t ntasks = til.tasks();
    for (int64_t task = xcd_major_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_id();
         task < ntasks; task += stride) {
        int ra, u0, u1;
        task_at_grouped(band, til, task, &ra, &u0, &u1);
        if (u0 < u1) f(ra, u0, u1);
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_count_i32(const int32_t *__restrict__ x,
                                                      const int32_t *__restrict__ y,
                                                      const int32_t *__restrict__ z,
                                                      const int32_t *__restrict__ r, int n,
                                                      int U, uint64_t *out) {
    __shared__ int64_t lds[kWavesPerBlock * kCountI32Lds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    for_each_task(band, til, [&](int ra, int u0, int u1) {
        TaskInputs<int32_t, K> in;
        load_task_inputs<int32_t, K, K, true>(x, y, z, r, 0, band, ra, u0, u1, in);
        uint32_t cnt = count_i32_task<K, K>(x, y, z, r, 0, band, ra, u0, u1,
                                            lds + wave * kCountI32Lds, in);
        if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
    });
}

// The exact int32 count with the Gram sums on the matrix cores (mfma.h):
// tasks of 64 rows (the broadcast tiling with one row per lane).
__global__ __launch_bounds__(kBlock) void k_count_i32_mfma(const int32_t *__restrict__ x,
                                                           const int32_t *__restrict__ y,
                                                           const int32_t *__restrict__ z,
                                                           const int32_t *__restrict__ r, int n,
                                                           int U, uint64_t *out) {
    __shared__ int64_t lds[kWavesPerBlock * kCountI32Lds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, 1, U);
    for_each_task(band, til, [&](int ra, int u0, int u1) {
        TaskInputs<int32_t, 1> in;
        load_task_inputs<int32_t, 1, 1, true>(x, y, z, r, 0, band, ra, u0, u1, in);
        const uint32_t cnt = count_i32_task_mfma(x, y, z, r, 0, band, ra, u0, u1,
                                                 lds + wave * kCountI32Lds, in);
        if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
    });
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
    for_each_task(band, til, [&](int ra, int u0, int u1) {
        TaskInputs<float, K> in;
        load_task_inputs<float, K, K, true>(x, y, z, r, 0, band, ra, u0, u1, in);
        uint32_t cnt = count_f32_task<K, K>(x, y, z, r, 0, band, ra, u0, u1,
                                            lds + wave * kCountF32Lds, in);
        if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)out, (unsigned long long)cnt);
    });
}

template <int K, bool PerObject>
__global__ __launch_bounds__(kBlock) void k_energy(const float *__restrict__ x,
                                                   const float *__restrict__ y,
                                                   const float *__restrict__ z, int n, int U,
                                                   float eps2, SumSink E, SumSink total) {
    __shared__ float lds[kWavesPerBlock * kEnergyLds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    for_each_task(band, til, [&](int ra, int u0, int u1) {
        TaskInputs<float, K> in;
        load_task_inputs<float, K, K, false>(x, y, z, nullptr, 0, band, ra, u0, u1, in);
        EnergyResult res = energy_task<K, K, PerObject, false>(
            x, y, z, nullptr, 0, band, ra, u0, u1, eps2, lds + wave * kEnergyLds, E, in);
        if (lane_id() == 0) total.add(0, res.energy);
    });
}

// The softened potential in double precision (energy64_task).
template <int K, bool PerObject>
__global__ __launch_bounds__(kBlock) void k_energy64(const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ z, int n, int U,
                                                     double eps2, SumSink E, SumSink total) {
    __shared__ double lds[kWavesPerBlock * kEnergy64Lds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    for_each_task(band, til, [&](int ra, int u0, int u1) {
        TaskInputs<double, K> in;
        load_task_inputs<double, K, K, false>(x, y, z, nullptr, 0, band, ra, u0, u1, in);
        const double e = energy64_task<K, PerObject>(x, y, z, 0, band, ra, u0, u1, eps2,
                                                     lds + wave * kEnergy64Lds, E, in);
        if (lane_id() == 0) total.add(0, e);
    });
}

// Forces of the softened potential on every object (force_task).
template <int K>
__global__ __launch_bounds__(kBlock) void k_force(const float *__restrict__ x,
                                                  const float *__restrict__ y,
                                                  const float *__restrict__ z, int n, int U,
                                                  float eps2, SumSink Fx, SumSink Fy, SumSink Fz) {
    __shared__ float lds[kWavesPerBlock * kForceLds];
    const int wave = wave_id();
    const Band band = Band::of(n);
    const Tiling til = Tiling::of(band, K, U);
    for_each_task(band, til, [&](int ra, int u0, int u1) {
        TaskInputs<float, K> in;
        load_task_inputs<float, K, K, false>(x, y, z, nullptr, 0, band, ra, u0, u1, in);
        force_task<K>(x, y, z, 0, band, ra, u0, u1, eps2, lds + wave * kForceLds, Fx, Fy, Fz,
                      in);
    });
}

// ---------------------------------------------------------- batched kernels --

// One wave task of a plan, resolved on the host.
//   broadcast form: set `set` (objects [base, base + n)), rows [a, a + 64K),
//     virtual partners [b, c);
//   stepping form, one row block: set `set` at base, rows [a, a + 64K), steps
//     [b, b + c) plus the extra step b + c when x is 1;
//   stepping form, a pack (set < 0): m whole sets of size n whose bases and
//     ids are the plan's pack entries [base, base + m); steps [b, b + c) and x.
struct TaskDesc {
    int64_t base;
    int32_t set;
    int32_t n;
    int32_t a;
    int32_t b;
    int32_t c;
    uint8_t K;
    uint8_t form;
    uint8_t m;
    uint8_t x;
};
static_assert(sizeof(TaskDesc) == 32, "one 32-byte scalar load per task");

// ------------------------------------------------------ unplanned schedule --
//
// An unplanned call schedules on the device.  It lists the sets that have
// pairs class by class (the largest sets first, set order within a class),
// with pre[j] the global index of the first task of listed set j, so the
// tasks of all sets form one range [0, T).  A bucket table maps every B-th
// task to its listed set (B = ceil(T / listed), so the table has at most
// `listed` + 1 entries and each bucket spans at most B + 1 listed sets): a
// wave finds the set of task t by one table lookup and a binary search over
// at most B + 1 entries of pre.
//
// The list is built by four kernels over blocks of kSchedBlock sets: class
// and task counts per block, a scan of the block counts (one block), the
// list and pre with block-local scans, and the bucket table.

constexpr int kSchedBlock = 1024;

// Workspace layout of an unplanned call of n_sets sets.
struct SchedLayout {
    size_t hdr, list, pre, tab, blk, total;
    int64_t nb;  // blocks of kSchedBlock sets
};

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr SchedLayout sched_layout(int64_t n_sets) {
    SchedLayout L{};
    const int64_t nb = (n_sets + kSchedBlock - 1) / kSchedBlock;
    size_t p = 0;
    L.hdr = p;
    p += 256;
    L.list = p;
    p += align256(4 * (size_t)n_sets);
    L.pre = p;
    p += align256(8 * (size_t)(n_sets + 1));
    L.tab = p;
    p += align256(4 * (size_t)(n_sets + 2));
    L.blk = p;
    p += align256(8 * 2 * kMaxClasses * (size_t)nb);
    L.nb = nb;
    L.total = p;
    return L;
}

// The header: class bases in the list and in the task range, and the totals.
struct SchedHeader {
    int64_t cbase[kMaxClasses + 1];  // first list index of each class
    int64_t tbase[kMaxClasses + 1];  // first task of each class
    int64_t T;                       // tasks in all
    int64_t listed;                  // sets with at least one task
    int64_t B;                       // tasks per bucket
    int64_t nbuckets;                // ceil(T / B)
};
static_assert(sizeof(SchedHeader) <= 256, "the header fits its slot");

// Class (or -1: no pairs) and task count of set s.
__device__ __forceinline__ int set_work(const int64_t *off, int64_t s, int64_t n_sets,
                                        int64_t n_total, const ClassTable &ct, int64_t *tasks) {
    *tasks = 0;
    if (s >= n_sets) return -1;
    int64_t b;
    int n;
    set_range(off, s, n_total, &b, &n);
    if (n < 2) return -1;
    const int c = ct.class_of(n);
    *tasks = ct.tasks(n, c);
    return *tasks > 0 ? c : -1;
}

// Per block: sets and tasks of each class (blk[b][c] and blk[b][kMaxClasses + c]).
__global__ __launch_bounds__(kSchedBlock) void k_sched_count(const int64_t *__restrict__ off,
                                                             int64_t n_sets, int64_t n_total,
                                                             ClassTable ct, int64_t *blk) {
    __shared__ unsigned long long acc[2 * kMaxClasses];
    if (threadIdx.x < 2 * kMaxClasses) acc[threadIdx.x] = 0;
    __syncthreads();
    int64_t t;
    const int c = set_work(off, (int64_t)blockIdx.x * kSchedBlock + threadIdx.x, n_sets, n_total,
                           ct, &t);
    if (c >= 0) {
        atomicAdd(&acc[c], 1ull);
        atomicAdd(&acc[kMaxClasses + c], (unsigned long long)t);
    }
    __syncthreads();
    if (threadIdx.x < 2 * kMaxClasses)
        blk[(int64_t)blockIdx.x * 2 * kMaxClasses + threadIdx.x] = (int64_t)acc[threadIdx.x];
}

// One block: exclusive scans of the block counts per class (in place), the
// class bases and the totals.
__global__ __launch_bounds__(kSchedBlock) void k_sched_scan(int64_t *blk, int64_t nb,
                                                            SchedHeader *hdr) {
    __shared__ int64_t wave_tot[kSchedBlock / kWave + 1];
    __shared__ int64_t total[2 * kMaxClasses];
    const int tid = threadIdx.x;
    const int64_t chunk = (nb + kSchedBlock - 1) / kSchedBlock;
    const int64_t b0 = min((int64_t)tid * chunk, nb), b1 = min(b0 + chunk, nb);
    for (int q = 0; q < 2 * kMaxClasses; ++q) {
        int64_t sum = 0;
        for (int64_t b = b0; b < b1; ++b) sum += blk[b * 2 * kMaxClasses + q];
        // exclusive scan of the thread sums across the block (wave shuffles,
        // then the wave totals)
        int64_t tot;
        int64_t run = block_exclusive_scan<kSchedBlock>(sum, wave_tot, &tot);
        if (tid == 0) total[q] = tot;
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t v = blk[b * 2 * kMaxClasses + q];
            blk[b * 2 * kMaxClasses + q] = run;
            run += v;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int64_t ls = 0, ts = 0;
        for (int c = 0; c < kMaxClasses; ++c) {
            hdr->cbase[c] = ls;
            hdr->tbase[c] = ts;
            ls += total[c];
            ts += total[kMaxClasses + c];
        }
        hdr->cbase[kMaxClasses] = ls;
        hdr->tbase[kMaxClasses] = ts;
        hdr->T = ts;
        hdr->listed = ls;
        const int64_t B = ls > 0 ? max((int64_t)1, (ts + ls - 1) / ls) : 1;
        hdr->B = B;
        hdr->nbuckets = (ts + B - 1) / B;
    }
}

// The list and the task prefixes.
__global__ __launch_bounds__(kSchedBlock) void k_sched_list(
    const int64_t *__restrict__ off, int64_t n_sets, int64_t n_total, ClassTable ct,
    const int64_t *__restrict__ blk, const SchedHeader *__restrict__ hdr,
    int32_t *__restrict__ list, int64_t *__restrict__ pre) {
    __shared__ int64_t wave_tot[kSchedBlock / kWave + 1];
    const int64_t s = (int64_t)blockIdx.x * kSchedBlock + threadIdx.x;
    int64_t t;
    const int c = set_work(off, s, n_sets, n_total, ct, &t);
    const int64_t *bb = blk + (int64_t)blockIdx.x * 2 * kMaxClasses;
    for (int q = 0; q < kMaxClasses; ++q) {
        int64_t sum;
        const int64_t rank = block_exclusive_scan<kSchedBlock>(c == q ? 1 : 0, wave_tot, &sum);
        const int64_t tpre = block_exclusive_scan<kSchedBlock>(c == q ? t : 0, wave_tot, &sum);
        if (c == q) {
            const int64_t j = hdr->cbase[q] + bb[q] + rank;
            list[j] = (int32_t)s;
            pre[j] = hdr->tbase[q] + bb[kMaxClasses + q] + tpre;
        }
    }
    if (s == 0) pre[hdr->listed] = hdr->T;
}

// The bucket table: tab[k] = the listed set holding task k B; a sentinel
// tab[nbuckets] = listed - 1.
__global__ void k_sched_tab(const int64_t *__restrict__ pre, const SchedHeader *__restrict__ hdr,
                            int32_t *__restrict__ tab) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nbk = hdr->nbuckets, listed = hdr->listed;
    if (k > nbk) return;
    if (k == nbk) {
        tab[k] = (int32_t)max((int64_t)0, listed - 1);
        return;
    }
    const int64_t t = k * hdr->B;
    int64_t lo = 0, hi = listed;  // pre[lo] <= t < pre[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    tab[k] = (int32_t)lo;
}

// Task source of an unplanned call, read by the scan kernels.
struct ScanSource {
    const SchedHeader *hdr;
    const int32_t *list;
    const int64_t *pre;
    const int32_t *tab;

    // Set (listed index j) and local task of global task t.
    __device__ __forceinline__ void decode(int64_t t, int64_t B, int64_t *set, int *local) const {
        const int64_t b = t / B;
        int64_t lo = tab[b], hi = (int64_t)tab[b + 1] + 1;  // pre[lo] <= t < pre[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (pre[mid] <= t) lo = mid; else hi = mid;
        }
        *set = list[lo];
        *local = (int)(t - pre[lo]);
    }
};

enum Kind { kCountI32 = 1, kCountF32 = 2, kEnergyF32 = 3 };

// LDS of one wave of the batched kernels, in bytes, for each kind: the larger
// of the broadcast window and the stepping window.
constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <int KindV>
constexpr int batched_lds_bytes() {
    return KindV == kCountI32 ? cmax(kCountI32Lds * 8, kStepCap * 24)
           : KindV == kCountF32 ? cmax(kCountF32Lds * 4, kStepCap * 16)
                                : cmax(kEnergyLds * 4, kStepCap * 16);
}
static_assert(batched_lds_bytes<kCountI32>() % 16 == 0 && batched_lds_bytes<kCountF32>() % 16 == 0 &&
                  batched_lds_bytes<kEnergyF32>() % 16 == 0,
              "LDS windows keep 16-byte alignment");

struct BatchIO {
    const void *x, *y, *z, *r;  // object arrays (r may be null for energies)
    const int64_t *off;
    int64_t n_total;
    uint64_t *counts;  // [n_sets] or null
    double *energy;    // [n_sets] (energies)
    float eps2;
    const int64_t *pack_base;  // plans: first object of each packed set
    const int32_t *pack_set;   // plans: id of each packed set
    double emax;               // > 0: fixed-point set energies (bound on one term)
};

// The sets' fixed-point energies back to doubles, each with its set's scale.
__global__ void k_finish_sets(double *E, const int64_t *off, int64_t n_sets, int64_t n_total,
                              double emax) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    int64_t b;
    int n;
    set_range(off, s, n_total, &b, &n);
    E[s] = (double)__double_as_longlong(E[s]) / fixed_scale(0.5 * n * (n - 1.0) * emax);
}

// Adds e to the energy of set `set` of n objects: a double atomic, or with
// io.emax > 0 a fixed-point one whose scale follows from the bound
// n (n - 1) / 2 * emax on the set's sum (k_finish_sets uses the same).
__device__ __forceinline__ void add_set_energy(const BatchIO &io, int64_t set, int n, double e) {
    const double scale = io.emax > 0.0 ? fixed_scale(0.5 * n * (n - 1.0) * io.emax) : 0.0;
    SumSink{io.energy, scale}.add(set, e);
}

// Object type of a kind.
template <int KindV>
using ObjT = typename std::conditional<KindV == kCountI32, int32_t, float>::type;

// Loads the inputs of a task of shape K (K <= KM); radii are loaded when the
// batch has them.
template <int K, int KM, int KindV>
__device__ __forceinline__ void batched_inputs(const BatchIO &io, int64_t base, const Band &band,
                                               int ra, int u0, int u1,
                                               TaskInputs<ObjT<KindV>, KM> &in) {
    using T = ObjT<KindV>;
    if (io.r)
        load_task_inputs<T, K, KM, true>((const T *)io.x, (const T *)io.y, (const T *)io.z,
                                         (const T *)io.r, base, band, ra, u0, u1, in);
    else
        load_task_inputs<T, K, KM, false>((const T *)io.x, (const T *)io.y, (const T *)io.z,
                                          nullptr, base, band, ra, u0, u1, in);
}

template <int K, int KM, int KindV>
__device__ __forceinline__ void batched_task(const BatchIO &io, int64_t base, const Band &band,
                                             int ra, int u0, int u1, int64_t set, void *win,
                                             const TaskInputs<ObjT<KindV>, KM> &in) {
    if constexpr (KindV == kCountI32) {
        uint32_t c = count_i32_task<K, KM>((const int32_t *)io.x, (const int32_t *)io.y,
                                           (const int32_t *)io.z, (const int32_t *)io.r, base,
                                           band, ra, u0, u1, win,
                                           in);
        if (lane_id() == 0 && c)
            atomicAdd((unsigned long long *)&io.counts[set], (unsigned long long)c);
    } else if constexpr (KindV == kCountF32) {
        uint32_t c = count_f32_task<K, KM>((const float *)io.x, (const float *)io.y,
                                           (const float *)io.z, (const float *)io.r, base, band,
                                           ra, u0, u1, (float *)win,
                                           in);
        if (lane_id() == 0 && c)
            atomicAdd((unsigned long long *)&io.counts[set], (unsigned long long)c);
    } else {
        EnergyResult res;
        if (io.r)
            res = energy_task<K, KM, false, true>((const float *)io.x, (const float *)io.y,
                                                  (const float *)io.z, (const float *)io.r, base,
                                                  band, ra, u0, u1, io.eps2, (float *)win,
                                                  SumSink{nullptr, 0.0}, in);
        else
            res = energy_task<K, KM, false, false>((const float *)io.x, (const float *)io.y,
                                                   (const float *)io.z, nullptr, base, band, ra,
                                                   u0, u1, io.eps2, (float *)win,
                                                   SumSink{nullptr, 0.0}, in);
        if (lane_id() == 0) {
            add_set_energy(io, set, band.n, res.energy);
            if (io.r && res.count)
                atomicAdd((unsigned long long *)&io.counts[set], (unsigned long long)res.count);
        }
    }
}

template <int K, int KindV>
__device__ __forceinline__ void run_shape(const BatchIO &io, int64_t base, const Band &band,
                                          int ra, int u0, int u1, int64_t set, void *win) {
    TaskInputs<ObjT<KindV>, K> in;
    batched_inputs<K, K, KindV>(io, base, band, ra, u0, u1, in);
    batched_task<K, K, KindV>(io, base, band, ra, u0, u1, set, win, in);
}

// Per-lane view of a stepping task's sets: the first object of the lane's
// own segment, and (packs) the set whose totals lane j < m reports.
struct StepSets {
    int64_t base;
    int64_t out_set;
};

__device__ __forceinline__ StepSets step_sets(const BatchIO &io, const TaskDesc &d) {
    StepSets s;
    if (d.set >= 0) {
        s.base = d.base;
        s.out_set = d.set;
        return s;
    }
    const int lane = lane_id();
    const int w = (d.n + d.K - 1) / d.K;
    const int j = lane / w < d.m ? lane / w : 0;
    s.base = io.pack_base[d.base + j];
    s.out_set = lane < d.m ? (int64_t)io.pack_set[d.base + lane] : 0;
    return s;
}

__device__ __forceinline__ StepGeom desc_geom(const TaskDesc &d) {
    return step_geom(d.n, d.K, d.a, d.b, d.c, d.x, d.m, d.set < 0);
}

// Issues the loads of a stepping task's raw inputs.
template <int KindV>
__device__ __forceinline__ StepRaw<ObjT<KindV>> step_load_task(const BatchIO &io,
                                                               const TaskDesc &d,
                                                               const StepSets &ss) {
    using T = ObjT<KindV>;
    const StepGeom g = desc_geom(d);
    const bool pack = d.set < 0;
    const StepLane p = pack ? step_lane<true>(g) : step_lane<false>(g);
    const T *X = (const T *)io.x, *Y = (const T *)io.y, *Z = (const T *)io.z,
            *R = (const T *)io.r;
    if (d.K == 2) {
        if (pack)
            return R ? step_load<T, 2, true, true>(X, Y, Z, R, ss.base, g, p)
                     : step_load<T, 2, false, true>(X, Y, Z, R, ss.base, g, p);
        return R ? step_load<T, 2, true, false>(X, Y, Z, R, ss.base, g, p)
                 : step_load<T, 2, false, false>(X, Y, Z, R, ss.base, g, p);
    }
    if (pack)
        return R ? step_load<T, 1, true, true>(X, Y, Z, R, ss.base, g, p)
                 : step_load<T, 1, false, true>(X, Y, Z, R, ss.base, g, p);
    return R ? step_load<T, 1, true, false>(X, Y, Z, R, ss.base, g, p)
             : step_load<T, 1, false, false>(X, Y, Z, R, ss.base, g, p);
}

// Stages and sweeps one stepping task whose raw inputs are loaded, and adds
// its totals to the outputs.  A single segment (a row block of one set)
// reports one total per wave; a pack sums per set over its segments.  hook()
// runs between staging and the sweep.
template <int K, int KindV, bool Pack, typename Hook>
__device__ __forceinline__ void step_run(const BatchIO &io, const StepGeom &g, const StepSets &ss,
                                         const StepRaw<ObjT<KindV>> &raw, void *win, Hook &&hook) {
    const int lane = lane_id();
    if constexpr (KindV == kCountI32 || KindV == kCountF32) {
        StepCountResult r;
        if constexpr (KindV == kCountI32)
            r = step_count_i32<K, Pack>(raw, g, win, hook);
        else
            r = step_count_f32<K, Pack>(raw, g, win, hook);
        if (Pack) {
            // collisions are usually rare: most packs have nothing to report
            if (__builtin_amdgcn_ballot_w64(r.lane != 0)) {
                const uint32_t c = segment_sum(r.lane, g, win);
                if (lane < g.m && c)
                    atomicAdd((unsigned long long *)&io.counts[ss.out_set],
                              (unsigned long long)c);
            }
        } else if (lane == 0 && r.wave) {
            atomicAdd((unsigned long long *)&io.counts[ss.out_set], (unsigned long long)r.wave);
        }
    } else {
        StepEnergyResult r;
        if (io.r)
            r = step_energy<K, Pack, true>(raw, g, io.eps2, win, hook);
        else
            r = step_energy<K, Pack, false>(raw, g, io.eps2, win, hook);
        if (Pack) {
            const double e = segment_sum(r.lane_energy, g, win);
            const uint32_t c = io.r && __builtin_amdgcn_ballot_w64(r.lane != 0)
                                   ? segment_sum(r.lane, g, win)
                                   : 0u;
            if (lane < g.m) {
                add_set_energy(io, ss.out_set, g.n, e);
                if (c)
                    atomicAdd((unsigned long long *)&io.counts[ss.out_set],
                              (unsigned long long)c);
            }
        } else {
            const double e = wave_sum(r.lane_energy);
            if (lane == 0) {
                add_set_energy(io, ss.out_set, g.n, e);
                if (io.r && r.wave)
                    atomicAdd((unsigned long long *)&io.counts[ss.out_set],
                              (unsigned long long)r.wave);
            }
        }
    }
}

template <int KindV, typename Hook>
__device__ __forceinline__ void step_run_task(const BatchIO &io, const TaskDesc &d,
                                              const StepSets &ss,
                                              const StepRaw<ObjT<KindV>> &raw, void *win,
                                              Hook &&hook) {
    const StepGeom g = desc_geom(d);
    const bool pack = d.set < 0;
    if (d.K == 2) {
        if (pack)
            step_run<2, KindV, true>(io, g, ss, raw, win, hook);
        else
            step_run<2, KindV, false>(io, g, ss, raw, win, hook);
    } else {
        if (pack)
            step_run<1, KindV, true>(io, g, ss, raw, win, hook);
        else
            step_run<1, KindV, false>(io, g, ss, raw, win, hook);
    }
}

// Runs one task with the compiled shape K (only shapes up to KMAX are compiled
// into a kernel, which keeps its register count, and so its occupancy, to
// what the largest shape it serves needs).
template <int KindV, int KMAX>
__device__ __forceinline__ void run_task(const BatchIO &io, int64_t base, const Band &band,
                                         int ra, int u0, int u1, int64_t set, int K, void *win) {
    if (KMAX >= 8 && K == 8)
        run_shape<(KMAX >= 8 ? 8 : 1), KindV>(io, base, band, ra, u0, u1, set, win);
    else if (KMAX >= 4 && K == 4)
        run_shape<(KMAX >= 4 ? 4 : 1), KindV>(io, base, band, ra, u0, u1, set, win);
    else if (KMAX >= 2 && K == 2)
        run_shape<(KMAX >= 2 ? 2 : 1), KindV>(io, base, band, ra, u0, u1, set, win);
    else if (K == 1)
        run_shape<1, KindV>(io, base, band, ra, u0, u1, set, win);
}

// Plans: wave w runs the tasks descs[wave_start[w] .. wave_start[w+1]), a list
// balanced across the waves on the host; the next descriptor is fetched while
// the current task runs.
// Wave lists of a plan per resident wave (short lists: the hardware starts a
// waiting workgroup as soon as a resident one finishes, which evens out what
// the host's cost estimate misses), and blocks of an unplanned call per
// resident block.
constexpr int kPlanWaveFactor = 64;
constexpr int kScanBlockFactor = 16;

// Waves per SIMD the batched kernels are compiled for: four where the
// largest compiled shape allows it without register spills (the stepping
// sweeps hide their per-task load latency behind the other waves).
template <int KindV, int KMAX>
constexpr int batched_min_waves() {
    return (KMAX <= 2 || (KindV == kEnergyF32 && KMAX <= 4)) ? 4 : 1;
}

template <int KindV, int KMAX>
__global__ __launch_bounds__(kBatchBlock, (batched_min_waves<KindV, KMAX>())) void k_batched_plan(BatchIO io,
                                                         const TaskDesc *__restrict__ descs,
                                                         const int32_t *__restrict__ wave_start,
                                                         int64_t n_waves) {
    constexpr int kLdsBytes = batched_lds_bytes<KindV>();
    __shared__ __align__(16) unsigned char lds[kBatchWaves * kLdsBytes];
    const int wave = batch_wave();
    void *win = lds + wave * kLdsBytes;
    const int64_t w = (int64_t)blockIdx.x * kBatchWaves + wave;
    if (w >= n_waves) return;
    int i = wave_start[w];
    const int e = wave_start[w + 1];
    if (i >= e) return;
    TaskDesc next = descs[i];
    for (; i < e; ++i) {
        const TaskDesc d = next;
        if (i + 1 < e) next = descs[i + 1];
        if (d.form == PAIRS_FORM_STEPPING) {
            const StepSets ss = step_sets(io, d);
            const StepRaw<ObjT<KindV>> raw = step_load_task<KindV>(io, d, ss);
            step_run_task<KindV>(io, d, ss, raw, win, []() PAIRS_INLINE {});
        } else {
            const Band band = Band::of(d.n);
            run_task<KindV, KMAX>(io, d.base, band, d.a, d.b, d.c, d.set, d.K, win);
        }
    }
}

// Unplanned calls: tasks decoded from the device-built prefix sums, taken by
// the waves with a grid stride.
template <int KindV, int KMAX>
__global__ __launch_bounds__(kBatchBlock, (batched_min_waves<KindV, KMAX>())) void k_batched_scan(BatchIO io, ScanSource src,
                                                         ClassTable ct) {
    constexpr int kLdsBytes = batched_lds_bytes<KindV>();
    __shared__ __align__(16) unsigned char lds[kBatchWaves * kLdsBytes];
    const int wave = batch_wave();
    void *win = lds + wave * kLdsBytes;
    const int64_t stride = (int64_t)gridDim.x * kBatchWaves;
    const int64_t ntasks = src.hdr->T, B = src.hdr->B;
    for (int64_t t = (int64_t)blockIdx.x * kBatchWaves + wave; t < ntasks; t += stride) {
        int64_t set;
        int local;
        src.decode(t, B, &set, &local);
        int64_t base;
        int n;
        set_range(io.off, set, io.n_total, &base, &n);
        if (n < 2) continue;
        const int c = ct.class_of(n);
        const Band band = Band::of(n);
        if (ct.form[c] == PAIRS_FORM_STEPPING) {
            const StepTiling til = StepTiling::of(band, ct.K[c], ct.U[c]);
            if (local < 0 || (int64_t)local >= til.tasks()) continue;
            int r0, s0, T, x;
            step_range(band, til, local / til.nchunks, local % til.nchunks, &r0, &s0, &T, &x);
            if (T + x == 0) continue;
            TaskDesc d{};
            d.base = base;
            d.set = (int32_t)set;
            d.n = n;
            d.a = r0;
            d.b = s0;
            d.c = T;
            // a last row block of at most 64 rows (a whole small set, or the
            // tail of a larger one) runs one row per lane, as in plans
            d.K = (uint8_t)(n - r0 <= kWave ? 1 : ct.K[c]);
            d.form = PAIRS_FORM_STEPPING;
            d.m = 1;
            d.x = (uint8_t)x;
            const StepSets ss{base, set};
            const StepRaw<ObjT<KindV>> raw = step_load_task<KindV>(io, d, ss);
            step_run_task<KindV>(io, d, ss, raw, win, []() PAIRS_INLINE {});
            continue;
        }
        const Tiling til = Tiling::of(band, ct.K[c], ct.U[c]);
        if (local < 0 || (int64_t)local >= til.tasks()) continue;
        int ra, u0, u1;
        task_range(band, til, local / til.nchunks, local % til.nchunks, &ra, &u0, &u1);
        if (u0 >= u1) continue;
        run_task<KindV, KMAX>(io, base, band, ra, u0, u1, set, ct.K[c], win);
    }
}

// ------------------------------------------- batched forces and fp64 energy --
//
// Unplanned batches of the two interactions whose results are per object or
// in double precision: forces of the softened potential (force_task) and the
// potential in double precision (energy64_task).  Tasks come from the same
// device-side schedule as the counts (ScanSource), in the broadcast form with
// the rows per lane of each set's class; per-object outputs are written at
// the set's base, so sets never touch each other's objects.

enum XKind { kForceF32 = 4, kEnergyF64 = 5 };

struct XBatchIO {
    const void *x, *y, *z;
    const int64_t *off;
    int64_t n_total;
    double eps2;
    SumSink f[3];        // forces: per-object components; energy: f[0] = per-object sums (or null)
    double *set_energy;  // energy: per-set totals
    double emax;         // energy: > 0 for fixed-point set totals (bound on one term)
};

template <int K, int KindV>
__device__ __forceinline__ void xbatched_task(const XBatchIO &io, int64_t base, const Band &band,
                                              int ra, int u0, int u1, int64_t set, void *win) {
    if constexpr (KindV == kForceF32) {
        const float *X = (const float *)io.x, *Y = (const float *)io.y, *Z = (const float *)io.z;
        TaskInputs<float, K> in;
        load_task_inputs<float, K, K, false>(X, Y, Z, nullptr, base, band, ra, u0, u1, in);
        force_task<K>(X, Y, Z, base, band, ra, u0, u1, (float)io.eps2, (float *)win, io.f[0],
                      io.f[1], io.f[2], in);
    } else {
        const double *X = (const double *)io.x, *Y = (const double *)io.y,
                     *Z = (const double *)io.z;
        TaskInputs<double, K> in;
        load_task_inputs<double, K, K, false>(X, Y, Z, nullptr, base, band, ra, u0, u1, in);
        double e;
        if (io.f[0].p)
            e = energy64_task<K, true>(X, Y, Z, base, band, ra, u0, u1, io.eps2, (double *)win,
                                       io.f[0], in);
        else
            e = energy64_task<K, false>(X, Y, Z, base, band, ra, u0, u1, io.eps2, (double *)win,
                                        io.f[0], in);
        if (lane_id() == 0) {
            const double scale =
                io.emax > 0.0 ? fixed_scale(0.5 * band.n * (band.n - 1.0) * io.emax) : 0.0;
            SumSink{io.set_energy, scale}.add(set, e);
        }
    }
}

template <int KindV>
__global__ __launch_bounds__(kBatchBlock) void k_xbatched_scan(XBatchIO io, ScanSource src,
                                                          ClassTable ct) {
    constexpr int kLdsBytes = KindV == kForceF32 ? kForceLds * 4 : kEnergy64Lds * 8;
    __shared__ __align__(16) unsigned char lds[kBatchWaves * kLdsBytes];
    const int wave = batch_wave();
    void *win = lds + wave * kLdsBytes;
    const int64_t stride = (int64_t)gridDim.x * kBatchWaves;
    const int64_t ntasks = src.hdr->T, B = src.hdr->B;
    for (int64_t t = (int64_t)blockIdx.x * kBatchWaves + wave; t < ntasks; t += stride) {
        int64_t set;
        int local;
        src.decode(t, B, &set, &local);
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
        if (ct.K[c] == 2)
            xbatched_task<2, KindV>(io, base, band, ra, u0, u1, set, win);
        else
            xbatched_task<1, KindV>(io, base, band, ra, u0, u1, set, win);
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

// Status words of the validation passes and the lattice kernels, in the
// library's own device memory: each device holds its copy from the time the
// library's code is loaded on it, so no call allocates for them.  Word 0
// takes the answer of a validation pass; word 16 takes bits nobody reads.
__device__ __align__(256) int g_status_words[64];

// Scratch of pairs_count_i32_batched_noalloc: the workspace of an unplanned
// batched call, in the library's own device memory (each device holds its
// copy until the process ends).  Host code never passes the array's name to
// a kernel or a copy: in host code it is a stand-in, not a device address.
// The device address is looked up once per device (device_state) and used
// instead.
constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per-device state: the addresses of that device's status words and scratch,
// and its CU count.
struct DeviceState {
    int *d_flag = nullptr;
    void *d_scratch = nullptr;
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

// Looks the state up on first use on a device (with that device current):
// the symbols' device addresses and an attribute query, none of which
// allocates.
pairs_status_t device_state(DeviceState **st) {
    int dev;
    PAIRS_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    DeviceState &d = g_dev[dev];
    if (!d.d_flag) {
        void *flag = nullptr, *scr = nullptr;
        PAIRS_HIP_CHECK(hipGetSymbolAddress(&flag, HIP_SYMBOL(g_status_words)));
        PAIRS_HIP_CHECK(hipGetSymbolAddress(&scr, HIP_SYMBOL(scratch)));
        int ncu = 0;
        PAIRS_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        d.n_cu = ncu;
        d.d_scratch = scr;
        d.d_flag = (int *)flag;
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
    int form;
};

// The double-precision energy and the forces run the float32 energy's shapes
// with at most 4 rows per lane: their rows and partner sums take twice the
// registers.
Shape single_set_shape(int kind, int64_t n, bool total_only = false) {
    const bool wide = kind == PAIRS_KIND_ENERGY_F64 || kind == PAIRS_KIND_FORCE_F32;
    const ClassTable t = shapes(wide ? PAIRS_KIND_ENERGY_F32 : kind,
                                !wide && total_only ? kModeTotalOnly : kModeSingle);
    const int c = t.class_of((int)n);
    return {wide ? std::min(t.K[c], 4) : t.K[c], t.U[c], t.form[c]};
}

// Blocks of a single-set launch: one wave per task, at most kMaxSingleBlocks
// (the waves then stride over the remaining tasks).
unsigned single_blocks(int n, int K, int U) {
    Tiling t = Tiling::of(Band::of(n), K, U);
    const int64_t need = (t.tasks() + kWavesPerBlock - 1) / kWavesPerBlock;
    return (unsigned)std::min<int64_t>(need, kMaxSingleBlocks);
}

template <int K>
void launch_count_i32(const int32_t *x, const int32_t *y, const int32_t *z, const int32_t *r,
                      int n, int U, uint64_t *out, hipStream_t s) {
    const unsigned blocks = single_blocks(n, K, U);
    if (blocks > 0) k_count_i32<K><<<blocks, kBlock, 0, s>>>(x, y, z, r, n, U, out);
}

template <int K>
void launch_count_f32(const float *x, const float *y, const float *z, const float *r, int n,
                      int U, uint64_t *out, hipStream_t s) {
    const unsigned blocks = single_blocks(n, K, U);
    if (blocks > 0) k_count_f32<K><<<blocks, kBlock, 0, s>>>(x, y, z, r, n, U, out);
}

template <int K>
void launch_energy(const float *x, const float *y, const float *z, int n, int U, float eps2,
                   SumSink E, SumSink total, hipStream_t s) {
    const unsigned blocks = single_blocks(n, K, U);
    if (blocks == 0) return;
    if (E.p)
        k_energy<K, true><<<blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
    else
        k_energy<K, false><<<blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
}

template <int K>
void launch_energy64(const double *x, const double *y, const double *z, int n, int U, double eps2,
                     SumSink E, SumSink total, hipStream_t s) {
    const unsigned blocks = single_blocks(n, K, U);
    if (blocks == 0) return;
    if (E.p)
        k_energy64<K, true><<<blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
    else
        k_energy64<K, false><<<blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, E, total);
}

template <int K>
void launch_force(const float *x, const float *y, const float *z, int n, int U, float eps2,
                  SumSink Fx, SumSink Fy, SumSink Fz, hipStream_t s) {
    const unsigned blocks = single_blocks(n, K, U);
    if (blocks == 0) return;
    k_force<K><<<blocks, kBlock, 0, s>>>(x, y, z, n, U, eps2, Fx, Fy, Fz);
}

// Bounds on one term of the potential, 1/sqrt(d2 + eps2) <= 1/sqrt(eps2), and
// of one force component, |d| / (d2 + eps2)^(3/2) <= 2 / (3 sqrt(3) eps2),
// with a margin for the float32 evaluation and partial sums.
double energy_term_bound(double eps2) { return 1.01 / sqrt(eps2); }
double force_term_bound(double eps2) { return 0.4 / eps2; }

constexpr unsigned kSumFlags = PAIRS_FLAG_VALIDATE | PAIRS_FLAG_DETERMINISTIC;

// Sinks of a single-set sum: double atomics, or under PAIRS_FLAG_DETERMINISTIC
// fixed point scaled for `bound`, the largest magnitude any partial sum of
// the output can reach.
SumSink sink(double *p, bool det, double bound) {
    return SumSink{p, det ? fixed_scale(bound) : 0.0};
}

// Converts fixed-point set energies back to doubles (no-op without the flag).
pairs_status_t finish_sets(const BatchIO &io, int64_t n_sets, hipStream_t s) {
    if (io.emax <= 0.0 || n_sets <= 0) return PAIRS_OK;
    k_finish_sets<<<blocks_for(n_sets, 256), 256, 0, s>>>(io.energy, io.off, n_sets, io.n_total,
                                                          io.emax);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

// Converts a fixed-point output back to doubles (no-op without the flag).
pairs_status_t finish(const SumSink &k, int64_t n, hipStream_t s) {
    if (k.scale <= 0.0 || !k.p || n <= 0) return PAIRS_OK;
    k_fixed_finish<<<blocks_for(n, 256), 256, 0, s>>>(k.p, n, 1.0 / k.scale);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

int max_rows(const ClassTable &ct) {
    int m = 1;
    for (int c = 0; c < ct.count; ++c) m = std::max(m, ct.K[c]);
    return m;
}

// Resident blocks of a kernel on the current device.
template <typename Kern>
int64_t resident_blocks(const DeviceState *st, Kern kern, int block = kBlock) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    return (int64_t)per_cu * (st->n_cu > 0 ? st->n_cu : 1);
}

// Calls f with the plan kernel of (kind, kmax).
template <typename F>
void with_plan_kernel(int kind, int kmax, F f) {
#define PAIRS_PLAN_K(KV, KM) f(k_batched_plan<KV, KM>)
    switch (kind * 16 + kmax) {
        case kCountI32 * 16 + 1: PAIRS_PLAN_K(kCountI32, 1); break;
        case kCountI32 * 16 + 2: PAIRS_PLAN_K(kCountI32, 2); break;
        case kCountI32 * 16 + 4: PAIRS_PLAN_K(kCountI32, 4); break;
        case kCountI32 * 16 + 8: PAIRS_PLAN_K(kCountI32, 8); break;
        case kCountF32 * 16 + 1: PAIRS_PLAN_K(kCountF32, 1); break;
        case kCountF32 * 16 + 2: PAIRS_PLAN_K(kCountF32, 2); break;
        case kCountF32 * 16 + 4: PAIRS_PLAN_K(kCountF32, 4); break;
        case kCountF32 * 16 + 8: PAIRS_PLAN_K(kCountF32, 8); break;
        case kEnergyF32 * 16 + 1: PAIRS_PLAN_K(kEnergyF32, 1); break;
        case kEnergyF32 * 16 + 2: PAIRS_PLAN_K(kEnergyF32, 2); break;
        case kEnergyF32 * 16 + 4: PAIRS_PLAN_K(kEnergyF32, 4); break;
        default: PAIRS_PLAN_K(kEnergyF32, 8); break;
    }
#undef PAIRS_PLAN_K
}

template <typename F>
void with_scan_kernel(int kind, int kmax, F f) {
#define PAIRS_SCAN_K(KV, KM) f(k_batched_scan<KV, KM>)
    switch (kind * 16 + kmax) {
        case kCountI32 * 16 + 1: PAIRS_SCAN_K(kCountI32, 1); break;
        case kCountI32 * 16 + 2: PAIRS_SCAN_K(kCountI32, 2); break;
        case kCountI32 * 16 + 4: PAIRS_SCAN_K(kCountI32, 4); break;
        case kCountI32 * 16 + 8: PAIRS_SCAN_K(kCountI32, 8); break;
        case kCountF32 * 16 + 1: PAIRS_SCAN_K(kCountF32, 1); break;
        case kCountF32 * 16 + 2: PAIRS_SCAN_K(kCountF32, 2); break;
        case kCountF32 * 16 + 4: PAIRS_SCAN_K(kCountF32, 4); break;
        case kCountF32 * 16 + 8: PAIRS_SCAN_K(kCountF32, 8); break;
        case kEnergyF32 * 16 + 1: PAIRS_SCAN_K(kEnergyF32, 1); break;
        case kEnergyF32 * 16 + 2: PAIRS_SCAN_K(kEnergyF32, 2); break;
        case kEnergyF32 * 16 + 4: PAIRS_SCAN_K(kEnergyF32, 4); break;
        default: PAIRS_SCAN_K(kEnergyF32, 8); break;
    }
#undef PAIRS_SCAN_K
}

pairs_status_t launch_scan(int kind, const BatchIO &io, const ScanSource &src,
                           const ClassTable &ct, hipStream_t s) {
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    // sixteen times the resident blocks: each block takes fewer grid-stride
    // tasks, and blocks that start as others finish even out the tail
    with_scan_kernel(kind, max_rows(ct), [&](auto kern) {
        const int64_t blocks = resident_blocks(st, kern, kBatchBlock) * kScanBlockFactor;
        kern<<<blocks, kBatchBlock, 0, s>>>(io, src, ct);
    });
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

constexpr size_t batched_ws_bytes(int64_t n_sets) { return sched_layout(n_sets).total; }

static_assert(batched_ws_bytes(PAIRS_NOALLOC_MAX_SETS) <= kScratchBytes,
              "the no-allocation count's largest batch fits its scratch");

pairs_status_t batched_common(int kind, const BatchIO &io, int64_t n_sets, void *ws,
                              size_t ws_bytes, hipStream_t s) {
    if (!ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    const SchedLayout L = sched_layout(n_sets);
    unsigned char *p = (unsigned char *)ws;
    SchedHeader *hdr = (SchedHeader *)(p + L.hdr);
    int32_t *list = (int32_t *)(p + L.list);
    int64_t *pre = (int64_t *)(p + L.pre);
    int32_t *tab = (int32_t *)(p + L.tab);
    int64_t *blk = (int64_t *)(p + L.blk);
    const ClassTable ct = shapes(kind == kCountI32   ? PAIRS_KIND_COUNT_I32
                                 : kind == kCountF32 ? PAIRS_KIND_COUNT_F32
                                                     : PAIRS_KIND_ENERGY_F32,
                                 kModeBatched);
    const unsigned nb = (unsigned)L.nb;
    k_sched_count<<<nb, kSchedBlock, 0, s>>>(io.off, n_sets, io.n_total, ct, blk);
    k_sched_scan<<<1, kSchedBlock, 0, s>>>(blk, L.nb, hdr);
    k_sched_list<<<nb, kSchedBlock, 0, s>>>(io.off, n_sets, io.n_total, ct, blk, hdr, list, pre);
    // at most n_sets + 1 buckets and the sentinel
    k_sched_tab<<<blocks_for(n_sets + 2, 256), 256, 0, s>>>(pre, hdr, tab);
    PAIRS_HIP_CHECK(hipGetLastError());
    ScanSource src{hdr, list, pre, tab};
    return launch_scan(kind, io, src, ct, s);
}

// Size classes of the batched forces and double-precision energies: the
// broadcast form, at most 2 rows per lane (three force components, or double
// rows, take the registers of two float rows, and one kernel serves every
// class, so its largest shape sets the occupancy of all).
ClassTable xbatched_table() {
    const int lo[3] = {1024, 128, 0}, K[3] = {2, 2, 1}, U[3] = {256, 128, 64};
    return make_table(3, lo, K, U, nullptr);
}

pairs_status_t xbatched_common(int kind, const XBatchIO &io, int64_t n_sets, void *ws,
                               size_t ws_bytes, hipStream_t s) {
    if (!ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    const SchedLayout L = sched_layout(n_sets);
    unsigned char *p = (unsigned char *)ws;
    SchedHeader *hdr = (SchedHeader *)(p + L.hdr);
    int32_t *list = (int32_t *)(p + L.list);
    int64_t *pre = (int64_t *)(p + L.pre);
    int32_t *tab = (int32_t *)(p + L.tab);
    int64_t *blk = (int64_t *)(p + L.blk);
    const ClassTable ct = xbatched_table();
    const unsigned nb = (unsigned)L.nb;
    k_sched_count<<<nb, kSchedBlock, 0, s>>>(io.off, n_sets, io.n_total, ct, blk);
    k_sched_scan<<<1, kSchedBlock, 0, s>>>(blk, L.nb, hdr);
    k_sched_list<<<nb, kSchedBlock, 0, s>>>(io.off, n_sets, io.n_total, ct, blk, hdr, list, pre);
    k_sched_tab<<<blocks_for(n_sets + 2, 256), 256, 0, s>>>(pre, hdr, tab);
    PAIRS_HIP_CHECK(hipGetLastError());
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    const ScanSource src{hdr, list, pre, tab};
    auto go = [&](auto kern) {
        const int64_t blocks = resident_blocks(st, kern, kBatchBlock) * kScanBlockFactor;
        kern<<<(unsigned)blocks, kBatchBlock, 0, s>>>(io, src, ct);
    };
    if (kind == kForceF32)
        go(k_xbatched_scan<kForceF32>);
    else
        go(k_xbatched_scan<kEnergyF64>);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t batched_args(const void *x, const void *y, const void *z,
                            const int64_t *d_offsets, int64_t n_sets, int64_t n_total,
                            unsigned flags, unsigned allowed = PAIRS_FLAG_VALIDATE) {
    if (n_sets < 0 || n_total < 0 || !d_offsets || (flags & ~allowed))
        return PAIRS_ERR_INVALID_ARG;
    if (n_sets >= INT32_MAX) return PAIRS_ERR_INVALID_ARG;
    if (n_total > 0 && (!x || !y || !z)) return PAIRS_ERR_INVALID_ARG;
    return PAIRS_OK;
}

// The unplanned batched count into a workspace of ws_bytes at ws (a caller's
// or the library's scratch); arguments already checked.  The schedule
// kernels write every workspace word the scan kernel reads, so nothing needs
// clearing between calls.
pairs_status_t count_i32_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                                 const int32_t *r, const int64_t *d_offsets, int64_t n_sets,
                                 int64_t n_total, uint64_t *d_counts, void *ws, size_t ws_bytes,
                                 unsigned flags, hipStream_t s) {
    if (flags & PAIRS_FLAG_VALIDATE) {
        PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
        PAIRS_TRY(validate_i32(x, y, z, r, n_total, s));
    }
    PAIRS_TRY(fill_u64(d_counts, n_sets, 0, s));
    if (n_sets == 0) return PAIRS_OK;
    BatchIO io{x, y, z, r, d_offsets, n_total, d_counts, nullptr, 0.0f};
    return batched_common(kCountI32, io, n_sets, ws, ws_bytes, s);
}

// ----------------------------------------------------------- binned count --

namespace bin = pairs_binning;

// Workspace layout of a binned count of n objects.
struct BinnedLayout {
    size_t obj, rec, perm, so, sq, ukeys, off, slot_bsum;
    size_t htags, hkeys, hvals, hsize, counters, items, item_pre, item_tab, item_hdr, item_bsum;
    size_t total;
    int blog;  // cell table of 2^blog buckets of 8 slots, at least 2n slots
};

// Bits per axis of a cell key: the fewest that hold the largest neighbour
// coordinate, 2^25 / cell + 2.
int binned_field_bits(int32_t cell) {
    const int64_t top = ((int64_t)1 << 25) / cell + 2;
    int fb = 1;
    while (((int64_t)1 << fb) <= top) ++fb;
    return fb;
}

// Bits of a batch's set index in a cell key (0 for one set).
int binned_set_bits(int64_t n_sets) {
    int sb = 0;
    while (sb < 63 && ((int64_t)1 << sb) < n_sets) ++sb;
    return sb;
}

pairs_status_t binned_layout(int64_t n, BinnedLayout *L) {
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p += align256(bytes);
        return at;
    };
    const size_t un = (size_t)n;
    L->obj = take(8 * un);
    L->rec = take(16 * un);
    L->perm = take(4 * un);
    L->so = take(16 * un);
    L->sq = take(8 * un);
    L->ukeys = take(8 * un);
    L->off = take(4 * (un + 1));
    // at least 2n slots, so the table is at most half full (n cells at most):
    // at 3/4 the lookups of the count kernel took a quarter longer
    L->blog = 1;
    while ((int64_t(bin::kSlots) << L->blog) < 2 * std::max<int64_t>(n, 1)) ++L->blog;
    const size_t slots = size_t(bin::kSlots) << L->blog;
    L->slot_bsum = take(8 * ((slots + bin::kSlotBlock - 1) / bin::kSlotBlock));
    L->htags = take(slots);
    L->hkeys = take(8 * slots);
    L->hvals = take(8 * slots);
    L->hsize = take(4 * slots);
    L->counters = take(8);  // cells, work items
    const size_t cap = (size_t)bin::item_capacity(n);
    L->items = take(sizeof(bin::Item) * cap);
    L->item_pre = take(8 * (cap + 1));
    L->item_tab = take(4 * (cap + 2));
    L->item_hdr = take(sizeof(bin::ItemSched));
    L->item_bsum = take(8 * ((cap + bin::kScanBlock - 1) / bin::kScanBlock));
    L->total = p;
    return PAIRS_OK;
}

// The binned count of n objects in n_sets sets (d_offsets null: one set)
// into d_counts[n_sets]; arguments already checked.
pairs_status_t binned_common(const int32_t *x, const int32_t *y, const int32_t *z,
                             const int32_t *r, const int64_t *d_offsets, int64_t n_sets,
                             int64_t n, int32_t cell, uint64_t *d_counts, void *d_ws,
                             size_t ws_bytes, unsigned flags, hipStream_t s) {
    const int fb = binned_field_bits(cell);
    if (3 * fb + binned_set_bits(n_sets) > 64) return PAIRS_ERR_INVALID_ARG;
    BinnedLayout L;
    PAIRS_TRY(binned_layout(n, &L));
    if (n > 0 && (!d_ws || ws_bytes < L.total)) return PAIRS_ERR_WORKSPACE;
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    if (flags & PAIRS_FLAG_VALIDATE) {
        if (d_offsets) PAIRS_TRY(validate_offsets(d_offsets, n_sets, n, s));
        PAIRS_TRY(run_validation(s, [&](int *flag) {
            if (n > 0)
                bin::k_bin_validate<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, r, n, cell, flag);
        }));
    }
    if (n < 2) return fill_u64(d_counts, n_sets, 0, s);
    unsigned char *w = (unsigned char *)d_ws;
    uint2 *obj = (uint2 *)(w + L.obj);
    int4 *rec = (int4 *)(w + L.rec);
    uint32_t *perm = (uint32_t *)(w + L.perm);
    int4 *so = (int4 *)(w + L.so);
    int64_t *sq = (int64_t *)(w + L.sq);
    uint32_t *off = (uint32_t *)(w + L.off);
    uint64_t *ukeys = (uint64_t *)(w + L.ukeys);
    int64_t *slot_bsum = (int64_t *)(w + L.slot_bsum);
    uint8_t *htags = (uint8_t *)(w + L.htags);
    uint64_t *hkeys = (uint64_t *)(w + L.hkeys);
    uint2 *hvals = (uint2 *)(w + L.hvals);
    uint32_t *hsize = (uint32_t *)(w + L.hsize);
    uint32_t *ncell = (uint32_t *)(w + L.counters), *item_n = ncell + 1;
    const bin::ItemList items{(bin::Item *)(w + L.items), item_n,
                              (uint32_t)bin::item_capacity(n)};
    int64_t *item_pre = (int64_t *)(w + L.item_pre);
    int32_t *item_tab = (int32_t *)(w + L.item_tab);
    bin::ItemSched *item_hdr = (bin::ItemSched *)(w + L.item_hdr);
    int64_t *item_bsum = (int64_t *)(w + L.item_bsum);
    const int64_t slots = int64_t(bin::kSlots) << L.blog;
    // 0. everything that starts at zero, by a kernel (no memset nodes when
    //    the call is captured into a graph)
    bin::ClearRanges cr = {{(uint32_t *)d_counts, (uint32_t *)hkeys, (uint32_t *)htags, hsize,
                            ncell},
                           {2 * n_sets, 2 * slots, slots / 4, slots, 2}};
    bin::k_bin_clear<<<dim3((unsigned)std::min<int64_t>(blocks_for(2 * slots, 256), 4096),
                            bin::kClearRanges),
                       256, 0, s>>>(cr);
    // 1. cells: find or insert, ranks
    const int nb = blocks_for(n, bin::kBlock);
    bin::k_bin_insert<<<nb, bin::kBlock, 0, s>>>(x, y, z, r, d_offsets, n_sets, n, cell, fb,
                                                L.blog, hkeys, htags, hsize, obj, rec);
    // 2. the cells in slot order and their first objects
    const unsigned snb = (unsigned)((slots + bin::kSlotBlock - 1) / bin::kSlotBlock);
    bin::k_bin_slot_sums<<<snb, bin::kScanBlock, 0, s>>>(htags, hsize, slots, slot_bsum);
    bin::k_bin_slot_scan<<<1, bin::kScanBlock, 0, s>>>(snb, slot_bsum, ncell);
    bin::k_bin_slot_prefix<<<snb, bin::kScanBlock, 0, s>>>(htags, hsize, hkeys, slots, slot_bsum,
                                                          ncell, n, off, ukeys, hvals);
    // 3. the records grouped by cell
    bin::k_bin_scatter<<<blocks_for(n, 256), 256, 0, s>>>(n, obj, hvals, perm);
    bin::k_bin_gather<<<blocks_for(n, 256), 256, 0, s>>>(rec, perm, n, so, sq);
    PAIRS_HIP_CHECK(hipGetLastError());
    // 4. 16 lanes per occupied cell, at most a few waves per SIMD of the
    //    device; 5. the work items' tasks, shared by every wave
    const int64_t blocks = std::min<int64_t>((n + 15) / 16, (int64_t)st->n_cu * 16);
    auto count = d_offsets ? bin::k_bin_count<true> : bin::k_bin_count<false>;
    count<<<(unsigned)blocks, bin::kBlock, 0, s>>>(so, ukeys, off, ncell, (const uint64_t *)htags,
                                                  hkeys, hvals, L.blog, fb, items, d_counts);
    const unsigned item_nb =
        (unsigned)((bin::item_capacity(n) + bin::kScanBlock - 1) / bin::kScanBlock);
    bin::k_bin_item_sums<<<item_nb, bin::kScanBlock, 0, s>>>(items, item_bsum);
    bin::k_bin_item_scan<<<1, bin::kScanBlock, 0, s>>>(items, item_bsum, item_hdr);
    bin::k_bin_item_prefix<<<item_nb, bin::kScanBlock, 0, s>>>(items, item_bsum, item_hdr,
                                                               item_pre);
    // at most cap buckets and the sentinel
    bin::k_bin_item_tab<<<blocks_for(bin::item_capacity(n) + 1, 256), 256, 0, s>>>(
        item_pre, item_hdr, item_tab);
    const int64_t item_blocks = std::min<int64_t>(n / (4 * bin::kBigCell) + 1,
                                                  (int64_t)st->n_cu * 8);
    bin::k_bin_count_items<<<(unsigned)item_blocks, bin::kBlock, 0, s>>>(
        so, sq, items, item_pre, item_tab, item_hdr, d_counts);
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

// ---------------------------------------------------------- lattice beads --

namespace lat = pairs_lattice;

size_t lattice_ws_bytes(int64_t n_total, int64_t max_n) {
    if (max_n > 0 && max_n <= lat::kMaxLdsBeads) return 0;
    return 256 + 32 * (size_t)n_total;
}

// Beads per thread and table size of the LDS kernel for vectors of at most m beads.
int lattice_bpt(int64_t m) {
    int b = 1;
    while (b < lat::kMaxBpt && (int64_t)b * lat::kBlock < m) b *= 2;
    return b;
}

int lattice_tlog(int64_t m) {
    int l = lat::kMinLog;
    while (l < lat::kMaxLog && (int64_t(1) << (l - 1)) < m) ++l;
    return l;
}

template <bool C, typename F>
void with_lattice_kernels(int bpt, F f) {
    switch (bpt) {
        case 1: f(lat::k_lattice_near<1, C, lat::kWaves>, lat::k_lattice<1, C, uint64_t>); break;
        case 2: f(lat::k_lattice_near<2, C, lat::kWaves>, lat::k_lattice<2, C, uint64_t>); break;
        case 4: f(lat::k_lattice_near<4, C, lat::kWaves>, lat::k_lattice<4, C, uint64_t>); break;
        case 8: f(lat::k_lattice_near<8, C, lat::kWaves>, lat::k_lattice<8, C, uint64_t>); break;
        default: f(lat::k_lattice_near<16, C, lat::kWaves>, lat::k_lattice<16, C, uint64_t>); break;
    }
}

// Vectors of at most kWaveBeads beads are counted one per wave.
constexpr int64_t kWaveBeads = 256;

template <bool C, typename F>
void with_lattice_wave_kernel(int bpt, F f) {
    switch (bpt) {
        case 1: f(lat::k_lattice_near<1, C, 1>); break;
        case 2: f(lat::k_lattice_near<2, C, 1>); break;
        default: f(lat::k_lattice_near<4, C, 1>); break;
    }
}

// The status word the lattice kernels raise bits in: the validation word
// under PAIRS_FLAG_VALIDATE (cleared first), else a word nobody reads.
pairs_status_t lattice_flag(DeviceState *st, bool validate, hipStream_t s, int **flag) {
    if (validate) {
        k_fill_u64<<<1, 1, 0, s>>>((uint64_t *)st->d_flag, 1, 0);
        PAIRS_HIP_CHECK(hipGetLastError());
        *flag = st->d_flag;
    } else {
        *flag = st->d_flag + 16;
    }
    return PAIRS_OK;
}

pairs_status_t lattice_status(DeviceState *st, hipStream_t s) {
    int bad = 0;
    PAIRS_HIP_CHECK(hipMemcpyAsync(&bad, st->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PAIRS_HIP_CHECK(hipStreamSynchronize(s));
    if (bad & lat::kFlagDomain) return PAIRS_ERR_DOMAIN;
    return bad ? PAIRS_ERR_INVALID_ARG : PAIRS_OK;
}

// LDS kernel over every vector of at most m beads; `defer` leaves longer
// vectors to k_lattice_global.
pairs_status_t lattice_lds(const lat::IO &io, int64_t m, bool defer, const DeviceState *st,
                           hipStream_t s) {
    const int bpt = lattice_bpt(m), tlog = lattice_tlog(m);
    const size_t lds = sizeof(uint64_t) << tlog;
    // the near pass sums into the outputs with atomics
    PAIRS_TRY(fill_u64(io.coll, io.n_sets, 0, s));
    PAIRS_TRY(fill_u64(io.cont, io.n_sets, 0, s));
    auto grid = [&](auto kern) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, lat::kBlock, lds) !=
                hipSuccess ||
            per_cu <= 0)
            per_cu = 1;
        const int64_t resident = (int64_t)per_cu * (st->n_cu > 0 ? st->n_cu : 1);
        return (unsigned)std::min<int64_t>(io.n_sets, resident * 4);
    };
    // keys relative to the first bead for every vector whose beads stay near
    // it, then box-based 64-bit keys for the vectors the first pass marked;
    // short vectors take the wave-per-vector near pass (four tables per block)
    const bool per_wave = m <= kWaveBeads;
    auto launch = [&](auto near, auto wide) {
        if (!per_wave) near<<<grid(near), lat::kBlock, lds, s>>>(io, tlog, defer ? 1 : 0);
        wide<<<grid(wide), lat::kBlock, lds, s>>>(io, tlog, defer ? 1 : 0);
    };
    auto launch_wave = [&](auto near) {
        const size_t lds4 = lds * lat::kWaves;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, near, lat::kBlock, lds4) !=
                hipSuccess ||
            per_cu <= 0)
            per_cu = 1;
        const int64_t resident = (int64_t)per_cu * (st->n_cu > 0 ? st->n_cu : 1);
        const int64_t need = (io.n_sets + lat::kWaves - 1) / lat::kWaves;
        near<<<(unsigned)std::min<int64_t>(need, resident * 4), lat::kBlock, lds4, s>>>(
            io, tlog, defer ? 1 : 0);
    };
    const int wbpt = (int)std::min<int64_t>(4, (m + lat::kWave - 1) / lat::kWave);
    const int wb = wbpt <= 1 ? 1 : wbpt <= 2 ? 2 : 4;
    if (io.cont) {
        if (per_wave) with_lattice_wave_kernel<true>(wb, launch_wave);
        with_lattice_kernels<true>(bpt, launch);
    } else {
        if (per_wave) with_lattice_wave_kernel<false>(wb, launch_wave);
        with_lattice_kernels<false>(bpt, launch);
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t lattice_args(const int32_t *x, const int32_t *y, const int32_t *z,
                            uint64_t *coll, uint64_t *cont, int64_t n_total, unsigned flags) {
    if (n_total < 0 || (flags & ~PAIRS_FLAG_VALIDATE)) return PAIRS_ERR_INVALID_ARG;
    if (n_total > 0 && (!x || !y || !z)) return PAIRS_ERR_INVALID_ARG;
    if (!coll && !cont) return PAIRS_ERR_INVALID_ARG;
    return PAIRS_OK;
}

}  // namespace

// ------------------------------------------------------------------- plans --

struct pairs_plan_s {
    int kind;
    bool det;  // fixed-point set energies (PAIRS_PLAN_DETERMINISTIC)
    int device;
    int64_t n_sets;
    int64_t n_total;
    int64_t ntasks;
    ClassTable classes;
    int kmax;          // largest rows-per-lane of the table
    int64_t n_waves;   // waves the task lists were balanced over
    int64_t *d_offsets;
    TaskDesc *d_descs;      // wave-major task descriptors
    int32_t *d_wave_start;  // [n_waves + 1]
    int64_t n_packed;       // sets placed in packs
    int64_t *d_pack_base;   // [n_packed] first object of each packed set
    int32_t *d_pack_set;    // [n_packed] its set id
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
    Shape sh = single_set_shape(PAIRS_KIND_COUNT_I32, n);
    if (sh.form == PAIRS_FORM_MATRIX) {
        const unsigned blocks = single_blocks((int)n, 1, sh.U);
        if (blocks > 0) k_count_i32_mfma<<<blocks, kBlock, 0, s>>>(x, y, z, r, (int)n, sh.U, d_count);
        PAIRS_HIP_CHECK(hipGetLastError());
        return PAIRS_OK;
    }
    switch (sh.K) {
        case 1: launch_count_i32<1>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        case 2: launch_count_i32<2>(x, y, z, r, (int)n, sh.U, d_count, s); break;
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
    Shape sh = single_set_shape(PAIRS_KIND_COUNT_F32, n);
    switch (sh.K) {
        case 1: launch_count_f32<1>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        case 2: launch_count_f32<2>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        case 4: launch_count_f32<4>(x, y, z, r, (int)n, sh.U, d_count, s); break;
        default: launch_count_f32<8>(x, y, z, r, (int)n, sh.U, d_count, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    return PAIRS_OK;
}

pairs_status_t pairs_energy_f32(const float *x, const float *y, const float *z, int64_t n,
                                float eps2, double *d_energy, double *d_total, unsigned flags,
                                pairs_stream_t stream) {
    if (!d_total || n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~kSumFlags))
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
    const bool det = flags & PAIRS_FLAG_DETERMINISTIC;
    const double emax = energy_term_bound(eps2), dn = (double)n;
    const SumSink E = sink(d_energy, det, (dn - 1.0) * emax);
    const SumSink T = sink(d_total, det, 0.5 * dn * (dn - 1.0) * emax);
    Shape sh = single_set_shape(PAIRS_KIND_ENERGY_F32, n, d_energy == nullptr);
    switch (sh.K) {
        case 1: launch_energy<1>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
        case 2: launch_energy<2>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
        case 4: launch_energy<4>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
        default: launch_energy<8>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    PAIRS_TRY(finish(E, n, s));
    return finish(T, 1, s);
}

pairs_status_t pairs_energy_f64(const double *x, const double *y, const double *z, int64_t n,
                                double eps2, double *d_energy, double *d_total, unsigned flags,
                                pairs_stream_t stream) {
    if (!d_total || n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~kSumFlags))
        return PAIRS_ERR_INVALID_ARG;
    if (!(eps2 > 0.0) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE)
        PAIRS_TRY(run_validation(s, [&](int *flag) {
            if (n > 0) k_validate_f64<<<blocks_for(n, 256), 256, 0, s>>>(x, y, z, n, flag);
        }));
    PAIRS_TRY(fill_f64(d_total, 1, 0.0, s));
    PAIRS_TRY(fill_f64(d_energy, n, 0.0, s));
    if (n < 2) return PAIRS_OK;
    const bool det = flags & PAIRS_FLAG_DETERMINISTIC;
    const double emax = energy_term_bound(eps2), dn = (double)n;
    const SumSink E = sink(d_energy, det, (dn - 1.0) * emax);
    const SumSink T = sink(d_total, det, 0.5 * dn * (dn - 1.0) * emax);
    const Shape sh = single_set_shape(PAIRS_KIND_ENERGY_F64, n);
    switch (sh.K) {
        case 1: launch_energy64<1>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
        case 2: launch_energy64<2>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
        default: launch_energy64<4>(x, y, z, (int)n, sh.U, eps2, E, T, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    PAIRS_TRY(finish(E, n, s));
    return finish(T, 1, s);
}

pairs_status_t pairs_force_f32(const float *x, const float *y, const float *z, int64_t n,
                               float eps2, double *d_fx, double *d_fy, double *d_fz,
                               unsigned flags, pairs_stream_t stream) {
    if (n < 0 || n > PAIRS_MAX_SET_SIZE || (flags & ~kSumFlags))
        return PAIRS_ERR_INVALID_ARG;
    if (!(eps2 > 0.0f) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z || !d_fx || !d_fy || !d_fz)) return PAIRS_ERR_INVALID_ARG;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) PAIRS_TRY(validate_f32(x, y, z, nullptr, n, s));
    PAIRS_TRY(fill_f64(d_fx, n, 0.0, s));
    PAIRS_TRY(fill_f64(d_fy, n, 0.0, s));
    PAIRS_TRY(fill_f64(d_fz, n, 0.0, s));
    if (n < 2) return PAIRS_OK;
    const bool det = flags & PAIRS_FLAG_DETERMINISTIC;
    // partial sums of a component never exceed the sum of |f| over n - 1 pairs
    const double bound = ((double)n - 1.0) * force_term_bound(eps2);
    const SumSink Fx = sink(d_fx, det, bound), Fy = sink(d_fy, det, bound),
                  Fz = sink(d_fz, det, bound);
    const Shape sh = single_set_shape(PAIRS_KIND_FORCE_F32, n);
    switch (sh.K) {
        case 1: launch_force<1>(x, y, z, (int)n, sh.U, eps2, Fx, Fy, Fz, s); break;
        case 2: launch_force<2>(x, y, z, (int)n, sh.U, eps2, Fx, Fy, Fz, s); break;
        default: launch_force<4>(x, y, z, (int)n, sh.U, eps2, Fx, Fy, Fz, s); break;
    }
    PAIRS_HIP_CHECK(hipGetLastError());
    PAIRS_TRY(finish(Fx, n, s));
    PAIRS_TRY(finish(Fy, n, s));
    return finish(Fz, n, s);
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
    return count_i32_batched(x, y, z, r, d_offsets, n_sets, n_total, d_counts, d_ws, ws_bytes,
                             flags, (hipStream_t)stream);
}

pairs_status_t pairs_count_i32_batched_noalloc(const int32_t *x, const int32_t *y,
                                               const int32_t *z, const int32_t *r,
                                               const int64_t *d_offsets, int64_t n_sets,
                                               int64_t n_total, uint64_t *d_counts,
                                               unsigned flags, pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags));
    if ((n_sets > 0 && !d_counts) || (n_total > 0 && !r)) return PAIRS_ERR_INVALID_ARG;
    if (n_sets > PAIRS_NOALLOC_MAX_SETS) return PAIRS_ERR_WORKSPACE;
    DeviceState *st;
    PAIRS_TRY(device_state(&st));  // the scratch's address on this device
    return count_i32_batched(x, y, z, r, d_offsets, n_sets, n_total, d_counts, st->d_scratch,
                             kScratchBytes, flags, (hipStream_t)stream);
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
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags, kSumFlags));
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
    if (flags & PAIRS_FLAG_DETERMINISTIC) io.emax = energy_term_bound(eps2);
    PAIRS_TRY(batched_common(kEnergyF32, io, n_sets, d_ws, ws_bytes, s));
    return finish_sets(io, n_sets, s);
}

pairs_status_t pairs_force_f32_batched(const float *x, const float *y, const float *z,
                                       const int64_t *d_offsets, int64_t n_sets,
                                       int64_t n_total, float eps2, double *d_fx, double *d_fy,
                                       double *d_fz, void *d_ws, size_t ws_bytes, unsigned flags,
                                       pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags, kSumFlags));
    if (!(eps2 > 0.0f) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
    if (n_total > 0 && (!d_fx || !d_fy || !d_fz)) return PAIRS_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
        PAIRS_TRY(validate_f32(x, y, z, nullptr, n_total, s));
    }
    PAIRS_TRY(fill_f64(d_fx, n_total, 0.0, s));
    PAIRS_TRY(fill_f64(d_fy, n_total, 0.0, s));
    PAIRS_TRY(fill_f64(d_fz, n_total, 0.0, s));
    if (n_sets == 0 || n_total < 2) return PAIRS_OK;
    // one scale for every object: the bound of the largest possible set
    const bool det = flags & PAIRS_FLAG_DETERMINISTIC;
    const double nmax = (double)std::min<int64_t>(n_total, PAIRS_MAX_BATCH_SET_SIZE);
    const double bound = (nmax - 1.0) * force_term_bound(eps2);
    XBatchIO io{x, y, z, d_offsets, n_total, eps2,
                {sink(d_fx, det, bound), sink(d_fy, det, bound), sink(d_fz, det, bound)},
                nullptr, 0.0};
    PAIRS_TRY(xbatched_common(kForceF32, io, n_sets, d_ws, ws_bytes, s));
    for (int c = 0; c < 3; ++c) PAIRS_TRY(finish(io.f[c], n_total, s));
    return PAIRS_OK;
}

pairs_status_t pairs_energy_f64_batched(const double *x, const double *y, const double *z,
                                        const int64_t *d_offsets, int64_t n_sets,
                                        int64_t n_total, double eps2, double *d_set_energy,
                                        double *d_energy, void *d_ws, size_t ws_bytes,
                                        unsigned flags, pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags, kSumFlags));
    if (!(eps2 > 0.0) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
    if (n_sets > 0 && !d_set_energy) return PAIRS_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < batched_ws_bytes(n_sets)) return PAIRS_ERR_WORKSPACE;
    int dev;
    PAIRS_TRY(current_device(&dev));
    hipStream_t s = (hipStream_t)stream;
    if (flags & PAIRS_FLAG_VALIDATE) {
        PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
        PAIRS_TRY(run_validation(s, [&](int *flag) {
            if (n_total > 0)
                k_validate_f64<<<blocks_for(n_total, 256), 256, 0, s>>>(x, y, z, n_total, flag);
        }));
    }
    PAIRS_TRY(fill_f64(d_set_energy, n_sets, 0.0, s));
    PAIRS_TRY(fill_f64(d_energy, n_total, 0.0, s));
    if (n_sets == 0) return PAIRS_OK;
    const bool det = flags & PAIRS_FLAG_DETERMINISTIC;
    const double emax = energy_term_bound(eps2);
    const double nmax = (double)std::min<int64_t>(n_total, PAIRS_MAX_BATCH_SET_SIZE);
    XBatchIO io{x, y, z, d_offsets, n_total, eps2,
                {sink(d_energy, det, (nmax - 1.0) * emax), SumSink{nullptr, 0.0},
                 SumSink{nullptr, 0.0}},
                d_set_energy, det ? emax : 0.0};
    PAIRS_TRY(xbatched_common(kEnergyF64, io, n_sets, d_ws, ws_bytes, s));
    PAIRS_TRY(finish(io.f[0], n_total, s));
    BatchIO bio{};
    bio.energy = d_set_energy;
    bio.off = d_offsets;
    bio.n_total = n_total;
    bio.emax = io.emax;
    return finish_sets(bio, n_sets, s);
}

pairs_status_t pairs_plan_create(int kind, const int64_t *h_offsets, int64_t n_sets,
                                 pairs_plan_t *out) {
    if (!out) return PAIRS_ERR_INVALID_ARG;
    *out = nullptr;
    const bool det = (kind & PAIRS_PLAN_DETERMINISTIC) != 0;
    kind &= ~PAIRS_PLAN_DETERMINISTIC;
    if (kind != PAIRS_KIND_COUNT_I32 && kind != PAIRS_KIND_COUNT_F32 &&
        kind != PAIRS_KIND_ENERGY_F32)
        return PAIRS_ERR_INVALID_ARG;
    if (det && kind != PAIRS_KIND_ENERGY_F32) return PAIRS_ERR_INVALID_ARG;
    if (n_sets < 0 || n_sets >= INT32_MAX || !h_offsets) return PAIRS_ERR_INVALID_ARG;
    if (h_offsets[0] != 0) return PAIRS_ERR_INVALID_ARG;
    for (int64_t s = 0; s < n_sets; ++s) {
        int64_t m = h_offsets[s + 1] - h_offsets[s];
        if (m < 0 || m > PAIRS_MAX_BATCH_SET_SIZE) return PAIRS_ERR_INVALID_ARG;
    }
    int dev;
    PAIRS_TRY(current_device(&dev));
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    const ClassTable ct = shapes(kind, kModeBatched);
    const int kmax = max_rows(ct);
    const int kk = kind == PAIRS_KIND_COUNT_I32 ? kCountI32
                   : kind == PAIRS_KIND_COUNT_F32 ? kCountF32 : kEnergyF32;
    int64_t n_waves = 0;
    // Task lists for kPlanWaveFactor times the resident waves: the lists are
    // balanced by a cost estimate, and as resident waves finish, the hardware
    // starts the waiting ones, which evens out what the estimate misses.
    with_plan_kernel(kk, kmax, [&](auto kern) {
        n_waves = resident_blocks(st, kern, kBatchBlock) * kBatchWaves * kPlanWaveFactor;
    });

    // every task with its cost in VALU issue slots.  Broadcast tasks: per
    // 64-partner group 5 instructions per row slice in a row block's core, 7
    // at the band edges.  Stepping tasks: about 6 per row and step, plus the
    // staging of the window.
    std::vector<TaskDesc> tasks;
    std::vector<int64_t> cost;
    std::vector<int64_t> pack_base;
    std::vector<int32_t> pack_set;
    // small sets of stepping classes, grouped by (n, K) for packing
    std::map<std::pair<int, int>, std::vector<int64_t>> packable;
    auto add = [&](const TaskDesc &d, int64_t w) -> bool {
        try {
            tasks.push_back(d);
            cost.push_back(w);
        } catch (const std::bad_alloc &) {
            return false;
        }
        return true;
    };
    auto step_cost = [](int K, int T, int x, int S, int w) -> int64_t {
        return 400 + (int64_t)(T + x + K) * K * 6 + (int64_t)K * ((S + w - 1) / w) * 40;
    };
    for (int64_t s = 0; s < n_sets; ++s) {
        const int n = (int)(h_offsets[s + 1] - h_offsets[s]);
        if (n < 2) continue;
        const int c = ct.class_of(n);
        const Band band = Band::of(n);
        if (ct.form[c] == PAIRS_FORM_STEPPING) {
            const int K = ct.K[c];
            if ((n + K - 1) / K <= kWave) {
                const int Kp = n < 4 * K ? 1 : K;  // tiny sets: one row per lane
                try {
                    packable[std::make_pair(n, Kp)].push_back(s);
                } catch (const std::bad_alloc &) {
                    return PAIRS_ERR_NO_MEMORY;
                }
                continue;
            }
            const StepTiling til = StepTiling::of(band, K, ct.U[c]);
            for (int b = 0; b < til.nblocks; ++b) {
                // a last row block of at most 64 rows runs one row per lane,
                // so that it does not leave half of its lanes' rows empty
                const int Kb = (K > 1 && n - b * til.rows <= kWave) ? 1 : K;
                for (int ch = 0; ch < til.nchunks; ++ch) {
                    int r0, s0, T, x;
                    step_range(band, til, b, ch, &r0, &s0, &T, &x);
                    if (T + x == 0) continue;
                    TaskDesc d{};
                    d.base = h_offsets[s];
                    d.set = (int32_t)s;
                    d.n = n;
                    d.a = r0;
                    d.b = s0;
                    d.c = T;
                    d.K = (uint8_t)Kb;
                    d.form = PAIRS_FORM_STEPPING;
                    d.m = 1;
                    d.x = (uint8_t)x;
                    if (!add(d, step_cost(Kb, T, x, step_window_entries(Kb, kWave, T, x), kWave)))
                        return PAIRS_ERR_NO_MEMORY;
                }
            }
            continue;
        }
        const Tiling til = Tiling::of(band, ct.K[c], ct.U[c]);
        for (int b = 0; b < til.nblocks; ++b)
            for (int ch = 0; ch < til.nchunks; ++ch) {
                int ra, u0, u1;
                task_range(band, til, b, ch, &ra, &u0, &u1);
                if (u0 >= u1) continue;
                TaskDesc d{};
                d.base = h_offsets[s];
                d.set = (int32_t)s;
                d.n = n;
                d.a = ra;
                d.b = u0;
                d.c = u1;
                d.K = (uint8_t)ct.K[c];
                d.form = PAIRS_FORM_BROADCAST;
                d.m = 1;
                const int rlast = std::min(ra + 64 * d.K, n) - 1;
                const int core_lo = rlast + 1, core_hi = ra + band.steps(ra);
                int64_t w = 600;
                for (int g0 = u0; g0 < u1; g0 += 64) {
                    const int gn = std::min(64, u1 - g0);
                    const bool full = g0 >= core_lo && g0 + gn - 1 <= core_hi;
                    w += 40 + (full ? 64 * 5 : gn * 7) * (int64_t)d.K;
                }
                if (!add(d, w)) return PAIRS_ERR_NO_MEMORY;
            }
    }
    // packs: whole sets of one size, as many per wave as lanes and window allow
    for (const auto &kv : packable) {
        const int n = kv.first.first, K = kv.first.second;
        const Band band = Band::of(n);
        const int w = (n + K - 1) / K;
        const int T = band.h, x = band.half > 0 ? 1 : 0;
        const int S = step_window_entries(K, w, T, x);
        const int mmax = std::max(1, std::min(kWave / w, kStepCap / (K * S)));
        const std::vector<int64_t> &sets = kv.second;
        for (size_t i0 = 0; i0 < sets.size(); i0 += (size_t)mmax) {
            const int m = (int)std::min<size_t>((size_t)mmax, sets.size() - i0);
            TaskDesc d{};
            d.base = (int64_t)pack_base.size();
            d.set = -1;
            d.n = n;
            d.a = 0;
            d.b = 1;
            d.c = T;
            d.K = (uint8_t)K;
            d.form = PAIRS_FORM_STEPPING;
            d.m = (uint8_t)m;
            d.x = (uint8_t)x;
            try {
                for (int j = 0; j < m; ++j) {
                    pack_base.push_back(h_offsets[sets[i0 + (size_t)j]]);
                    pack_set.push_back((int32_t)sets[i0 + (size_t)j]);
                }
            } catch (const std::bad_alloc &) {
                return PAIRS_ERR_NO_MEMORY;
            }
            if (!add(d, step_cost(K, T, x, S, w) + 40 * (int64_t)m)) return PAIRS_ERR_NO_MEMORY;
        }
    }
    const int64_t ntasks = (int64_t)tasks.size();
    if (ntasks >= INT32_MAX) return PAIRS_ERR_INVALID_ARG;
    if (n_waves < 1) n_waves = 1;
    n_waves = std::min<int64_t>(n_waves, std::max<int64_t>(ntasks, 1));

    // Wave list w runs as workgroup w, which the dispatcher deals to XCD
    // w % kXcds; each XCD has its own L2.  All tasks of one set go to the
    // lists of one XCD, so that a set's objects are fetched into one L2 only:
    // sets (and packs) are dealt to the XCDs by longest processing time first,
    // then within each XCD every task, largest first, goes to the list with
    // the least work so far.
    const int groups = n_waves >= kXcds ? kXcds : 1;
    std::vector<int32_t> order((size_t)ntasks);
    for (int64_t k = 0; k < ntasks; ++k) order[(size_t)k] = (int32_t)k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cost[(size_t)a] > cost[(size_t)b]; });
    std::vector<int8_t> group_of((size_t)ntasks, 0);
    if (groups > 1) {
        // a unit is a set split into row-block tasks (id: the set), or one
        // pack (id: n_sets + its first entry in pack_base)
        const int64_t nunits = n_sets + (int64_t)pack_base.size();
        auto unit = [&](int64_t t) -> int64_t {
            const TaskDesc &d = tasks[(size_t)t];
            return d.set >= 0 ? (int64_t)d.set : n_sets + d.base;
        };
        std::vector<int64_t> unit_cost;
        std::vector<int64_t> units;
        std::vector<int8_t> unit_group;
        try {
            unit_cost.assign((size_t)nunits, 0);
            unit_group.assign((size_t)nunits, 0);
            for (int64_t t = 0; t < ntasks; ++t) unit_cost[(size_t)unit(t)] += cost[(size_t)t];
            for (int64_t u = 0; u < nunits; ++u)
                if (unit_cost[(size_t)u] > 0) units.push_back(u);
        } catch (const std::bad_alloc &) {
            return PAIRS_ERR_NO_MEMORY;
        }
        std::stable_sort(units.begin(), units.end(), [&](int64_t a, int64_t b) {
            return unit_cost[(size_t)a] > unit_cost[(size_t)b];
        });
        int64_t load[kXcds] = {0};
        for (const int64_t u : units) {
            const int g = (int)(std::min_element(load, load + groups) - load);
            load[g] += unit_cost[(size_t)u];
            unit_group[(size_t)u] = (int8_t)g;
        }
        for (int64_t t = 0; t < ntasks; ++t) group_of[(size_t)t] = unit_group[(size_t)unit(t)];
    }
    std::vector<int32_t> owner((size_t)ntasks);
    std::vector<int32_t> per_wave((size_t)n_waves, 0);
    {
        typedef std::pair<int64_t, int32_t> Load;  // (work, wave)
        auto cmp = [](const Load &a, const Load &b) { return a > b; };  // min-heap
        std::vector<std::vector<Load>> heaps((size_t)groups);
        for (int64_t w = 0; w < n_waves; ++w)
            heaps[(size_t)(w % groups)].push_back(Load(0, (int32_t)w));
        for (int64_t k = 0; k < ntasks; ++k) {
            const int32_t t = order[(size_t)k];
            std::vector<Load> &heap = heaps[(size_t)group_of[(size_t)t]];
            std::pop_heap(heap.begin(), heap.end(), cmp);
            Load &l = heap.back();
            owner[(size_t)t] = l.second;
            per_wave[(size_t)l.second]++;
            l.first += cost[(size_t)t];
            std::push_heap(heap.begin(), heap.end(), cmp);
        }
    }
    std::vector<int32_t> wave_start((size_t)n_waves + 1, 0);
    for (int64_t w = 0; w < n_waves; ++w) wave_start[(size_t)w + 1] = wave_start[(size_t)w] + per_wave[(size_t)w];
    std::vector<TaskDesc> laid((size_t)ntasks);
    {
        std::vector<int32_t> cur(wave_start.begin(), wave_start.end() - 1);
        for (int64_t k = 0; k < ntasks; ++k) {  // largest first within each wave
            const int32_t t = order[(size_t)k];
            laid[(size_t)cur[(size_t)owner[(size_t)t]]++] = tasks[(size_t)t];
        }
    }

    pairs_plan_s *p = new (std::nothrow) pairs_plan_s();
    if (!p) return PAIRS_ERR_NO_MEMORY;
    p->kind = kind;
    p->det = det;
    p->device = dev;
    p->n_sets = n_sets;
    p->n_total = h_offsets[n_sets];
    p->ntasks = ntasks;
    p->classes = ct;
    p->kmax = kmax;
    p->n_waves = n_waves;
    p->d_offsets = nullptr;
    p->d_descs = nullptr;
    p->d_wave_start = nullptr;
    p->n_packed = (int64_t)pack_base.size();
    p->d_pack_base = nullptr;
    p->d_pack_set = nullptr;
    hipError_t e = hipMalloc(&p->d_offsets, sizeof(int64_t) * (size_t)(n_sets + 1));
    if (e == hipSuccess && p->n_packed > 0)
        e = hipMalloc(&p->d_pack_base, sizeof(int64_t) * (size_t)p->n_packed);
    if (e == hipSuccess && p->n_packed > 0)
        e = hipMalloc(&p->d_pack_set, sizeof(int32_t) * (size_t)p->n_packed);
    if (e == hipSuccess && p->n_packed > 0)
        e = hipMemcpy(p->d_pack_base, pack_base.data(), sizeof(int64_t) * (size_t)p->n_packed,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && p->n_packed > 0)
        e = hipMemcpy(p->d_pack_set, pack_set.data(), sizeof(int32_t) * (size_t)p->n_packed,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMalloc(&p->d_wave_start, sizeof(int32_t) * (size_t)(n_waves + 1));
    if (e == hipSuccess && ntasks > 0)
        e = hipMalloc(&p->d_descs, sizeof(TaskDesc) * (size_t)ntasks);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_offsets, h_offsets, sizeof(int64_t) * (size_t)(n_sets + 1),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_wave_start, wave_start.data(), sizeof(int32_t) * (size_t)(n_waves + 1),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && ntasks > 0)
        e = hipMemcpy(p->d_descs, laid.data(), sizeof(TaskDesc) * (size_t)ntasks,
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_offsets) (void)hipFree(p->d_offsets);
        if (p->d_wave_start) (void)hipFree(p->d_wave_start);
        if (p->d_descs) (void)hipFree(p->d_descs);
        if (p->d_pack_base) (void)hipFree(p->d_pack_base);
        if (p->d_pack_set) (void)hipFree(p->d_pack_set);
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
    io.pack_base = plan->d_pack_base;
    io.pack_set = plan->d_pack_set;
    if (plan->n_total > 0 && (!io.x || !io.y || !io.z)) return PAIRS_ERR_INVALID_ARG;
    if (plan->kind == PAIRS_KIND_ENERGY_F32) {
        if (!(eps2 > 0.0f) || !isfinite(eps2)) return PAIRS_ERR_INVALID_ARG;
        io.energy = (double *)out[0];
        io.counts = (uint64_t *)out[1];
        io.eps2 = eps2;
        if (plan->det) io.emax = energy_term_bound(eps2);
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
    const int kind = plan->kind == PAIRS_KIND_COUNT_I32   ? kCountI32
                     : plan->kind == PAIRS_KIND_COUNT_F32 ? kCountF32
                                                          : kEnergyF32;
    const int64_t blocks = (plan->n_waves + kBatchWaves - 1) / kBatchWaves;
    with_plan_kernel(kind, plan->kmax, [&](auto kern) {
        kern<<<blocks, kBatchBlock, 0, s>>>(io, plan->d_descs, plan->d_wave_start,
                                                  plan->n_waves);
    });
    PAIRS_HIP_CHECK(hipGetLastError());
    return finish_sets(io, plan->n_sets, s);
}

pairs_status_t pairs_plan_destroy(pairs_plan_t plan) {
    if (!plan) return PAIRS_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(plan->device);
    if (plan->d_offsets) (void)hipFree(plan->d_offsets);
    if (plan->d_descs) (void)hipFree(plan->d_descs);
    if (plan->d_wave_start) (void)hipFree(plan->d_wave_start);
    if (plan->d_pack_base) (void)hipFree(plan->d_pack_base);
    if (plan->d_pack_set) (void)hipFree(plan->d_pack_set);
    (void)hipSetDevice(cur);
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
        (void)hipStreamDestroy(cs);
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
    (void)hipStreamDestroy(cs);
    if (st != PAIRS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e);
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e);
    }
    pairs_graph_s *pg = new (std::nothrow) pairs_graph_s{g, ex, dev};
    if (!pg) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
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
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
    return PAIRS_OK;
}

// A shape mode exists for every kind but the total-only one, which only the
// float32 energy has.
bool valid_mode(int kind, int mode) {
    return mode == kModeSingle || mode == kModeBatched ||
           (mode == kModeTotalOnly && kind == PAIRS_KIND_ENERGY_F32);
}

pairs_status_t pairs_get_shapes(int kind, int batched, pairs_shape_table_t *out) {
    if (!out || kind < PAIRS_KIND_COUNT_I32 || kind > PAIRS_KIND_ENERGY_F32 ||
        !valid_mode(kind, batched))
        return PAIRS_ERR_INVALID_ARG;
    const ClassTable t = shapes(kind, batched);
    out->count = t.count;
    for (int c = 0; c < 4; ++c) {
        out->min_n[c] = t.lo[c];
        out->rows_per_lane[c] = t.K[c];
        out->chunk[c] = t.U[c];
        out->form[c] = t.form[c];
    }
    return PAIRS_OK;
}

pairs_status_t pairs_set_shapes(int kind, int batched, const pairs_shape_table_t *table) {
    if (kind < PAIRS_KIND_COUNT_I32 || kind > PAIRS_KIND_ENERGY_F32 || !valid_mode(kind, batched))
        return PAIRS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_shape_mutex);
    if (!table) {
        g_shapes_set[kind - 1][batched] = false;
        return PAIRS_OK;
    }
    if (table->count < 1 || table->count > kMaxClasses) return PAIRS_ERR_INVALID_ARG;
    ClassTable t = make_table(table->count, table->min_n, table->rows_per_lane, table->chunk,
                              table->form);
    if (!valid_table(t, batched == kModeBatched, kind)) return PAIRS_ERR_INVALID_ARG;
    g_shapes[kind - 1][batched] = t;
    g_shapes_set[kind - 1][batched] = true;
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

pairs_status_t pairs_debug_task_at(int64_t n, int rows_per_lane, int chunk,
                                   const int64_t *tasks, int64_t count, int64_t *out) {
    if (n < 0 || n > PAIRS_MAX_SET_SIZE || count < 0 || (count > 0 && (!tasks || !out)) ||
        (rows_per_lane != 1 && rows_per_lane != 2 && rows_per_lane != 4 && rows_per_lane != 8) ||
        chunk < 64 || chunk % 64 != 0 || chunk > (1 << 22))
        return PAIRS_ERR_INVALID_ARG;
    const Band band = Band::of((int)n);
    const Tiling til = Tiling::of(band, rows_per_lane, chunk);
    for (int64_t k = 0; k < count; ++k)
        if (tasks[k] < 0 || tasks[k] >= til.tasks()) return PAIRS_ERR_INVALID_ARG;
    for (int64_t k = 0; k < count; ++k) {
        int ra, u0, u1;
        task_at_grouped(band, til, tasks[k], &ra, &u0, &u1);
        out[3 * k] = ra;
        out[3 * k + 1] = u0;
        out[3 * k + 2] = u1;
    }
    return PAIRS_OK;
}

pairs_status_t pairs_debug_single_launch(int kind, int64_t n, int64_t *n_tasks,
                                         int64_t *n_blocks, int32_t *threads) {
    if (kind < PAIRS_KIND_COUNT_I32 || kind > PAIRS_KIND_FORCE_F32 || n < 0 ||
        n > PAIRS_MAX_SET_SIZE || !n_tasks || !n_blocks || !threads)
        return PAIRS_ERR_INVALID_ARG;
    *n_tasks = 0;
    *n_blocks = 0;
    *threads = kBlock;
    if (n < 2) return PAIRS_OK;
    const Shape sh = single_set_shape(kind, n);
    *n_tasks = Tiling::of(Band::of((int)n), sh.K, sh.U).tasks();
    *n_blocks = single_blocks((int)n, sh.K, sh.U);
    return PAIRS_OK;
}

pairs_status_t pairs_binned_workspace_size(int64_t n, size_t *bytes) {
    if (!bytes || n < 0 || n > PAIRS_BINNED_MAX_SET_SIZE) return PAIRS_ERR_INVALID_ARG;
    BinnedLayout L;
    PAIRS_TRY(binned_layout(n, &L));
    *bytes = L.total;
    return PAIRS_OK;
}

pairs_status_t pairs_count_i32_binned(const int32_t *x, const int32_t *y, const int32_t *z,
                                      const int32_t *r, int64_t n, int32_t cell,
                                      uint64_t *d_count, void *d_ws, size_t ws_bytes,
                                      unsigned flags, pairs_stream_t stream) {
    if (n < 0 || n > PAIRS_BINNED_MAX_SET_SIZE || !d_count || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (cell < PAIRS_BINNED_MIN_CELL || cell > PAIRS_BINNED_MAX_CELL) return PAIRS_ERR_INVALID_ARG;
    if (n > 0 && (!x || !y || !z || !r)) return PAIRS_ERR_INVALID_ARG;
    return binned_common(x, y, z, r, nullptr, 1, n, cell, d_count, d_ws, ws_bytes, flags,
                         (hipStream_t)stream);
}

pairs_status_t pairs_count_i32_binned_batched(const int32_t *x, const int32_t *y,
                                              const int32_t *z, const int32_t *r,
                                              const int64_t *d_offsets, int64_t n_sets,
                                              int64_t n_total, int32_t cell, uint64_t *d_counts,
                                              void *d_ws, size_t ws_bytes, unsigned flags,
                                              pairs_stream_t stream) {
    if (n_sets < 0 || n_sets >= INT32_MAX || n_total < 0 || n_total > PAIRS_BINNED_MAX_SET_SIZE ||
        !d_offsets || (flags & ~PAIRS_FLAG_VALIDATE))
        return PAIRS_ERR_INVALID_ARG;
    if (n_sets > 0 && !d_counts) return PAIRS_ERR_INVALID_ARG;
    if (cell < PAIRS_BINNED_MIN_CELL || cell > PAIRS_BINNED_MAX_CELL) return PAIRS_ERR_INVALID_ARG;
    if (n_total > 0 && (!x || !y || !z || !r)) return PAIRS_ERR_INVALID_ARG;
    if (n_sets == 0) return n_total == 0 ? PAIRS_OK : PAIRS_ERR_INVALID_ARG;
    return binned_common(x, y, z, r, d_offsets, n_sets, n_total, cell, d_counts, d_ws, ws_bytes,
                         flags, (hipStream_t)stream);
}

pairs_status_t pairs_lattice_workspace_size(int64_t n_sets, int64_t n_total, int64_t max_n,
                                            size_t *bytes) {
    if (!bytes || n_sets < 0 || n_total < 0 || max_n < 0) return PAIRS_ERR_INVALID_ARG;
    *bytes = lattice_ws_bytes(n_total, max_n);
    return PAIRS_OK;
}

pairs_status_t pairs_lattice_count(const int32_t *x, const int32_t *y, const int32_t *z,
                                   int64_t n, uint64_t *d_collisions, uint64_t *d_contacts,
                                   void *d_ws, size_t ws_bytes, unsigned flags,
                                   pairs_stream_t stream) {
    PAIRS_TRY(lattice_args(x, y, z, d_collisions, d_contacts, n, flags));
    if (n > PAIRS_LATTICE_MAX_BEADS) return PAIRS_ERR_INVALID_ARG;
    const bool global = n > lat::kMaxLdsBeads;
    if (global && (!d_ws || ws_bytes < lattice_ws_bytes(n, n))) return PAIRS_ERR_WORKSPACE;
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    hipStream_t s = (hipStream_t)stream;
    const bool validate = flags & PAIRS_FLAG_VALIDATE;
    lat::IO io{x, y, z, nullptr, 1, n, d_collisions, d_contacts, nullptr};
    PAIRS_TRY(lattice_flag(st, validate, s, &io.flag));
    if (!global) {
        PAIRS_TRY(lattice_lds(io, std::max<int64_t>(n, 2), false, st, s));
    } else {
        int tlog = 1;
        while ((int64_t(1) << tlog) < 2 * n) ++tlog;
        lat::SingleState *g = (lat::SingleState *)d_ws;
        uint64_t *table = (uint64_t *)((unsigned char *)d_ws + 256);
        const unsigned blocks =
            (unsigned)std::min<int64_t>(blocks_for(n, lat::kBlock), (int64_t)st->n_cu * 8);
        const unsigned clear_blocks = (unsigned)std::min<int64_t>(
            blocks_for(int64_t(1) << tlog, lat::kBlock), (int64_t)st->n_cu * 8);
        lat::k_lattice_single_init<<<1, 64, 0, s>>>(g, d_collisions, d_contacts);
        lat::k_lattice_single_box<<<blocks, lat::kBlock, 0, s>>>(io, g);
        lat::k_lattice_single_clear<<<clear_blocks, lat::kBlock, 0, s>>>(io, g, table, tlog);
        lat::k_lattice_single_pass<false><<<blocks, lat::kBlock, 0, s>>>(io, g, table, tlog);
        if (d_contacts)
            lat::k_lattice_single_pass<true><<<blocks, lat::kBlock, 0, s>>>(io, g, table, tlog);
        PAIRS_HIP_CHECK(hipGetLastError());
    }
    return validate ? lattice_status(st, s) : PAIRS_OK;
}

pairs_status_t pairs_lattice_count_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                                           const int64_t *d_offsets, int64_t n_sets,
                                           int64_t n_total, int64_t max_n,
                                           uint64_t *d_collisions, uint64_t *d_contacts,
                                           void *d_ws, size_t ws_bytes, unsigned flags,
                                           pairs_stream_t stream) {
    PAIRS_TRY(batched_args(x, y, z, d_offsets, n_sets, n_total, flags));
    PAIRS_TRY(lattice_args(x, y, z, d_collisions, d_contacts, n_total, flags));
    if (max_n < 0) return PAIRS_ERR_INVALID_ARG;
    const bool global = max_n == 0 || max_n > lat::kMaxLdsBeads;
    if (global && (!d_ws || ws_bytes < lattice_ws_bytes(n_total, max_n)))
        return PAIRS_ERR_WORKSPACE;
    DeviceState *st;
    PAIRS_TRY(device_state(&st));
    hipStream_t s = (hipStream_t)stream;
    const bool validate = flags & PAIRS_FLAG_VALIDATE;
    if (validate) PAIRS_TRY(validate_offsets(d_offsets, n_sets, n_total, s));
    if (n_sets == 0) return PAIRS_OK;
    lat::IO io{x, y, z, d_offsets, n_sets, n_total, d_collisions, d_contacts, nullptr};
    PAIRS_TRY(lattice_flag(st, validate, s, &io.flag));
    const int64_t m = global ? lat::kMaxLdsBeads : std::max<int64_t>(max_n, 2);
    PAIRS_TRY(lattice_lds(io, m, global, st, s));
    if (global) {
        const unsigned blocks = (unsigned)std::min<int64_t>(n_sets, (int64_t)st->n_cu * 4);
        uint64_t *table = (uint64_t *)((unsigned char *)d_ws + 256);
        if (d_contacts)
            lat::k_lattice_global<true><<<blocks, lat::kBlock, 0, s>>>(io, table);
        else
            lat::k_lattice_global<false><<<blocks, lat::kBlock, 0, s>>>(io, table);
        PAIRS_HIP_CHECK(hipGetLastError());
    }
    return validate ? lattice_status(st, s) : PAIRS_OK;
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

pairs_status_t pairs_debug_step_ranges(int n, int rows_per_lane, int chunk, int32_t *out,
                                       int64_t capacity, int64_t *n_tasks) {
    if (n < 0 || !n_tasks || (rows_per_lane != 1 && rows_per_lane != 2) || chunk <= 0)
        return PAIRS_ERR_INVALID_ARG;
    const Band band = Band::of(n);
    const StepTiling til = StepTiling::of(band, rows_per_lane, chunk);
    *n_tasks = til.tasks();
    if (!out) return PAIRS_OK;
    if (capacity < til.tasks()) return PAIRS_ERR_WORKSPACE;
    int64_t k = 0;
    for (int b = 0; b < til.nblocks; ++b)
        for (int c = 0; c < til.nchunks; ++c, ++k) {
            int r0, s0, T, x;
            step_range(band, til, b, c, &r0, &s0, &T, &x);
            out[4 * k] = r0;
            out[4 * k + 1] = s0;
            out[4 * k + 2] = T;
            out[4 * k + 3] = x;
        }
    return PAIRS_OK;
}
