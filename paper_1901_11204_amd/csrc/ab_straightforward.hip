// The benchmark's assignment comparison (declared in pairs_ab.h): the
// balanced circular assignment against the straightforward triangular one,
// run by the same wave task body, one wave per row block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "band.h"
#include "device.h"
#include "pairs_ab.h"
#include "tasks.h"

using namespace pairs_dev;

namespace {

constexpr int kWavesPerBlock = 4;

__global__ void k_zero(uint64_t *p) { *p = 0; }

// One wave per row block [ra, ra + 64K): all of the block's pairs in one task.
// times (optional): the wave's start and end on the device's constant-rate
// wall clock, at times[2 blk] and times[2 blk + 1].
template <int K, typename BandT>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void k_ab_count(
    const int32_t *__restrict__ x, const int32_t *__restrict__ y, const int32_t *__restrict__ z,
    const int32_t *__restrict__ r, int n, uint64_t *out, uint64_t *times) {
    const uint64_t t0 = times ? wall_clock64() : 0;
    constexpr int kLds = 5 * kWave;  // words of the wider (double) partner record
    __shared__ double lds[kWavesPerBlock * kLds];
    const int wave = wave_id();
    const int64_t blk = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    const int ra = (int)blk * kWave * K;
    if (ra >= n) return;
    struct Stamp {
        uint64_t *t;
        int64_t b;
        uint64_t t0;
        __device__ ~Stamp() {
            if (t && lane_id() == 0) {
                t[2 * b] = t0;
                t[2 * b + 1] = wall_clock64();
            }
        }
    } stamp{times, blk, t0};
    const BandT band = BandT::of(n);
    const int rlast = min(ra + kWave * K, n) - 1;
    const int u0 = ra + 1;
    const int u1 = rlast + band.steps(rlast) + 1;  // last row's last partner, exclusive
    if (u0 >= u1) return;
    TaskInputs<int32_t, K> in;
    load_task_inputs<int32_t, K, K, true, BandT>(x, y, z, r, 0, band, ra, u0, u1, in);
    const uint32_t c = count_i32_task<K, K, BandT>(x, y, z, r, 0, band, ra, u0, u1,
                                                   lds + wave * kLds, in);
    if (lane_id() == 0 && c) atomicAdd((unsigned long long *)out, (unsigned long long)c);
}

int64_t ab_waves(int64_t n, int K) { return (n + kWave * K - 1) / (kWave * K); }

template <int K, typename BandT>
void launch(const int32_t *x, const int32_t *y, const int32_t *z, const int32_t *r, int n,
            uint64_t *out, uint64_t *times, hipStream_t s) {
    const int64_t blocks = (ab_waves(n, K) + kWavesPerBlock - 1) / kWavesPerBlock;
    k_ab_count<K, BandT><<<(unsigned)blocks, kWave * kWavesPerBlock, 0, s>>>(x, y, z, r, n, out,
                                                                            times);
}

int ab_run(int variant, const int32_t *x, const int32_t *y, const int32_t *z, const int32_t *r,
           int64_t n, int rows_per_lane, uint64_t *d_count, uint64_t *d_times, void *stream) {
    if ((variant != 0 && variant != 1) || n < 0 || n > (1 << 30) || !d_count ||
        (rows_per_lane != 1 && rows_per_lane != 8) || (n > 0 && (!x || !y || !z || !r)))
        return -1;
    hipStream_t s = (hipStream_t)stream;
    k_zero<<<1, 1, 0, s>>>(d_count);
    if (n >= 2) {
        const int nn = (int)n;
        if (variant == 0) {
            if (rows_per_lane == 8) launch<8, Band>(x, y, z, r, nn, d_count, d_times, s);
            else launch<1, Band>(x, y, z, r, nn, d_count, d_times, s);
        } else {
            if (rows_per_lane == 8) launch<8, TriBand>(x, y, z, r, nn, d_count, d_times, s);
            else launch<1, TriBand>(x, y, z, r, nn, d_count, d_times, s);
        }
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : -(int)e;
}

}  // namespace

extern "C" int pairs_ab_count_i32(int variant, const int32_t *x, const int32_t *y,
                                  const int32_t *z, const int32_t *r, int64_t n, int rows_per_lane,
                                  uint64_t *d_count, void *stream) {
    return ab_run(variant, x, y, z, r, n, rows_per_lane, d_count, nullptr, stream);
}

extern "C" int64_t pairs_ab_waves(int64_t n, int rows_per_lane) {
    if (n < 2 || (rows_per_lane != 1 && rows_per_lane != 8)) return 0;
    return ab_waves(n, rows_per_lane);
}

extern "C" int pairs_ab_count_i32_timed(int variant, const int32_t *x, const int32_t *y,
                                        const int32_t *z, const int32_t *r, int64_t n,
                                        int rows_per_lane, uint64_t *d_count, uint64_t *d_times,
                                        void *stream) {
    if (!d_times) return -1;
    return ab_run(variant, x, y, z, r, n, rows_per_lane, d_count, d_times, stream);
}

extern "C" int pairs_ab_wall_clock_khz(int64_t *khz) {
    int dev = 0, v = 0;
    if (!khz || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return -1;
    *khz = v;
    return 0;
}
