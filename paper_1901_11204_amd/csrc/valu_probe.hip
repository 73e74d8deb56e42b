// Issue-rate probe of the gfx950 vector instructions the pair kernels use.
//
// Each probe kernel runs kChains independent dependency chains of one
// instruction pattern per lane, kIters times, on a grid that fills every CU.
// The host times each kernel with HIP events; lane-operations per second
// against 256 CUs x 64 lanes x clock gives the issue cost of the pattern.
// Used to measure the per-pair cost of the predicates (not on the hot path).
//
// The LDS probes time wave-wide reads of 8 or 16 bytes per lane, every lane
// at one address (a broadcast) or at consecutive addresses (a gather), with
// one three-input add per 8 bytes to consume the data; their "lane
// operations" are lane reads.  The random-address LDS probes time the reads
// and atomics of a hash table.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kIters = 4096;

__global__ void p_fma_f64(double *out, double a, double b) {
    double c[kChains];
    for (int k = 0; k < kChains; ++k) c[k] = threadIdx.x * 1e-3 + k;
    for (int it = 0; it < kIters; ++it)
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = __builtin_fma(c[k], a, b);
    double s = 0;
    for (int k = 0; k < kChains; ++k) s += c[k];
    if (s == 12345.0) out[threadIdx.x] = s;
}

__global__ void p_fma_f32(float *out, float a, float b) {
    float c[kChains];
    for (int k = 0; k < kChains; ++k) c[k] = threadIdx.x * 1e-3f + k;
    for (int it = 0; it < kIters; ++it)
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = __builtin_fmaf(c[k], a, b);
    float s = 0;
    for (int k = 0; k < kChains; ++k) s += c[k];
    if (s == 12345.0f) out[threadIdx.x] = s;
}

// reciprocal square root alone
__global__ void p_rsq_f32(float *out, float a) {
    float c[2 * kChains];
    for (int k = 0; k < 2 * kChains; ++k) c[k] = threadIdx.x * 1e-3f + k + a;
    for (int it = 0; it < kIters / 2; ++it)
#pragma unroll
        for (int k = 0; k < 2 * kChains; ++k) c[k] = __builtin_amdgcn_rsqf(c[k]);
    float s = 0;
    for (int k = 0; k < 2 * kChains; ++k) s += c[k];
    if (s == 12345.0f) out[threadIdx.x] = s;
}

// the energy pattern: 3 fma + 1 rsq per step (4 instructions)
__global__ void p_fma3_rsq(float *out, float a, float b) {
    float c[kChains];
    for (int k = 0; k < kChains; ++k) c[k] = threadIdx.x * 1e-3f + k + 1.0f;
    for (int it = 0; it < kIters / 4; ++it)
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            float d = __builtin_fmaf(c[k], a, b);
            d = __builtin_fmaf(d, a, b);
            d = __builtin_fmaf(d, a, b);
            c[k] = __builtin_amdgcn_rsqf(d);
        }
    float s = 0;
    for (int k = 0; k < kChains; ++k) s += c[k];
    if (s == 12345.0f) out[threadIdx.x] = s;
}

// the count pattern: 4 fma_f64 + 1 cmp_f64, ballot + popcount into 32 bits
__global__ void p_count_f64(unsigned *out, double a, double b, double h) {
    double c[kChains];
    uint32_t cnt = 0;
    for (int k = 0; k < kChains; ++k) c[k] = threadIdx.x * 1e-3 + k;
    for (int it = 0; it < kIters / 5; ++it)
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            double v = __builtin_fma(c[k], a, b);
            v = __builtin_fma(v, a, b);
            v = __builtin_fma(v, a, b);
            c[k] = __builtin_fma(v, a, b);
            cnt += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(c[k] >= h));
        }
    if (cnt == 12345u) out[threadIdx.x] = cnt;
}

__global__ void p_mad_u64_u32(unsigned long long *out, unsigned a) {
    unsigned long long c[kChains];
    for (int k = 0; k < kChains; ++k) c[k] = threadIdx.x + k;
    for (int it = 0; it < kIters; ++it)
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = (unsigned long long)(unsigned)c[k] * a + c[k];
    unsigned long long s = 0;
    for (int k = 0; k < kChains; ++k) s += c[k];
    if (s == 12345ull) out[threadIdx.x] = s;
}

typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
constexpr int kLdsWords = 8192;  // 32 KB per block
constexpr int kLdsIters = 2048;  // 8 reads each

// Mode: 0 broadcast b128, 1 gather b128, 2 broadcast b64, 3 gather b64.
// Largest byte offset read: 63 * 16 + 7 * 2048 + 7 * 256 + 16 < 32 KB.
template <int Mode>
__global__ __launch_bounds__(256) void p_lds_read(uint32_t *out) {
    __shared__ __align__(16) uint32_t buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += 256) buf[i] = i * 2654435761u;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int lane_off = Mode == 1 ? lane * 16 : Mode == 3 ? lane * 8 : 0;
    const char *b = (const char *)buf;
    uint32_t acc = 0;
    for (int it = 0; it < kLdsIters; ++it) {
        const char *p = b + lane_off + (it & 7) * 2048;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (Mode <= 1) {
                const u4 v = *(const u4 *)(p + k * 256);
                acc = acc + v.x + v.y;  // v_add3_u32
                acc = acc + v.z + v.w;
            } else {
                const u2 v = *(const u2 *)(p + k * 256);
                acc = acc + v.x + v.y;
            }
        }
    }
    if (acc == 0x12345678u) out[threadIdx.x] = acc;
}

// Random-address LDS operations, as a hash table makes them: Mode 0 a
// 16-byte read, 1 a 32-bit atomic add returning the old value, 2 a 32-bit
// compare-and-swap (whose compare mostly fails), 3 a 32-bit atomic add
// without return.  Each lane draws its addresses from its own xorshift
// sequence; eight independent operations per step.  Indices stay inside the
// 32 KB buffer (masked).
template <int Mode>
__global__ __launch_bounds__(256) void p_lds_rand(uint32_t *out) {
    __shared__ __align__(16) uint32_t buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += 256) buf[i] = i * 2654435761u;
    __syncthreads();
    uint32_t h = (threadIdx.x + 1) * 0x9E3779B1u ^ (blockIdx.x * 0x85EBCA6Bu);
    uint32_t acc = 0;
    for (int it = 0; it < kLdsIters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            h ^= h << 13;
            h ^= h >> 17;
            h ^= h << 5;
            if (Mode == 0) {
                const u4 v = *(const u4 *)&buf[4 * ((h >> 8) & (kLdsWords / 4 - 1))];
                acc = acc + v.x + v.y;
                acc = acc + v.z + v.w;
            } else if (Mode == 1) {
                acc += atomicAdd(&buf[(h >> 8) & (kLdsWords - 1)], 1u);
            } else if (Mode == 2) {
                acc += atomicCAS(&buf[(h >> 8) & (kLdsWords - 1)], 0x12345u, h);
            } else {
                atomicAdd(&buf[(h >> 8) & (kLdsWords - 1)], 1u);
            }
        }
    }
    if (Mode == 3) acc = buf[threadIdx.x];
    if (acc == 0x12345678u) out[threadIdx.x] = acc;
}

}  // namespace

extern "C" {

// Probe names in order; pattern instruction counts per chain step.
const char *valu_probe_names =
    "fma_f64,fma_f32,rsq_f32,fma3_rsq_f32,count_f64,mad_u64_u32,"
    "lds_bcast_b128,lds_gather_b128,lds_bcast_b64,lds_gather_b64,"
    "lds_rand_b128,lds_rand_add_rtn_b32,lds_rand_cas_b32,lds_rand_add_b32";

// Runs probe `which` once (after one warm-up) on blocks x 256 threads and
// returns its duration in milliseconds in *ms and the number of lane
// instructions it issued in *lane_ops; returns a hipError_t.
int valu_probe_run(int which, int blocks, double *ms, double *lane_ops) {
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, 1 << 20);
    if (e != hipSuccess) return (int)e;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const double lanes = (double)blocks * 256;
    double per_lane = 0;
    for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0);
        switch (which) {
            case 0: p_fma_f64<<<blocks, 256>>>((double *)buf, 0.999, 1e-3); per_lane = kIters * kChains; break;
            case 1: p_fma_f32<<<blocks, 256>>>((float *)buf, 0.999f, 1e-3f); per_lane = kIters * kChains; break;
            case 2: p_rsq_f32<<<blocks, 256>>>((float *)buf, 1.0f); per_lane = (kIters / 2) * 2 * kChains; break;
            case 3: p_fma3_rsq<<<blocks, 256>>>((float *)buf, 0.999f, 1e-3f); per_lane = (kIters / 4) * kChains * 4; break;
            case 4: p_count_f64<<<blocks, 256>>>((unsigned *)buf, 0.999, 1e-3, 3.0); per_lane = (kIters / 5) * kChains * 5; break;
            case 5: p_mad_u64_u32<<<blocks, 256>>>((unsigned long long *)buf, 12345u); per_lane = kIters * kChains; break;
            case 6: p_lds_read<0><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 7: p_lds_read<1><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 8: p_lds_read<2><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 9: p_lds_read<3><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 10: p_lds_rand<0><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 11: p_lds_rand<1><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 12: p_lds_rand<2><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            case 13: p_lds_rand<3><<<blocks, 256>>>((uint32_t *)buf); per_lane = kLdsIters * 8; break;
            default: (void)hipFree(buf); return (int)hipErrorInvalidValue;
        }
        (void)hipEventRecord(e1);
        (void)hipEventSynchronize(e1);
    }
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t;
    *lane_ops = lanes * per_lane;
    e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return (int)e;
}

}  // extern "C"
