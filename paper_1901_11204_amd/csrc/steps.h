// Row-stepping wave tasks for batches of sets.
//
// This is the paper's own form of the balanced assignment (Section 4): every
// row is a work item and at step s it evaluates the pair with object
// (row + s) mod n.  Here each lane holds K (1 or 2) consecutive rows, so the
// partner of its row k at step s is object r0 + K l + (s + k) and the sweep
// position tau = s - s0 + k addresses the same object for all K rows: one
// window read feeds K pair tests.  The window of the task's partners is
// staged once into wave-private LDS in a K-interleaved layout (residue
// c = tau mod K, entry l + tau div K), so the 64 lanes read 64 consecutive
// entries.  Unlike the broadcast sweep, no lane idles at the band edges: each
// row runs exactly its own steps, and only the extra step of an even n needs
// a per-row mask.
//
// A task holds m segments of w lanes.  A row block of one set is one segment
// of 64 lanes.  A pack is m whole sets of the same size n, ceil(n/K) lanes
// each, so that many small sets share a wave.
//
// A task runs in three phases: load (the lane's raw rows and window objects
// into registers), stage (convert them into LDS records) and sweep.  Keeping
// the load apart lets a persistent wave issue the next task's loads before
// it sweeps the current one.
#pragma once

#include <math.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "band.h"
#include "device.h"
#include "tasks.h"

namespace pairs_dev {

// Lambdas of the task bodies are inlined like the bodies themselves, so that
// what they capture stays in registers.
#define PAIRS_INLINE __attribute__((always_inline))

// Window capacity of one wave in records (m * K * S <= kStepCap): 416
// records of 24 bytes keep four waves of the int32 count per SIMD within the
// 160 KB of LDS of a CU.
constexpr int kStepCap = 416;

// What a stepping task covers.  Segment j holds rows [r0, r0 + K w) of its set
// in lanes [j w, (j + 1) w); every row runs the steps [s0, s0 + T), and the
// rows below half also run the step s0 + T when x is 1.
struct StepGeom {
    int n, half;
    int r0, s0, T, x;
    int m, w, S;
};

// Window entries per residue for K rows per lane over w lanes: the sweep
// position tau runs over [0, T + x + K - 1).
__host__ __device__ constexpr int step_window_entries(int K, int w, int T, int x) {
    return w + (T + x + K - 1 + K - 1) / K;
}

// Window entries one lane stages per residue: ceil(S / w) is at most 6 for
// K = 1 (row blocks with at most 288 steps) and 4 for K = 2 (at most 272
// steps); packs of whole sets need at most 3 for either K.
template <int K>
__host__ __device__ constexpr int step_iters() {
    return K == 1 ? 6 : 4;
}

__device__ __forceinline__ StepGeom step_geom(int n, int K, int r0, int s0, int T, int x, int m,
                                              bool pack) {
    StepGeom g;
    g.n = n;
    g.half = (n % 2 == 0) ? n / 2 : 0;
    g.r0 = r0;
    g.s0 = s0;
    g.T = T;
    g.x = x;
    g.m = m;
    g.w = pack ? (n + K - 1) / K : kWave;
    g.S = step_window_entries(K, g.w, T, x);
    return g;
}

// Per-lane placement: segment j, lane l within it, and whether the lane holds
// any set at all.  Idle lanes read segment 0's first entries.
struct StepLane {
    int j, l;
    bool live;
};

template <bool Pack>
__device__ __forceinline__ StepLane step_lane(const StepGeom &g) {
    const int lane = lane_id();
    StepLane p;
    if (!Pack) {  // one segment of all 64 lanes
        p.j = 0;
        p.l = lane;
        p.live = true;
        return p;
    }
    p.j = lane / g.w;
    p.l = lane - p.j * g.w;
    p.live = p.j < g.m;
    if (!p.live) {
        p.j = 0;
        p.l = 0;
    }
    return p;
}

// Object of window entry q of residue c (mod n); n or more marks a sentinel
// (past 2n, only ever read by padding rows).
__device__ __forceinline__ int step_entry_object(const StepGeom &g, int K, int q, int c) {
    int o = g.r0 + g.s0 + K * q + c;
    return o >= g.n ? o - g.n : o;
}

// ------------------------------------------------------------------ load --

// The raw values one lane needs: its K rows and its window entries
// ent[c * step_iters<K>() + i] (entry q = l + w i of residue c); each holds
// x, y, z, r.  Slots outside the task stay unread.
template <typename T>
struct Vec4;
template <>
struct Vec4<int32_t> {
    typedef int4 type;
    static __device__ __forceinline__ int4 make(int32_t a, int32_t b, int32_t c, int32_t d) {
        return make_int4(a, b, c, d);
    }
};
template <>
struct Vec4<float> {
    typedef float4 type;
    static __device__ __forceinline__ float4 make(float a, float b, float c, float d) {
        return make_float4(a, b, c, d);
    }
};

template <typename T>
struct StepRaw {
    typename Vec4<T>::type row0, row1;
    typename Vec4<T>::type ent0, ent1, ent2, ent3, ent4, ent5, ent6, ent7;
};

// Slot S of a raw struct, resolved at compile time so that the struct stays
// in registers.
template <int S, typename R>
__device__ __forceinline__ auto &raw_slot(R &r) {
    static_assert(S >= 0 && S < 8, "eight window slots");
    if constexpr (S == 0) return r.ent0;
    else if constexpr (S == 1) return r.ent1;
    else if constexpr (S == 2) return r.ent2;
    else if constexpr (S == 3) return r.ent3;
    else if constexpr (S == 4) return r.ent4;
    else if constexpr (S == 5) return r.ent5;
    else if constexpr (S == 6) return r.ent6;
    else return r.ent7;
}

template <int S, typename R>
__device__ __forceinline__ auto &raw_row(R &r) {
    if constexpr (S == 0) return r.row0;
    else return r.row1;
}

// Calls f(std::integral_constant<int, I>) for I = 0 .. N-1.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Returns the loaded values by value (not through a reference), so that the
// two shapes' loads of one task merge as register values.  A pack covers whole
// sets, so its window holds only objects of its own rows: only the rows are
// loaded, and staging places each row in the window (step_stage).
template <typename T, int K, bool WithR, bool Pack>
__device__ __forceinline__ StepRaw<T> step_load(const T *__restrict__ X, const T *__restrict__ Y,
                                                const T *__restrict__ Z, const T *__restrict__ R,
                                                int64_t base, const StepGeom &g,
                                                const StepLane &p) {
    StepRaw<T> raw{};
    static_for<K>([&](auto kc) PAIRS_INLINE {
        constexpr int k = decltype(kc)::value;
        const int r = g.r0 + K * p.l + k;
        if (p.live && r < g.n) {
            const int64_t o = base + r;
            raw_row<k>(raw) = Vec4<T>::make(X[o], Y[o], Z[o], WithR ? R[o] : T(0));
        }
    });
    if (Pack) return raw;
    static_for<K * step_iters<K>()>([&](auto sc) PAIRS_INLINE {
        constexpr int slot = decltype(sc)::value;
        constexpr int c = slot / step_iters<K>(), i = slot % step_iters<K>();
        const int q = p.l + g.w * i;
        const int o = step_entry_object(g, K, q, c);
        if (p.live && q < g.S && o < g.n) {
            const int64_t go = base + o;
            raw_slot<slot>(raw) = Vec4<T>::make(X[go], Y[go], Z[go], WithR ? R[go] : T(0));
        }
    });
    return raw;
}

// Stage, then synchronise the wave.  rec(e, valid, vals) writes entry e.
// Row blocks write every staged entry (a converted record or a sentinel).  A
// pack (whole sets, r0 = 0, s0 = 1) writes each of its rows o to the window
// positions v = o - 1 and v = o - 1 + n that exist: every position below
// 2n - 1 holds object (v + 1) mod n, and no row of a pack reads past it.
template <typename T, int K, bool Pack, typename Rec>
__device__ __forceinline__ void step_stage(const StepGeom &g, const StepLane &p,
                                           const StepRaw<T> &raw, Rec &&rec) {
    if (Pack) {
        static_for<K>([&](auto kc) PAIRS_INLINE {
            constexpr int k = decltype(kc)::value;
            const int o = K * p.l + k;
            if (p.live && o < g.n) {
                const auto &v = raw_row<k>(raw);
                const int v1 = o - 1, v2 = o - 1 + g.n, lim = K * g.S;
                const int seg = p.j * K * g.S;
                if (v1 >= 0 && v1 < lim) rec(seg + (v1 % K) * g.S + v1 / K, true, v);
                if (v2 < lim) rec(seg + (v2 % K) * g.S + v2 / K, true, v);
            }
        });
        wave_sync();
        return;
    }
    static_for<K * step_iters<K>()>([&](auto sc) PAIRS_INLINE {
        constexpr int slot = decltype(sc)::value;
        constexpr int c = slot / step_iters<K>(), i = slot % step_iters<K>();
        const int q = p.l + g.w * i;
        if (p.live && q < g.S) {
            const int o = step_entry_object(g, K, q, c);
            rec((p.j * K + c) * g.S + q, o < g.n, raw_slot<slot>(raw));
        }
    });
    wave_sync();
}

// ----------------------------------------------------------------- sweep --
//
// test(e, k, masked) evaluates window entry e for row slice k; masked asks
// for the even-n extra step (rows below half only).  e0 is the lane's entry
// of sweep position 0.  Position tau is entry e0 + (tau mod K) S + tau div K;
// every (tau, k) with 0 <= tau - k < T is tested unmasked, and (T + k, k)
// masked when x is 1.  The main loop tests kStepUnroll positions per row and
// iteration (which bounds the window records in flight, and so the
// registers); fold() runs at least once every kStepUnroll + 2 tests of a row.
constexpr int kStepUnroll = 8;

//
// group(ea, eb) tests every row slice against both entries ea and eb, all
// unmasked; the main loops use it so that a kind can interleave the
// independent dependency chains of several tests.
template <int K, typename Test, typename Group, typename Fold>
__device__ __forceinline__ void step_sweep(const StepGeom &g, int e0, Test &&test, Group &&group,
                                           Fold &&fold) {
    const int T = g.T;
    if (K == 1) {
        int tau = 0;
        for (; tau + kStepUnroll <= T; tau += kStepUnroll) {
#pragma unroll
            for (int d = 0; d < kStepUnroll; d += 2) group(e0 + tau + d, e0 + tau + d + 1);
            fold();
        }
        for (; tau < T; ++tau) test(e0 + tau, 0, false);
        if (g.x) test(e0 + T, 0, true);
        fold();
    } else {
        // tau = 0: row 0 only (entry e0)
        if (T > 0) test(e0, 0, false);
        // tau in [1, T) in pairs: tau = 2u + 1 is entry e0 + S + u (residue
        // 1), tau = 2u + 2 is entry e0 + 1 + u (residue 0)
        const int b1 = e0 + g.S, b0 = e0 + 1;
        const int pairs = (T - 1) / 2;  // both positions below T
        int u = 0;
        for (; u + kStepUnroll / 2 <= pairs; u += kStepUnroll / 2) {
#pragma unroll
            for (int d = 0; d < kStepUnroll / 2; ++d) group(b1 + u + d, b0 + u + d);
            fold();
        }
        for (; u < pairs; ++u) {
            test(b1 + u, 0, false);
            test(b1 + u, 1, false);
            test(b0 + u, 0, false);
            test(b0 + u, 1, false);
        }
        fold();
        // an odd last position tau = T - 1 (when T - 1 is odd)
        if (T >= 2 && ((T - 1) & 1)) {
            test(b1 + pairs, 0, false);
            test(b1 + pairs, 1, false);
        }
        // tau = T: row 1's last common step, and row 0's extra step
        const int eT = e0 + (T & 1) * g.S + T / 2;
        if (T > 0) test(eT, 1, false);
        if (g.x) {
            test(eT, 0, true);
            const int eT1 = e0 + ((T + 1) & 1) * g.S + (T + 1) / 2;
            test(eT1, 1, true);
        }
        fold();
    }
}

// ------------------------------------------------------------- int32 count --

struct StepCountResult {
    uint32_t wave;  // hits summed over the wave (single-segment tasks)
    uint32_t lane;  // hits of this lane's rows (packs)
};

// The Gram test of a row against a window record.  The empty asm statement
// makes the row's 32-bit values loop-carried, so that their sign extension is
// not hoisted out of the sweep; with it in the loop body each product is
// selected as a single 32x32->64-bit multiply-add instead of a full
// 64x64-bit product.  It emits no instruction.
__device__ __forceinline__ bool step_hit_i32(RowI32 &r, int4 b, int64_t qb) {
    asm("" : "+v"(r.ax), "+v"(r.ay), "+v"(r.az), "+v"(r.ar));
    int64_t v = r.nq + (int64_t)r.ax * b.x;
    v += (int64_t)r.ay * b.y;
    v += (int64_t)r.az * b.z;
    v += (int64_t)r.ar * b.w;
    return v >= qb;
}

// Exact int32 count of one stepping task (int64 Gram form, as the broadcast
// sweep's narrow blocks).  Pack counts per lane (multi-segment tasks); a
// single segment counts with wave ballots.  hook() runs between staging and
// the sweep.
template <int K, bool Pack, typename Hook>
__device__ __forceinline__ StepCountResult step_count_i32(const StepRaw<int32_t> &raw,
                                                          const StepGeom &g, void *__restrict__ lds,
                                                          Hook &&hook) {
    int4 *wa = (int4 *)lds;
    int64_t *wq = (int64_t *)((char *)lds + kStepCap * sizeof(int4));
    const StepLane p = step_lane<Pack>(g);
    RowI32 rows[K];
    bool extra[K];
    bool in = true;  // rows and staged entries of this lane inside the plain test's box
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int r = g.r0 + K * p.l + k;
        extra[k] = r < g.half;
        if (p.live && r < g.n) {
            const int4 v = k == 0 ? raw.row0 : raw.row1;  // k is a constant here
            rows[k] = gram_row(v.x, v.y, v.z, v.w);
            in = in && in_box<kBoxBitsI64>(v.x, v.y, v.z, v.w);
        } else {
            rows[k].ax = rows[k].ay = rows[k].az = rows[k].ar = 0;
            rows[k].nq = -((int64_t)1 << 62);  // never hits
        }
    }
    step_stage<int32_t, K, Pack>(g, p, raw, [&](int e, bool valid, const int4 &v) PAIRS_INLINE {
        wa[e] = valid ? v : make_int4(0, 0, 0, 0);
        wq[e] = valid ? gram_q(v.x, v.y, v.z, v.w) : INT64_MAX;  // sentinel: never reached
        in = in && (!valid || in_box<kBoxBitsI64>(v.x, v.y, v.z, v.w));
    });
    hook();
    const int e0 = (p.j * K) * g.S + p.l;
    StepCountResult res{0u, 0u};
    auto tally = [&](bool hit) PAIRS_INLINE {
        if (Pack)
            res.lane += hit ? 1u : 0u;
        else
            res.wave += count_bits(hit);
    };
    if (!wave_all(in)) {
        // a row or window object outside the plain test's box: the wide test
        // for the whole task (sentinel entries, q = INT64_MAX, are read only
        // by padding rows, whose results are not counted)
        auto wide = [&](int e, int k, bool masked) PAIRS_INLINE {
            const int4 v = wa[e];
            bool hit = gram_hit_wide(rows[k], PartnerI32{v.x, v.y, v.z, v.w}, wq[e]);
            if (masked) hit = hit && extra[k];
            tally(hit && (p.live && g.r0 + K * p.l + k < g.n));
        };
        step_sweep<K>(
            g, e0, wide,
            [&](int ea, int eb) PAIRS_INLINE {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    wide(ea, k, false);
                    wide(eb, k, false);
                }
            },
            []() PAIRS_INLINE {});
        wave_sync();
        return res;
    }
    step_sweep<K>(
        g, e0,
        [&](int e, int k, bool masked) PAIRS_INLINE {
            bool hit = step_hit_i32(rows[k], wa[e], wq[e]);
            if (masked) hit = hit && extra[k];
            tally(hit);
        },
        [&](int ea, int eb) PAIRS_INLINE {
            // 2K independent multiply-add chains, advanced in lockstep: a
            // dependent 64-bit multiply-add waits on its predecessor, so a
            // wave needs several chains in flight to issue every cycle
            const int4 a = wa[ea], b = wa[eb];
            const int64_t qa = wq[ea], qb = wq[eb];
            int64_t va[K], vb[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                asm("" : "+v"(rows[k].ax), "+v"(rows[k].ay), "+v"(rows[k].az), "+v"(rows[k].ar));
                va[k] = rows[k].nq + (int64_t)rows[k].ax * a.x;
                vb[k] = rows[k].nq + (int64_t)rows[k].ax * b.x;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                va[k] += (int64_t)rows[k].ay * a.y;
                vb[k] += (int64_t)rows[k].ay * b.y;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                va[k] += (int64_t)rows[k].az * a.z;
                vb[k] += (int64_t)rows[k].az * b.z;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                va[k] += (int64_t)rows[k].ar * a.w;
                vb[k] += (int64_t)rows[k].ar * b.w;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                tally(va[k] >= qa);
                tally(vb[k] >= qb);
            }
        },
        []() PAIRS_INLINE {});
    wave_sync();  // the window is reused by the next task
    return res;
}

// ------------------------------------------------------------- float32 kinds --

// Pinned binary32 count (Pack and hook as above).
template <int K, bool Pack, typename Hook>
__device__ __forceinline__ StepCountResult step_count_f32(const StepRaw<float> &raw,
                                                          const StepGeom &g, void *__restrict__ lds,
                                                          Hook &&hook) {
    float4 *wa = (float4 *)lds;
    const StepLane p = step_lane<Pack>(g);
    float xr[K], yr[K], zr[K], rr[K];
    bool extra[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int r = g.r0 + K * p.l + k;
        extra[k] = r < g.half;
        if (p.live && r < g.n) {
            const float4 v = k == 0 ? raw.row0 : raw.row1;
            xr[k] = v.x; yr[k] = v.y; zr[k] = v.z; rr[k] = v.w;
        } else {
            xr[k] = INFINITY;  // infinite distance: never hits
            yr[k] = zr[k] = rr[k] = 0.0f;
        }
    }
    step_stage<float, K, Pack>(g, p, raw, [&](int e, bool valid, const float4 &v) PAIRS_INLINE {
        wa[e] = valid ? v : make_float4(-INFINITY, 0.0f, 0.0f, 0.0f);
    });
    hook();
    const int e0 = (p.j * K) * g.S + p.l;
    StepCountResult res{0u, 0u};
    auto test = [&](int e, int k, bool masked) PAIRS_INLINE {
        const float4 b = wa[e];
        bool hit = hit_f32(xr[k], yr[k], zr[k], rr[k], b.x, b.y, b.z, b.w);
        if (masked) hit = hit && extra[k];
        if (Pack) {
            res.lane += hit ? 1u : 0u;
        } else {
            res.wave += count_bits(hit);
        }
    };
    step_sweep<K>(
        g, e0, test,
        [&](int ea, int eb) PAIRS_INLINE {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                test(ea, k, false);
                test(eb, k, false);
            }
        },
        []() PAIRS_INLINE {});
    wave_sync();
    return res;
}

struct StepEnergyResult {
    double lane_energy;  // energy of this lane's rows (row side: each pair once)
    uint32_t wave;       // hits over the wave (single segment, WithCount)
    uint32_t lane;       // hits of this lane's rows (packs, WithCount)
};

// Softened potential summed over the task's pairs, optionally with the pinned
// binary32 count on the same differences (WithCount); float32 partials of at
// most kFoldEvery terms per row are folded into double accumulators.
template <int K, bool Pack, bool WithCount, typename Hook>
__device__ __forceinline__ StepEnergyResult step_energy(const StepRaw<float> &raw,
                                                        const StepGeom &g, float eps2,
                                                        void *__restrict__ lds, Hook &&hook) {
    float4 *wa = (float4 *)lds;
    const StepLane p = step_lane<Pack>(g);
    float xr[K], yr[K], zr[K], rr[K], part[K];
    double acc[K];
    bool extra[K], live_row[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int r = g.r0 + K * p.l + k;
        extra[k] = r < g.half;
        live_row[k] = p.live && r < g.n;
        if (live_row[k]) {
            const float4 v = k == 0 ? raw.row0 : raw.row1;
            xr[k] = v.x; yr[k] = v.y; zr[k] = v.z;
            rr[k] = WithCount ? v.w : 0.0f;
        } else {
            xr[k] = INFINITY;  // infinite distance: e is exactly 0, never hits
            yr[k] = zr[k] = rr[k] = 0.0f;
        }
        part[k] = 0.0f;
        acc[k] = 0.0;
    }
    step_stage<float, K, Pack>(g, p, raw, [&](int e, bool valid, const float4 &v) PAIRS_INLINE {
        wa[e] = valid ? make_float4(v.x, v.y, v.z, WithCount ? v.w : 0.0f)
                      : make_float4(-INFINITY, 0.0f, 0.0f, 0.0f);
    });
    hook();
    const int e0 = (p.j * K) * g.S + p.l;
    StepEnergyResult res{0.0, 0u, 0u};
    auto test = [&](int ent, int k, bool masked) PAIRS_INLINE {
        const float4 b = wa[ent];
        const float dx = xr[k] - b.x, dy = yr[k] - b.y, dz = zr[k] - b.z;
        float e;
        if (WithCount) {
            const float d2 = sq_dist_f32(dx, dy, dz);
            const float Rs = __fadd_rn(rr[k], b.w);
            bool hit = d2 <= __fmul_rn(Rs, Rs);
            if (masked) hit = hit && extra[k];
            if (Pack) {
                res.lane += hit ? 1u : 0u;
            } else {
                res.wave += count_bits(hit);
            }
            e = __builtin_amdgcn_rsqf(d2 + eps2);
        } else {
            float d2 = __builtin_fmaf(dx, dx, eps2);
            d2 = __builtin_fmaf(dy, dy, d2);
            d2 = __builtin_fmaf(dz, dz, d2);
            e = __builtin_amdgcn_rsqf(d2);
        }
        if (masked) e = extra[k] ? e : 0.0f;
        part[k] += e;
    };
    step_sweep<K>(
        g, e0, test,
        [&](int ea, int eb) PAIRS_INLINE {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                test(ea, k, false);
                test(eb, k, false);
            }
        },
        [&]() PAIRS_INLINE {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                acc[k] += (double)part[k];
                part[k] = 0.0f;
            }
        });
    wave_sync();
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (live_row[k]) tot += acc[k];
    res.lane_energy = tot;
    return res;
}

// Sums of per-lane values over each segment of w lanes, through the window
// (after the sweep): on return lane j < m holds the sum of segment j.  Four
// independent partial sums keep the LDS reads of a segment in flight together.
template <typename T>
__device__ __forceinline__ T segment_sum(T v, const StepGeom &g, void *__restrict__ lds) {
    T *s = (T *)lds;
    const int lane = lane_id();
    s[lane] = v;
    wave_sync();
    T tot = T(0);
    if (lane < g.m) {
        const T *seg = s + lane * g.w;
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
        int i = 0;
        for (; i + 4 <= g.w; i += 4) {
            a0 += seg[i];
            a1 += seg[i + 1];
            a2 += seg[i + 2];
            a3 += seg[i + 3];
        }
        for (; i < g.w; ++i) a0 += seg[i];
        tot = (a0 + a1) + (a2 + a3);
    }
    wave_sync();
    return tot;
}

}  // namespace pairs_dev
