// The exact int32 count on the matrix cores.
//
// The Gram form of the collision test (tasks.h) decides
//   x_i x_j + y_i y_j + z_i z_j + r_i r_j - h_i >= h_j,   h = (|p|^2 - r^2) / 2,
// and its sum of four products is one entry of the product of a 16 x 4 tile
// of rows (x, y, z, r) and a 4 x 16 tile of partners: v_mfma_f64_16x16x4f64
// computes 256 of them at once, with -h_i as the accumulator input, and the
// VALU is left one comparison per pair.  Inside the double form's box
// (coordinates in [-2^24, 2^24), radii in [0, 2^25)) every product and every
// partial sum is an integer below 2^52, so the matrix unit's fused
// multiply-adds are exact whatever order it sums in, and the result is the
// same integer predicate as the VALU forms'.  A group of partners (or a task
// of rows) outside that box takes the VALU's wide test instead.
//
// Operand layout of v_mfma_f64_16x16x4f64 (one double per lane for A and B,
// four for the accumulator), with l the lane:
//   A: lane l holds A[i = l % 16][k = l / 16]   (row i, coordinate k)
//   B: lane l holds B[k = l / 16][j = l % 16]   (coordinate k, partner j)
//   D: lane l holds D[i = l / 16 + 4 v][j = l % 16] for v = 0 .. 3.
//
// A task is the broadcast form's (band.h Tiling with one row per lane): 64
// consecutive rows, as four 16-row tiles, against a chunk of virtual
// partners staged 64 at a time in LDS as five arrays (x, y, z, r, h) of
// doubles, each group read as four 16-partner tiles.
#pragma once

#include "tasks.h"

namespace pairs_dev {

typedef double mfma_d4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaRowTiles = 4;  // 16-row tiles per task: 64 rows

template <typename BandT = Band>
__device__ __forceinline__ uint32_t count_i32_task_mfma(const int32_t *__restrict__ px,
                                                        const int32_t *__restrict__ py,
                                                        const int32_t *__restrict__ pz,
                                                        const int32_t *__restrict__ pr,
                                                        int64_t base, const BandT band, int ra,
                                                        int u0, int u1, void *__restrict__ lds,
                                                        const TaskInputs<int32_t, 1> &in) {
    double *win = (double *)lds;
    const int lane = lane_id();
    const int li = lane & 15, lk = lane >> 4;
    // The tiles' A operands (coordinate lk of row 16 t + li) and accumulator
    // inputs (-h of rows 16 t + lk + 4 v); padding rows have A = 0 and
    // -h = -inf, so they never hit.
    double a[kMfmaRowTiles];
    mfma_d4 c[kMfmaRowTiles];
    bool rows_in = true;
#pragma unroll
    for (int t = 0; t < kMfmaRowTiles; ++t) {
        const int i = ra + 16 * t + li;
        double X = 0.0, Y = 0.0, Z = 0.0, R = 0.0, H = INFINITY;
        if (i < band.n) {
            const int64_t g = base + i;
            const int32_t x = px[g], y = py[g], z = pz[g], r = pr[g];
            gram_features(x, y, z, r, X, Y, Z, R, H);
            rows_in = rows_in && in_box<kBoxBitsF64>(x, y, z, r);
        }
        a[t] = lk == 0 ? X : lk == 1 ? Y : lk == 2 ? Z : R;
#pragma unroll
        for (int v = 0; v < 4; ++v) c[t][v] = -__shfl(H, lk + 4 * v, kWave);
    }
    const bool rows_plain = wave_all(rows_in);
    // the lane's own row (ra + lane), for groups that take the wide test
    const int row = ra + lane;
    const bool row_live = row < band.n;
    const double xr = row_live ? (double)in.x[0] : 0.0, yr = row_live ? (double)in.y[0] : 0.0,
                 zr = row_live ? (double)in.z[0] : 0.0, rr = row_live ? (double)in.r[0] : 0.0;
    const int nsteps = row_live ? band.steps(row) : 0;
    const int rlast = min(ra + kWave, band.n) - 1;
    const int core_lo = rlast + 1;            // every row has u - 1 >= row
    const int core_hi = ra + band.steps(ra);  // every row has u <= row + steps(row)

    uint32_t cnt = 0, lane_cnt = 0;
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
            const int u = g0 + kWave + lane;
            if (u < u1) {
                const int64_t g = partner_index(base, band, u);
                qx = px[g]; qy = py[g]; qz = pz[g]; qr = pr[g];
            }
        }
        wave_sync();
        const int gn = __builtin_amdgcn_readfirstlane(min(kWave, u1 - g0));
        if (!plain) {
            for (int t = 0; t < gn; ++t) {
                const double jx = win[t], jy = win[kWave + t], jz = win[2 * kWave + t],
                             jr = win[3 * kWave + t];
                cnt += count_bits_both(wide_hit_f64(xr, yr, zr, rr, jx, jy, jz, jr),
                                       owns(g0 + t, row, nsteps));
            }
        } else if (g0 >= core_lo && g0 + gn - 1 <= core_hi) {
            // every row owns every partner of the group (padding partners
            // have h = inf and never hit)
            // all sixteen products of the group first, so that the matrix
            // unit's latency is covered before the comparisons read them
            double b[4], hj[4];
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) {
                b[pt] = win[lk * kWave + 16 * pt + li];
                hj[pt] = win[4 * kWave + 16 * pt + li];
            }
            mfma_d4 d[4][kMfmaRowTiles];
#pragma unroll
            for (int pt = 0; pt < 4; ++pt)
#pragma unroll
                for (int t = 0; t < kMfmaRowTiles; ++t)
                    d[pt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[pt], c[t], 0, 0, 0);
            // hits tallied per lane on the VALU, which has slack beside the
            // matrix unit, rather than by ballots on the shared scalar unit
#pragma unroll
            for (int pt = 0; pt < 4; ++pt)
#pragma unroll
                for (int t = 0; t < kMfmaRowTiles; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) lane_cnt += d[pt][t][v] >= hj[pt] ? 1u : 0u;
        } else {
            // a band edge: each result also needs its row to own the partner
            for (int pt = 0; pt < 4; ++pt) {
                if (16 * pt >= gn) break;
                const double b = win[lk * kWave + 16 * pt + li];
                const double hj = win[4 * kWave + 16 * pt + li];
                const int u = g0 + 16 * pt + li;
#pragma unroll
                for (int t = 0; t < kMfmaRowTiles; ++t) {
                    const mfma_d4 d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b, c[t], 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = ra + 16 * t + lk + 4 * v;
                        cnt += count_bits_both(d[v] >= hj, owns(u, i, band.steps(i)));
                    }
                }
            }
        }
        wave_sync();
    }
    if (__builtin_amdgcn_ballot_w64(lane_cnt != 0))
        for (int o = kWave / 2; o >= 1; o >>= 1) lane_cnt += __shfl_xor(lane_cnt, o, kWave);
    return cnt + __builtin_amdgcn_readfirstlane(lane_cnt);
}

}  // namespace pairs_dev
