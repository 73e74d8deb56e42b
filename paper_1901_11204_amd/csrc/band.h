// Balanced circular pair assignment of one set (paper, Section 4: algorithm
// "Proposed algorithm for calculating SPI", the stopping step derived from the
// crossing of reach(s) and reached(s), and the even-N rule after
// Proposition 2).
//
// Row i of a set of n objects evaluates partners (i + s) mod n for
// s = 1 .. steps(i), steps(i) = floor((n-1)/2), plus one step s = n/2 for the
// rows i < n/2 when n is even.  Every unordered pair is evaluated once.
//
// The kernels sweep a "virtual partner" u = i + s in [i+1, i+steps(i)] (so
// u < 2n and the partner is u or u - n).  For a fixed u the rows that evaluate
// a partner at u form the contiguous range [first_row(u), u-1], because
// i + steps(i) never decreases as i grows (at the even-N boundary,
// (n/2 - 1) + n/2 = n/2 + (n/2 - 1)).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define PAIRS_HD __host__ __device__ __forceinline__
#else
#define PAIRS_HD inline
#endif

struct Band {
    int n;     // objects in the set
    int h;     // floor((n-1)/2) steps for every row
    int half;  // n/2 when n is even (rows below it take one extra step), else 0

    PAIRS_HD static Band of(int n) {
        Band b;
        b.n = n;
        b.h = n > 0 ? (n - 1) / 2 : 0;
        b.half = (n % 2 == 0) ? n / 2 : 0;
        return b;
    }
    PAIRS_HD int steps(int i) const { return h + (i < half ? 1 : 0); }
    // Smallest row whose last virtual partner i + steps(i) is >= u (may be <= 0).
    PAIRS_HD int first_row(int u) const {
        int c = u - h - 1;
        return (c >= 0 && c < half) ? c : u - h;
    }
    PAIRS_HD int64_t pairs() const { return (int64_t)n * (n - 1) / 2; }
};

// The straightforward assignment that the paper measures its method against
// (Section 5): row i evaluates every j in (i, n), so row i does n-1-i steps
// and the "virtual partner" u is j itself.  Only the comparison kernels of the
// benchmark use it.
struct TriBand {
    int n;

    PAIRS_HD static TriBand of(int n) {
        TriBand b;
        b.n = n;
        return b;
    }
    PAIRS_HD int steps(int i) const { return n - 1 - i; }
};

// Work decomposition of one set into wave tasks.  A task is a block of 64*K
// consecutive rows [ra, ra + 64K) and a chunk of at most U consecutive virtual
// partners; chunk c of row block b covers u in [ra+1 + c*U, ra+1 + (c+1)*U)
// clipped to the block's last virtual partner.
struct Tiling {
    int rows;    // 64*K
    int chunk;   // U, a multiple of 64
    int nblocks; // row blocks
    int nchunks; // chunks per row block (enough for the longest block)

    PAIRS_HD static Tiling of(const Band &b, int K, int U) {
        Tiling t;
        t.rows = 64 * K;
        t.chunk = U;
        if (b.n < 2) {
            t.nblocks = 0;
            t.nchunks = 0;
            return t;
        }
        t.nblocks = (b.n + t.rows - 1) / t.rows;
        // a block's virtual partners span [ra+1, rlast + steps(rlast)]:
        // at most min(rows, n) - 1 + steps(0) values
        int64_t span = (int64_t)(t.rows < b.n ? t.rows : b.n) - 1 + b.steps(0);
        t.nchunks = (int)((span + U - 1) / U);
        return t;
    }
    PAIRS_HD int64_t tasks() const { return (int64_t)nblocks * nchunks; }
};

// The u-range [u0, u1) of task (block, c); empty when u0 >= u1.
PAIRS_HD void task_range(const Band &b, const Tiling &t, int block, int c, int *ra, int *u0,
                         int *u1) {
    int a = block * t.rows;
    int rlast = (a + t.rows < b.n ? a + t.rows : b.n) - 1;
    int uend = rlast + b.steps(rlast) + 1;
    int lo = a + 1 + c * t.chunk;
    int hi = lo + t.chunk;
    *ra = a;
    *u0 = lo;
    *u1 = hi < uend ? hi : uend;
}

// Task `task` of the tiling, enumerated row block by chunk:
// block = task / nchunks, chunk = task % nchunks.
PAIRS_HD void task_at(const Band &b, const Tiling &t, int64_t task, int *ra, int *u0, int *u1) {
    const int block = (int)(task / t.nchunks), c = (int)(task % t.nchunks);
    task_range(b, t, block, c, ra, u0, u1);
}

// The single-set launch order of the same tasks.  The row blocks form
// kTaskGroups groups of R = ceil(nblocks / kTaskGroups) consecutive blocks
// (the last group may be smaller); a group's tasks are enumerated chunk by
// chunk across its blocks, block fastest.  Tasks that run at the same time
// then read one narrow window of partners (a group's blocks are R*64K rows
// apart at most, and neighbouring chunks are U partners apart), which an
// L2 cache of a few MB holds, where the block-major order has every chunk of
// the set in flight.  A bijection on [0, tasks()).
constexpr int kTaskGroups = 16;

PAIRS_HD void task_at_grouped(const Band &b, const Tiling &t, int64_t task, int *ra, int *u0,
                              int *u1) {
    const int R = (t.nblocks + kTaskGroups - 1) / kTaskGroups;
    const int64_t per_group = (int64_t)R * t.nchunks;
    const int g = (int)(task / per_group);
    const int64_t w = task - (int64_t)g * per_group;
    const int rg = t.nblocks - g * R < R ? t.nblocks - g * R : R;  // blocks in group g
    const int c = (int)(w / rg), block = g * R + (int)(w % rg);
    task_range(b, t, block, c, ra, u0, u1);
}

// Row-stepping decomposition (the paper's own form: row i visits partners
// (i + s) mod n for s = 1, 2, ...).  A stepping task holds K consecutive rows
// per lane, rows [r0, r0 + 64K), and runs the steps [s0, s0 + T) for all its
// rows, plus, when x is set, the extra step s0 + T (= n/2) for the rows below
// n/2 of an even n.  Chunk c of a row block covers the steps
// [1 + c*U, 1 + (c+1)*U) clipped to the set's last step.
struct StepTiling {
    int rows;     // 64*K
    int chunk;    // U
    int nblocks;  // row blocks
    int nchunks;  // step chunks per row block

    PAIRS_HD static StepTiling of(const Band &b, int K, int U) {
        StepTiling t;
        t.rows = 64 * K;
        t.chunk = U;
        if (b.n < 2) {
            t.nblocks = 0;
            t.nchunks = 0;
            return t;
        }
        t.nblocks = (b.n + t.rows - 1) / t.rows;
        const int smax = b.h + (b.half > 0 ? 1 : 0);  // largest step of any row
        t.nchunks = (smax + U - 1) / U;
        return t;
    }
    PAIRS_HD int64_t tasks() const { return (int64_t)nblocks * nchunks; }
};

// Steps of chunk c: [*s0, *s0 + *T) for every row of the block, plus the
// extra step *s0 + *T for the rows below n/2 when *x is 1.
PAIRS_HD void step_range(const Band &b, const StepTiling &t, int block, int c, int *r0, int *s0,
                         int *T, int *x) {
    *r0 = block * t.rows;
    const int lo = 1 + c * t.chunk;
    const int hi = lo + t.chunk;                     // exclusive
    const int common_end = b.h + 1;                  // steps 1..h belong to every row
    const bool has_extra = b.half > 0 && hi > common_end && lo <= common_end;
    const int end = hi < common_end ? hi : common_end;
    *s0 = lo;
    *T = end > lo ? end - lo : 0;
    *x = has_extra ? 1 : 0;
}
