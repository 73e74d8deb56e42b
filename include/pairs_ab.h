/*
 * pairs_ab.h: the assignment comparison of the benchmark (not part of the
 * pairs library's interface).
 *
 * Section 5 of the paper compares its balanced circular assignment with the
 * straightforward parallelisation of the triangular loop, in which row i
 * evaluates every j in (i, n) and so does n-1-i pair tests.  These entry
 * points run both assignments with the same wave task body as the library's
 * exact int32 count (broadcast form, rows_per_lane rows per lane), one wave per
 * row block and no partner chunking, so that the only difference is the
 * assignment:
 *   variant 0 (balanced): the rows of a block evaluate their virtual partners
 *     u = i + s, s = 1 .. steps(i) (equal work per row);
 *   variant 1 (straightforward): the rows of a block evaluate j in (i, n).
 * Both count every unordered pair with |p_i - p_j|^2 <= (r_i + r_j)^2 once
 * and give the same result.
 *
 * Arguments: device pointers to n int32 values each (x, y, z, r; the exact
 * domain of pairs_count_i32 applies), rows_per_lane in {1, 8}, d_count a
 * device uint64 that is overwritten.  Launches on `stream` (a hipStream_t, 0
 * for the null stream) and returns 0, -1 for invalid arguments or a negative
 * hipError_t on a launch failure.  Nothing is allocated.
 */
#ifndef PAIRS_AB_H
#define PAIRS_AB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int pairs_ab_count_i32(int variant, const int32_t *x, const int32_t *y, const int32_t *z,
                       const int32_t *r, int64_t n, int rows_per_lane, uint64_t *d_count,
                       void *stream);

/*
 * The same run with the start and end of every wave on the device's
 * constant-rate wall clock (the dispatch-order evidence of the comparison):
 * d_times is a device uint64 array of 2 * pairs_ab_waves(n, rows_per_lane)
 * entries, the start of wave w (row block w) at [2w] and its end at [2w+1].
 * Returns as pairs_ab_count_i32, and -1 for a null d_times.
 */
int64_t pairs_ab_waves(int64_t n, int rows_per_lane);
int pairs_ab_count_i32_timed(int variant, const int32_t *x, const int32_t *y, const int32_t *z,
                             const int32_t *r, int64_t n, int rows_per_lane, uint64_t *d_count,
                             uint64_t *d_times, void *stream);

/* Ticks per millisecond of that clock on the current device (0 on success). */
int pairs_ab_wall_clock_khz(int64_t *khz);

#ifdef __cplusplus
}
#endif

#endif
