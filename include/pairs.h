/*
 * pairs.h -- C ABI of libpairs, brute-force all-pairs interactions within sets
 * of objects on AMD Instinct MI355X (gfx950).
 *
 * Method: Saldanha & de Souza, "High Performance Algorithms for Counting
 * Collisions and Pairwise Interactions", ICCS 2019, Section 4.  Every
 * unordered pair {i, j} of a set of n objects is evaluated exactly once, under
 * the paper's balanced circular assignment: object i evaluates partners
 * (i + s) mod n for s = 1 .. floor((n-1)/2), and when n is even the objects
 * i < n/2 also evaluate s = n/2 (the even-N rule after Proposition 2).  Every
 * object therefore owns floor((n-1)/2) or n/2 pairs (Proposition 1, and the
 * work/depth paragraph).  The per-pair interaction is symmetric (the paper's
 * "symmetric pairwise interaction"), so the reduced result does not depend on
 * which of the two objects evaluates a pair.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments named d_* and all object arrays are DEVICE pointers
 *   (memory of the current HIP device).  Host pointers are named h_*.
 * - Objects are structure-of-arrays: x[k], y[k], z[k] (and r[k]) describe
 *   object k.  Arrays must not overlap any output.
 * - The caller owns every input and output buffer.  Outputs are overwritten
 *   (the library clears them in-stream first), never accumulated into.
 * - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *   the call returns without waiting for it, except where a flag below asks
 *   for a synchronous check.
 * - Argument errors are detected on the host and returned before anything is
 *   enqueued.  A HIP failure returns PAIRS_ERR_HIP; pairs_last_hip_error()
 *   then gives the hipError_t code for the calling thread.
 * - Sets with fewer than 2 objects have no pairs: their results are 0.
 * - Calls are reentrant and may run concurrently on different streams.
 */
#ifndef PAIRS_H
#define PAIRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PAIRS_OK = 0,
    PAIRS_ERR_INVALID_ARG = -1, /* null pointer, negative size, bad offsets, bad flag */
    PAIRS_ERR_DOMAIN = -2,      /* input outside the exact domain (PAIRS_FLAG_VALIDATE) */
    PAIRS_ERR_HIP = -3,         /* a HIP runtime call failed */
    PAIRS_ERR_NO_MEMORY = -4,   /* device or host allocation failed */
    PAIRS_ERR_WORKSPACE = -5,   /* caller workspace missing or too small */
    PAIRS_ERR_NO_DEVICE = -6    /* no usable HIP device */
} pairs_status_t;

/* A hipStream_t passed as an opaque pointer; NULL is the null stream. */
typedef void *pairs_stream_t;

/* Flags. */
enum {
    /* Check the inputs against the exact domain on the device before the
     * computation and return PAIRS_ERR_DOMAIN if any object is outside it.
     * This waits for the stream (a synchronous call). */
    PAIRS_FLAG_VALIDATE = 1u
};

/* Exact domain of the int32 collision count: every coordinate in
 * [-2^24, 2^24] and every radius in [0, 2^24].  Inside it the GPU evaluates
 * the predicate exactly (see pairs_count_i32). */
#define PAIRS_I32_COORD_LIMIT (1 << 24)
#define PAIRS_I32_RADIUS_LIMIT (1 << 24)

/* Largest number of objects in one set (single-set calls and each set of a
 * batch): row and partner indices are 32-bit inside the kernels. */
#define PAIRS_MAX_SET_SIZE ((int64_t)1 << 30)

/* ------------------------------------------------------------ single set -- */

/*
 * Collision count of one set of n spheres with int32 centres (x, y, z) and
 * int32 radii r (Section 4 with interact() the sphere-overlap test; contact
 * at distance exactly r_i + r_j counts):
 *
 *   *d_count = #{ i < j : (x_i-x_j)^2 + (y_i-y_j)^2 + (z_i-z_j)^2 <= (r_i+r_j)^2 }
 *
 * The result is exact for inputs in the exact domain (PAIRS_I32_*_LIMIT);
 * outside it the result is undefined unless PAIRS_FLAG_VALIDATE is given, in
 * which case the call returns PAIRS_ERR_DOMAIN and writes nothing.
 * d_count: one uint64 in device memory.  n >= 0, n <= PAIRS_MAX_SET_SIZE.
 */
pairs_status_t pairs_count_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                               const int32_t *r, int64_t n, uint64_t *d_count,
                               unsigned flags, pairs_stream_t stream);

/*
 * Collision count of one set of float32 spheres, the predicate evaluated by
 * one fixed IEEE binary32 sequence (round to nearest even, subnormals kept):
 *   dx = fl(x_i - x_j) (dy, dz likewise),
 *   d2 = fl(fma(dz, dz, fl(fma(dy, dy, fl(dx*dx))))),
 *   R = fl(r_i + r_j), R2 = fl(R*R), hit iff d2 <= R2.
 * fl(a - b) = -fl(b - a), so the answer does not depend on which object of a
 * pair evaluates it.  Inputs must be finite (PAIRS_FLAG_VALIDATE checks it).
 */
pairs_status_t pairs_count_f32(const float *x, const float *y, const float *z,
                               const float *r, int64_t n, uint64_t *d_count,
                               unsigned flags, pairs_stream_t stream);

/*
 * Softened pairwise potential of one set of n float32 particles,
 * e_ij = 1 / sqrt(|p_i - p_j|^2 + eps2), in float32 pair arithmetic with
 * double-precision accumulation:
 *   *d_total = sum over i < j of e_ij                       (one double)
 *   d_energy[i] = sum over j != i of e_ij   (n doubles; may be NULL)
 * Each unordered pair is evaluated once and its value is added to both
 * objects.  Accuracy against an exact evaluation of the same inputs: relative
 * error of the total at most 1e-6, of each d_energy[i] at most 1e-5.
 * eps2 > 0; inputs finite (PAIRS_FLAG_VALIDATE checks it).
 */
pairs_status_t pairs_energy_f32(const float *x, const float *y, const float *z, int64_t n,
                                float eps2, double *d_energy, double *d_total,
                                unsigned flags, pairs_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PAIRS_H */
