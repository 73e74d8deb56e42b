/*
 * pairs.h -- C ABI of libpairs, brute-force all-pairs interactions within sets
 * of objects on AMD Instinct MI355X (gfx950), and the linear-time collision
 * and contact counts of lattice beads (paper Section 3, at the end).
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
    PAIRS_FLAG_VALIDATE = 1u,
    /* Sums of doubles (energies, forces; not counts, which are exact
     * integers in any order) reproducible bit for bit from run to run, in
     * graphs as in eager calls: every partial sum is rounded once to a
     * multiple of 2^-S and added as a 64-bit integer, where 2^S is the
     * largest power of two that keeps the output's largest possible sum
     * below 2^61 units (a bound computed from n and eps2: (n-1)/sqrt(eps2)
     * per object, n(n-1)/2 /sqrt(eps2) per set or in total, and
     * (n-1) * 0.4/eps2 per force component).  The added error is at most
     * half a unit per partial sum; it stays far below float32 rounding unless
     * the sums are many orders of magnitude below their bound (terms much
     * smaller than 1/sqrt(eps2)).  Accepted by pairs_energy_f32,
     * pairs_energy_f64, pairs_force_f32 and pairs_energy_f32_batched; plans
     * take it as PAIRS_PLAN_DETERMINISTIC in their kind. */
    PAIRS_FLAG_DETERMINISTIC = 2u
};

/* Exact domain of the int32 collision counts (single set and batched):
 * every coordinate in [PAIRS_I32_COORD_MIN, PAIRS_I32_COORD_MAX] =
 * [-2^30, 2^30 - 1] and every radius in [0, PAIRS_I32_RADIUS_MAX] = [0, 2^30].
 * Differences then fit in int32, and squared distances (below 3 * 2^62) and
 * squared radius sums (at most 2^62) in uint64: inside it the GPU evaluates
 * the predicate exactly, with no check needed (see pairs_count_i32). */
#define PAIRS_I32_COORD_MIN (-(1 << 30))
#define PAIRS_I32_COORD_MAX ((1 << 30) - 1)
#define PAIRS_I32_RADIUS_MAX (1 << 30)

/* Largest number of objects in one set of a single-set call: row and
 * partner indices are 32-bit inside the kernels. */
#define PAIRS_MAX_SET_SIZE ((int64_t)1 << 30)

/* Largest number of objects in one set of a batch. */
#define PAIRS_MAX_BATCH_SET_SIZE ((int64_t)1 << 24)

/* Kinds of batched work (plans). */
enum {
    PAIRS_KIND_COUNT_I32 = 1, /* per-set exact int32 collision counts */
    PAIRS_KIND_COUNT_F32 = 2, /* per-set pinned-binary32 collision counts */
    PAIRS_KIND_ENERGY_F32 = 3, /* per-set potential totals, optionally with counts */
    /* the two kinds below name single-set calls for pairs_debug_single_launch
       only; plans and shape tables do not take them */
    PAIRS_KIND_ENERGY_F64 = 4, /* pairs_energy_f64 */
    PAIRS_KIND_FORCE_F32 = 5   /* pairs_force_f32 */
};

/* Or'ed into the kind of pairs_plan_create (PAIRS_KIND_ENERGY_F32 only): the
 * plan's set energies are reduced as under PAIRS_FLAG_DETERMINISTIC. */
#define PAIRS_PLAN_DETERMINISTIC 0x100

typedef struct pairs_plan_s *pairs_plan_t;
typedef struct pairs_graph_s *pairs_graph_t;

/* ------------------------------------------------------------ single set -- */

/*
 * Collision count of one set of n spheres with int32 centres (x, y, z) and
 * int32 radii r (Section 4 with interact() the sphere-overlap test; contact
 * at distance exactly r_i + r_j counts):
 *
 *   *d_count = #{ i < j : (x_i-x_j)^2 + (y_i-y_j)^2 + (z_i-z_j)^2 <= (r_i+r_j)^2 }
 *
 * The result is exact for every input in the exact domain (PAIRS_I32_COORD_MIN
 * .. PAIRS_I32_COORD_MAX, radii 0 .. PAIRS_I32_RADIUS_MAX), with no flag and
 * no host synchronisation: objects in a smaller box take a cheaper test, and
 * a wave switches to the full-width test for a task or a group of 64
 * partners that leaves it.  Outside the domain the result is undefined unless
 * PAIRS_FLAG_VALIDATE is given, in which case the call returns
 * PAIRS_ERR_DOMAIN and writes nothing.
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

/*
 * The same softened potential with double inputs and double arithmetic:
 * e_ij = 1/sqrt(|p_i - p_j|^2 + eps2) from the hardware reciprocal square
 * root refined by one Newton step, summed in double; outputs as for
 * pairs_energy_f32 (d_energy may be NULL).  Accuracy against an exact
 * evaluation: relative error at most 1e-12 for the total and for each
 * d_energy[i].  eps2 > 0; inputs finite with |coordinates| well below 1e150
 * (PAIRS_FLAG_VALIDATE checks finiteness).
 */
pairs_status_t pairs_energy_f64(const double *x, const double *y, const double *z, int64_t n,
                                double eps2, double *d_energy, double *d_total,
                                unsigned flags, pairs_stream_t stream);

/*
 * Forces of the same softened potential on every object of one set, a
 * symmetric interaction with a vector value (Section 4 leaves interact()
 * open): the force on i from j is
 *   f_ij = (p_i - p_j) / (|p_i - p_j|^2 + eps2)^(3/2),   f_ji = -f_ij,
 * and d_f*[i] = the components of F_i = sum over j != i of f_ij (n doubles
 * each).  Each unordered pair is evaluated once, in float32 with the
 * hardware reciprocal square root, and added to i and subtracted from j
 * (Newton's third law) in double accumulators.  Accuracy against an exact
 * evaluation of the same inputs: every component within 1e-5 of
 * S_i = sum over j != i of |f_ij| (the forces cancel, so their own size is
 * no scale).  eps2 > 0; inputs finite (PAIRS_FLAG_VALIDATE checks it).
 */
pairs_status_t pairs_force_f32(const float *x, const float *y, const float *z, int64_t n,
                               float eps2, double *d_fx, double *d_fy, double *d_fz,
                               unsigned flags, pairs_stream_t stream);

/* --------------------------------------------------------------- batches -- */
/*
 * A batch is a CSR list of independent sets (the pruned sets that a spatial
 * partition or a bounding-volume hierarchy produces, paper Sections 1 and 6):
 * set s owns objects [offsets[s], offsets[s+1]) of the object arrays, with
 * offsets[0] = 0, offsets non-decreasing, offsets[n_sets] = n_total and every
 * set at most PAIRS_MAX_BATCH_SET_SIZE objects.  Each set is the single-set
 * problem above; all sets are processed by one persistent kernel launch.
 *
 * Unplanned calls take the offsets in device memory (d_offsets, int64
 * [n_sets + 1]) and a caller workspace of at least
 * pairs_batched_workspace_size() bytes (device memory, 256-byte aligned, not
 * shared with a concurrent call).  They schedule the work on the device and
 * never wait for the host.  Offsets that break the rules above give undefined
 * per-set results (never an access outside the arrays) unless
 * PAIRS_FLAG_VALIDATE is given, which returns PAIRS_ERR_INVALID_ARG for bad
 * offsets and PAIRS_ERR_DOMAIN for bad values.
 */
pairs_status_t pairs_batched_workspace_size(int64_t n_sets, int64_t n_total, size_t *bytes);

/* d_counts[s] = collision count of set s (the pairs_count_i32 predicate). */
pairs_status_t pairs_count_i32_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                                       const int32_t *r, const int64_t *d_offsets,
                                       int64_t n_sets, int64_t n_total, uint64_t *d_counts,
                                       void *d_ws, size_t ws_bytes, unsigned flags,
                                       pairs_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * unplanned batched count above with no workspace argument.  Its workspace is
 * a scratch array of 8 MiB in the library's own device memory, one per
 * device, held until the process ends; the call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine), and nothing it uses
 * needs clearing between calls.  Batches of more than PAIRS_NOALLOC_MAX_SETS
 * sets return PAIRS_ERR_WORKSPACE with nothing enqueued.  Every call on a
 * device shares that device's scratch: calls that overlap on one device (on
 * different streams, or from different threads) race and give undefined
 * counts; calls ordered on one stream are safe.  Arguments, flags and results
 * are those of pairs_count_i32_batched.
 */
#define PAIRS_NOALLOC_MAX_SETS ((int64_t)250000)
pairs_status_t pairs_count_i32_batched_noalloc(const int32_t *x, const int32_t *y,
                                               const int32_t *z, const int32_t *r,
                                               const int64_t *d_offsets, int64_t n_sets,
                                               int64_t n_total, uint64_t *d_counts,
                                               unsigned flags, pairs_stream_t stream);

/* d_counts[s] = collision count of set s (the pairs_count_f32 predicate). */
pairs_status_t pairs_count_f32_batched(const float *x, const float *y, const float *z,
                                       const float *r, const int64_t *d_offsets,
                                       int64_t n_sets, int64_t n_total, uint64_t *d_counts,
                                       void *d_ws, size_t ws_bytes, unsigned flags,
                                       pairs_stream_t stream);

/* d_set_energy[s] = sum over the pairs of set s of 1/sqrt(d^2 + eps2) (double;
 * relative error at most 1e-6 per set), and, if r is not NULL, d_set_counts[s]
 * = the set's pinned-binary32 collision count.  r and d_set_counts are both
 * NULL or both non-NULL.  With r given, e uses fl(d2 + eps2) with d2 the
 * pinned squared distance. */
pairs_status_t pairs_energy_f32_batched(const float *x, const float *y, const float *z,
                                        const float *r, const int64_t *d_offsets,
                                        int64_t n_sets, int64_t n_total, float eps2,
                                        double *d_set_energy, uint64_t *d_set_counts, void *d_ws,
                                        size_t ws_bytes, unsigned flags, pairs_stream_t stream);

/* ----------------------------------------------------------------- plans -- */
/*
 * Forces of the softened potential (pairs_force_f32) within every set of a
 * CSR batch, on the balanced assignment of each set (Section 4: any
 * symmetric pairwise interaction; each pair evaluated once, added to one
 * object and subtracted from the other): d_fx, d_fy, d_fz (double[n_total])
 * receive, for every object, the sum over the other objects of its own set.
 * Offsets, workspace (pairs_batched_workspace_size) and validation as for
 * the batched counts; eps2 > 0; inputs finite.  PAIRS_FLAG_DETERMINISTIC
 * reduces the components in fixed point, with one scale for all objects
 * (the bound of the largest possible set).
 */
pairs_status_t pairs_force_f32_batched(const float *x, const float *y, const float *z,
                                       const int64_t *d_offsets, int64_t n_sets,
                                       int64_t n_total, float eps2, double *d_fx, double *d_fy,
                                       double *d_fz, void *d_ws, size_t ws_bytes, unsigned flags,
                                       pairs_stream_t stream);

/*
 * The potential in double precision (pairs_energy_f64) within every set of a
 * CSR batch: d_set_energy[s] = the sum over pairs of set s (double[n_sets]);
 * d_energy (double[n_total] or NULL) = each object's sum over the other
 * objects of its set.  Offsets, workspace and validation as for the batched
 * counts; eps2 > 0.  PAIRS_FLAG_DETERMINISTIC as for pairs_energy_f32_batched
 * (per-set scales for the set totals, one scale for the per-object sums).
 */
pairs_status_t pairs_energy_f64_batched(const double *x, const double *y, const double *z,
                                        const int64_t *d_offsets, int64_t n_sets,
                                        int64_t n_total, double eps2, double *d_set_energy,
                                        double *d_energy, void *d_ws, size_t ws_bytes,
                                        unsigned flags, pairs_stream_t stream);

/*
 * A plan fixes the set sizes of a batch (h_offsets: HOST int64[n_sets + 1],
 * same rules as above, checked on the host) and precomputes its schedule: a
 * task table ordered so that the tasks of the largest sets run first.  The
 * plan owns that table and a device copy of the offsets (allocated by create,
 * freed by destroy) on the device current at create.  The task table must
 * have fewer than 2^31 entries (PAIRS_ERR_INVALID_ARG otherwise).
 *
 * execute enqueues the batch on `stream` with no allocation and no host
 * wait, so it may be captured into a HIP graph.  in[] and out[] by kind:
 *   PAIRS_KIND_COUNT_I32: in = {x, y, z, r} (int32),  out = {counts (uint64[n_sets])}
 *   PAIRS_KIND_COUNT_F32: in = {x, y, z, r} (float),  out = {counts}
 *   PAIRS_KIND_ENERGY_F32: in = {x, y, z, r or NULL} (float),
 *                          out = {energy (double[n_sets]), counts or NULL}
 * eps2 is used by PAIRS_KIND_ENERGY_F32 only.  A plan must not execute on two
 * streams at once.
 */
pairs_status_t pairs_plan_create(int kind, const int64_t *h_offsets, int64_t n_sets,
                                 pairs_plan_t *plan);
pairs_status_t pairs_plan_execute(pairs_plan_t plan, const void *const *in, void *const *out,
                                  float eps2, pairs_stream_t stream);
pairs_status_t pairs_plan_info(pairs_plan_t plan, int64_t *n_sets, int64_t *n_total,
                               int64_t *n_tasks);
pairs_status_t pairs_plan_destroy(pairs_plan_t plan);

/* ------------------------------------------------------- repeated steps -- */
/*
 * Per-step perturbation of moving objects (paper, Introduction: objects in
 * motion whose interactions are recomputed every small time step).  Object k
 * (global index first_index + k, below 2^32) gets, per axis a, the
 * zero-mean perturbation of standard deviation sigma
 *   delta = fl32(fl32(S) * c),  c = fl32(sigma / sqrt((4/3)(2^48 - 1))),
 *   S = 2 (w0>>8 + w1>>8 + w2>>8 + w3>>8) - 4 (2^24 - 1)
 * where w = Philox4x32-10 (Salmon et al., SC 2011) of the counter
 * (global index, step, a, 0) under the key (seed low 32 bits, seed high 32
 * bits); then x = fl32(x + delta).  S is an Irwin-Hall(4) variate, an
 * approximation of a normal variate bounded at about 3.46 standard
 * deviations; every step is exactly rounded, so the result is reproducible
 * bit for bit.  Coordinates are updated in place.
 */
pairs_status_t pairs_jitter_f32(float *x, float *y, float *z, int64_t n, uint64_t seed,
                                uint32_t step, float sigma, int64_t first_index,
                                pairs_stream_t stream);

/*
 * Captures n_steps repeated steps of an energy plan into one HIP graph: for
 * k = 0 .. n_steps-1, jitter all plan objects with step first_step + k, then
 * execute the plan into row k of d_energy (double[n_steps][n_sets]) and, if r
 * is not NULL, of d_counts (uint64[n_steps][n_sets]).  Launching the graph
 * runs all steps with no host involvement; positions accumulate across steps
 * and launches.  The graph keeps the pointers given here.
 */
pairs_status_t pairs_plan_capture_steps(pairs_plan_t plan, float *x, float *y, float *z,
                                        const float *r, uint64_t seed, float sigma,
                                        uint32_t first_step, int n_steps, float eps2,
                                        double *d_energy, uint64_t *d_counts,
                                        pairs_graph_t *graph);
pairs_status_t pairs_graph_launch(pairs_graph_t graph, pairs_stream_t stream);
pairs_status_t pairs_graph_destroy(pairs_graph_t graph);

/* ------------------------------------------------------------ tile shapes -- */
/*
 * Tile shapes of the kernels, chosen per size class.  Entry c of a table
 * applies to sets with n > min_n[c] that no earlier entry takes; the last
 * entry takes the rest.  Entries are listed from the largest sets down
 * (min_n strictly decreasing).  Each entry names one of three wave-task
 * forms of the balanced assignment (Section 4):
 *
 * PAIRS_FORM_BROADCAST: a wave holds 64 * rows_per_lane consecutive rows of a
 *   set, K = rows_per_lane per lane in lane-major order, and sweeps a chunk of
 *   at most `chunk` virtual partners u = row + s, each broadcast to every
 *   lane.  rows_per_lane is 1, 2, 4 or 8; chunk a multiple of 64 in
 *   [64, 2^22].
 * PAIRS_FORM_STEPPING: the paper's own per-row form.  Each lane holds K =
 *   rows_per_lane (1 or 2) consecutive rows and steps through their partners
 *   (row + s) mod n, `chunk` steps per task.  chunk is a multiple of 16 in
 *   [16, 288] for K = 1 and in [16, 272] for K = 2.  Batched tables only.  A
 *   plan packs whole sets of equal size that fit one wave (ceil(n/K) <= 64)
 *   into shared waves; unplanned calls give each set its own waves.
 *
 * PAIRS_FORM_MATRIX: the exact int32 count of single sets only (kind
 *   PAIRS_KIND_COUNT_I32, batched = 0).  A wave holds 64 consecutive rows as
 *   four 16-row tiles, and the Gram sums of each tile with 16 partners are
 *   one double-precision matrix instruction (exact inside the double form's
 *   box, the wide VALU test outside it); the VALU compares.  rows_per_lane
 *   is 1; chunk as for the broadcast form.  The default tables do not use
 *   it: on gfx950 it runs slower than the broadcast form.
 *
 * Tables are per kind (PAIRS_KIND_*) and per mode, the `batched` argument:
 * PAIRS_SHAPES_SINGLE (0) single-set calls, PAIRS_SHAPES_BATCHED (1) batched
 * calls and plans, and PAIRS_SHAPES_TOTAL_ONLY (2) single-set calls of
 * pairs_energy_f32 with d_energy = NULL (kind PAIRS_KIND_ENERGY_F32 only: a
 * total alone has no partner-side sums, and runs best with one row per lane).
 * Other values give PAIRS_ERR_INVALID_ARG.  A plan keeps the table of its
 * creation.  set(NULL) restores the defaults.  Results never depend on the
 * shapes; only the speed does.
 */
#define PAIRS_SHAPES_SINGLE 0
#define PAIRS_SHAPES_BATCHED 1
#define PAIRS_SHAPES_TOTAL_ONLY 2
#define PAIRS_FORM_BROADCAST 0
#define PAIRS_FORM_STEPPING 1
#define PAIRS_FORM_MATRIX 2

typedef struct {
    int32_t count;            /* entries used, 1..4 */
    int32_t min_n[4];
    int32_t rows_per_lane[4];
    int32_t chunk[4];
    int32_t form[4];          /* PAIRS_FORM_* */
} pairs_shape_table_t;

pairs_status_t pairs_get_shapes(int kind, int batched, pairs_shape_table_t *out);
pairs_status_t pairs_set_shapes(int kind, int batched, const pairs_shape_table_t *table);

/* ----------------------------------------------------------- binned count -- */
/*
 * Collision count of one set of int32 spheres (the same result as
 * pairs_count_i32) through a uniform grid of cubic cells of side `cell`:
 * the pruning step that produces the paper's pruned sets (Sections 1 and 6),
 * with the pairwise count inside each cell on the balanced assignment.  With
 * every radius at most cell/2, touching spheres lie in the same or in
 * neighbouring cells, so only the pairs inside a cell and between each cell
 * and its 13 forward neighbours are tested.  The objects are grouped by cell
 * on the device through a hash table of the occupied cells, so the time
 * grows with n times the objects per cell rather than with n^2.
 *
 * Domain: coordinates in [-2^24, 2^24], radii in [0, cell/2],
 * PAIRS_BINNED_MIN_CELL <= cell <= PAIRS_BINNED_MAX_CELL, at most
 * PAIRS_BINNED_MAX_SET_SIZE objects.  Outside it the result is undefined
 * unless PAIRS_FLAG_VALIDATE is given (then PAIRS_ERR_DOMAIN).
 * Workspace: pairs_binned_workspace_size(n) bytes of device memory, owned by
 * the caller (about 120 to 160 bytes per object, with the cell table
 * rounded up to a power of two of at least 2n slots); the size query needs
 * no device.
 * Every call clears what it needs, so a workspace serves calls in a row.
 * Stream-ordered, with no host synchronisation and no allocation; the call
 * can be captured into a HIP graph (without PAIRS_FLAG_VALIDATE, whose check
 * waits on the host), since it clears its state with kernels, not memsets.
 * The counts are exact, so they do not depend on the order in which the
 * device groups the objects.
 */
#define PAIRS_BINNED_MIN_CELL 32
#define PAIRS_BINNED_MAX_CELL (1 << 25)
#define PAIRS_BINNED_MAX_SET_SIZE ((int64_t)1 << 30)

pairs_status_t pairs_binned_workspace_size(int64_t n, size_t *bytes);

pairs_status_t pairs_count_i32_binned(const int32_t *x, const int32_t *y, const int32_t *z,
                                      const int32_t *r, int64_t n, int32_t cell,
                                      uint64_t *d_count, void *d_ws, size_t ws_bytes,
                                      unsigned flags, pairs_stream_t stream);

/*
 * The binned count of every set of a CSR batch (the objects of set s are
 * [d_offsets[s], d_offsets[s+1]), d_offsets[n_sets] = n_total, on the device)
 * into d_counts[n_sets] (uint64, device): pairs of objects of different sets
 * are never counted.  A set's cells are keyed by the set index above the
 * cells' 3 fb bits, fb = the fewest bits that hold 2^25 / cell + 2 (11 for
 * cells of 2^15, 16 for cells of 1024), so 3 fb + ceil(log2 n_sets) must not
 * pass 64 (else PAIRS_ERR_INVALID_ARG).  Same domain, workspace
 * (pairs_binned_workspace_size(n_total)) and stream behaviour as
 * pairs_count_i32_binned; PAIRS_FLAG_VALIDATE also checks the offsets.
 */
pairs_status_t pairs_count_i32_binned_batched(const int32_t *x, const int32_t *y,
                                              const int32_t *z, const int32_t *r,
                                              const int64_t *d_offsets, int64_t n_sets,
                                              int64_t n_total, int32_t cell, uint64_t *d_counts,
                                              void *d_ws, size_t ws_bytes, unsigned flags,
                                              pairs_stream_t stream);

/* --------------------------------------------------------- lattice beads -- */
/*
 * Collision and contact counts of bead vectors on the integer lattice Z^3
 * (Section 3, algorithms countColls and countContacts).  Beads are points
 * (x, y, z) of int32 coordinates; for each vector
 *
 *   collisions = #{ i < j : bead i and bead j occupy the same site }
 *   contacts   = #{ i < j : |x_i-x_j| + |y_i-y_j| + |z_i-z_j| == 1 }
 *
 * i.e. the pairs on one site and the pairs on sites one unit apart along one
 * axis.  The paper counts both with an occupancy array over the bounded
 * lattice in O(n) time; here the occupancy lives in a hash table per vector
 * (LDS for vectors of at most PAIRS_LATTICE_LDS_BEADS beads, device memory
 * from the workspace for longer ones), so no bound on the lattice is needed
 * beyond the domain below.  Counts are exact integers.
 *
 * Domain, per vector: at most PAIRS_LATTICE_MAX_BEADS beads, and a bounding
 * box that, padded by one site on every side, holds fewer than 2^40 sites:
 * (max x - min x + 3)(max y - min y + 3)(max z - min z + 3) < 2^40.  Any
 * chain of unit steps shorter than about 30 000 beads is inside.  A vector
 * outside the domain gets UINT64_MAX in both of its outputs; with
 * PAIRS_FLAG_VALIDATE the call then waits for the stream and returns
 * PAIRS_ERR_DOMAIN (box) or PAIRS_ERR_INVALID_ARG (length).
 *
 * Workspace: pairs_lattice_workspace_size() bytes of device memory, owned by
 * the caller; zero bytes (d_ws may be NULL) when every vector has at most
 * PAIRS_LATTICE_LDS_BEADS beads and the call is told so through max_n.
 */
#define PAIRS_LATTICE_LDS_BEADS 4096
#define PAIRS_LATTICE_MAX_BEADS (((int64_t)1 << 24) - 1)

/* Workspace bytes for a batch whose vectors have at most max_n beads each
 * (max_n = 0: unknown).  A single vector of n beads is (1, n, n). */
pairs_status_t pairs_lattice_workspace_size(int64_t n_sets, int64_t n_total, int64_t max_n,
                                            size_t *bytes);

/* One vector of n beads.  d_collisions, d_contacts: one uint64 each in device
 * memory; either may be NULL (its pass is skipped: the collision count costs
 * less alone).  Vectors longer than PAIRS_LATTICE_LDS_BEADS use the whole
 * grid with the table in the workspace. */
pairs_status_t pairs_lattice_count(const int32_t *x, const int32_t *y, const int32_t *z,
                                   int64_t n, uint64_t *d_collisions, uint64_t *d_contacts,
                                   void *d_ws, size_t ws_bytes, unsigned flags,
                                   pairs_stream_t stream);

/* A CSR batch of vectors (offsets as for the sphere batches), one workgroup
 * per vector.  max_n: an upper bound of every vector's length, or 0 if
 * unknown; it sizes the LDS tables.  A vector longer than a non-zero max_n
 * is a caller error (UINT64_MAX outputs; PAIRS_ERR_INVALID_ARG under
 * PAIRS_FLAG_VALIDATE).  d_collisions, d_contacts: uint64[n_sets] each,
 * either may be NULL. */
pairs_status_t pairs_lattice_count_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                                           const int64_t *d_offsets, int64_t n_sets,
                                           int64_t n_total, int64_t max_n,
                                           uint64_t *d_collisions, uint64_t *d_contacts,
                                           void *d_ws, size_t ws_bytes, unsigned flags,
                                           pairs_stream_t stream);

/* ---------------------------------------------------------- introspection -- */
/*
 * Host-only: the wave tasks of a single set of n objects for the tile shape
 * (rows_per_lane in {1, 2, 4, 8}, chunk a positive multiple of 64).  Task k is
 * written as out[3k] = first row ra, out[3k+1] = u0, out[3k+2] = u1: rows
 * [ra, ra + 64*rows_per_lane) evaluate their balanced-assignment partners
 * (row + s) mod n for every virtual partner u = row + s in [u0, u1).
 * *n_tasks receives the task count; out may be NULL to query it only.
 */
pairs_status_t pairs_debug_task_ranges(int n, int rows_per_lane, int chunk, int32_t *out,
                                       int64_t capacity, int64_t *n_tasks);

/*
 * Host-only: the stepping-form tasks of a single set of n objects (Section 4:
 * row i visits (i + s) mod n for s = 1 .. steps(i)) for rows_per_lane K in
 * {1, 2} and chunk steps per task (chunk >= 1).  Task k is written as
 * out[4k] = first row r0, out[4k+1] = s0, out[4k+2] = T, out[4k+3] = x: the
 * rows [r0, r0 + 64K) that exist run the steps [s0, s0 + T), and when x is 1
 * the rows below n/2 also run step s0 + T (the extra step of an even n).
 */
pairs_status_t pairs_debug_step_ranges(int n, int rows_per_lane, int chunk, int32_t *out,
                                       int64_t capacity, int64_t *n_tasks);

/*
 * Host-only: tasks[k] (an index below the tiling's task count) of a single set
 * of n <= PAIRS_MAX_SET_SIZE objects decoded as the single-set kernels decode
 * it: out[3k] = first row, out[3k+1] = u0, out[3k+2] = u1.  rows_per_lane in
 * {1, 2, 4, 8}; chunk a multiple of 64 in [64, 2^22].  For sets too large to
 * list every task with pairs_debug_task_ranges.  The kernels' order: the row
 * blocks form 16 groups of R = ceil(blocks / 16) consecutive blocks (the last
 * may be smaller), and inside a group task index g*R*chunks + c*R_g + j is
 * chunk c of the group's block j (R_g = the group's block count).
 */
pairs_status_t pairs_debug_task_at(int64_t n, int rows_per_lane, int chunk,
                                   const int64_t *tasks, int64_t count, int64_t *out);

/*
 * Host-only: the launch a single-set call of `kind` (PAIRS_KIND_COUNT_I32,
 * _COUNT_F32, _ENERGY_F32, _ENERGY_F64 or _FORCE_F32) makes for n objects
 * with the current tile shapes: *n_tasks wave tasks of the balanced
 * assignment (Section 4) on *n_blocks blocks of *threads work-items.  Up to
 * 2^22 blocks each wave runs one task; a larger tiling launches 2^22 blocks
 * whose waves stride over the tasks, so no launch exceeds 2^32 work-items for
 * any n <= PAIRS_MAX_SET_SIZE.  0 tasks and 0 blocks for n < 2.
 */
pairs_status_t pairs_debug_single_launch(int kind, int64_t n, int64_t *n_tasks,
                                         int64_t *n_blocks, int32_t *threads);

/* ---------------------------------------------------------------- errors -- */

/* Static text for a status code. */
const char *pairs_status_string(pairs_status_t status);

/* hipError_t of the last failing HIP call on the calling thread. */
int pairs_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PAIRS_H */
