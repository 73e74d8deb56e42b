/*
 * CPU oracle for all-pairs interaction counts and sums.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this code.  The GPU library
 * never links it, includes it or calls it, and shares no code with it.
 *
 * What it computes is the plain definition: the standard pairwise loop of the
 * paper (Section 4, algorithm "Standard algorithm for calculating SPI"), in
 * which every object i is paired with every later object j > i and the
 * interaction of each unordered pair is accumulated exactly once.  The
 * balanced (circular) assignment of the paper (Section 4, algorithm "Proposed
 * algorithm for calculating SPI", with the even-N rule stated after
 * Proposition 2) evaluates the same N(N-1)/2 unordered pairs (Propositions 1
 * and 2), so its reduced result equals this loop's exactly for counts, and up
 * to rounding order for floating-point sums.
 *
 * Interactions (the paper leaves interact() open; Section 4 asks only that it
 * be symmetric):
 *   - sphere collision, integer inputs: hit iff |p_i - p_j|^2 <= (r_i + r_j)^2,
 *     evaluated in 128-bit integers, exact for every int32 input;
 *   - sphere collision, float32 inputs: the same predicate evaluated by one
 *     pinned IEEE binary32 sequence (round to nearest even, no flush to zero):
 *       dx = fl(x_i - x_j), dy, dz likewise,
 *       d2 = fl(fma(dz, dz, fl(fma(dy, dy, fl(dx * dx))))),
 *       R  = fl(r_i + r_j),  R2 = fl(R * R),  hit iff d2 <= R2;
 *     fl(a - b) = -fl(b - a) under round-to-nearest-even, so the sequence gives
 *     the same answer for (i, j) and (j, i);
 *   - softened potential: e_ij = 1 / sqrt(|p_i - p_j|^2 + eps2), with the
 *     float32 inputs and the float32 eps2 promoted exactly to double and all
 *     arithmetic in double.  total = sum over i < j of e_ij; the per-object
 *     value E_i = sum over j != i of e_ij receives the full e_ij from every
 *     partner, so sum_i E_i = 2 * total.  Both sums use Neumaier's compensated
 *     summation;
 *   - forces of that potential, f_ij = (p_i - p_j) / (d2 + eps2)^(3/2), with
 *     F_i = sum over j != i of f_ij (see oracle_force_rows).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp (see build.py).
 * OpenMP only splits the outer loop over i between threads; the body is the
 * plain loop.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

static int nthreads_or_default(int threads) {
#ifdef _OPENMP
    return threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* Number of threads an OpenMP region of this library would use. */
int oracle_threads(int threads) { return nthreads_or_default(threads); }

/* ---------------------------------------------------------------- counts -- */

static inline int hit_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                          const int32_t *r, int64_t i, int64_t j) {
    i128 dx = (i128)x[i] - (i128)x[j];
    i128 dy = (i128)y[i] - (i128)y[j];
    i128 dz = (i128)z[i] - (i128)z[j];
    i128 d2 = dx * dx + dy * dy + dz * dz;
    i128 R = (i128)r[i] + (i128)r[j];
    return d2 <= R * R;
}

static inline int hit_f32(const float *x, const float *y, const float *z,
                          const float *r, int64_t i, int64_t j) {
    float dx = x[i] - x[j];
    float dy = y[i] - y[j];
    float dz = z[i] - z[j];
    float d2 = dx * dx;
    d2 = fmaf(dy, dy, d2);
    d2 = fmaf(dz, dz, d2);
    float R = r[i] + r[j];
    float R2 = R * R;
    return d2 <= R2;
}

/* Collision count of one set of n int32 spheres (plain i < j loop). */
uint64_t oracle_count_i32(const int32_t *x, const int32_t *y, const int32_t *z,
                          const int32_t *r, int64_t n, int threads) {
    uint64_t c = 0;
#pragma omp parallel for reduction(+ : c) schedule(dynamic, 16) num_threads(nthreads_or_default(threads))
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            c += (uint64_t)hit_i32(x, y, z, r, i, j);
    return c;
}

/* Collision count of one set of n float32 spheres, pinned binary32 predicate. */
uint64_t oracle_count_f32(const float *x, const float *y, const float *z,
                          const float *r, int64_t n, int threads) {
    uint64_t c = 0;
#pragma omp parallel for reduction(+ : c) schedule(dynamic, 16) num_threads(nthreads_or_default(threads))
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            c += (uint64_t)hit_f32(x, y, z, r, i, j);
    return c;
}

/* Count of colliding pairs (a, b) with a in set A and b in set B (int32). */
uint64_t oracle_cross_count_i32(const int32_t *ax, const int32_t *ay, const int32_t *az,
                                const int32_t *ar, int64_t na,
                                const int32_t *bx, const int32_t *by, const int32_t *bz,
                                const int32_t *br, int64_t nb, int threads) {
    uint64_t c = 0;
#pragma omp parallel for reduction(+ : c) schedule(dynamic, 16) num_threads(nthreads_or_default(threads))
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j) {
            i128 dx = (i128)ax[i] - (i128)bx[j];
            i128 dy = (i128)ay[i] - (i128)by[j];
            i128 dz = (i128)az[i] - (i128)bz[j];
            i128 R = (i128)ar[i] + (i128)br[j];
            c += (uint64_t)(dx * dx + dy * dy + dz * dz <= R * R);
        }
    return c;
}

/* ------------------------------------------------------------- energies -- */

/* Neumaier's improvement of Kahan summation (Neumaier 1974). */
typedef struct { double s, c; } nsum_t;

static inline void nsum_add(nsum_t *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double nsum_value(const nsum_t *a) { return a->s + a->c; }

static inline double pair_energy(const float *x, const float *y, const float *z,
                                 double eps2, int64_t i, int64_t j) {
    double dx = (double)x[i] - (double)x[j];
    double dy = (double)y[i] - (double)y[j];
    double dz = (double)z[i] - (double)z[j];
    double d2 = dx * dx + dy * dy + dz * dz;
    return 1.0 / sqrt(d2 + eps2);
}

/* Total softened potential of one set: sum over i < j of e_ij. */
double oracle_energy_total(const float *x, const float *y, const float *z, int64_t n,
                           float eps2f, int threads) {
    const double eps2 = (double)eps2f;
    int nt = nthreads_or_default(threads);
    nsum_t *part = (nsum_t *)calloc((size_t)nt, sizeof(nsum_t));
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        nsum_t acc = {0.0, 0.0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                nsum_add(&acc, pair_energy(x, y, z, eps2, i, j));
        part[t] = acc;
    }
    nsum_t tot = {0.0, 0.0};
    for (int t = 0; t < nt; ++t) {
        nsum_add(&tot, part[t].s);
        nsum_add(&tot, part[t].c);
    }
    free(part);
    return nsum_value(&tot);
}

/* Per-object energy E_i = sum over j != i of e_ij, for the listed objects only
 * (rows == NULL means every object 0..n-1, written to E[0..n-1]). */
void oracle_energy_rows(const float *x, const float *y, const float *z, int64_t n,
                        float eps2f, const int64_t *rows, int64_t nrows, double *E,
                        int threads) {
    const double eps2 = (double)eps2f;
    int64_t m = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(threads))
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        nsum_t acc = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j)
            if (j != i) nsum_add(&acc, pair_energy(x, y, z, eps2, i, j));
        E[k] = nsum_value(&acc);
    }
}

/* The same potential for double inputs (the double-precision variant): the
 * pair term and the sums exactly as above, the inputs used as given. */
static inline double pair_energy64(const double *x, const double *y, const double *z,
                                   double eps2, int64_t i, int64_t j) {
    double dx = x[i] - x[j];
    double dy = y[i] - y[j];
    double dz = z[i] - z[j];
    double d2 = dx * dx + dy * dy + dz * dz;
    return 1.0 / sqrt(d2 + eps2);
}

double oracle_energy_f64_total(const double *x, const double *y, const double *z, int64_t n,
                               double eps2, int threads) {
    int nt = nthreads_or_default(threads);
    nsum_t *part = (nsum_t *)calloc((size_t)nt, sizeof(nsum_t));
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        nsum_t acc = {0.0, 0.0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                nsum_add(&acc, pair_energy64(x, y, z, eps2, i, j));
        part[t] = acc;
    }
    nsum_t tot = {0.0, 0.0};
    for (int t = 0; t < nt; ++t) {
        nsum_add(&tot, part[t].s);
        nsum_add(&tot, part[t].c);
    }
    free(part);
    return nsum_value(&tot);
}

void oracle_energy_f64_rows(const double *x, const double *y, const double *z, int64_t n,
                            double eps2, const int64_t *rows, int64_t nrows, double *E,
                            int threads) {
    int64_t m = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(threads))
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        nsum_t acc = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j)
            if (j != i) nsum_add(&acc, pair_energy64(x, y, z, eps2, i, j));
        E[k] = nsum_value(&acc);
    }
}

/* Forces of the same softened potential (a symmetric pairwise interaction
 * with a vector value, Section 4's interact() returning a vector): the force
 * on object i from object j is minus the gradient of e_ij in p_i,
 *   f_ij = (p_i - p_j) / (|p_i - p_j|^2 + eps2)^(3/2),   f_ji = -f_ij,
 * and F_i = sum over j != i of f_ij, each component summed with Neumaier's
 * compensation in double.  S_i = sum over j != i of |f_ij| (the Euclidean
 * norm of each term) is the scale against which cancellation in F_i is
 * measured.  rows: the objects to compute (NULL: all n, in order). */
void oracle_force_rows(const float *x, const float *y, const float *z, int64_t n, float eps2f,
                       const int64_t *rows, int64_t nrows, double *Fx, double *Fy, double *Fz,
                       double *S, int threads) {
    const double eps2 = (double)eps2f;
    int64_t m = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(threads))
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        nsum_t ax = {0.0, 0.0}, ay = {0.0, 0.0}, az = {0.0, 0.0}, as = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = (double)x[i] - (double)x[j];
            double dy = (double)y[i] - (double)y[j];
            double dz = (double)z[i] - (double)z[j];
            double d2 = dx * dx + dy * dy + dz * dz + eps2;
            double w = 1.0 / (d2 * sqrt(d2));
            nsum_add(&ax, dx * w);
            nsum_add(&ay, dy * w);
            nsum_add(&az, dz * w);
            nsum_add(&as, sqrt(dx * dx + dy * dy + dz * dz) * w);
        }
        Fx[k] = nsum_value(&ax);
        Fy[k] = nsum_value(&ay);
        Fz[k] = nsum_value(&az);
        S[k] = nsum_value(&as);
    }
}

/* ---------------------------------------------------------------- batches -- */
/* A batch is CSR: set s owns objects [off[s], off[s+1]).  Each set is an
 * independent instance of the single-set problem. */

void oracle_count_i32_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                              const int32_t *r, const int64_t *off, int64_t n_sets,
                              uint64_t *out, int threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(threads))
    for (int64_t s = 0; s < n_sets; ++s) {
        int64_t b = off[s], n = off[s + 1] - off[s];
        out[s] = oracle_count_i32(x + b, y + b, z + b, r + b, n, 1);
    }
}

void oracle_energy_count_f32_batched(const float *x, const float *y, const float *z,
                                     const float *r, const int64_t *off, int64_t n_sets,
                                     float eps2f, double *energy, uint64_t *counts,
                                     int threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(threads))
    for (int64_t s = 0; s < n_sets; ++s) {
        int64_t b = off[s], n = off[s + 1] - off[s];
        if (energy) energy[s] = oracle_energy_total(x + b, y + b, z + b, n, eps2f, 1);
        if (counts) counts[s] = oracle_count_f32(x + b, y + b, z + b, r + b, n, 1);
    }
}

/* ----------------------------------------------------------------- jitter -- */
/*
 * Per-step position perturbation of the repeated-step workload.
 *
 * Random numbers come from Philox4x32-10, the counter-based generator of
 * Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC 2011): a 4x32-bit counter is passed through 10 rounds, each of which
 * multiplies two counter words by the constants 0xD2511F53 and 0xCD9E8D57,
 * takes the high and low halves of the 64-bit products, exchanges words and
 * xors in the 2x32-bit key; the key is advanced by the Weyl increments
 * 0x9E3779B9 and 0xBB67AE85 between rounds.
 *
 * Counter (global object index, step, axis, 0); key (seed low word, seed high
 * word).  The four output words w_k give u_k = w_k >> 8, uniform on [0, 2^24);
 * S = 2 (u_0 + u_1 + u_2 + u_3) - 4 (2^24 - 1) is a zero-mean Irwin-Hall(4)
 * variate (an approximation of a normal variate bounded at about 3.46 standard
 * deviations) with variance (4/3)(2^48 - 1).  The perturbation is
 * delta = fl32(fl32(S) * c) with c = fl32(sigma / sqrt((4/3)(2^48 - 1))) and
 * the coordinate becomes fl32(x + delta).  Every step is an exactly rounded
 * IEEE operation, so any correct implementation reproduces it bit for bit.
 */
static inline void philox_round(uint32_t ctr[4], const uint32_t key[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * ctr[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    uint32_t n3 = lo0;
    ctr[0] = n0; ctr[1] = n1; ctr[2] = n2; ctr[3] = n3;
}

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t ctr[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            key[0] += 0x9E3779B9u;
            key[1] += 0xBB67AE85u;
        }
        philox_round(ctr, key);
    }
    out[0] = ctr[0]; out[1] = ctr[1]; out[2] = ctr[2]; out[3] = ctr[3];
}

float oracle_jitter_scale(float sigma) {
    return (float)((double)sigma / sqrt(4.0 / 3.0 * (ldexp(1.0, 48) - 1.0)));
}

/* Apply one step of perturbation to objects [0, n) whose global indices are
 * first_index + k. */
void oracle_jitter_f32(float *x, float *y, float *z, int64_t n, uint64_t seed,
                       uint32_t step, float sigma, int64_t first_index) {
    const float c = oracle_jitter_scale(sigma);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    float *coord[3] = {x, y, z};
    for (int64_t k = 0; k < n; ++k) {
        for (uint32_t axis = 0; axis < 3; ++axis) {
            uint32_t ctr[4] = {(uint32_t)(first_index + k), step, axis, 0u};
            uint32_t w[4];
            oracle_philox4x32_10(ctr, key, w);
            int32_t sum = 0;
            for (int q = 0; q < 4; ++q) sum += (int32_t)(w[q] >> 8);
            int32_t S = 2 * sum - 4 * ((1 << 24) - 1);
            float delta = (float)S * c;
            coord[axis][k] = coord[axis][k] + delta;
        }
    }
}

/* ---------------------------------------------------------- lattice beads -- */
/* Beads are points of the integer lattice Z^3 (Section 3).  For one vector of
 * beads the paper counts
 *   - collisions: pairs of beads on the same lattice site (its countColls
 *     accumulates, bead by bead, how many earlier beads occupy the site; the
 *     total is the number of unordered pairs with equal coordinates), and
 *   - contacts: pairs of beads on neighbouring sites, the six sites at unit
 *     distance along one axis (its countContacts sums the occupancy of the six
 *     neighbours of every bead and halves the result, so each unordered pair
 *     counts once).
 * This is that plain definition over the unordered pairs i < j of a vector,
 * with the coordinate differences taken in 64 bits so that any int32 input is
 * exact.  Vectors are CSR like the sphere batches. */

void oracle_lattice_counts(const int32_t *x, const int32_t *y, const int32_t *z,
                           int64_t n, uint64_t *collisions, uint64_t *contacts) {
    uint64_t coll = 0, cont = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            int64_t dx = (int64_t)x[i] - x[j];
            int64_t dy = (int64_t)y[i] - y[j];
            int64_t dz = (int64_t)z[i] - z[j];
            int64_t l1 = llabs(dx) + llabs(dy) + llabs(dz);
            coll += l1 == 0;
            cont += l1 == 1;
        }
    }
    *collisions = coll;
    *contacts = cont;
}

void oracle_lattice_batched(const int32_t *x, const int32_t *y, const int32_t *z,
                            const int64_t *off, int64_t n_sets, uint64_t *collisions,
                            uint64_t *contacts, int threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(threads))
    for (int64_t s = 0; s < n_sets; ++s) {
        int64_t b = off[s];
        oracle_lattice_counts(x + b, y + b, z + b, off[s + 1] - b, collisions + s, contacts + s);
    }
}
