/*
 * oracle.h -- plain CPU oracle for the STREAM hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load or call this library.
 * The GPU library (libtstream) never includes, links or loads it; the two
 * share no source, header, table or helper.
 *
 * What it computes: the four element-wise maps of the generic STREAM
 * benchmark in Section 5 (Listing 4) of Heller et al., "Closing the
 * Performance Gap with Modern C++" -- copy, scale, add, triad -- over plain
 * host arrays, in that order, with scalar 3.0 in the paper's runs.
 *
 *   copy   c[j] <- a[j]
 *   scale  b[j] <- q * c[j]
 *   add    c[j] <- a[j] + b[j]
 *   triad  a[j] <- b[j] + q * c[j], computed as fma(q, c[j], b[j]):
 *          one rounding (the reading taken for the listing's b + c*scalar).
 *
 * Binary64 results are exact IEEE-754 round-to-nearest-even results of each
 * operation, so every output element is uniquely defined.  The file is built
 * by gcc with -O2 -ffp-contract=off -fno-fast-math on x86-64 (SSE2, no
 * excess precision): no operation is contracted, reassociated or blocked.
 *
 * Reduced-precision storage (not in the paper; a storage form of the same
 * maps): elements stored as binary32, bfloat16 or binary16 are widened
 * exactly to binary32, the map is evaluated in binary32 (fmaf for triad,
 * q rounded once to binary32), and the result is narrowed back by
 * round-to-nearest-even with this file's own converters.
 *
 * Pins (tests under tests/ that need no GPU): the closed form of the
 * iteration from (1, 2, 0) with q = 3, and the closed form (Binet) of the
 * variant whose copy is a <- b; exact rational arithmetic rounded once, for
 * every op and storage type on tiny random and special inputs and for chains
 * of up to 80 iterations (which also tells one rounding of the triad from
 * two); the converters against numpy and torch over every rounding class
 * (all 2^32 inputs with TS_EXHAUSTIVE=1); checksums against math.fsum; and
 * the stored fixtures in tests/golden/.
 */
#ifndef STREAM_ORACLE_H
#define STREAM_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage types (the oracle's own numbering). */
enum { ORACLE_F64 = 0, ORACLE_F32 = 1, ORACLE_BF16 = 2, ORACLE_F16 = 3 };
/* Operations of Listing 4, in the order the benchmark runs them. */
enum { ORACLE_COPY = 0, ORACLE_SCALE = 1, ORACLE_ADD = 2, ORACLE_TRIAD = 3 };

/* --- Binary64 maps (Section 5, Listing 4) ------------------------------ */
void oracle_copy_f64(const double *src, double *dst, size_t n);
void oracle_scale_f64(const double *src, double *dst, size_t n, double q);
void oracle_add_f64(const double *x, const double *y, double *dst, size_t n);
/* dst[j] = fma(q, y[j], x[j]) = x[j] + q*y[j] with one rounding. */
void oracle_triad_f64(const double *x, const double *y, double *dst, size_t n,
                      double q);

/* One benchmark iteration over arrays a, b, c in the listing's order:
 * copy (a -> c), scale (c -> b), add (a, b -> c), triad (b, c -> a). */
void oracle_stream_iteration_f64(double *a, double *b, double *c, size_t n,
                                 double q);
void oracle_stream_run_f64(double *a, double *b, double *c, size_t n, double q,
                           int iterations);
/* The variant whose copy runs a <- b (the direction some one-line summaries
 * of STREAM write); scale, add and triad as in the listing:
 * copy (b -> a), scale (c -> b), add (a, b -> c), triad (b, c -> a). */
void oracle_stream_iteration_copyb_f64(double *a, double *b, double *c,
                                       size_t n, double q);
void oracle_stream_run_copyb_f64(double *a, double *b, double *c, size_t n,
                                 double q, int iterations);

/* --- Reduced-precision storage ------------------------------------------ */
/* Round-to-nearest-even narrowing of a binary32 value; NaN stays NaN (quiet,
 * sign kept), overflow goes to infinity, binary16 subnormals are produced. */
uint16_t oracle_f32_to_bf16(float x);
uint16_t oracle_f32_to_f16(float x);
/* Exact widening to binary32. */
float oracle_bf16_to_f32(uint16_t h);
float oracle_f16_to_f32(uint16_t h);
/* Array forms of the converters (for exhaustive tests). */
void oracle_f32_to_bf16_array(const float *x, uint16_t *out, size_t n);
void oracle_f32_to_f16_array(const float *x, uint16_t *out, size_t n);
void oracle_bf16_to_f32_array(const uint16_t *x, float *out, size_t n);
void oracle_f16_to_f32_array(const uint16_t *x, float *out, size_t n);

/* One map over arrays of storage type `dtype`.  `y` is unused by copy and
 * scale; `q` is unused by copy and add.  Copy moves the stored bits
 * unchanged.  Returns 0, or -1 for an unknown dtype/op. */
int oracle_op(int dtype, int op, const void *x, const void *y, void *dst,
              size_t n, double q);
/* `iterations` benchmark iterations (listing order) in storage type dtype. */
int oracle_stream_run(int dtype, void *a, void *b, void *c, size_t n, double q,
                      int iterations);

/* --- Validation ------------------------------------------------------------ */
typedef struct {
    double sum;          /* sum of x[j] widened to binary64, j = 0..n-1 in order */
    double abs_dev_sum;  /* sum of |x[j] - expected|                              */
    double max_abs_dev;  /* max of |x[j] - expected| (NaN terms ignored, as fmax) */
    uint64_t mismatches; /* count of x[j] whose binary64 value differs in bits
                            from `expected`; NaN matches NaN                   */
} oracle_checksum;

int oracle_checksum_array(int dtype, const void *x, size_t n, double expected,
                          oracle_checksum *out);
/* Count of j where x[j] and ref[j] differ in stored bits (NaN matches NaN). */
int oracle_mismatch_count(int dtype, const void *x, const void *ref, size_t n,
                          uint64_t *out);

/* --- Timed mode (host baseline) ------------------------------------------- */
/* Runs `iterations` binary64 benchmark iterations over three freshly
 * allocated arrays of n elements with `threads` POSIX threads.  Thread t owns
 * the contiguous block [t*n/T, (t+1)*n/T) of every array, is pinned to the
 * t-th CPU of the process's affinity set, and writes the initial values
 * (1, 2, 0) into its own block itself (first touch).  The four maps run in
 * listing order with a barrier around each; op_seconds[4*it + op] receives
 * the wall time of map `op` in iteration `it`.  final_abc receives
 * a[0], b[0], c[0], a[n-1], b[n-1], c[n-1] at the end.  T is the number of
 * threads the system let the call create (at most `threads`, reported in
 * *threads_used): the blocks and the barrier are sized to them before any
 * of them starts, so a partial start still runs to the end.
 * Returns 0, -1 on bad arguments, -2 on allocation failure or when no
 * thread could be created. */
int oracle_stream_timed_f64(size_t n, int iterations, int threads, double q,
                            double *op_seconds, double *final_abc,
                            int *threads_used);

#ifdef __cplusplus
}
#endif
#endif
