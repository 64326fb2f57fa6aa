/*
 * oracle.c -- plain CPU oracle for the STREAM hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE: loaded only by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg.  Shares nothing with the
 * GPU library.  The contract of every function is in oracle.h.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        -pthread oracle.c -lm
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <sched.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Binary64 maps: Section 5, Listing 4.                                     */
/* ------------------------------------------------------------------------ */

/* Listing 4, "Copy": copy(as -> cs). */
void oracle_copy_f64(const double *src, double *dst, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        dst[j] = src[j];
}

/* Listing 4, "Scale": transform(cs -> bs, c * scalar). */
void oracle_scale_f64(const double *src, double *dst, size_t n, double q)
{
    for (size_t j = 0; j < n; ++j)
        dst[j] = q * src[j];
}

/* Listing 4, "Add": transform(as, bs -> cs, a + b). */
void oracle_add_f64(const double *x, const double *y, double *dst, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        dst[j] = x[j] + y[j];
}

/* Listing 4, "Triad": transform(bs, cs -> as, b + c * scalar), read as a
 * single fused multiply-add (one rounding). */
void oracle_triad_f64(const double *x, const double *y, double *dst, size_t n,
                      double q)
{
    for (size_t j = 0; j < n; ++j)
        dst[j] = fma(q, y[j], x[j]);
}

/* Listing 4 as a whole: the four maps in the order the benchmark runs them. */
void oracle_stream_iteration_f64(double *a, double *b, double *c, size_t n,
                                 double q)
{
    oracle_copy_f64(a, c, n);        /* c = a         */
    oracle_scale_f64(c, b, n, q);    /* b = q * c     */
    oracle_add_f64(a, b, c, n);      /* c = a + b     */
    oracle_triad_f64(b, c, a, n, q); /* a = b + q * c */
}

void oracle_stream_run_f64(double *a, double *b, double *c, size_t n, double q,
                           int iterations)
{
    for (int it = 0; it < iterations; ++it)
        oracle_stream_iteration_f64(a, b, c, n, q);
}

void oracle_stream_iteration_copyb_f64(double *a, double *b, double *c,
                                       size_t n, double q)
{
    oracle_copy_f64(b, a, n);        /* a = b         */
    oracle_scale_f64(c, b, n, q);    /* b = q * c     */
    oracle_add_f64(a, b, c, n);      /* c = a + b     */
    oracle_triad_f64(b, c, a, n, q); /* a = b + q * c */
}

void oracle_stream_run_copyb_f64(double *a, double *b, double *c, size_t n,
                                 double q, int iterations)
{
    for (int it = 0; it < iterations; ++it)
        oracle_stream_iteration_copyb_f64(a, b, c, n, q);
}

/* ------------------------------------------------------------------------ */
/* Storage-format converters, written from the IEEE-754 format definitions. */
/* ------------------------------------------------------------------------ */

static uint32_t f32_bits(float x)
{
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

static float f32_from_bits(uint32_t u)
{
    float x;
    memcpy(&x, &u, sizeof x);
    return x;
}

static uint64_t f64_bits(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

/* bfloat16 is the upper half of a binary32 pattern (8 exponent bits, 7
 * stored fraction bits).  Narrowing keeps the upper 16 bits and rounds on the
 * lower 16: up when they exceed one half of the last kept place, or equal it
 * and the kept pattern is odd.  A carry out of the fraction moves into the
 * exponent, which is exactly the next representable value (infinity past the
 * largest finite). */
uint16_t oracle_f32_to_bf16(float x)
{
    uint32_t u = f32_bits(x);
    if ((u & 0x7fffffffu) > 0x7f800000u)          /* NaN: keep sign, quiet it */
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t keep = u >> 16;
    uint32_t rest = u & 0xffffu;
    if (rest > 0x8000u || (rest == 0x8000u && (keep & 1u)))
        keep += 1u;
    return (uint16_t)keep;
}

float oracle_bf16_to_f32(uint16_t h)
{
    return f32_from_bits((uint32_t)h << 16);
}

/* binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits.
 * Normal values are s * 2^(e-10) with 2^10 <= s < 2^11 and -14 <= e <= 15;
 * subnormals are s * 2^-24 with 0 < s < 2^10. */
uint16_t oracle_f32_to_f16(float x)
{
    uint32_t u = f32_bits(x);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    uint32_t mag = u & 0x7fffffffu;
    if (mag > 0x7f800000u)                       /* NaN: quiet, sign kept */
        return (uint16_t)(sign | 0x7e00u | ((mag >> 13) & 0x03ffu));
    if (mag == 0x7f800000u)                      /* infinity */
        return (uint16_t)(sign | 0x7c00u);
    uint32_t biased = mag >> 23;
    if (biased == 0)          /* zero or binary32 subnormal: below 2^-126,   */
        return sign;          /* far under half the least binary16 subnormal */
    int e = (int)biased - 127;                   /* |x| = sig * 2^(e-23)    */
    uint32_t sig = (mag & 0x7fffffu) | 0x800000u; /* 2^23 <= sig < 2^24     */
    if (e < -25)                                 /* |x| < 2^-25: rounds to 0 */
        return sign;
    /* Number of low bits of sig below the binary16 quantum: 2^(e-10) for
     * normal results, 2^-24 for subnormal ones. */
    int shift = (e >= -14) ? 13 : (-e - 1);
    uint32_t q = sig >> shift;
    uint32_t rest = sig & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1);
    if (rest > half || (rest == half && (q & 1u)))
        q += 1u;
    uint32_t bits;
    if (e >= -14)
        bits = ((uint32_t)(e + 14) << 10) + q;   /* q carries the hidden bit */
    else
        bits = q;                                /* subnormal, or 2^-14 on carry */
    if (bits >= 0x7c00u)
        bits = 0x7c00u;                          /* overflow to infinity */
    return (uint16_t)(sign | bits);
}

float oracle_f16_to_f32(uint16_t h)
{
    int negative = (h & 0x8000u) != 0;
    int biased = (h >> 10) & 0x1f;
    int frac = h & 0x3ff;
    float mag;
    if (biased == 0)
        mag = ldexpf((float)frac, -24);
    else if (biased == 31)
        mag = frac ? NAN : INFINITY;
    else
        mag = ldexpf((float)(frac + 1024), biased - 25);
    return negative ? -mag : mag;
}

void oracle_f32_to_bf16_array(const float *x, uint16_t *out, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        out[j] = oracle_f32_to_bf16(x[j]);
}

void oracle_f32_to_f16_array(const float *x, uint16_t *out, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        out[j] = oracle_f32_to_f16(x[j]);
}

void oracle_bf16_to_f32_array(const uint16_t *x, float *out, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        out[j] = oracle_bf16_to_f32(x[j]);
}

void oracle_f16_to_f32_array(const uint16_t *x, float *out, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        out[j] = oracle_f16_to_f32(x[j]);
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision storage: widen exactly, evaluate in binary32, narrow.  */
/* ------------------------------------------------------------------------ */

static size_t elem_size(int dtype)
{
    switch (dtype) {
    case ORACLE_F64: return 8;
    case ORACLE_F32: return 4;
    case ORACLE_BF16:
    case ORACLE_F16: return 2;
    default: return 0;
    }
}

static float load_f32(int dtype, const void *p, size_t j)
{
    if (dtype == ORACLE_F32)
        return ((const float *)p)[j];
    uint16_t h = ((const uint16_t *)p)[j];
    return dtype == ORACLE_BF16 ? oracle_bf16_to_f32(h) : oracle_f16_to_f32(h);
}

static void store_f32(int dtype, void *p, size_t j, float v)
{
    if (dtype == ORACLE_F32)
        ((float *)p)[j] = v;
    else if (dtype == ORACLE_BF16)
        ((uint16_t *)p)[j] = oracle_f32_to_bf16(v);
    else
        ((uint16_t *)p)[j] = oracle_f32_to_f16(v);
}

int oracle_op(int dtype, int op, const void *x, const void *y, void *dst,
              size_t n, double q)
{
    size_t es = elem_size(dtype);
    if (es == 0 || op < ORACLE_COPY || op > ORACLE_TRIAD)
        return -1;
    if (dtype == ORACLE_F64) {
        switch (op) {
        case ORACLE_COPY: oracle_copy_f64(x, dst, n); break;
        case ORACLE_SCALE: oracle_scale_f64(x, dst, n, q); break;
        case ORACLE_ADD: oracle_add_f64(x, y, dst, n); break;
        default: oracle_triad_f64(x, y, dst, n, q); break;
        }
        return 0;
    }
    if (op == ORACLE_COPY) {                   /* stored bits move unchanged */
        memmove(dst, x, n * es);
        return 0;
    }
    float qf = (float)q;                       /* one RNE rounding of q */
    for (size_t j = 0; j < n; ++j) {
        float r;
        if (op == ORACLE_SCALE)
            r = qf * load_f32(dtype, x, j);
        else if (op == ORACLE_ADD)
            r = load_f32(dtype, x, j) + load_f32(dtype, y, j);
        else
            r = fmaf(qf, load_f32(dtype, y, j), load_f32(dtype, x, j));
        store_f32(dtype, dst, j, r);
    }
    return 0;
}

int oracle_stream_run(int dtype, void *a, void *b, void *c, size_t n, double q,
                      int iterations)
{
    if (elem_size(dtype) == 0)
        return -1;
    for (int it = 0; it < iterations; ++it) {
        oracle_op(dtype, ORACLE_COPY, a, NULL, c, n, q);
        oracle_op(dtype, ORACLE_SCALE, c, NULL, b, n, q);
        oracle_op(dtype, ORACLE_ADD, a, b, c, n, q);
        oracle_op(dtype, ORACLE_TRIAD, b, c, a, n, q);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Validation sums.                                                          */
/* ------------------------------------------------------------------------ */

static double load_f64(int dtype, const void *p, size_t j)
{
    if (dtype == ORACLE_F64)
        return ((const double *)p)[j];
    return (double)load_f32(dtype, p, j);
}

static int same_value_bits(double v, double expected)
{
    if (isnan(v) && isnan(expected))
        return 1;
    return f64_bits(v) == f64_bits(expected);
}

int oracle_checksum_array(int dtype, const void *x, size_t n, double expected,
                          oracle_checksum *out)
{
    if (elem_size(dtype) == 0 || out == NULL)
        return -1;
    oracle_checksum r = {0.0, 0.0, NAN, 0};
    for (size_t j = 0; j < n; ++j) {
        double v = load_f64(dtype, x, j);
        double d = fabs(v - expected);
        r.sum += v;
        r.abs_dev_sum += d;
        r.max_abs_dev = fmax(r.max_abs_dev, d);
        if (!same_value_bits(v, expected))
            r.mismatches += 1;
    }
    if (n == 0)
        r.max_abs_dev = 0.0;
    *out = r;
    return 0;
}

int oracle_mismatch_count(int dtype, const void *x, const void *ref, size_t n,
                          uint64_t *out)
{
    size_t es = elem_size(dtype);
    if (es == 0 || out == NULL)
        return -1;
    uint64_t count = 0;
    for (size_t j = 0; j < n; ++j) {
        double v = load_f64(dtype, x, j);
        double r = load_f64(dtype, ref, j);
        if (isnan(v) && isnan(r))
            continue;
        if (memcmp((const char *)x + j * es, (const char *)ref + j * es, es) != 0)
            count += 1;
    }
    *out = count;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Timed mode: block-partitioned, pinned threads, first-touch placement.     */
/* The block scheme follows the paper's NUMA allocator/executor (Section    */
/* 4.1): bytes divided evenly over the targets, work pinned to its block.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *a, *b, *c;
    size_t n;
    int threads;
    int iterations;
    double q;
    double *op_seconds;
    pthread_barrier_t barrier;
    cpu_set_t allowed;
    int n_allowed;
    /* Start gate: workers wait until every thread that could be created
     * exists; `go` is then 1 (threads = that number) or -1 (give up). */
    pthread_mutex_t gate_mu;
    pthread_cond_t gate_cv;
    int go;
} timed_shared;

typedef struct {
    timed_shared *s;
    int tid;
} timed_arg;

static double now_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void pin_to_allowed_cpu(const timed_shared *s, int tid)
{
    if (s->n_allowed <= 0)
        return;
    int want = tid % s->n_allowed, seen = 0;
    for (int cpu = 0; cpu < CPU_SETSIZE; ++cpu) {
        if (!CPU_ISSET(cpu, &s->allowed))
            continue;
        if (seen++ == want) {
            cpu_set_t one;
            CPU_ZERO(&one);
            CPU_SET(cpu, &one);
            sched_setaffinity(0, sizeof one, &one); /* best effort */
            return;
        }
    }
}

static void *timed_worker(void *p)
{
    timed_arg *arg = p;
    timed_shared *s = arg->s;
    int t = arg->tid;
    pthread_mutex_lock(&s->gate_mu);
    while (s->go == 0)
        pthread_cond_wait(&s->gate_cv, &s->gate_mu);
    int go = s->go;
    pthread_mutex_unlock(&s->gate_mu);
    if (go < 0)
        return NULL;
    pin_to_allowed_cpu(s, t);
    size_t lo = (size_t)t * s->n / (size_t)s->threads;
    size_t hi = (size_t)(t + 1) * s->n / (size_t)s->threads;
    size_t len = hi - lo;
    double *a = s->a + lo, *b = s->b + lo, *c = s->c + lo;
    for (size_t j = 0; j < len; ++j) {  /* first touch of this block */
        a[j] = 1.0;
        b[j] = 2.0;
        c[j] = 0.0;
    }
    for (int it = 0; it < s->iterations; ++it) {
        for (int op = ORACLE_COPY; op <= ORACLE_TRIAD; ++op) {
            double t0 = 0.0;
            pthread_barrier_wait(&s->barrier);
            if (t == 0)
                t0 = now_seconds();
            switch (op) {
            case ORACLE_COPY: oracle_copy_f64(a, c, len); break;
            case ORACLE_SCALE: oracle_scale_f64(c, b, len, s->q); break;
            case ORACLE_ADD: oracle_add_f64(a, b, c, len); break;
            default: oracle_triad_f64(b, c, a, len, s->q); break;
            }
            pthread_barrier_wait(&s->barrier);
            if (t == 0)
                s->op_seconds[4 * it + op] = now_seconds() - t0;
        }
    }
    return NULL;
}

int oracle_stream_timed_f64(size_t n, int iterations, int threads, double q,
                            double *op_seconds, double *final_abc,
                            int *threads_used)
{
    if (n == 0 || iterations < 0 || threads < 1 || threads > 1024 ||
        op_seconds == NULL || final_abc == NULL || threads_used == NULL)
        return -1;
    *threads_used = 0;
    timed_shared s;
    memset(&s, 0, sizeof s);
    size_t bytes = ((n * sizeof(double)) + 4095u) & ~(size_t)4095u;
    s.a = aligned_alloc(4096, bytes);
    s.b = aligned_alloc(4096, bytes);
    s.c = aligned_alloc(4096, bytes);
    pthread_t *tids = calloc((size_t)threads, sizeof *tids);
    timed_arg *args = calloc((size_t)threads, sizeof *args);
    if (!s.a || !s.b || !s.c || !tids || !args) {
        free(s.a);
        free(s.b);
        free(s.c);
        free(tids);
        free(args);
        return -2;
    }
    s.n = n;
    s.iterations = iterations;
    s.q = q;
    s.op_seconds = op_seconds;
    CPU_ZERO(&s.allowed);
    if (sched_getaffinity(0, sizeof s.allowed, &s.allowed) == 0)
        s.n_allowed = CPU_COUNT(&s.allowed);
    pthread_mutex_init(&s.gate_mu, NULL);
    pthread_cond_init(&s.gate_cv, NULL);
    int started = 0;
    for (int t = 0; t < threads; ++t) {
        args[t].s = &s;
        args[t].tid = t;
        if (pthread_create(&tids[t], NULL, timed_worker, &args[t]) != 0)
            break;
        ++started;
    }
    /* The run uses the threads that exist: the blocks and the barrier are
     * sized to them before any worker passes the gate. */
    s.threads = started;
    if (started > 0)
        pthread_barrier_init(&s.barrier, NULL, (unsigned)started);
    pthread_mutex_lock(&s.gate_mu);
    s.go = started > 0 ? 1 : -1;
    pthread_cond_broadcast(&s.gate_cv);
    pthread_mutex_unlock(&s.gate_mu);
    for (int t = 0; t < started; ++t)
        pthread_join(tids[t], NULL);
    int rc = -2;
    if (started > 0) {
        pthread_barrier_destroy(&s.barrier);
        final_abc[0] = s.a[0];
        final_abc[1] = s.b[0];
        final_abc[2] = s.c[0];
        final_abc[3] = s.a[n - 1];
        final_abc[4] = s.b[n - 1];
        final_abc[5] = s.c[n - 1];
        *threads_used = started;
        rc = 0;
    }
    pthread_cond_destroy(&s.gate_cv);
    pthread_mutex_destroy(&s.gate_mu);
    free(tids);
    free(args);
    free(s.a);
    free(s.b);
    free(s.c);
    return rc;
}
