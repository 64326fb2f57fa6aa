/*
 * stream_client.c -- a plain C consumer of libtstream, with no Python and no
 * torch in the process: it includes only the public header and links only
 * the library.  It runs the STREAM iteration (Section 5, Listing 4) from
 * (1, 2, 0) with q = 3 and checks STREAM's closed form a = 15^k,
 * b = 3 * 15^(k-1), c = 4 * 15^(k-1) (exact in binary64 for k <= 13) on the
 * device and on elements copied back, then runs a small ragged batch through
 * a captured multi-iteration graph and checks each instance's closed form.
 *
 * Usage: stream_client [n] [host]   (default n = 1000003).  With "host" the
 * same STREAM checks run on a host-CPU target (no GPU needed), followed by
 * a run-time-compiled transform (to_upper over bytes); batches and graphs
 * must then report TS_E_UNSUPPORTED.  Exit status 0 when every check
 * passes; each step prints one line.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tstream.h"

#define CHECK(call)                                                            \
    do {                                                                       \
        int st_ = (call);                                                      \
        if (st_ != TS_OK) {                                                    \
            fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__,      \
                    #call, st_, ts_last_error());                              \
            exit(2);                                                           \
        }                                                                      \
    } while (0)

static int fail_count = 0;

static void expect(int ok, const char *what)
{
    printf("%s: %s\n", ok ? "ok  " : "FAIL", what);
    fflush(stdout);
    if (!ok)
        ++fail_count;
}

/* Closed form from (1, 2, 0) with scalar q: one iteration maps a to
 * q(2 + q) a, b to q a, c to (1 + q) a, so after k >= 1 iterations
 * a = g^k, b = q g^(k-1), c = (1 + q) g^(k-1) with g = q(2 + q).  For the
 * scalars used here (3, 1/2, 5/4, 2) and k = 8 every factor and product is a
 * dyadic rational with a short significand, so each value is exact. */
static void closed_form(double q, int k, double *a, double *b, double *c)
{
    const double g = q * (2.0 + q);
    double p = 1.0; /* g^(k-1) */
    for (int i = 1; i < k; ++i)
        p *= g;
    *a = p * g;
    *b = q * p;
    *c = (1.0 + q) * p;
}

int main(int argc, char **argv)
{
    size_t n = argc > 1 ? (size_t)strtoull(argv[1], NULL, 10) : 1000003u;
    const int on_host = argc > 2 && strcmp(argv[2], "host") == 0;
    int major = 0, minor = 0;
    CHECK(ts_version(&major, &minor));
    printf("libtstream %d.%d, n = %zu, %s target\n", major, minor, n, on_host ? "host" : "GPU");

    ts_target tgt;
    if (on_host)
        CHECK(ts_target_create_host(NULL, 0, &tgt));
    else
        CHECK(ts_target_create_owned(0, &tgt));
    ts_array arr[3];
    const double init[3] = {1.0, 2.0, 0.0};
    for (int k = 0; k < 3; ++k) {
        CHECK(ts_array_alloc(tgt, TS_F64, n, 1, &arr[k])); /* one element past an aligned base */
        CHECK(ts_fill(arr[k], init[k]));
    }

    const int iters = 10;
    for (int i = 0; i < iters; ++i)
        CHECK(ts_stream_iteration(tgt, arr[0], arr[1], arr[2], 3.0));
    CHECK(ts_target_synchronize(tgt));

    const double expected[3] = {576650390625.0, 115330078125.0, 153773437500.0};
    for (int k = 0; k < 3; ++k) {
        ts_checksum_out cs;
        CHECK(ts_checksum(tgt, arr[k], expected[k], &cs));
        char msg[128];
        snprintf(msg, sizeof msg, "array %c: closed form at every element (%llu mismatches)", "abc"[k],
                 (unsigned long long)cs.mismatches);
        expect(cs.mismatches == 0 && cs.max_abs_dev == 0.0, msg);
    }
    double *host = malloc(n * sizeof(double));
    if (!host)
        return 2;
    CHECK(ts_copy_to_host(host, arr[0], n));
    CHECK(ts_target_synchronize(tgt));
    expect(host[0] == expected[0] && host[n / 2] == expected[0] && host[n - 1] == expected[0],
           "copied-back elements of a equal 15^10");
    free(host);

    if (on_host) {
        /* Listing 3 on the host: upper-case a byte array in place. */
        const char text[] = "hello world";
        ts_array s;
        CHECK(ts_array_alloc(tgt, TS_U8, sizeof text - 1, 0, &s));
        CHECK(ts_copy_from_host(s, text, sizeof text - 1));
        ts_transform up;
        CHECK(ts_transform_create(tgt, "(x >= 'a' && x <= 'z') ? x - ('a' - 'A') : x", 1, TS_U8, &up));
        CHECK(ts_transform_apply(tgt, up, s, NULL, s, 0.0));
        char back[sizeof text] = {0};
        CHECK(ts_copy_to_host(back, s, sizeof text - 1));
        expect(strcmp(back, "HELLO WORLD") == 0, "to_upper transform on the host target");
        CHECK(ts_transform_destroy(up));
        CHECK(ts_array_free(s));
        ts_batch none;
        ts_batch_desc d0 = {NULL, NULL, NULL, 0, 1.0};
        ts_graph g0;
        expect(ts_batch_create(tgt, TS_F64, &d0, 1, &none) == TS_E_UNSUPPORTED &&
                   ts_graph_capture_arrays_iteration(tgt, arr[0], arr[1], arr[2], 3.0, &g0) == TS_E_UNSUPPORTED,
               "batches and graphs are GPU-only (TS_E_UNSUPPORTED)");
        for (int k = 0; k < 3; ++k)
            CHECK(ts_array_free(arr[k]));
        CHECK(ts_target_destroy(tgt));
        printf("%s\n", fail_count ? "FAILED" : "all checks passed");
        return fail_count ? 1 : 0;
    }

    /* A ragged batch carved out of the three arrays: instance i covers
     * elements [off_i, off_i + len_i) of each, with its own scalar. */
    enum { COUNT = 5 };
    const uint64_t lens[COUNT] = {0, 1, 777, 4099, 65537};
    const double qs[COUNT] = {3.0, 0.5, 1.25, 3.0, 2.0};
    void *base[3];
    for (int k = 0; k < 3; ++k)
        CHECK(ts_array_info(arr[k], &base[k], NULL, NULL));
    ts_batch_desc descs[COUNT];
    uint64_t off = 0;
    for (int i = 0; i < COUNT; ++i) {
        descs[i].a = (char *)base[0] + off * 8;
        descs[i].b = (char *)base[1] + off * 8;
        descs[i].c = (char *)base[2] + off * 8;
        descs[i].len = lens[i];
        descs[i].q = qs[i];
        off += lens[i] + 3;
    }
    if (off > n) {
        fprintf(stderr, "n = %zu is too small for the batch (needs %llu)\n", n, (unsigned long long)off);
        return 2;
    }
    ts_batch batch;
    CHECK(ts_batch_create(tgt, TS_F64, descs, COUNT, &batch));
    for (int k = 0; k < 3; ++k)
        CHECK(ts_batch_fill(tgt, batch, k, init[k]));
    ts_graph graph;
    CHECK(ts_graph_capture_stream_iterations(tgt, batch, 4, &graph));
    CHECK(ts_graph_launch(tgt, graph, 2)); /* 8 iterations */
    CHECK(ts_target_synchronize(tgt));
    for (int k = 0; k < 3; ++k) {
        double exp_k[COUNT];
        uint64_t counts[COUNT];
        for (int i = 0; i < COUNT; ++i) {
            double v[3];
            closed_form(qs[i], 8, &v[0], &v[1], &v[2]);
            exp_k[i] = v[k];
        }
        CHECK(ts_batch_mismatch_count(tgt, batch, k, exp_k, counts));
        uint64_t total = 0;
        for (int i = 0; i < COUNT; ++i)
            total += counts[i];
        char msg[128];
        snprintf(msg, sizeof msg, "batched graph, array %c: every instance at its closed form (%llu mismatches)",
                 "abc"[k], (unsigned long long)total);
        expect(total == 0, msg);
    }

    /* The allocation-free checksum: the same reductions as ts_checksum, the
     * result written in stream order to device memory the caller owns. */
    {
        ts_array out_arr;
        void *out_ptr = NULL;
        ts_checksum_out ref, got;
        CHECK(ts_array_alloc(tgt, TS_F64, 4, 0, &out_arr)); /* 32 bytes: one ts_checksum_out */
        CHECK(ts_array_info(out_arr, &out_ptr, NULL, NULL));
        CHECK(ts_checksum(tgt, arr[1], 1.0, &ref));
        CHECK(ts_checksum_noalloc(tgt, arr[1], 1.0, (ts_checksum_out *)out_ptr));
        CHECK(ts_copy_to_host(&got, out_arr, 4));
        CHECK(ts_target_synchronize(tgt));
        expect(memcmp(&ref, &got, sizeof ref) == 0 && got.mismatches == n,
               "allocation-free checksum equals ts_checksum bit for bit");
        CHECK(ts_array_free(out_arr));
    }

    /* Errors come back as status codes with a message, never as crashes. */
    ts_array short_arr;
    CHECK(ts_array_alloc(tgt, TS_F64, n - 1, 0, &short_arr));
    expect(ts_copy(tgt, arr[0], short_arr) == TS_E_SHAPE && ts_last_error()[0] != '\0',
           "a short destination is TS_E_SHAPE with a message");

    CHECK(ts_array_free(short_arr));
    CHECK(ts_graph_destroy(graph));
    CHECK(ts_batch_destroy(batch));
    for (int k = 0; k < 3; ++k)
        CHECK(ts_array_free(arr[k]));
    CHECK(ts_target_destroy(tgt));
    printf("%s\n", fail_count ? "FAILED" : "all checks passed");
    return fail_count ? 1 : 0;
}
