/* Sanitizer driver for the CPU oracle (built with gcc -fsanitize=... by
 * tests/test_sanitizers.py; test infrastructure only).  Every oracle entry
 * point runs on random values of every storage type, then the threaded
 * timed mode runs with several workers. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t state = 0x9e3779b97f4a7c15ull;

static uint64_t next(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

int main(int argc, char **argv)
{
    const size_t n = argc > 1 ? (size_t)strtoull(argv[1], NULL, 10) : 100003;
    const int threads = argc > 2 ? atoi(argv[2]) : 4;
    for (int dt = 0; dt < 4; ++dt) {
        const size_t es = dt == 0 ? 8 : dt == 1 ? 4 : 2;
        unsigned char *buf[3];
        for (int k = 0; k < 3; ++k) {
            buf[k] = malloc(n * es);
            if (!buf[k])
                return 2;
            for (size_t j = 0; j < n * es; ++j)
                buf[k][j] = (unsigned char)next();
        }
        for (int op = 0; op < 4; ++op)
            if (oracle_op(dt, op, buf[0], buf[1], buf[2], n, 3.0))
                return 1;
        if (oracle_stream_run(dt, buf[0], buf[1], buf[2], n, 3.0, 3))
            return 1;
        oracle_checksum cs;
        uint64_t m;
        if (oracle_checksum_array(dt, buf[0], n, 1.0, &cs) || oracle_mismatch_count(dt, buf[0], buf[1], n, &m))
            return 1;
        for (int k = 0; k < 3; ++k)
            free(buf[k]);
    }
    double secs[4 * 4], fin[6];
    int used = 0;
    if (oracle_stream_timed_f64(1u << 18, 4, threads, 3.0, secs, fin, &used) || used != threads)
        return 1;
    printf("oracle ok: a = %g after the timed run\n", fin[0]);
    return 0;
}
