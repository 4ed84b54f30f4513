/*
 * fzo_sanitize.c -- drives the oracle (oracle/fzo.c) under AddressSanitizer
 * and UndefinedBehaviorSanitizer: compress / decompress round trips over
 * ragged shapes of every rank, every bound mode, fp64 input, the
 * field-global predictor, escapes up to and past the per-chunk cap, the
 * error statuses, and decompression of truncated and corrupted streams
 * (which must be rejected or decoded without any out-of-bounds access).
 * Test infrastructure: built and run by tests/test_oracle_sanitize.py.
 * Prints one line per failed check and exits nonzero if any failed.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fzo.h"

static int failures = 0;
#define CHECK(cond, ...)                       \
    do {                                       \
        if (!(cond)) {                         \
            printf("FAIL %s:%d ", __FILE__, __LINE__); \
            printf(__VA_ARGS__);               \
            printf("\n");                      \
            failures++;                        \
        }                                      \
    } while (0)

static uint64_t lcg = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(lcg >> 33);
}
static double urand(void) { return (rnd() + 0.5) / 2147483648.0; }

static int64_t numel(int rank, const int64_t *d)
{
    int64_t n = 1;
    for (int i = 0; i < rank; i++) n *= d[i];
    return n;
}

/* a smooth field with a little noise; `offset` shifts it (forces escapes) */
static void fill(float *x, int rank, const int64_t *d, float offset)
{
    int64_t n = numel(rank, d);
    double a = urand() * 0.3 + 0.05, b = urand() * 0.2 + 0.03, c = urand() * 6.0;
    for (int64_t i = 0; i < n; i++)
        x[i] = (float)(sin(a * (double)(i % 997) + c) + cos(b * (double)(i / 37)) + 1e-3 * (urand() - 0.5)) + offset;
}

static void roundtrip(int rank, const int64_t *d, double eb, int mode, int global, int threads, float offset)
{
    int64_t n = numel(rank, d);
    float *x = malloc((size_t)n * sizeof(float)), *y = malloc((size_t)n * sizeof(float));
    fill(x, rank, d, offset);
    int64_t cap = fzo_bound(rank, d);
    uint8_t *s = malloc((size_t)cap);
    uint32_t st = 99;
    int64_t len = fzo_compress_pred(x, rank, d, eb, mode, global, s, cap, &st, threads);
    CHECK(len > 0, "compress rank %d mode %d global %d -> %lld", rank, mode, global, (long long)len);
    if (len > 0 && st == 0) {
        int err = fzo_decompress(s, len, y, rank, d);
        CHECK(err == 0, "decompress rank %d mode %d -> %d", rank, mode, err);
        float *y4 = malloc((size_t)n * sizeof(float));
        CHECK(fzo_decompress_threads(s, len, y4, rank, d, 4) == 0 && memcmp(y, y4, (size_t)n * sizeof(float)) == 0,
              "threaded decompress rank %d mode %d", rank, mode);
        free(y4);
        float ebx2, inv;
        memcpy(&ebx2, s + 48, 4);
        memcpy(&inv, s + 52, 4);
        for (int64_t i = 0; i < n && err == 0; i++) {
            double e = fabs((double)x[i] - (double)y[i]);
            double lim = mode == FZO_EB_PWREL ? eb * fmax(fabs((double)x[i]), 1.1754943508222875e-38)
                                               : 0.5 * ebx2 + fabs((double)x[i]) * 1.2e-7 + 1e-30;
            if (!(e <= lim)) {
                CHECK(0, "bound rank %d mode %d at %lld: %g > %g", rank, mode, (long long)i, e, lim);
                break;
            }
        }
        /* the same stream cut short, and with bytes changed, must not be
         * read out of bounds */
        for (int64_t cut = 0; cut < len; cut += 1 + len / 13) (void)fzo_decompress(s, cut, y, rank, d);
        uint8_t *t = malloc((size_t)len);
        for (int k = 0; k < 60; k++) {
            memcpy(t, s, (size_t)len);
            int flips = 1 + (int)(rnd() % 4);
            for (int f = 0; f < flips; f++) t[rnd() % (uint32_t)len] ^= (uint8_t)(1u << (rnd() % 8));
            (void)fzo_decompress(t, len, y, rank, d);
            (void)fzo_decompress_threads(t, len, y, rank, d, 3);
        }
        free(t);
    }
    free(x); free(y); free(s);
}

static void roundtrip_f64(int rank, const int64_t *d, double eb, int mode)
{
    int64_t n = numel(rank, d);
    double *x = malloc((size_t)n * sizeof(double)), *y = malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; i++) x[i] = sin(0.013 * (double)i) * 1.000000123 + 1e-9 * (double)(i % 7);
    int64_t cap = fzo_bound(rank, d);
    uint8_t *s = malloc((size_t)cap);
    uint32_t st = 99;
    int64_t len = fzo_compress_f64(x, rank, d, eb, mode, s, cap, &st, 1);
    CHECK(len > 0 && st == 0, "f64 compress rank %d -> %lld status %u", rank, (long long)len, st);
    if (len > 0 && st == 0) {
        CHECK(fzo_decompress_f64(s, len, y, rank, d) == 0, "f64 decompress rank %d", rank);
        float yf[4];
        CHECK(fzo_decompress(s, len, yf, 1, (const int64_t[]){4}) != 0, "fp64 stream read as fp32");
        for (int64_t cut = 0; cut < len; cut += 1 + len / 7) (void)fzo_decompress_f64(s, cut, y, rank, d);
    }
    free(x); free(y); free(s);
}

/* 1-D chunk of zeros with spikes of 100000 at even positions from `lo`,
 * `gap` apart: two escapes per spike under eb 0.5 */
static void spikes(int count, int lo, int gap, int extra_step, uint32_t expect_status)
{
    int64_t d[1] = {32768};
    float *x = calloc(32768, sizeof(float)), *y = malloc(32768 * sizeof(float));
    for (int i = 0; i < count; i++) x[lo + gap * i] = 100000.0f;
    if (extra_step)
        for (int i = extra_step; i < 32768; i++) x[i] = 100000.0f;
    int64_t cap = fzo_bound(1, d);
    uint8_t *s = malloc((size_t)cap);
    uint32_t st = 99;
    int64_t len = fzo_compress(x, 1, d, 0.5, FZO_EB_ABS, s, cap, &st, 1);
    CHECK(len > 0 && st == expect_status, "spikes %d: status %u, expected %u", count, st, expect_status);
    if (len > 0 && st == 0) {
        CHECK(fzo_decompress(s, len, y, 1, d) == 0, "spikes %d decompress", count);
        CHECK(memcmp(x, y, 32768 * sizeof(float)) == 0, "spikes %d reconstruction", count);
    }
    free(x); free(y); free(s);
}

int main(void)
{
    static const int64_t shapes[][4] = {
        {1, 1, 0, 0}, {1, 70001, 0, 0}, {1, 32768, 0, 0}, {2, 33, 1100, 0}, {2, 1, 1, 0},
        {2, 65, 2049, 0}, {3, 17, 33, 65}, {3, 1, 1, 1}, {3, 20, 64, 130}, {3, 5, 3, 2},
    };
    for (size_t k = 0; k < sizeof(shapes) / sizeof(shapes[0]); k++) {
        int rank = (int)shapes[k][0];
        const int64_t *d = &shapes[k][1];
        roundtrip(rank, d, 1e-3, FZO_EB_REL, 0, 1, 0.0f);
        roundtrip(rank, d, 1e-4, FZO_EB_REL, 0, 4, 0.0f);
        roundtrip(rank, d, 1e-3, FZO_EB_ABS, 0, 1, 1000.0f); /* offset: escapes at chunk origins */
        roundtrip(rank, d, 1e-2, FZO_EB_PWREL, 0, 1, 0.0f);
        roundtrip(rank, d, 1e-3, FZO_EB_REL, 1, 1, 0.0f);
        roundtrip_f64(rank, d, 1e-3, FZO_EB_REL);
    }
    spikes(150, 2, 50, 0, 0);                      /* 300 escapes in layer 0 */
    spikes(512, 16386, 16, 0, 0);                  /* 1024 in layer 2 */
    spikes(512, 16386, 16, 30000, FZO_ERR_OUTLIER_CAP); /* 1025: the chunk cap */

    /* statuses */
    {
        int64_t d[3] = {10, 10, 10};
        float x[1000];
        int64_t cap = fzo_bound(3, d);
        uint8_t *s = malloc((size_t)cap);
        uint32_t st = 0;
        for (int i = 0; i < 1000; i++) x[i] = (float)i;
        x[345] = NAN;
        CHECK(fzo_compress(x, 3, d, 1e-3, FZO_EB_REL, s, cap, &st, 1) > 0 && st == FZO_ERR_NONFINITE, "NaN status %u", st);
        x[345] = 1e30f;
        CHECK(fzo_compress(x, 3, d, 1e-10, FZO_EB_ABS, s, cap, &st, 1) > 0 && st == FZO_ERR_EB_RANGE, "range status %u", st);
        CHECK(fzo_compress(x, 3, d, -1.0, FZO_EB_ABS, s, cap, &st, 1) < 0, "negative bound accepted");
        CHECK(fzo_compress(x, 3, d, 1e-3, 7, s, cap, &st, 1) < 0, "unknown mode accepted");
        CHECK(fzo_compress(x, 3, d, 1e-3, FZO_EB_REL, s, 10, &st, 1) < 0, "short output accepted");
        free(s);
    }
    printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
