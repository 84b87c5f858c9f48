/*
 * plain_loops.c — plain serial binary32 / int64 loops over the benchmark's
 * operations: the cost of the arithmetic alone, timed beside the oracle
 * (whose binary64 / compensated reference arithmetic costs more). Not an
 * oracle and not checked against anything: TIMING BASELINE ONLY, test
 * infrastructure like the rest of oracle/.
 *
 * Built with gcc -O2 -ffp-contract=off and without fast-math, so the
 * binary32 sums stay sequential (no reassociation, no vectorised sums).
 */
#include <stdint.h>
#include <string.h>

static float bf16(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

void plain_triad(int64_t n, const float* b, const float* c, float* a, float s) {
    for (int64_t i = 0; i < n; ++i) a[i] = b[i] + s * c[i];
}

double plain_dot_f32(int64_t n, const float* x, const float* y) {
    float acc = 0.0f;
    for (int64_t i = 0; i < n; ++i) acc += x[i] * y[i];
    return acc;
}

double plain_sumsq_f32(int64_t n, const float* x) {
    float acc = 0.0f;
    for (int64_t i = 0; i < n; ++i) acc += x[i] * x[i];
    return acc;
}

double plain_dot_bf16(int64_t n, const uint16_t* x, const uint16_t* y) {
    float acc = 0.0f;
    for (int64_t i = 0; i < n; ++i) acc += bf16(x[i]) * bf16(y[i]);
    return acc;
}

double plain_sumsq_bf16(int64_t n, const uint16_t* x) {
    float acc = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        const float v = bf16(x[i]);
        acc += v * v;
    }
    return acc;
}

void plain_scan_i32_i64(int64_t n, const int32_t* x, int64_t* y) {
    int64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) y[i] = acc += x[i];
}

void plain_scan_i32_i32(int64_t n, const int32_t* x, int32_t* y) {
    uint32_t acc = 0;
    for (int64_t i = 0; i < n; ++i) y[i] = (int32_t)(acc += (uint32_t)x[i]);
}

void plain_scan_f32(int64_t n, const float* x, float* y) {
    float acc = 0.0f;
    for (int64_t i = 0; i < n; ++i) y[i] = acc += x[i];
}

/* BATCH: m ranges of lens[k] consecutive elements each. */
void plain_scan_f32_batch(int64_t m, const int64_t* lens, const float* x, float* y, int reverse) {
    int64_t o = 0;
    for (int64_t k = 0; k < m; ++k) {
        float acc = 0.0f;
        if (reverse)
            for (int64_t i = o + lens[k] - 1; i >= o; --i) y[i] = acc += x[i];
        else
            for (int64_t i = o; i < o + lens[k]; ++i) y[i] = acc += x[i];
        o += lens[k];
    }
}

void plain_dot_f32_batch(int64_t m, const int64_t* lens, const float* x, const float* y, double* out) {
    int64_t o = 0;
    for (int64_t k = 0; k < m; ++k) {
        out[k] = plain_dot_f32(lens[k], x + o, y + o);
        o += lens[k];
    }
}

void plain_bcast_mul_batch(int64_t m, const int64_t* lens, const float* x, const float* y, const double* g,
                           float* gx, float* gy) {
    int64_t o = 0;
    for (int64_t k = 0; k < m; ++k) {
        const float gk = (float)g[k];
        for (int64_t i = o; i < o + lens[k]; ++i) {
            gx[i] = gk * y[i];
            gy[i] = gk * x[i];
        }
        o += lens[k];
    }
}
