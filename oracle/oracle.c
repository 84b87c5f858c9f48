/*
 * Plain serial CPU oracle for the segmented for_each / transform_reduce /
 * inclusive_scan path of the distributed-ranges model (Brock et al.,
 * "Distributed Ranges: A Model for Distributed Data Structures, Algorithms,
 * and Views").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do. It shares no code, header or constant with the GPU
 * library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -march=native, no
 * fast-math), so that float arithmetic is plain IEEE binary32/binary64 with
 * one rounding per operation and no fused multiply-add.
 *
 * Model. A distributed range is a list of segments; concatenated in order
 * they form the logical range (section 3, "Distributed Range"). Zipping
 * aligned ranges pairs element j of segment k of every input (section 4.4,
 * "Zip", aligned case), and a transform view applies an element-wise
 * function on the fly (section 4.4, "Transform"; Algorithm 1 builds the dot
 * product from zip, transform(l * r) and reduce). In this oracle a segment k
 * is given by one pointer per zipped input and a length n_k, and the view
 * element is v = op(x0, x1).
 *
 * Two modes. CONCAT (mode 0): the segments are one distributed range, the
 * paper's setting; a reduction has one result and a scan carries across
 * segment boundaries. BATCH (mode 1): every segment is a range of its own;
 * one result per segment, and the scan restarts at every segment.
 *
 * Readings where the paper is silent or inconsistent:
 *  - The reduce pseudocode (Algorithm 3) accumulates into init inside a
 *    parallel loop and returns from a void function; the prose (section
 *    4.3, "reduce") says the per-segment partial results are combined after
 *    all of them are complete. Here: R = init + sum over all elements.
 *  - The inclusive_scan pseudocode (Algorithm 4) never resets its segment
 *    counter and reads partial_sums[-1] for the first segment; the prose
 *    (section 4.3, "inclusive_scan") says the offset of segment i is the
 *    scanned total of segments 0..i-1. Here: the offset of segment 0 is 0.
 *  - The paper states no accumulation type. Integer data accumulate in
 *    int64 exactly. Floating-point data are summed in binary64 with
 *    Neumaier's compensated summation of the exact element values, which is
 *    the reference the GPU results are measured against.
 *  - for_each stores op(...) in the output type, each arithmetic operation
 *    rounded once in that type and no fused multiply-add (the stream triad
 *    a = b + s*c is therefore fl(b + fl(s*c))).
 *
 * Parity pins (tests/test_oracle_pins.py): closed forms (scan of ones is
 * iota, sum of 0..N-1 is N(N-1)/2, scan of a constant), brute force over
 * all segmentations of tiny ranges, segmentation invariance of integer
 * results, batch == per-range concat, math.fsum (correctly rounded) for the
 * binary64 references, numpy float32 arithmetic for the triad, the
 * hand-worked examples in tests/golden/.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

enum { OR_I32 = 0, OR_F32 = 1, OR_BF16 = 2, OR_F64 = 3, OR_I64 = 4 };
enum { OR_IDENTITY = 0, OR_SQUARE = 1, OR_MUL = 2, OR_AXPY = 3 };
enum { OR_CONCAT = 0, OR_BATCH = 1 };

enum { OR_OK = 0, OR_EBADARG = -1 };

static int op_arity(int op)
{
    switch (op) {
    case OR_IDENTITY: return 1;
    case OR_SQUARE: return 1;
    case OR_MUL: return 2;
    case OR_AXPY: return 2;
    default: return -1;
    }
}

/* ---- element decoding ---------------------------------------------------- */

/* bfloat16 is the upper half of a binary32 pattern; decoding is exact. */
static float bf16_value(uint16_t bits)
{
    uint32_t w = ((uint32_t)bits) << 16;
    float f;
    memcpy(&f, &w, sizeof f);
    return f;
}

static double load_fp(const void* base, int64_t j, int dtype)
{
    switch (dtype) {
    case OR_F32: return (double)((const float*)base)[j];
    case OR_BF16: return (double)bf16_value(((const uint16_t*)base)[j]);
    case OR_F64: return ((const double*)base)[j];
    default: return NAN;
    }
}

static float load_f32(const void* base, int64_t j, int dtype)
{
    switch (dtype) {
    case OR_F32: return ((const float*)base)[j];
    case OR_BF16: return bf16_value(((const uint16_t*)base)[j]);
    default: return NAN;
    }
}

/* ---- view element -------------------------------------------------------- */

/*
 * v = op(x0, x1) in binary64. For FP32 and BF16 inputs the identity, the
 * square and the product are exact in binary64 (at most 48 significand
 * bits); x0 + alpha*x1 is exact too when alpha has few significand bits.
 */
static double view_fp(const void* in0, const void* in1, int64_t j, int dtype, int op, double alpha)
{
    double a = load_fp(in0, j, dtype);
    switch (op) {
    case OR_IDENTITY: return a;
    case OR_SQUARE: return a * a;
    case OR_MUL: return a * load_fp(in1, j, dtype);
    case OR_AXPY: return a + alpha * load_fp(in1, j, dtype);
    default: return NAN;
    }
}

/* Integer view element, exact in int64 for int32 inputs. */
static int64_t view_int(const void* in0, const void* in1, int64_t j, int op, int64_t alpha)
{
    int64_t a = ((const int32_t*)in0)[j];
    switch (op) {
    case OR_IDENTITY: return a;
    case OR_SQUARE: return a * a;
    case OR_MUL: return a * (int64_t)((const int32_t*)in1)[j];
    case OR_AXPY: return a + alpha * (int64_t)((const int32_t*)in1)[j];
    default: return 0;
    }
}

/* ---- Neumaier summation in binary64 ------------------------------------- */

typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum* a)
{
    if (!isfinite(a->s))
        return a->s;
    return a->s + a->c;
}

/* ---- argument checks ----------------------------------------------------- */

static int check_common(int m, const void* const* in0, const void* const* in1,
                        const int64_t* len, int op)
{
    int ar = op_arity(op);
    if (m < 0 || ar < 0 || len == 0)
        return OR_EBADARG;
    for (int k = 0; k < m; ++k) {
        if (len[k] < 0)
            return OR_EBADARG;
        if (len[k] > 0 && in0[k] == 0)
            return OR_EBADARG;
        if (ar == 2 && len[k] > 0 && (in1 == 0 || in1[k] == 0))
            return OR_EBADARG;
    }
    return OR_OK;
}

/* ---- for_each (section 4.3, "for_each") --------------------------------- */

/*
 * out_k[j] = op(in0_k[j], in1_k[j]) for every segment k and index j,
 * evaluated in the output type with one rounding per operation.
 * Input/output types: F32 or BF16 -> F32, F64 -> F64, I32 -> I32 (two's
 * complement wrap) or I64.
 */
int oracle_for_each(int m, const void* const* in0, const void* const* in1,
                    void* const* out, const int64_t* len, int in_dtype, int op,
                    double alpha, int out_dtype)
{
    int rc = check_common(m, in0, in1, len, op);
    if (rc != OR_OK)
        return rc;
    for (int k = 0; k < m; ++k) {
        const void* a = in0[k];
        const void* b = in1 ? in1[k] : 0;
        for (int64_t j = 0; j < len[k]; ++j) {
            if (out_dtype == OR_F32 && (in_dtype == OR_F32 || in_dtype == OR_BF16)) {
                float x = load_f32(a, j, in_dtype), r;
                if (op == OR_IDENTITY) {
                    r = x;
                } else if (op == OR_SQUARE) {
                    r = x * x;
                } else if (op == OR_MUL) {
                    r = x * load_f32(b, j, in_dtype);
                } else {
                    float t = (float)alpha * load_f32(b, j, in_dtype);
                    r = x + t;
                }
                ((float*)out[k])[j] = r;
            } else if (out_dtype == OR_F64 && in_dtype == OR_F64) {
                double x = ((const double*)a)[j], r;
                if (op == OR_IDENTITY) {
                    r = x;
                } else if (op == OR_SQUARE) {
                    r = x * x;
                } else if (op == OR_MUL) {
                    r = x * ((const double*)b)[j];
                } else {
                    double t = alpha * ((const double*)b)[j];
                    r = x + t;
                }
                ((double*)out[k])[j] = r;
            } else if (in_dtype == OR_I32 && (out_dtype == OR_I32 || out_dtype == OR_I64)) {
                int64_t v = view_int(a, b, j, op, (int64_t)alpha);
                if (out_dtype == OR_I64)
                    ((int64_t*)out[k])[j] = v;
                else
                    ((int32_t*)out[k])[j] = (int32_t)(uint32_t)(uint64_t)v;
            } else {
                return OR_EBADARG;
            }
        }
    }
    return OR_OK;
}

/* ---- transform_reduce (section 4.3, "reduce"; Algorithms 1 and 3) ------- */

/*
 * Integer inputs (I32): result_i64[r] = init + sum of v, exact in int64.
 * Floating inputs: result_f64[r] = init + sum of v, Neumaier in binary64;
 * abs_sum[r] (optional) = init magnitude excluded, sum of |v|, for the
 * condition number sum|v| / |sum v|.
 * CONCAT: one result. BATCH: one result per segment.
 */
int oracle_reduce(int m, const void* const* in0, const void* const* in1,
                  const int64_t* len, int in_dtype, int op, double alpha, int mode,
                  int64_t init_i, double init_f, int64_t* result_i64,
                  double* result_f64, double* abs_sum)
{
    int rc = check_common(m, in0, in1, len, op);
    if (rc != OR_OK || (mode != OR_CONCAT && mode != OR_BATCH))
        return OR_EBADARG;
    if (in_dtype == OR_I32) {
        if (result_i64 == 0)
            return OR_EBADARG;
        int64_t acc = init_i;
        for (int k = 0; k < m; ++k) {
            if (mode == OR_BATCH)
                acc = init_i;
            for (int64_t j = 0; j < len[k]; ++j)
                acc += view_int(in0[k], in1 ? in1[k] : 0, j, op, (int64_t)alpha);
            if (mode == OR_BATCH)
                result_i64[k] = acc;
        }
        if (mode == OR_CONCAT)
            result_i64[0] = acc;
        return OR_OK;
    }
    if (in_dtype != OR_F32 && in_dtype != OR_BF16 && in_dtype != OR_F64)
        return OR_EBADARG;
    if (result_f64 == 0)
        return OR_EBADARG;
    nsum acc = { init_f, 0.0 };
    nsum mag = { 0.0, 0.0 };
    for (int k = 0; k < m; ++k) {
        if (mode == OR_BATCH) {
            acc.s = init_f;
            acc.c = 0.0;
            mag.s = 0.0;
            mag.c = 0.0;
        }
        for (int64_t j = 0; j < len[k]; ++j) {
            double v = view_fp(in0[k], in1 ? in1[k] : 0, j, in_dtype, op, alpha);
            nsum_add(&acc, v);
            nsum_add(&mag, fabs(v));
        }
        if (mode == OR_BATCH) {
            result_f64[k] = nsum_value(&acc);
            if (abs_sum)
                abs_sum[k] = nsum_value(&mag);
        }
    }
    if (mode == OR_CONCAT) {
        result_f64[0] = nsum_value(&acc);
        if (abs_sum)
            abs_sum[0] = nsum_value(&mag);
    }
    return OR_OK;
}

/* ---- inclusive_scan (section 4.3, "inclusive_scan"; Algorithm 4) -------- */

/*
 * out_k[j] = sum of v over every element at or before (k, j) in the
 * logical range (forward), or at or after it (reverse = 1). CONCAT carries
 * across segments (segment k starts from the total of segments before it,
 * 0 for the first); BATCH restarts at every segment.
 *
 * I32 input: out is int64 (out_dtype I64) or int32 holding the int64 value
 * modulo 2^32 (out_dtype I32). Floating input: out is the binary64
 * reference (Neumaier running sum), and abs_prefix (optional, same shape)
 * receives the running sum of |v| in the same direction, the scale of the
 * rounding error a scan can make at that position.
 */
int oracle_scan(int m, const void* const* in0, const void* const* in1,
                void* const* out, double* const* abs_prefix, const int64_t* len,
                int in_dtype, int op, double alpha, int mode, int reverse, int out_dtype)
{
    int rc = check_common(m, in0, in1, len, op);
    if (rc != OR_OK || (mode != OR_CONCAT && mode != OR_BATCH))
        return OR_EBADARG;
    int is_int = (in_dtype == OR_I32);
    if (is_int && out_dtype != OR_I64 && out_dtype != OR_I32)
        return OR_EBADARG;
    if (!is_int && (in_dtype != OR_F32 && in_dtype != OR_BF16 && in_dtype != OR_F64))
        return OR_EBADARG;
    if (!is_int && out_dtype != OR_F64)
        return OR_EBADARG;

    int64_t iacc = 0;
    nsum facc = { 0.0, 0.0 };
    nsum mag = { 0.0, 0.0 };
    for (int kk = 0; kk < m; ++kk) {
        int k = reverse ? (m - 1 - kk) : kk;
        if (mode == OR_BATCH) {
            iacc = 0;
            facc.s = facc.c = 0.0;
            mag.s = mag.c = 0.0;
        }
        for (int64_t jj = 0; jj < len[k]; ++jj) {
            int64_t j = reverse ? (len[k] - 1 - jj) : jj;
            const void* b = in1 ? in1[k] : 0;
            if (is_int) {
                iacc += view_int(in0[k], b, j, op, (int64_t)alpha);
                if (out_dtype == OR_I64)
                    ((int64_t*)out[k])[j] = iacc;
                else
                    ((int32_t*)out[k])[j] = (int32_t)(uint32_t)(uint64_t)iacc;
            } else {
                double v = view_fp(in0[k], b, j, in_dtype, op, alpha);
                nsum_add(&facc, v);
                nsum_add(&mag, fabs(v));
                ((double*)out[k])[j] = nsum_value(&facc);
                if (abs_prefix)
                    abs_prefix[k][j] = nsum_value(&mag);
            }
        }
    }
    return OR_OK;
}

/* ---- adjoints ------------------------------------------------------------ */

/*
 * Adjoint of a transform_reduce with respect to one input: for every
 * element, grad[j] = g_r * d v / d x_which, where g_r is the upstream
 * gradient of the segment's result r (g[0] for CONCAT, g[k] for BATCH).
 * d(x0*x1)/dx0 = x1, d(x0*x1)/dx1 = x0, d(x0^2)/dx0 = 2*x0,
 * d(x0)/dx0 = 1, d(x0 + alpha*x1)/dx1 = alpha. Output binary64.
 */
int oracle_reduce_grad(int m, const void* const* in0, const void* const* in1,
                       double* const* grad, const int64_t* len, int in_dtype, int op,
                       double alpha, int mode, const double* g, int which)
{
    int rc = check_common(m, in0, in1, len, op);
    if (rc != OR_OK || in_dtype == OR_I32 || which < 0 || which >= op_arity(op))
        return OR_EBADARG;
    for (int k = 0; k < m; ++k) {
        double gk = (mode == OR_BATCH) ? g[k] : g[0];
        for (int64_t j = 0; j < len[k]; ++j) {
            double d;
            if (op == OR_IDENTITY)
                d = 1.0;
            else if (op == OR_SQUARE)
                d = 2.0 * load_fp(in0[k], j, in_dtype);
            else if (op == OR_MUL)
                d = load_fp(which == 0 ? in1[k] : in0[k], j, in_dtype);
            else
                d = (which == 0) ? 1.0 : alpha;
            grad[k][j] = gk * d;
        }
    }
    return OR_OK;
}

/* ---- generic reduce and scan (section 4.3) -------------------------------- */

/*
 * The paper's reduce and scan take any commutative binary operator (the
 * footnote to section 4.3, "reduce"; its listings show +), reduce takes an
 * initial value (Algorithm 3), and exclusive_scan is built like
 * inclusive_scan (end of section 4.3, "inclusive_scan"). combine: 0 = sum,
 * 1 = max, 2 = min.
 *
 * Readings:
 *  - sum: as oracle_reduce / oracle_scan (exact view values, Neumaier
 *    binary64), started from init instead of 0.
 *  - max / min compare the view values as for_each would store them
 *    (binary32 arithmetic with one rounding per operation for F32 and BF16
 *    inputs, binary64 for F64, exact int64 for I32). Rounding is monotone,
 *    so this is also the rounding of the exact maximum for identity, square
 *    and mul views. NaN values are ignored (fmax / fmin) unless all are NaN.
 *  - Without an initial value the identity of the operator is used:
 *    0, -inf / INT64_MIN (max), +inf / INT64_MAX (min).
 *  - exclusive: element i receives init combined with the elements strictly
 *    before it (after it, in reverse); the first receives init.
 */
enum { OR_SUM = 0, OR_MAX = 1, OR_MIN = 2 };

static double view_stored_fp(const void* in0, const void* in1, int64_t j, int dtype, int op, double alpha)
{
    if (dtype == OR_F64) {
        double x = ((const double*)in0)[j];
        switch (op) {
        case OR_IDENTITY: return x;
        case OR_SQUARE: return x * x;
        case OR_MUL: return x * ((const double*)in1)[j];
        default: { double t = alpha * ((const double*)in1)[j]; return x + t; }
        }
    }
    float x = load_f32(in0, j, dtype);
    switch (op) {
    case OR_IDENTITY: return x;
    case OR_SQUARE: { float r = x * x; return r; }
    case OR_MUL: { float r = x * load_f32(in1, j, dtype); return r; }
    default: { float t = (float)alpha * load_f32(in1, j, dtype); float r = x + t; return r; }
    }
}

static double comb_fp(int combine, double a, double b)
{
    return combine == OR_MAX ? fmax(a, b) : fmin(a, b);
}

static int64_t comb_int(int combine, int64_t a, int64_t b)
{
    if (combine == OR_MAX)
        return a > b ? a : b;
    return a < b ? a : b;
}

/*
 * Results as oracle_reduce (int64 for I32 inputs, binary64 otherwise), with
 * the operator `combine` and, when has_init is 0, its identity as init.
 */
int oracle_reduce_ex(int m, const void* const* in0, const void* const* in1,
                     const int64_t* len, int in_dtype, int op, double alpha, int mode,
                     int combine, int has_init, int64_t init_i, double init_f,
                     int64_t* result_i64, double* result_f64)
{
    if (combine == OR_SUM)
        return oracle_reduce(m, in0, in1, len, in_dtype, op, alpha, mode,
                             has_init ? init_i : 0, has_init ? init_f : 0.0,
                             result_i64, result_f64, 0);
    int rc = check_common(m, in0, in1, len, op);
    if (rc != OR_OK || (mode != OR_CONCAT && mode != OR_BATCH) || (combine != OR_MAX && combine != OR_MIN))
        return OR_EBADARG;
    int is_int = (in_dtype == OR_I32);
    if ((is_int && result_i64 == 0) || (!is_int && result_f64 == 0))
        return OR_EBADARG;
    if (!is_int && in_dtype != OR_F32 && in_dtype != OR_BF16 && in_dtype != OR_F64)
        return OR_EBADARG;
    int64_t i0 = has_init ? init_i : (combine == OR_MAX ? INT64_MIN : INT64_MAX);
    double f0 = has_init ? init_f : (combine == OR_MAX ? -INFINITY : INFINITY);
    int64_t ia = i0;
    double fa = f0;
    for (int k = 0; k < m; ++k) {
        if (mode == OR_BATCH) {
            ia = i0;
            fa = f0;
        }
        const void* b = in1 ? in1[k] : 0;
        for (int64_t j = 0; j < len[k]; ++j) {
            if (is_int)
                ia = comb_int(combine, ia, view_int(in0[k], b, j, op, (int64_t)alpha));
            else
                fa = comb_fp(combine, fa, view_stored_fp(in0[k], b, j, in_dtype, op, alpha));
        }
        if (mode == OR_BATCH) {
            if (is_int)
                result_i64[k] = ia;
            else
                result_f64[k] = fa;
        }
    }
    if (mode == OR_CONCAT) {
        if (is_int)
            result_i64[0] = ia;
        else
            result_f64[0] = fa;
    }
    return OR_OK;
}

/*
 * Outputs as oracle_scan (I32 input: int64 or int32-wrapped; floating
 * input: binary64), with the operator `combine`, an optional initial value,
 * and exclusive = 1 for the exclusive scan. abs_prefix (sum only, optional)
 * receives the running sum of |v| including |init|, the scale of the
 * rounding error.
 */
int oracle_scan_ex(int m, const void* const* in0, const void* const* in1,
                   void* const* out, double* const* abs_prefix, const int64_t* len,
                   int in_dtype, int op, double alpha, int mode, int reverse, int out_dtype,
                   int combine, int exclusive, int has_init, int64_t init_i, double init_f)
{
    int rc = check_common(m, in0, in1, len, op);
    if (rc != OR_OK || (mode != OR_CONCAT && mode != OR_BATCH))
        return OR_EBADARG;
    if (combine != OR_SUM && combine != OR_MAX && combine != OR_MIN)
        return OR_EBADARG;
    int is_int = (in_dtype == OR_I32);
    if (is_int && out_dtype != OR_I64 && out_dtype != OR_I32)
        return OR_EBADARG;
    if (!is_int && (in_dtype != OR_F32 && in_dtype != OR_BF16 && in_dtype != OR_F64))
        return OR_EBADARG;
    if (!is_int && out_dtype != OR_F64)
        return OR_EBADARG;
    if (combine != OR_SUM && abs_prefix)
        return OR_EBADARG;
    int64_t i0 = has_init ? init_i : (combine == OR_SUM ? 0 : combine == OR_MAX ? INT64_MIN : INT64_MAX);
    double f0 = has_init ? init_f : (combine == OR_SUM ? 0.0 : combine == OR_MAX ? -INFINITY : INFINITY);

    int64_t iacc = i0;
    double facc_m = f0;                 /* max / min */
    nsum facc = { f0, 0.0 };            /* sum */
    nsum mag = { fabs(f0), 0.0 };
    for (int kk = 0; kk < m; ++kk) {
        int k = reverse ? (m - 1 - kk) : kk;
        if (mode == OR_BATCH) {
            iacc = i0;
            facc_m = f0;
            facc.s = f0;
            facc.c = 0.0;
            mag.s = fabs(f0);
            mag.c = 0.0;
        }
        const void* b = in1 ? in1[k] : 0;
        for (int64_t jj = 0; jj < len[k]; ++jj) {
            int64_t j = reverse ? (len[k] - 1 - jj) : jj;
            if (is_int) {
                int64_t before = iacc;
                int64_t v = view_int(in0[k], b, j, op, (int64_t)alpha);
                iacc = combine == OR_SUM ? iacc + v : comb_int(combine, iacc, v);
                int64_t y = exclusive ? before : iacc;
                if (out_dtype == OR_I64)
                    ((int64_t*)out[k])[j] = y;
                else
                    ((int32_t*)out[k])[j] = (int32_t)(uint32_t)(uint64_t)y;
            } else if (combine == OR_SUM) {
                double before = nsum_value(&facc), mbefore = nsum_value(&mag);
                double v = view_fp(in0[k], b, j, in_dtype, op, alpha);
                nsum_add(&facc, v);
                nsum_add(&mag, fabs(v));
                ((double*)out[k])[j] = exclusive ? before : nsum_value(&facc);
                if (abs_prefix)
                    abs_prefix[k][j] = exclusive ? mbefore : nsum_value(&mag);
            } else {
                double before = facc_m;
                facc_m = comb_fp(combine, facc_m, view_stored_fp(in0[k], b, j, in_dtype, op, alpha));
                ((double*)out[k])[j] = exclusive ? before : facc_m;
            }
        }
    }
    return OR_OK;
}

/* ---- Black-Scholes for_each (section 5, "Black Scholes") ----------------- */

/*
 * The paper's Black Scholes benchmark is a for_each over a zip of option
 * arrays that prices European options. The price is the standard closed-form
 * solution of the Black-Scholes equation: for spot S, strike K, time to
 * expiry T (years), volatility sigma and risk-free rate r,
 *   d1 = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt(T)),   d2 = d1 - sigma sqrt(T),
 *   call = S N(d1) - K exp(-rT) N(d2),   put = K exp(-rT) N(-d2) - S N(-d1),
 * N the standard normal distribution function, N(x) = erfc(-x / sqrt(2)) / 2.
 * Inputs are the stored binary32 values; the prices are evaluated in
 * binary64 with the C library's log, sqrt, exp and erfc.
 */
int oracle_black_scholes(int m, const float* const* S, const float* const* K, const float* const* T,
                         const float* const* V, double* const* call, double* const* put,
                         const int64_t* len, double r)
{
    if (m < 0 || len == 0)
        return OR_EBADARG;
    const double rs2 = 0.70710678118654752440;   /* 1 / sqrt(2) */
    for (int k = 0; k < m; ++k) {
        if (len[k] < 0)
            return OR_EBADARG;
        if (len[k] > 0 && (!S[k] || !K[k] || !T[k] || !V[k] || !call[k] || !put[k]))
            return OR_EBADARG;
        for (int64_t j = 0; j < len[k]; ++j) {
            double s = S[k][j], x = K[k][j], t = T[k][j], v = V[k][j];
            double vst = v * sqrt(t);
            double d1 = (log(s / x) + (r + 0.5 * v * v) * t) / vst;
            double d2 = d1 - vst;
            double disc = exp(-r * t);
            call[k][j] = s * 0.5 * erfc(-d1 * rs2) - x * disc * 0.5 * erfc(-d2 * rs2);
            put[k][j] = x * disc * 0.5 * erfc(d2 * rs2) - s * 0.5 * erfc(d1 * rs2);
        }
    }
    return OR_OK;
}

int oracle_abi_version(void) { return 1; }
