/* Quad-precision etalon for the accuracy acceptance of the twofold functions
 * -- TEST INFRASTRUCTURE ONLY (loaded by tests/ through oracle/qref.py).
 *
 * The paper measures the twofold functions on about a million random
 * arguments against quad precision for the double version (section
 * "Analysis > Accuracy"); this file is that etalon, here for both formats.
 * It uses binary128 (__float128, libquadmath: 113-bit significand) and shares
 * nothing with the oracle or the GPU library.
 *
 * The exact argument is the real sum x0 + x1.  Its quad rounding would perturb
 * exp near |x| = 745 by up to 2^-103.5 of the result, so each function is split
 * into a part of x0 alone and a correction from x1, both exact identities:
 *   exp(x0 + x1)   = e + e*expm1(x1),           e = exp(x0)
 *   expm1(x0 + x1) = m + (m + 1)*expm1(x1),     m = expm1(x0)
 *   log(x0 + x1)   = log(x0) + log1p(x1/x0)
 *   log1p(x0 + x1) = log1p(x0) + log1p(x1/(1 + x0))
 * The corrections are at most about 2^-52 of the result, so the rounding of
 * their own arguments costs nothing visible; every term is computed to about
 * one quad ulp (2^-112 relative).
 *
 * qref_check(fn, fmt, x0, x1, z0, z1, n, l0, rel, cls, threads) measures, per
 * element, the relative error |z0 + z1 - f| / |f| of a result pair against
 * f = fn(x0 + x1):
 *   fn  0 exp, 1 expm1, 2 log, 3 log1p;  fmt 0 binary64 arrays, 1 binary32
 *   rel[i]  the relative error, rounded to double (0 when f = 0 and z0 + z1 = 0)
 *   cls[i]  0: measured (rel[i] holds it)
 *           1: result in the subnormal-second-part range (|f| below 2^-969,
 *              binary32 2^-102) and |z0 + z1 - f| <= l0*|f| + one subnormal ulp
 *           2: such a result that fails that bar
 *           3: not measured: x0 + x1 not finite, outside the function's domain,
 *              f beyond the format's largest finite value, or z0 not finite
 * qref_quad(fn, x, out, n) and qref_libm(fn, x, out, n) call one libquadmath
 * function (expq, expm1q, logq, log1pq) or one C library function (exp, expm1,
 * log, log1p) per element, for the benchmark's context timing of the paper's
 * comparison of twofold functions with quad precision (section "Analysis >
 * Performance").
 * qref_eval(fn, x0, x1, out, ex, n) returns f(x0 + x1) (binary64 x0, x1) as
 * (out[3i] + out[3i+1] + out[3i+2])*2^ex[i], the quad significand m = f*2^-ex
 * in [1/2, 1) cut into three doubles (exactly: 113 bits fit in three), for
 * pinning this etalon itself at any magnitude.
 */
#include <math.h>
#include <quadmath.h>
#include <stddef.h>
#include <stdint.h>

typedef __float128 q;

/* f(x0 + x1), or NaN outside the domain (as a NaN quad). */
static q ref(int fn, q x0, q x1)
{
    switch (fn) {
    case 0: {
        q e = expq(x0);
        return e + e * expm1q(x1);
    }
    case 1: {
        q m = expm1q(x0);
        return m + (m + 1) * expm1q(x1);
    }
    case 2:
        if (x0 + x1 <= 0 || !(x0 > 0)) return nanq("");
        return logq(x0) + log1pq(x1 / x0);
    default: {
        q u = 1 + x0;
        if (u + x1 <= 0 || !(u > 0)) return nanq("");
        return log1pq(x0) + log1pq(x1 / u);
    }
    }
}

static int finiteq_(q v) { return !isnanq(v) && !isinfq(v); }

static void one(int fn, int fmt, q x0, q x1, q z0, q z1, double l0, double* rel, int8_t* cls)
{
    const q big = fmt ? (q)3.4028234663852886e38 : (q)1.7976931348623157e308;
    const q subnormal_f = fmt ? ldexpq(1, -102) : ldexpq(1, -969);
    const q tiny = fmt ? ldexpq(1, -149) : ldexpq(1, -1074);
    *rel = 0;
    *cls = 3;
    if (!finiteq_(x0) || !finiteq_(x1) || !finiteq_(z0)) return;
    q f = ref(fn, x0, x1);
    if (!finiteq_(f) || fabsq(f) > big) return;
    if (!finiteq_(z1)) {            /* a finite f with a non-finite second part */
        *rel = INFINITY;
        *cls = 0;
        return;
    }
    q err = fabsq((z0 + z1) - f);
    if (f != 0 && fabsq(f) < subnormal_f) {
        *cls = err <= (q)l0 * fabsq(f) + tiny ? 1 : 2;
        return;
    }
    *cls = 0;
    if (f == 0)
        *rel = err == 0 ? 0.0 : INFINITY;
    else
        *rel = (double)(err / fabsq(f));
}

void qref_check(int fn, int fmt, const void* x0, const void* x1, const void* z0,
                const void* z1, size_t n, double l0, double* rel, int8_t* cls, int threads)
{
    long long i, m = (long long)n;
    if (fmt == 0) {
        const double *a = (const double*)x0, *b = (const double*)x1;
        const double *c = (const double*)z0, *d = (const double*)z1;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(threads)
        for (i = 0; i < m; i++) one(fn, 0, a[i], b[i], c[i], d[i], l0, rel + i, cls + i);
    } else {
        const float *a = (const float*)x0, *b = (const float*)x1;
        const float *c = (const float*)z0, *d = (const float*)z1;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(threads)
        for (i = 0; i < m; i++) one(fn, 1, a[i], b[i], c[i], d[i], l0, rel + i, cls + i);
    }
}

void qref_quad(int fn, const double* x, double* out, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        q v = x[i], r;
        switch (fn) {
        case 0: r = expq(v); break;
        case 1: r = expm1q(v); break;
        case 2: r = logq(v); break;
        default: r = log1pq(v); break;
        }
        out[i] = (double)r;
    }
}

void qref_libm(int fn, const double* x, double* out, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        double v = x[i];
        switch (fn) {
        case 0: out[i] = exp(v); break;
        case 1: out[i] = expm1(v); break;
        case 2: out[i] = log(v); break;
        default: out[i] = log1p(v); break;
        }
    }
}

void qref_eval(int fn, const double* x0, const double* x1, double* out, int* ex, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        q f = ref(fn, x0[i], x1[i]);
        int e = 0;
        q m = finiteq_(f) ? frexpq(f, &e) : f;
        for (int k = 0; k < 3; k++) {
            out[3 * i + k] = (double)m;
            m = finiteq_(m) ? m - (q)out[3 * i + k] : 0;
        }
        ex[i] = e;
    }
}
