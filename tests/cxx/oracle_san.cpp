// Sanitizer driver of the CPU oracle (test infrastructure): built together
// with oracle/tfo.cpp and the binary128 etalon oracle/qref.c under
// AddressSanitizer and UndefinedBehaviorSanitizer, host code only
// (tests/test_oracle_sanitized.py).  It calls every function the two export
// (scalar, array with two OpenMP threads, and operation-counting builds) on
// random bit patterns of every class (NaN, signed infinities and zeros,
// subnormals, huge and tiny normals) and on the arguments the functions are
// meant for.  Any sanitizer report aborts the program; on success it prints
// "SANITIZED OK" and the number of element evaluations.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

extern "C" {
#define DECL_TW(NAME, T)                                                                    \
    T tfo_##NAME(T, T, T*);                                                                 \
    void tfo_##NAME##_n(const T*, const T*, T*, T*, size_t, int);                           \
    void tfo_count_##NAME##_n(const T*, const T*, size_t, unsigned long long*);
#define DECL_D(NAME, T)                                                                     \
    T tfo_##NAME(T, T*);                                                                    \
    void tfo_##NAME##_n(const T*, T*, T*, size_t, int);                                     \
    void tfo_count_##NAME##_n(const T*, size_t, unsigned long long*);
#define DECL_1X(NAME, T)                                                                    \
    T tfo_##NAME(T);                                                                        \
    void tfo_##NAME##_n(const T*, T*, size_t, int);
#define DECL_BWD(NAME, T)                                                                   \
    void tfo_##NAME##_n(const T*, const T*, const T*, const T*, T*, T*, size_t, int);      \
    void tfo_count_##NAME##_n(const T*, const T*, const T*, const T*, size_t,               \
                              unsigned long long*);
#define EACH_TW(X)                                                                          \
    X(texp, double) X(texpm1, double) X(tlog, double) X(tlog1p, double)                     \
    X(texpf, float) X(texpm1f, float) X(tlogf, float) X(tlog1pf, float)                     \
    X(texpp, double) X(pexp, double) X(texpm1p, double) X(pexpm1, double)                  \
    X(tlogp, double) X(plog, double) X(tlog1pp, double) X(plog1p, double)                  \
    X(texppf, float) X(pexpf, float) X(texpm1pf, float) X(pexpm1f, float)                  \
    X(tlogpf, float) X(plogf, float) X(tlog1ppf, float) X(plog1pf, float)                  \
    X(tsqrt, double) X(trenorm, double) X(tsqrtf, float) X(trenormf, float)
#define EACH_D(X)                                                                           \
    X(pexp0, double) X(texp0, double) X(pexpm10, double) X(texpm10, double)                \
    X(plog0, double) X(tlog0, double) X(plog1p0, double) X(tlog1p0, double)                \
    X(pexp0f, float) X(texp0f, float) X(pexpm10f, float) X(texpm10f, float)                \
    X(plog0f, float) X(tlog0f, float) X(plog1p0f, float) X(tlog1p0f, float)
#define EACH_1X(X)                                                                          \
    X(exp1x, double) X(expm1_1x, double) X(log1x, double) X(log1p_1x, double)               \
    X(exp1xf, float) X(expm1_1xf, float) X(log1xf, float) X(log1p_1xf, float)
#define EACH_BWD(X)                                                                         \
    X(texp_bwd, double) X(texpm1_bwd, double) X(tlog_bwd, double) X(tlog1p_bwd, double)     \
    X(texpf_bwd, float) X(texpm1f_bwd, float) X(tlogf_bwd, float) X(tlog1pf_bwd, float)     \
    X(tadd, double) X(tsub, double) X(tmul, double) X(tdiv, double)                         \
    X(taddf, float) X(tsubf, float) X(tmulf, float) X(tdivf, float)
EACH_TW(DECL_TW)
EACH_D(DECL_D)
EACH_1X(DECL_1X)
EACH_BWD(DECL_BWD)
void tfo_eft_n(int, const double*, const double*, double*, double*, size_t);
int tfo_abi_version(void);
void qref_check(int, int, const void*, const void*, const void*, const void*, size_t, double,
                double*, int8_t*, int);
void qref_quad(int, const double*, double*, size_t);
void qref_libm(int, const double*, double*, size_t);
void qref_eval(int, const double*, const double*, double*, int*, size_t);
}

namespace {

uint64_t g_state = 0x9e3779b97f4a7c15ull;
uint64_t next_u64() {  // splitmix64
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <class T> T from_bits(uint64_t b) {
    T v;
    if (sizeof(T) == 8) {
        std::memcpy(&v, &b, 8);
    } else {
        uint32_t w = (uint32_t)b;
        std::memcpy(&v, &w, 4);
    }
    return v;
}

// Arguments of every class: raw bit patterns, scaled uniform values over the
// functions' ranges, and fixed edges.
template <class T> std::vector<T> arguments(size_t n) {
    std::vector<T> v;
    const T edges[] = {T(0), -T(0), T(1), T(-1), T(0.5), T(2), T(-0.5), T(0.693147),
                       T(709.78), T(-745.13), T(88.72), T(-103.97), T(1e-300), T(-1e-300),
                       INFINITY, -INFINITY, NAN, std::numeric_limits<T>::denorm_min(),
                       -std::numeric_limits<T>::denorm_min(), std::numeric_limits<T>::max(),
                       -std::numeric_limits<T>::max(), std::numeric_limits<T>::min()};
    for (T e : edges) v.push_back(e);
    for (size_t i = 0; i < n; ++i) {
        const uint64_t r = next_u64();
        switch (i % 3) {
            case 0: v.push_back(from_bits<T>(r)); break;
            case 1: v.push_back(T((double)(r >> 11) * 0x1p-53 * 1600.0 - 800.0)); break;
            default: v.push_back(T(std::ldexp((double)(r >> 11) * 0x1p-53, (int)(r % 130) - 64) *
                                   ((r >> 7) & 1 ? -1 : 1)));
        }
    }
    return v;
}

}  // namespace

int main() {
    size_t calls = 0;
    const auto xd = arguments<double>(6000);
    const auto xf = arguments<float>(6000);
    // second parts: zero, tiny, coupled-size and arbitrary
    auto second = [](auto x, size_t i) {
        using T = decltype(x);
        switch (i % 4) {
            case 0: return T(0);
            case 1: return T(x * T(1e-17));
            case 2: return from_bits<T>(next_u64());
            default: return T(std::numeric_limits<T>::denorm_min());
        }
    };
#define RUN_TW(NAME, T)                                                                    \
    {                                                                                      \
        const auto& xs = sizeof(T) == 8 ? (const void*)&xd : (const void*)&xf;             \
        const auto& x = *(const std::vector<T>*)xs;                                        \
        std::vector<T> x1(x.size());                                                       \
        for (size_t i = 0; i < x.size(); ++i) {                                            \
            x1[i] = second(x[i], i);                                                       \
            T z1;                                                                          \
            (void)tfo_##NAME(x[i], x1[i], &z1);                                            \
            ++calls;                                                                       \
        }                                                                                  \
        std::vector<T> z0(x.size()), z1(x.size());                                         \
        tfo_##NAME##_n(x.data(), x1.data(), z0.data(), z1.data(), x.size(), 2);            \
        unsigned long long cnt[4];                                                         \
        tfo_count_##NAME##_n(x.data(), x1.data(), x.size(), cnt);                          \
        calls += 2 * x.size();                                                             \
    }
#define RUN_D(NAME, T)                                                                     \
    {                                                                                      \
        const auto& x = *(const std::vector<T>*)(sizeof(T) == 8 ? (const void*)&xd         \
                                                                 : (const void*)&xf);      \
        for (size_t i = 0; i < x.size(); ++i) {                                            \
            T z1;                                                                          \
            (void)tfo_##NAME(x[i], &z1);                                                   \
            ++calls;                                                                       \
        }                                                                                  \
        std::vector<T> z0(x.size()), z1(x.size());                                         \
        tfo_##NAME##_n(x.data(), z0.data(), z1.data(), x.size(), 2);                       \
        unsigned long long cnt[4];                                                         \
        tfo_count_##NAME##_n(x.data(), x.size(), cnt);                                     \
        calls += 2 * x.size();                                                             \
    }
#define RUN_1X(NAME, T)                                                                    \
    {                                                                                      \
        const auto& x = *(const std::vector<T>*)(sizeof(T) == 8 ? (const void*)&xd         \
                                                                 : (const void*)&xf);      \
        for (size_t i = 0; i < x.size(); ++i) {                                            \
            (void)tfo_##NAME(x[i]);                                                        \
            ++calls;                                                                       \
        }                                                                                  \
        std::vector<T> z(x.size());                                                        \
        tfo_##NAME##_n(x.data(), z.data(), x.size(), 2);                                   \
        calls += x.size();                                                                 \
    }
#define RUN_BWD(NAME, T)                                                                   \
    {                                                                                      \
        const auto& x = *(const std::vector<T>*)(sizeof(T) == 8 ? (const void*)&xd         \
                                                                 : (const void*)&xf);      \
        const size_t n = x.size();                                                         \
        std::vector<T> a1(n), b0(n), b1(n), g0(n), g1(n);                                  \
        for (size_t i = 0; i < n; ++i) {                                                   \
            a1[i] = second(x[i], i);                                                       \
            b0[i] = x[(i * 7919) % n];                                                     \
            b1[i] = second(b0[i], i + 1);                                                  \
        }                                                                                  \
        tfo_##NAME##_n(x.data(), a1.data(), b0.data(), b1.data(), g0.data(), g1.data(), n,  \
                       2);                                                                 \
        unsigned long long cnt[4];                                                         \
        tfo_count_##NAME##_n(x.data(), a1.data(), b0.data(), b1.data(), n, cnt);           \
        calls += 2 * n;                                                                    \
    }
    EACH_TW(RUN_TW)
    EACH_D(RUN_D)
    EACH_1X(RUN_1X)
    EACH_BWD(RUN_BWD)
    {
        const size_t n = xd.size();
        std::vector<double> b(n), s(n), t(n);
        for (size_t i = 0; i < n; ++i) b[i] = xd[(i * 104729) % n];
        for (int which = 0; which < 3; ++which) tfo_eft_n(which, xd.data(), b.data(), s.data(),
                                                           t.data(), n);
        calls += 3 * n;
    }
    // the etalon: its accuracy check on the twofold results of both formats,
    // its three-part evaluation, and the context functions
    {
        const auto& x = xd;
        const size_t n = x.size();
        std::vector<double> x1(n), z0(n), z1(n), rel(n), parts(3 * n), out(n);
        std::vector<int8_t> cls(n);
        std::vector<int> ex(n);
        void (*const fd[4])(const double*, const double*, double*, double*, size_t, int) = {
            tfo_texp_n, tfo_texpm1_n, tfo_tlog_n, tfo_tlog1p_n};
        for (int fn = 0; fn < 4; ++fn) {
            for (size_t i = 0; i < n; ++i) x1[i] = second(x[i], i);
            fd[fn](x.data(), x1.data(), z0.data(), z1.data(), n, 2);
            qref_check(fn, 0, x.data(), x1.data(), z0.data(), z1.data(), n, 0x1p-95,
                       rel.data(), cls.data(), 2);
            qref_eval(fn, x.data(), x1.data(), parts.data(), ex.data(), n);
            qref_quad(fn, x.data(), out.data(), n);
            qref_libm(fn, x.data(), out.data(), n);
            calls += 4 * n;
        }
        const size_t m = xf.size();
        std::vector<float> f1(m), w0(m), w1(m);
        void (*const ff[4])(const float*, const float*, float*, float*, size_t, int) = {
            tfo_texpf_n, tfo_texpm1f_n, tfo_tlogf_n, tfo_tlog1pf_n};
        for (int fn = 0; fn < 4; ++fn) {
            for (size_t i = 0; i < m; ++i) f1[i] = second(xf[i], i);
            ff[fn](xf.data(), f1.data(), w0.data(), w1.data(), m, 2);
            qref_check(fn, 1, xf.data(), f1.data(), w0.data(), w1.data(), m, 0x1p-38,
                       rel.data(), cls.data(), 2);
            calls += m;
        }
    }
    if (tfo_abi_version() != 1) return 1;
    std::printf("SANITIZED OK %zu calls\n", calls);
    return 0;
}
