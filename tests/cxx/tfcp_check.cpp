// Check of the C++ convenience layer (include/twofold.hpp) against the C ABI.
//
//   tfcp_check cpu   argument handling only, no GPU work: every overload with
//                    n = 0 returns TF_OK, arrays of different lengths and NULL
//                    arrays with n > 0 return TF_EINVAL.
//   tfcp_check gpu   every overload on device arrays of 100003 elements, its
//                    outputs compared bit for bit with the C entry point's.
// Prints one line per check and "ALL OK" at the end; exit status 0 on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/twofold.hpp"

using tfcp::twofold_array;

static int failures = 0;

static void expect(bool ok, const char* what) {
    std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    std::fflush(stdout);
    if (!ok) ++failures;
}

template <class T> static int cpu_checks() {
    T* fake = reinterpret_cast<T*>(uintptr_t(0x1000));
    twofold_array<T> e{nullptr, nullptr, 0}, a{fake, fake, 10}, b{fake, fake, 11};
    twofold_array<T> nul{nullptr, fake, 10};
    const char* dn = sizeof(T) == 8 ? "double" : "float";
    char what[128];
#define CPU_UNARY(NAME)                                                                      \
    std::snprintf(what, sizeof what, "%s %s n=0 / length mismatch / NULL", #NAME, dn);        \
    expect(tfcp::NAME(e, e) == TF_OK && tfcp::NAME(a, b) == TF_EINVAL &&                      \
               tfcp::NAME(nul, a) == TF_EINVAL,                                               \
           what);
    CPU_UNARY(texp) CPU_UNARY(texpm1) CPU_UNARY(tlog) CPU_UNARY(tlog1p)
    CPU_UNARY(texpp) CPU_UNARY(pexp) CPU_UNARY(texpm1p) CPU_UNARY(pexpm1)
    CPU_UNARY(tlogp) CPU_UNARY(plog) CPU_UNARY(tlog1pp) CPU_UNARY(plog1p)
    CPU_UNARY(tsqrt) CPU_UNARY(trenorm) CPU_UNARY(exp) CPU_UNARY(expm1) CPU_UNARY(log)
    CPU_UNARY(log1p)
#undef CPU_UNARY
#define CPU_DOTTED(NAME)                                                                     \
    std::snprintf(what, sizeof what, "%s %s n=0 / NULL", #NAME, dn);                          \
    expect(tfcp::NAME(static_cast<const T*>(nullptr), e) == TF_OK &&                          \
               tfcp::NAME(static_cast<const T*>(nullptr), a) == TF_EINVAL,                    \
           what);
    CPU_DOTTED(pexp0) CPU_DOTTED(texp0) CPU_DOTTED(pexpm10) CPU_DOTTED(texpm10)
    CPU_DOTTED(plog0) CPU_DOTTED(tlog0) CPU_DOTTED(plog1p0) CPU_DOTTED(tlog1p0)
#undef CPU_DOTTED
#define CPU_BINARY(NAME)                                                                     \
    std::snprintf(what, sizeof what, "%s %s n=0 / length mismatch / NULL", #NAME, dn);        \
    expect(tfcp::NAME(e, e, e) == TF_OK && tfcp::NAME(a, a, b) == TF_EINVAL &&                \
               tfcp::NAME(a, b, a) == TF_EINVAL && tfcp::NAME(a, nul, a) == TF_EINVAL,        \
           what);
    CPU_BINARY(tadd) CPU_BINARY(tsub) CPU_BINARY(tmul) CPU_BINARY(tdiv)
#undef CPU_BINARY
    return 0;
}

#define HIP_OK(call)                                                                         \
    do {                                                                                     \
        if ((call) != hipSuccess) {                                                          \
            std::printf("FAIL HIP call %s\n", #call);                                        \
            return 1;                                                                        \
        }                                                                                    \
    } while (0)

// Device arrays of n elements: inputs x (positive, in every function's domain),
// y, and two output pairs.
template <class T> struct Dev {
    size_t n;
    T *x0, *x1, *y0, *y1, *a0, *a1, *b0, *b1;
};

template <class T> static bool same(const Dev<T>& d) {
    std::vector<T> h[4];
    const T* p[4] = {d.a0, d.a1, d.b0, d.b1};
    for (int k = 0; k < 4; ++k) {
        h[k].resize(d.n);
        if (hipMemcpy(h[k].data(), p[k], d.n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
            return false;
    }
    return std::memcmp(h[0].data(), h[2].data(), d.n * sizeof(T)) == 0 &&
           std::memcmp(h[1].data(), h[3].data(), d.n * sizeof(T)) == 0;
}

template <class T> static int gpu_checks() {
    Dev<T> d;
    d.n = 100003;
    T** all[8] = {&d.x0, &d.x1, &d.y0, &d.y1, &d.a0, &d.a1, &d.b0, &d.b1};
    for (T** q : all) HIP_OK(hipMalloc(reinterpret_cast<void**>(q), d.n * sizeof(T)));
    std::vector<T> hx0(d.n), hx1(d.n), hy0(d.n), hy1(d.n);
    const T eps = sizeof(T) == 8 ? T(0x1p-54) : T(0x1p-25);
    for (size_t i = 0; i < d.n; ++i) {
        hx0[i] = T(0.001) + T(0.6) * T(i % 1000) / T(1000);      // in (0, ln 2): every domain
        hx1[i] = hx0[i] * eps * (T(i % 7) - T(3)) / T(3);       // coupled second part
        hy0[i] = T(1.5) + T(i % 13);
        hy1[i] = hy0[i] * eps * (T(i % 5) - T(2)) / T(2);
    }
    HIP_OK(hipMemcpy(d.x0, hx0.data(), d.n * sizeof(T), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d.x1, hx1.data(), d.n * sizeof(T), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d.y0, hy0.data(), d.n * sizeof(T), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d.y1, hy1.data(), d.n * sizeof(T), hipMemcpyHostToDevice));
    twofold_array<T> x{d.x0, d.x1, d.n}, y{d.y0, d.y1, d.n}, za{d.a0, d.a1, d.n};
    const char* dn = sizeof(T) == 8 ? "double" : "float";
    const bool dbl = sizeof(T) == 8;
    char what[128];
    // the C entry point of the format: the binary64 name, or the binary32 twin
#define CFN(NAME) (dbl ? reinterpret_cast<decltype(&tf_##NAME)>(&tf_##NAME)                  \
                       : reinterpret_cast<decltype(&tf_##NAME)>(&tf_##NAME##f))
#define GPU_UNARY(NAME, CNAME)                                                               \
    {                                                                                        \
        tf_status s1 = tfcp::NAME(x, za);                                                    \
        tf_status s2 = reinterpret_cast<tf_status (*)(const T*, const T*, T*, T*, size_t,   \
                                                      void*)>(CFN(CNAME))(d.x0, d.x1, d.b0,  \
                                                                           d.b1, d.n,         \
                                                                           nullptr);          \
        HIP_OK(hipDeviceSynchronize());                                                      \
        std::snprintf(what, sizeof what, "%s %s equals tf_%s", #NAME, dn, #CNAME);          \
        expect(s1 == TF_OK && s2 == TF_OK && same(d), what);                                 \
    }
    GPU_UNARY(texp, texp) GPU_UNARY(texpm1, texpm1) GPU_UNARY(tlog, tlog)
    GPU_UNARY(tlog1p, tlog1p) GPU_UNARY(texpp, texpp) GPU_UNARY(pexp, pexp)
    GPU_UNARY(texpm1p, texpm1p) GPU_UNARY(pexpm1, pexpm1) GPU_UNARY(tlogp, tlogp)
    GPU_UNARY(plog, plog) GPU_UNARY(tlog1pp, tlog1pp) GPU_UNARY(plog1p, plog1p)
    GPU_UNARY(tsqrt, tsqrt) GPU_UNARY(trenorm, trenorm) GPU_UNARY(exp, texp)
    GPU_UNARY(expm1, texpm1) GPU_UNARY(log, tlog) GPU_UNARY(log1p, tlog1p)
#undef GPU_UNARY
#define GPU_DOTTED(NAME)                                                                     \
    {                                                                                        \
        tf_status s1 = tfcp::NAME(static_cast<const T*>(d.x0), za);                          \
        tf_status s2 = reinterpret_cast<tf_status (*)(const T*, T*, T*, size_t, void*)>(    \
            CFN(NAME))(d.x0, d.b0, d.b1, d.n, nullptr);                                      \
        HIP_OK(hipDeviceSynchronize());                                                      \
        std::snprintf(what, sizeof what, "%s %s equals tf_%s", #NAME, dn, #NAME);           \
        expect(s1 == TF_OK && s2 == TF_OK && same(d), what);                                 \
    }
    GPU_DOTTED(pexp0) GPU_DOTTED(texp0) GPU_DOTTED(pexpm10) GPU_DOTTED(texpm10)
    GPU_DOTTED(plog0) GPU_DOTTED(tlog0) GPU_DOTTED(plog1p0) GPU_DOTTED(tlog1p0)
#undef GPU_DOTTED
#define GPU_BINARY(NAME)                                                                     \
    {                                                                                        \
        tf_status s1 = tfcp::NAME(x, y, za);                                                 \
        tf_status s2 = reinterpret_cast<tf_status (*)(const T*, const T*, const T*,         \
                                                      const T*, T*, T*, size_t, void*)>(    \
            CFN(NAME))(d.x0, d.x1, d.y0, d.y1, d.b0, d.b1, d.n, nullptr);                    \
        HIP_OK(hipDeviceSynchronize());                                                      \
        std::snprintf(what, sizeof what, "%s %s equals tf_%s", #NAME, dn, #NAME);           \
        expect(s1 == TF_OK && s2 == TF_OK && same(d), what);                                 \
    }
    GPU_BINARY(tadd) GPU_BINARY(tsub) GPU_BINARY(tmul) GPU_BINARY(tdiv)
#undef GPU_BINARY
#undef CFN
    for (T** q : all) HIP_OK(hipFree(*q));
    return 0;
}

int main(int argc, char** argv) {
    const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
    int rc = gpu ? (gpu_checks<double>() | gpu_checks<float>())
                 : (cpu_checks<double>() | cpu_checks<float>());
    if (rc != 0 || failures != 0) {
        std::printf("FAILED %d\n", failures);
        return 1;
    }
    std::printf("ALL OK\n");
    return 0;
}
