// Check library of the device value type of include/twofold_device.hpp (test
// infrastructure): one kernel per function that reads twofold arguments from
// split arrays, evaluates them with tfcp::twofold<T> values and the header's
// functions and operators, and writes the result pairs.  tests/
// test_cxx_device.py compares these with the library's array entry points.
//
//   tfcp_dev_apply(op, dtype, x0, x1, y0, y1, z0, z1, n, stream)
//     op:    0 exp  1 expm1  2 log  3 log1p   (the standard-like names)
//            4 pexp0  5 texp0  6 pexpm10  7 texpm10  8 plog0  9 tlog0
//            10 plog1p0  11 tlog1p0                 (dotted: x0 only)
//            12 texpp  13 pexp  14 texpm1p  15 pexpm1  16 tlogp  17 plog
//            18 tlog1pp  19 plog1p                  (coupled argument)
//            20 +  21 -  22 *  23 /                 (x op y)
//            24 sqrt  25 renorm
//     dtype: 0 binary64, 1 binary32; device pointers; returns 0, or -1 for an
//     unknown op or dtype, or the HIP error of the launch.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "twofold_device.hpp"

namespace {

template <class T, int OP>
__device__ __forceinline__ tfcp::twofold<T> apply(tfcp::twofold<T> x, tfcp::twofold<T> y) {
    using namespace tfcp;
    if constexpr (OP == 0) return exp(x);
    else if constexpr (OP == 1) return expm1(x);
    else if constexpr (OP == 2) return log(x);
    else if constexpr (OP == 3) return log1p(x);
    else if constexpr (OP == 4) return pexp0(x.value);
    else if constexpr (OP == 5) return texp0(x.value);
    else if constexpr (OP == 6) return pexpm10(x.value);
    else if constexpr (OP == 7) return texpm10(x.value);
    else if constexpr (OP == 8) return plog0(x.value);
    else if constexpr (OP == 9) return tlog0(x.value);
    else if constexpr (OP == 10) return plog1p0(x.value);
    else if constexpr (OP == 11) return tlog1p0(x.value);
    else if constexpr (OP == 12) return texpp(x);
    else if constexpr (OP == 13) return pexp(x);
    else if constexpr (OP == 14) return texpm1p(x);
    else if constexpr (OP == 15) return pexpm1(x);
    else if constexpr (OP == 16) return tlogp(x);
    else if constexpr (OP == 17) return plog(x);
    else if constexpr (OP == 18) return tlog1pp(x);
    else if constexpr (OP == 19) return plog1p(x);
    else if constexpr (OP == 20) return x + y;
    else if constexpr (OP == 21) return x - y;
    else if constexpr (OP == 22) return x * y;
    else if constexpr (OP == 23) return x / y;
    else if constexpr (OP == 24) return tfcp::sqrt(x);
    else return tfcp::renorm(x);
}

template <class T, int OP>
__global__ __launch_bounds__(256) void k_dev(const T* x0, const T* x1, const T* y0, const T* y1,
                                             T* z0, T* z1, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        tfcp::twofold<T> x{x0[i], x1 ? x1[i] : T(0)};
        tfcp::twofold<T> y{y0 ? y0[i] : T(0), y1 ? y1[i] : T(0)};
        tfcp::twofold<T> z = apply<T, OP>(x, y);
        z0[i] = z.value;
        z1[i] = z.error;
    }
}

template <class T, int OP>
int launch(const void* x0, const void* x1, const void* y0, const void* y1, void* z0, void* z1,
           size_t n, hipStream_t s) {
    if (n == 0) return 0;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_dev<T, OP><<<(unsigned)blocks, 256, 0, s>>>((const T*)x0, (const T*)x1, (const T*)y0,
                                                 (const T*)y1, (T*)z0, (T*)z1, n);
    return (int)hipGetLastError();
}

template <class T, int... OPS> struct Table;
template <class T> struct Table<T> {
    static int run(int, const void*, const void*, const void*, const void*, void*, void*, size_t,
                   hipStream_t) {
        return -1;
    }
};
template <class T, int OP, int... REST> struct Table<T, OP, REST...> {
    static int run(int op, const void* x0, const void* x1, const void* y0, const void* y1,
                   void* z0, void* z1, size_t n, hipStream_t s) {
        if (op == OP) return launch<T, OP>(x0, x1, y0, y1, z0, z1, n, s);
        return Table<T, REST...>::run(op, x0, x1, y0, y1, z0, z1, n, s);
    }
};
template <class T>
using All = Table<T, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20,
                  21, 22, 23, 24, 25>;

}  // namespace

extern "C" int tfcp_dev_apply(int op, int dtype, const void* x0, const void* x1, const void* y0,
                              const void* y1, void* z0, void* z1, size_t n, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (dtype == 0) return All<double>::run(op, x0, x1, y0, y1, z0, z1, n, s);
    if (dtype == 1) return All<float>::run(op, x0, x1, y0, y1, z0, z1, n, s);
    return -1;
}
