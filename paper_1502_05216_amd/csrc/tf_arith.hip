// Twofold arithmetic over arrays for gfx950: z = x op y for twofolds
// x = x0 + x1, y = y0 + y1 (tadd, tsub, tmul, tdiv), z = sqrt(x) (tsqrt) and
// the renormalization of x (trenorm) --
// the paper's second measured workload (section "Twofolds update").  The main
// part is the 1x operation on the main parts (IEEE +, -, *, / and sqrt,
// correctly rounded); z1 is the twofold error term: the exact error of the
// main operation from an error-free transform (two_sum, the corrected
// subtraction, the FMA product) or the FMA remainder of a quotient / square
// root, plus the first-order terms of the low parts.  Then the rule for a
// non-finite main part.  Each kernel streams its arrays once: 48 B per
// binary64 element for the binary operations, 32 B for tsqrt and trenorm.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/twofold_hip.h"
#include "tf_common.hpp"

using namespace tfk;

namespace {

// y0, y1 are not read for tsqrt and trenorm (they may be null).
template <int OP> constexpr bool kUnary = OP == OP_SQRT || OP == OP_RENORM;

template <class T, int OP, int EPT>
__global__ __launch_bounds__(kBlock) void k_arith(const T* x0, const T* x1, const T* y0,
                                                  const T* y1, T* z0, T* z1, size_t n) {
    constexpr bool UNARY = kUnary<OP>;
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    const size_t off = (size_t)threadIdx.x * EPT;
    for (size_t t = blockIdx.x; t < nfull; t += gridDim.x) {
        const size_t base = t * TILE + off;
        Vec<T, EPT> a, b, c, d, r0, r1;
        vload<kStreamNT>(a, x0 + base);
        vload<kStreamNT>(b, x1 + base);
        if constexpr (!UNARY) {
            vload<kStreamNT>(c, y0 + base);
            vload<kStreamNT>(d, y1 + base);
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            Tw<T> y = UNARY ? Tw<T>{T(0), T(0)} : Tw<T>{c.v[e], d.v[e]};
            Tw<T> r = arith_elem<OP>(Tw<T>{a.v[e], b.v[e]}, y);
            r0.v[e] = r.x0;
            r1.v[e] = r.x1;
        }
        vstore<kStreamNT>(z0 + base, r0);
        vstore<kStreamNT>(z1 + base, r1);
    }
    const size_t rbase = nfull * TILE;
    if (rbase < n && blockIdx.x == nfull % gridDim.x) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const size_t i = rbase + off + e;
            if (i < n) {
                Tw<T> y = UNARY ? Tw<T>{T(0), T(0)} : Tw<T>{y0[i], y1[i]};
                Tw<T> r = arith_elem<OP>(Tw<T>{x0[i], x1[i]}, y);
                z0[i] = r.x0;
                z1[i] = r.x1;
            }
        }
    }
}

template <class T, int OP>
tf_status launch_arith(const T* x0, const T* x1, const T* y0, const T* y1, T* z0, T* z1, size_t n,
                       void* stream) {
    constexpr bool UNARY = kUnary<OP>;
    if (n == 0) return TF_OK;
    if (!x0 || !x1 || (!UNARY && (!y0 || !y1)) || !z0 || !z1) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    const bool al = aligned16(x0) && aligned16(x1) && (UNARY || (aligned16(y0) && aligned16(y1))) &&
                    aligned16(z0) && aligned16(z1);
    constexpr int EPT = 16 / sizeof(T);
    const size_t tile = (size_t)kBlock * (al ? EPT : 1);
    const size_t tiles = n / tile, cap = (size_t)cus * kStreamBpc;
    const unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    hipStream_t s = (hipStream_t)stream;
    if (al)
        hipLaunchKernelGGL((k_arith<T, OP, EPT>), dim3(grid), dim3(kBlock), 0, s, x0, x1, y0, y1,
                           z0, z1, n);
    else
        hipLaunchKernelGGL((k_arith<T, OP, 1>), dim3(grid), dim3(kBlock), 0, s, x0, x1, y0, y1,
                           z0, z1, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

}  // namespace

extern "C" {

#define TF_ARITH_ENTRY(NAME, T, OP)                                                           \
    tf_status NAME(const T* x0, const T* x1, const T* y0, const T* y1, T* z0, T* z1, size_t n, \
                   void* stream) {                                                            \
        return launch_arith<T, OP>(x0, x1, y0, y1, z0, z1, n, stream);                        \
    }

TF_ARITH_ENTRY(tf_tadd, double, OP_ADD)
TF_ARITH_ENTRY(tf_tsub, double, OP_SUB)
TF_ARITH_ENTRY(tf_tmul, double, OP_MUL)
TF_ARITH_ENTRY(tf_tdiv, double, OP_DIV)
TF_ARITH_ENTRY(tf_taddf, float, OP_ADD)
TF_ARITH_ENTRY(tf_tsubf, float, OP_SUB)
TF_ARITH_ENTRY(tf_tmulf, float, OP_MUL)
TF_ARITH_ENTRY(tf_tdivf, float, OP_DIV)

tf_status tf_tsqrt(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                   void* stream) {
    return launch_arith<double, OP_SQRT>(x0, x1, nullptr, nullptr, z0, z1, n, stream);
}
tf_status tf_tsqrtf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                    void* stream) {
    return launch_arith<float, OP_SQRT>(x0, x1, nullptr, nullptr, z0, z1, n, stream);
}
tf_status tf_trenorm(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                     void* stream) {
    return launch_arith<double, OP_RENORM>(x0, x1, nullptr, nullptr, z0, z1, n, stream);
}
tf_status tf_trenormf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                      void* stream) {
    return launch_arith<float, OP_RENORM>(x0, x1, nullptr, nullptr, z0, z1, n, stream);
}

}  // extern "C"
