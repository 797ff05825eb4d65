/* twofold.hpp -- C++ convenience layer over the C ABI of twofold_hip.h.
 *
 * The paper's C++ interface (section "Experimental code > C/C++ interface")
 * wraps its functions in a generic twofold<T> type with the fields "value"
 * and "error", uses one function name for float and double, and overloads
 * the standard exp, expm1, log and log1p for twofold arguments.  This header
 * gives the same interface for twofold ARRAYS on the device:
 *
 *   tfcp::twofold_array<T> {T* value; T* error; size_t n;}
 *       n numbers value[i] + error[i], each array a device allocation of n
 *       elements owned by the caller (the library neither allocates nor
 *       frees them);
 *   tfcp::texp(x, z, stream), tfcp::exp(x, z, stream), tfcp::pexp0(x0, z, stream),
 *   tfcp::tadd(x, y, z, stream), ...  -- float and double alike, no suffix.
 *
 * Every function is an inline call of the C entry point of the same name
 * (the binary32 one for T = float), so the results are those of the library,
 * bit for bit, and the calls are asynchronous on `stream` (a hipStream_t, or
 * null for the default stream).  They return the library's tf_status, plus
 * TF_EINVAL when the arrays of one call have different lengths.
 *
 * Plain C++ (no HIP headers needed): link against libtwofold_hip.so.
 */
#ifndef TWOFOLD_HPP
#define TWOFOLD_HPP

#include <cstddef>

#include "twofold_hip.h"

namespace tfcp {

template <class T> struct twofold_array {
    T* value;
    T* error;
    size_t n;
};

namespace detail {
template <class T> inline bool same_n(const twofold_array<T>& a, const twofold_array<T>& b) {
    return a.n == b.n;
}
}  // namespace detail

/* Functions of a twofold argument (the four twofold functions and the
 * coupled-argument entry points), square root and renormalization:
 * z = NAME(x). */
#define TFCP_UNARY(NAME)                                                                      \
    inline tf_status NAME(const twofold_array<double>& x, const twofold_array<double>& z,    \
                          void* stream = nullptr) {                                           \
        if (!detail::same_n(x, z)) return TF_EINVAL;                                          \
        return tf_##NAME(x.value, x.error, z.value, z.error, x.n, stream);                    \
    }                                                                                         \
    inline tf_status NAME(const twofold_array<float>& x, const twofold_array<float>& z,      \
                          void* stream = nullptr) {                                           \
        if (!detail::same_n(x, z)) return TF_EINVAL;                                          \
        return tf_##NAME##f(x.value, x.error, z.value, z.error, x.n, stream);                 \
    }

TFCP_UNARY(texp)
TFCP_UNARY(texpm1)
TFCP_UNARY(tlog)
TFCP_UNARY(tlog1p)
TFCP_UNARY(texpp)
TFCP_UNARY(pexp)
TFCP_UNARY(texpm1p)
TFCP_UNARY(pexpm1)
TFCP_UNARY(tlogp)
TFCP_UNARY(plog)
TFCP_UNARY(tlog1pp)
TFCP_UNARY(plog1p)
TFCP_UNARY(tsqrt)
TFCP_UNARY(trenorm)
#undef TFCP_UNARY

/* Functions of a dotted argument (the value part alone, as the paper's
 * pexp0(x.value)): z = NAME(x0), with z.n elements of x0. */
#define TFCP_DOTTED(NAME)                                                                     \
    inline tf_status NAME(const double* x0, const twofold_array<double>& z,                   \
                          void* stream = nullptr) {                                           \
        return tf_##NAME(x0, z.value, z.error, z.n, stream);                                  \
    }                                                                                         \
    inline tf_status NAME(const float* x0, const twofold_array<float>& z,                     \
                          void* stream = nullptr) {                                           \
        return tf_##NAME##f(x0, z.value, z.error, z.n, stream);                               \
    }

TFCP_DOTTED(pexp0)
TFCP_DOTTED(texp0)
TFCP_DOTTED(pexpm10)
TFCP_DOTTED(texpm10)
TFCP_DOTTED(plog0)
TFCP_DOTTED(tlog0)
TFCP_DOTTED(plog1p0)
TFCP_DOTTED(tlog1p0)
#undef TFCP_DOTTED

/* Twofold arithmetic: z = x op y. */
#define TFCP_BINARY(NAME)                                                                     \
    inline tf_status NAME(const twofold_array<double>& x, const twofold_array<double>& y,    \
                          const twofold_array<double>& z, void* stream = nullptr) {          \
        if (!detail::same_n(x, y) || !detail::same_n(x, z)) return TF_EINVAL;                 \
        return tf_##NAME(x.value, x.error, y.value, y.error, z.value, z.error, x.n, stream);  \
    }                                                                                         \
    inline tf_status NAME(const twofold_array<float>& x, const twofold_array<float>& y,      \
                          const twofold_array<float>& z, void* stream = nullptr) {            \
        if (!detail::same_n(x, y) || !detail::same_n(x, z)) return TF_EINVAL;                 \
        return tf_##NAME##f(x.value, x.error, y.value, y.error, z.value, z.error, x.n,       \
                            stream);                                                          \
    }

TFCP_BINARY(tadd)
TFCP_BINARY(tsub)
TFCP_BINARY(tmul)
TFCP_BINARY(tdiv)
#undef TFCP_BINARY

/* Standard-like names: for a twofold argument they are the twofold functions
 * (texp, texpm1, tlog, tlog1p), whose value parts reproduce the library's 1x
 * exp, expm1, log and log1p bit for bit. */
template <class T>
inline tf_status exp(const twofold_array<T>& x, const twofold_array<T>& z, void* stream = nullptr) {
    return texp(x, z, stream);
}
template <class T>
inline tf_status expm1(const twofold_array<T>& x, const twofold_array<T>& z,
                       void* stream = nullptr) {
    return texpm1(x, z, stream);
}
template <class T>
inline tf_status log(const twofold_array<T>& x, const twofold_array<T>& z, void* stream = nullptr) {
    return tlog(x, z, stream);
}
template <class T>
inline tf_status log1p(const twofold_array<T>& x, const twofold_array<T>& z,
                       void* stream = nullptr) {
    return tlog1p(x, z, stream);
}

}  // namespace tfcp

#endif  // TWOFOLD_HPP
