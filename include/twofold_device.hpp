/* twofold_device.hpp -- the paper's twofold<T> value type for HIP device code.
 *
 * The paper's C++ interface (section "Experimental code > C/C++ interface")
 * is a generic type twofold<T> with the fields "value" and "error" (the number
 * is value + error), one function name for float and double, and the standard
 * exp, expm1, log and log1p overloaded for twofold arguments.  This header
 * gives that interface to device code: a kernel holds tfcp::twofold<double>
 * (or <float>) values in registers and calls
 *
 *   z = tfcp::exp(x);   z = tfcp::texp(x);         twofold exp of a twofold (texp)
 *   tfcp::expm1 / texpm1, tfcp::log / tlog, tfcp::log1p / tlog1p
 *   tfcp::pexp0(v), texp0, pexpm10, texpm10, plog0, tlog0, plog1p0, tlog1p0
 *                                                   dotted argument v (a T)
 *   tfcp::texpp(x), pexp, texpm1p, pexpm1, tlogp, plog, tlog1pp, plog1p
 *                                                   coupled argument x
 *   x + y, x - y, x * y, x / y, tfcp::sqrt(x), tfcp::renorm(x)
 *                                                   twofold arithmetic
 *
 * Each function runs the element function the library's kernels run (the
 * general form, which takes any argument), so its result equals the array
 * entry point's of include/twofold_hip.h bit for bit, special values
 * included.  The range-reduction tables are this translation unit's own copy
 * in device global memory, read through the caches (the library's kernels
 * stage the same tables in LDS); they are a few kilobytes per format.
 *
 * Built with hipcc for gfx950 with -ffp-contract=off (every fused
 * multiply-add of the method is explicit; a contracted a*b + c would change
 * the bits) and, for binary32, -fno-gpu-flush-denormals-to-zero.  Include
 * path: the repository's include/ directory.  No library link is needed: the
 * functions are header-only and inline.
 */
#ifndef TWOFOLD_DEVICE_HPP
#define TWOFOLD_DEVICE_HPP

#include <hip/hip_runtime.h>

#include "../paper_1502_05216_amd/csrc/tf_device.hpp"

namespace tfcp {

template <class T> struct twofold {
    T value;
    T error;
};

namespace detail {

using tfh::Tw;

// Views of this translation unit's tables (tf_tables.inc, global memory).
template <class T> struct tabs;
template <> struct tabs<double> {
    __device__ static tfh::ExpTab<double> et() { return {TFH_D_S}; }
    __device__ static tfh::Pexp0Tab<double> pt() { return {TFH_D_E, TFH_D_EK, tfh::pexp0_c_table(0.0)}; }
    __device__ static tfh::Pm1Tab<double> mt() { return {TFH_D_CM1}; }
    __device__ static tfh::LogTab<double> lt() { return {TFH_D_LOG_INVC, TFH_D_LOG}; }
};
template <> struct tabs<float> {
    __device__ static tfh::ExpTab<float> et() { return {TFH_F_S}; }
    __device__ static tfh::Pexp0Tab<float> pt() { return {TFH_F_E, TFH_F_EK, tfh::pexp0_c_table(0.0f)}; }
    __device__ static tfh::Pm1Tab<float> mt() { return {TFH_F_CM1}; }
    __device__ static tfh::LogTab<float> lt() { return {TFH_F_LOG_INVC, TFH_F_LOG}; }
};

template <class T> __device__ __forceinline__ bool tiny(T x1) {
    return tfh::fabs_(x1) < tfh::P<T>::EXPM1_TINY;
}
template <class T> __device__ __forceinline__ Tw<T> in(twofold<T> x) { return {x.value, x.error}; }

}  // namespace detail

// --- the four twofold functions (section "Twofold exponent / logarithm:
// Algorithm summary"): z0 is the 1x function of x.value ------------------
template <class T> __device__ __forceinline__ twofold<T> texp(twofold<T> x) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::texp_elem<false, true>(x.value, x.error, detail::tiny(x.error), D::et(), D::pt(), z0, z1);
    return {z0, z1};
}
template <class T> __device__ __forceinline__ twofold<T> texpm1(twofold<T> x) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::texpm1_elem(x.value, x.error, detail::tiny(x.error), D::et(), D::pt(), D::mt(), z0, z1);
    return {z0, z1};
}
template <class T> __device__ __forceinline__ twofold<T> tlog(twofold<T> x) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::tlog_elem<false>(x.value, x.error, D::lt(), D::mt(), z0, z1);
    return {z0, z1};
}
template <class T> __device__ __forceinline__ twofold<T> tlog1p(twofold<T> x) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::tlog1p_elem<false>(x.value, x.error, D::lt(), D::mt(), z0, z1);
    return {z0, z1};
}

// The standard-like names of the paper's C++ interface.
template <class T> __device__ __forceinline__ twofold<T> exp(twofold<T> x) { return texp(x); }
template <class T> __device__ __forceinline__ twofold<T> expm1(twofold<T> x) { return texpm1(x); }
template <class T> __device__ __forceinline__ twofold<T> log(twofold<T> x) { return tlog(x); }
template <class T> __device__ __forceinline__ twofold<T> log1p(twofold<T> x) { return tlog1p(x); }

// --- functions of a dotted argument v (second part 0) --------------------
template <class T> __device__ __forceinline__ twofold<T> pexp0(T v) {
    T z0, z1;
    tfh::pexp0_p<false>(v, detail::tabs<T>::pt(), z0, z1);
    return {z0, z1};
}
template <class T> __device__ __forceinline__ twofold<T> texp0(T v) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::texp0_elem<false>(v, D::et(), D::pt(), z0, z1);
    return {z0, z1};
}
template <class T> __device__ __forceinline__ twofold<T> pexpm10(T v) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::pexpm10_p<false>(v, D::pt(), D::mt(), z0, z1);
    return {z0, z1};
}
template <class T> __device__ __forceinline__ twofold<T> texpm10(T v) {
    using D = detail::tabs<T>;
    T z0, z1;
    tfh::texpm10_elem<false>(v, D::et(), D::pt(), D::mt(), z0, z1);
    return {z0, z1};
}

namespace detail {
template <int KIND, bool PFN, class T> __device__ __forceinline__ twofold<T> logf_(T y0, T y1) {
    T z0, z1;
    tfh::log_iface_elem<KIND, PFN, false>(y0, y1, tabs<T>::lt(), tabs<T>::mt(), z0, z1);
    return {z0, z1};
}
}  // namespace detail

template <class T> __device__ __forceinline__ twofold<T> plog0(T v) {
    return detail::logf_<tfh::LK_LOG0, true>(v, T(0));
}
template <class T> __device__ __forceinline__ twofold<T> tlog0(T v) {
    return detail::logf_<tfh::LK_LOG0, false>(v, T(0));
}
template <class T> __device__ __forceinline__ twofold<T> plog1p0(T v) {
    return detail::logf_<tfh::LK_LOG1P0, true>(v, T(0));
}
template <class T> __device__ __forceinline__ twofold<T> tlog1p0(T v) {
    return detail::logf_<tfh::LK_LOG1P0, false>(v, T(0));
}

// --- functions of a coupled argument (x.value + x.error rounds to x.value) --
template <class T> __device__ __forceinline__ twofold<T> texpp(twofold<T> x) { return texp(x); }
template <class T> __device__ __forceinline__ twofold<T> texpm1p(twofold<T> x) { return texpm1(x); }
// pexp keeps pexp0's all-twofold Horner (its renormalised second part would
// expose the last bits of the 1x Horner tail that texp uses)
template <class T> __device__ __forceinline__ twofold<T> pexp(twofold<T> x) {
    using D = detail::tabs<T>;
    T z0, z1, r0, r1;
    tfh::texp_elem<false, false>(x.value, x.error, detail::tiny(x.error), D::et(), D::pt(), z0,
                                 z1);
    tfh::renorm_out(z0, z1, r0, r1);
    return {r0, r1};
}
template <class T> __device__ __forceinline__ twofold<T> pexpm1(twofold<T> x) {
    twofold<T> z = texpm1(x);
    T r0, r1;
    tfh::renorm_out(z.value, z.error, r0, r1);
    return {r0, r1};
}
template <class T> __device__ __forceinline__ twofold<T> tlogp(twofold<T> x) {
    return detail::logf_<tfh::LK_LOGC, false>(x.value, x.error);
}
template <class T> __device__ __forceinline__ twofold<T> plog(twofold<T> x) {
    return detail::logf_<tfh::LK_LOGC, true>(x.value, x.error);
}
template <class T> __device__ __forceinline__ twofold<T> tlog1pp(twofold<T> x) {
    return detail::logf_<tfh::LK_LOG1PC, false>(x.value, x.error);
}
template <class T> __device__ __forceinline__ twofold<T> plog1p(twofold<T> x) {
    return detail::logf_<tfh::LK_LOG1PC, true>(x.value, x.error);
}

// --- twofold arithmetic (section "Twofolds update"): the main part is the 1x
// operation on the main parts, then the rule for a non-finite main part ----
namespace detail {
template <int OP, class T> __device__ __forceinline__ twofold<T> ar(twofold<T> x, twofold<T> y) {
    Tw<T> z = tfh::arith_elem<OP>(in(x), in(y));
    return {z.x0, z.x1};
}
}  // namespace detail

template <class T> __device__ __forceinline__ twofold<T> operator+(twofold<T> x, twofold<T> y) {
    return detail::ar<tfh::OP_ADD>(x, y);
}
template <class T> __device__ __forceinline__ twofold<T> operator-(twofold<T> x, twofold<T> y) {
    return detail::ar<tfh::OP_SUB>(x, y);
}
template <class T> __device__ __forceinline__ twofold<T> operator*(twofold<T> x, twofold<T> y) {
    return detail::ar<tfh::OP_MUL>(x, y);
}
template <class T> __device__ __forceinline__ twofold<T> operator/(twofold<T> x, twofold<T> y) {
    return detail::ar<tfh::OP_DIV>(x, y);
}
template <class T> __device__ __forceinline__ twofold<T> sqrt(twofold<T> x) {
    return detail::ar<tfh::OP_SQRT>(x, x);
}
template <class T> __device__ __forceinline__ twofold<T> renorm(twofold<T> x) {
    return detail::ar<tfh::OP_RENORM>(x, x);
}

}  // namespace tfcp

#endif  // TWOFOLD_DEVICE_HPP
