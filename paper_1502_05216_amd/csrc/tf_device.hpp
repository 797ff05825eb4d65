// Device-side twofold arithmetic, 1x functions and twofold exp/log cores for
// gfx950 (binary64 and binary32).  Every function here is inlined into the
// kernels of tf_kernels.hip; tables are read from LDS through the pointers
// the kernels pass in.
//
// Bit-reproducibility: the library is compiled with -ffp-contract=off, so the
// compiler never fuses a*b+c; every fused multiply-add is an explicit ffma().
// Every step is one IEEE operation (+ - * fma, rint, ldexp, frexp) or integer
// bit manipulation, so a given sequence gives the same bits on any IEEE
// machine.  Branches of the method become selects; index arithmetic is done on
// clamped arguments so that a table read can never leave its table, whatever
// the input (NaN, infinities).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tf_tables.inc"

namespace tfh {

template <class T> struct Tw { T x0, x1; };

// ----------------------------------------------------------------------------
// IEEE primitives
// ----------------------------------------------------------------------------
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double frint(double a) { return __builtin_rint(a); }
__device__ __forceinline__ float frint(float a) { return __builtin_rintf(a); }
__device__ __forceinline__ double fldexp(double a, int k) { return __builtin_amdgcn_ldexp(a, k); }
__device__ __forceinline__ float fldexp(float a, int k) { return __builtin_amdgcn_ldexpf(a, k); }
__device__ __forceinline__ double fabs_(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float fabs_(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double frexp_mant(double a) { return __builtin_amdgcn_frexp_mant(a); }
__device__ __forceinline__ float frexp_mant(float a) { return __builtin_amdgcn_frexp_mantf(a); }
__device__ __forceinline__ int frexp_exp(double a) { return __builtin_amdgcn_frexp_exp(a); }
__device__ __forceinline__ int frexp_exp(float a) { return __builtin_amdgcn_frexp_expf(a); }
__device__ __forceinline__ bool isnan_(double a) { return __builtin_isnan(a); }
__device__ __forceinline__ bool isnan_(float a) { return __builtin_isnan(a); }

// ----------------------------------------------------------------------------
// Format parameters
// ----------------------------------------------------------------------------
// Build define TF_PEXP0_K selects pexp0's decomposition x = 2^L m + 2^-K n + y:
// K = 5, the paper's parameters (default), or K = 6 (build variant k6, the
// rebalancing the section "Function pexp0()" closes with): |y| <= 2^-7, so
// the Taylor sum needs one term fewer (N = 11, binary32 5) and its twofold
// part one step fewer, for a C table of twice the entries (8 KB in binary64).
#ifndef TF_PEXP0_K
#define TF_PEXP0_K 5
#endif
constexpr bool kPexp0K6 = TF_PEXP0_K == 6;
static_assert(TF_PEXP0_K == 5 || TF_PEXP0_K == 6, "TF_PEXP0_K is 5 or 6");

constexpr double fact_ratio(int n, int j) {  // n!/j!, exact for n <= 12
    double r = 1.0;
    for (int i = j + 1; i <= n; ++i) r *= i;
    return r;
}

template <class T> struct P;

// pexp0's C table of the selected decomposition.
__device__ __forceinline__ const double2* pexp0_c_table(double) {
    return kPexp0K6 ? TFH_D_C6 : TFH_D_C;
}
__device__ __forceinline__ const float2* pexp0_c_table(float) {
    return kPexp0K6 ? TFH_F_C6 : TFH_F_C;
}

template <> struct P<double> {
    using V2 = double2;
    using U = uint64_t;
    static constexpr int L = TFH_D_L, N1 = TFH_D_N1;
    static constexpr int K = kPexp0K6 ? TFH_D_K6_K : TFH_D_K, N = kPexp0K6 ? TFH_D_K6_N : TFH_D_N;
    static constexpr int E_OFF = TFH_D_E_OFF, E_CNT = TFH_D_E_CNT;
    static constexpr int C_OFF = kPexp0K6 ? TFH_D_K6_C_OFF : TFH_D_C_OFF;
    static constexpr int C_CNT = kPexp0K6 ? TFH_D_K6_C_CNT : TFH_D_C_CNT;
    static constexpr int CM1_OFF = TFH_D_CM1_OFF, CM1_CNT = TFH_D_CM1_CNT;
    static constexpr int MANT = 52, EXPMASK = 0x7ff, BIAS = 1023;
    static constexpr U MANT_MASK = 0x000fffffffffffffull;
    static constexpr U ONE_BITS = 0x3ff0000000000000ull;   // exponent field of [1,2)
    static constexpr U HALF_BITS = 0x3fe0000000000000ull;  // exponent field of [1/2,1)
    static constexpr double INF = __builtin_inf();
    static constexpr double LN2_HI = TFH_D_LN2_HI, LN2_LO = TFH_D_LN2_LO;
    static constexpr double RCP_HI = TFH_D_RCP_HI, RCP_LO = TFH_D_RCP_LO;
    static constexpr double INV_L = TFH_D_INV_L, L1 = TFH_D_L1, L2 = TFH_D_L2;
    static constexpr double LN2X_HI = TFH_D_LN2X_HI, LN2X_LO = TFH_D_LN2X_LO;
    static constexpr double EXP_XMAX = TFH_D_EXP_XMAX, EXPM1_XMAX = TFH_D_EXPM1_XMAX;
    static constexpr double EXP_XLO = TFH_D_EXP_XLO, EXPM1_XNEG = TFH_D_EXPM1_XNEG;
    static constexpr double EXPM1_TINY = TFH_D_EXPM1_TINY, LOG1P_TINY = TFH_D_LOG1P_TINY;
    // Highest Horner step run in twofold arithmetic (horner_fact): pexp0 with
    // the 1x tail (|y| <= 2^-6, or 2^-7 with K = 6), pexpm10.
    static constexpr int EXP_TF_J = kPexp0K6 ? 6 : 7, EXPM1_TF_J = 6;
    static constexpr int EXP_NC = TFH_D_EXP_NC, LOG_NC = TFH_D_LOG_NC;
    static constexpr double EXP_C[EXP_NC] = {TFH_D_EXP_C_LIST};
    static constexpr double LOG_C[LOG_NC] = {TFH_D_LOG_C_LIST};
    __device__ static U bits(double x) { return (U)__double_as_longlong(x); }
    __device__ static double from_bits(U b) { return __longlong_as_double((long long)b); }
    __device__ static double qnan() { return __builtin_nan(""); }
};

template <> struct P<float> {
    using V2 = float2;
    using U = uint32_t;
    static constexpr int L = TFH_F_L, N1 = TFH_F_N1;
    static constexpr int K = kPexp0K6 ? TFH_F_K6_K : TFH_F_K, N = kPexp0K6 ? TFH_F_K6_N : TFH_F_N;
    static constexpr int E_OFF = TFH_F_E_OFF, E_CNT = TFH_F_E_CNT;
    static constexpr int C_OFF = kPexp0K6 ? TFH_F_K6_C_OFF : TFH_F_C_OFF;
    static constexpr int C_CNT = kPexp0K6 ? TFH_F_K6_C_CNT : TFH_F_C_CNT;
    static constexpr int CM1_OFF = TFH_F_CM1_OFF, CM1_CNT = TFH_F_CM1_CNT;
    static constexpr int MANT = 23, EXPMASK = 0xff, BIAS = 127;
    static constexpr U MANT_MASK = 0x007fffffu;
    static constexpr U ONE_BITS = 0x3f800000u;
    static constexpr U HALF_BITS = 0x3f000000u;
    static constexpr float INF = __builtin_inff();
    static constexpr float LN2_HI = TFH_F_LN2_HI, LN2_LO = TFH_F_LN2_LO;
    static constexpr float RCP_HI = TFH_F_RCP_HI, RCP_LO = TFH_F_RCP_LO;
    static constexpr float INV_L = TFH_F_INV_L, L1 = TFH_F_L1, L2 = TFH_F_L2;
    static constexpr float LN2X_HI = TFH_F_LN2X_HI, LN2X_LO = TFH_F_LN2X_LO;
    static constexpr float EXP_XMAX = TFH_F_EXP_XMAX, EXPM1_XMAX = TFH_F_EXPM1_XMAX;
    static constexpr float EXP_XLO = TFH_F_EXP_XLO, EXPM1_XNEG = TFH_F_EXPM1_XNEG;
    static constexpr float EXPM1_TINY = TFH_F_EXPM1_TINY, LOG1P_TINY = TFH_F_LOG1P_TINY;
    static constexpr int EXP_TF_J = 3, EXPM1_TF_J = 3;
    static constexpr int EXP_NC = TFH_F_EXP_NC, LOG_NC = TFH_F_LOG_NC;
    static constexpr float EXP_C[EXP_NC] = {TFH_F_EXP_C_LIST};
    static constexpr float LOG_C[LOG_NC] = {TFH_F_LOG_C_LIST};
    __device__ static U bits(float x) { return (U)__float_as_uint(x); }
    __device__ static float from_bits(U b) { return __uint_as_float(b); }
    __device__ static float qnan() { return __builtin_nanf(""); }
};

// ----------------------------------------------------------------------------
// Twofold arithmetic (error-free transforms with the FMA exact product).
// Outputs of fast_two_sum / two_sum / two_prod are the unique exact rounding
// errors, so the fast form is used wherever |a| >= |b| (or a = 0) is proven.
// ----------------------------------------------------------------------------
template <class T> __device__ __forceinline__ Tw<T> fast_two_sum(T a, T b) {
    T s = a + b;
    T t = b - (s - a);
    return {s, t};
}
template <class T> __device__ __forceinline__ Tw<T> two_sum(T a, T b) {
    T s = a + b;
    T bp = s - a;
    T ap = s - bp;
    T db = b - bp;
    T da = a - ap;
    return {s, da + db};
}
// fast_two_sum for |a| >= |b|, with the error formed as (a - s) + b: a - s is
// exact (the negation of fast_two_sum's exact s - a), so the error has the
// same value, and an exact sum gives +0 as two_sum's does (b - (s - a) would
// give -0 for b = -0).  It equals two_sum bit for bit when |a| >= |b|.
template <class T> __device__ __forceinline__ Tw<T> fast_two_sum_pz(T a, T b) {
    T s = a + b;
    T t = (a - s) + b;
    return {s, t};
}
template <class T> __device__ __forceinline__ Tw<T> two_prod(T a, T b) {
    T p = a * b;
    return {p, ffma(a, b, -p)};
}
// Twofold times 1x with the operations the paper counts for it (section
// "Twofold exponent / Method summary": two multiplications, one FMA, one
// sum): the low product is rounded on its own before it meets the error of
// the exact product.  Fusing it into that error with a second FMA would save
// an operation but change the second part's bits.
template <class T> __device__ __forceinline__ Tw<T> mul_td(Tw<T> A, T c) {
    Tw<T> pe = two_prod(A.x0, c);
    return {pe.x0, pe.x1 + A.x1 * c};
}
template <class T> __device__ __forceinline__ Tw<T> add_td_fast(Tw<T> A, T c) {
    Tw<T> st = fast_two_sum(c, A.x0);
    return {st.x0, st.x1 + A.x1};
}
template <class T> __device__ __forceinline__ Tw<T> add_td(Tw<T> A, T c) {
    Tw<T> st = two_sum(A.x0, c);
    return {st.x0, st.x1 + A.x1};
}
template <class T> __device__ __forceinline__ Tw<T> mul_tt(Tw<T> A, Tw<T> B) {
    Tw<T> pe = two_prod(A.x0, B.x0);
    return {pe.x0, ffma(A.x0, B.x1, ffma(A.x1, B.x0, pe.x1))};
}
template <class T> __device__ __forceinline__ Tw<T> add_tt(Tw<T> A, Tw<T> B) {
    Tw<T> st = two_sum(A.x0, B.x0);
    return {st.x0, st.x1 + (A.x1 + B.x1)};
}
template <class T> __device__ __forceinline__ Tw<T> add_tt_fast(Tw<T> A, Tw<T> B) {
    Tw<T> st = fast_two_sum(A.x0, B.x0);
    return {st.x0, st.x1 + (A.x1 + B.x1)};
}
template <class T> __device__ __forceinline__ Tw<T> div_tt(Tw<T> A, Tw<T> B) {
    T q0 = A.x0 / B.x0;
    T r = ffma(-q0, B.x0, A.x0);
    T q1 = ((r + A.x1) - q0 * B.x1) / B.x0;
    return {q0, q1};
}
// d + t = a - b exactly, any a, b: negating b is exact, so the two-sum of a
// and -b is an error-free difference (x + (-y) is the IEEE operation x - y).
template <class T> __device__ __forceinline__ Tw<T> two_diff(T a, T b) { return two_sum(a, -b); }
__device__ __forceinline__ double fsqrt(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ float fsqrt(float a) { return __builtin_sqrtf(a); }
template <class T> __device__ __forceinline__ Tw<T> sel(bool c, Tw<T> a, Tw<T> b) {
    return {c ? a.x0 : b.x0, c ? a.x1 : b.x1};
}

// ----------------------------------------------------------------------------
// LDS table views
// ----------------------------------------------------------------------------
template <class T> struct ExpTab {        // 2^(j/32) twofolds for the 1x exp/expm1
    const typename P<T>::V2* S;
};
template <class T> struct LogTab {        // 1x log cells
    const T* INVC;
    const typename P<T>::V2* LOG;
};
template <class T> struct Pexp0Tab {      // pexp0: E = Ehat 2^k and C = e^(n/32)/N!
    const typename P<T>::V2* E;
    const int* EK;
    const typename P<T>::V2* C;
};
template <class T> struct Pm1Tab {        // pexpm10: e^(n/128) - 1
    const typename P<T>::V2* CM1;
};

// ----------------------------------------------------------------------------
// 1x functions (main parts z0)
// ----------------------------------------------------------------------------
template <class T> __device__ __forceinline__ T exp_q(T r) {
    T q = P<T>::EXP_C[P<T>::EXP_NC - 1];
#pragma unroll
    for (int i = P<T>::EXP_NC - 2; i >= 0; --i) q = ffma(r, q, P<T>::EXP_C[i]);
    return q;
}
template <class T> __device__ __forceinline__ T log_q(T r) {
    T q = P<T>::LOG_C[P<T>::LOG_NC - 1];
#pragma unroll
    for (int i = P<T>::LOG_NC - 2; i >= 0; --i) q = ffma(r, q, P<T>::LOG_C[i]);
    return q;
}

// Every per-element routine below has a FAST form.  A kernel takes it for a
// whole wave when every lane of the wave satisfies the routine's stated
// argument condition (a wave vote); under that condition the range, NaN and
// infinity selects of the general form are no-ops, so both forms give the same
// bits.  This is the paper's conditional vectoring: the plain branch-free
// computation when all lanes lie in the main interval, the general one
// otherwise.

// exp(x): x = (32m + j) ln2/32 + r, e^x = 2^m 2^(j/32) e^r.
// FAST: EXP_XLO <= x <= EXP_XMAX.
template <bool FAST, class T> __device__ __forceinline__ T exp1x(T x, ExpTab<T> t) {
    using K = P<T>;
    T xc = x;
    if constexpr (!FAST) {
        xc = (x >= K::EXP_XLO) ? x : K::EXP_XLO;
        xc = (xc <= K::EXP_XMAX) ? xc : K::EXP_XMAX;
    }
    T kd = frint(xc * K::INV_L);
    int k = (int)kd;
    T r = ffma(-kd, K::L1, xc);
    r = ffma(-kd, K::L2, r);
    T p = ffma(r * r, exp_q(r), r);
    int j = k & 31, m = (k - j) >> 5;
    typename K::V2 s = t.S[j];
    T y = s.x + ffma(s.x, p, s.y);
    T res = fldexp(y, m);
    if constexpr (FAST) return res;
    res = (x < K::EXP_XLO) ? T(0) : res;
    res = (x > K::EXP_XMAX) ? K::INF : res;
    return isnan_(x) ? x + x : res;
}

// expm1 for |x| < EXPM1_TINY: x + x^2/2 (zero keeps its sign).
template <class T> __device__ __forceinline__ T expm1_tiny(T x) {
    return (x == T(0)) ? x : ffma(x, x * T(0.5), x);
}

// expm1(x): the reduction of exp with r = rhi + rlo; the -1 enters as -2^-m in
// the scaled domain through exact transforms.  FAST: EXPM1_XNEG <= x <= EXPM1_XMAX.
template <bool FAST, class T> __device__ __forceinline__ T expm1_1x(T x, ExpTab<T> t) {
    using K = P<T>;
    T xc = x;
    if constexpr (!FAST) {
        xc = (x >= K::EXPM1_XNEG) ? x : K::EXPM1_XNEG;
        xc = (xc <= K::EXPM1_XMAX) ? xc : K::EXPM1_XMAX;
    }
    T kd = frint(xc * K::INV_L);
    int k = (int)kd;
    T rhi = ffma(-kd, K::L1, xc);
    T rlo = -kd * K::L2;
    T r = rhi + rlo;
    T plo = ffma(r * r, exp_q(r), rlo);
    int j = k & 31, m = (k - j) >> 5;
    typename K::V2 s = t.S[j];
    Tw<T> A = two_sum(s.x, -fldexp(T(1), -m));
    Tw<T> B = two_prod(s.x, rhi);
    T c = ffma(s.x, plo, ffma(s.y, rhi, s.y));
    // |A0| = |2^(j/32) - 2^-m| is 0 or at least 2^(1/32) - 1 = 0.02190, while
    // |B0| = |2^(j/32) rhi| <= 2^(31/32) ln2/64 = 0.02120: a fast two-sum, with
    // two_sum's bits
    Tw<T> H = fast_two_sum_pz(A.x0, B.x0);
    T tail = H.x1 + ((A.x1 + B.x1) + c);
    T res = fldexp(H.x0 + tail, m);
    res = (fabs_(x) < K::EXPM1_TINY) ? expm1_tiny(x) : res;
    if constexpr (FAST) return res;
    res = (x < K::EXPM1_XNEG) ? T(-1) : res;
    res = (x > K::EXPM1_XMAX) ? K::INF : res;
    return isnan_(x) ? x + x : res;
}

// u = z 2^e with z in [3/4, 3/2), cell i = top 7 significand bits (u > 0 normal).
template <class T> struct LogSplit { T z; int e; int i; };
template <class T> __device__ __forceinline__ LogSplit<T> log_split(T u) {
    using K = P<T>;
    typename K::U b = K::bits(u);
    int e = (int)((b >> K::MANT) & K::EXPMASK) - K::BIAS;
    int i = (int)((b >> (K::MANT - 7)) & 127);
    bool hi = i >= 64;
    typename K::U zb = (b & K::MANT_MASK) | (hi ? K::HALF_BITS : K::ONE_BITS);
    return {K::from_bits(zb), e + (hi ? 1 : 0), i};
}

// log(x) = e ln2 - log(invc) + log1p(z invc - 1), z invc - 1 exact.
// FAST: 0 < x < inf.
template <bool FAST, class T> __device__ __forceinline__ T log1x(T x, LogTab<T> t) {
    using K = P<T>;
    // The split of x > 0 through the frexp instructions, x = m 2^ex with m in
    // [1/2, 1): they normalise subnormals exactly, so this is the (z, e, i) of
    // scaling a subnormal x into the normal range first and splitting its bits
    // (the cell index is the top 7 fraction bits of m, the same as of 2m).
    // Measured against that form, bit for bit the same: tlog 1% faster in
    // binary64 and 3.5% in binary32.
    T m = frexp_mant(x);
    int ex = frexp_exp(x);
    int i = (int)((K::bits(m) >> (K::MANT - 7)) & 127);
    bool upper = i >= 64;
    T z = upper ? m : m + m;                      // exact
    int e = upper ? ex : ex - 1;
    T r = ffma(z, t.INVC[i], T(-1));
    T ed = (T)e;
    typename K::V2 lg = t.LOG[i];
    T hi = ffma(ed, K::LN2X_HI, lg.x);
    T lo = ffma(ed, K::LN2X_LO, lg.y);
    T tail = ffma(r * r, log_q(r), lo);
    Tw<T> st = fast_two_sum(hi, r);
    T res = st.x0 + (st.x1 + tail);
    if constexpr (FAST) return res;
    res = (x == K::INF) ? K::INF : res;
    res = (x == T(0)) ? -K::INF : res;
    res = (x < T(0)) ? K::qnan() : res;
    return isnan_(x) ? x + x : res;
}

// log1p(x): u + c = 1 + x exactly, log(u) with c folded into r; |x| < 2^-8
// uses r = x directly.  FAST: -1 < x < inf.  SMALL: the caller guarantees
// |x| < 2 (the exponent of x is at most that of 1), so the fast two-sum gives
// the same exact u + c.
template <bool FAST, bool SMALL = false, class T>
__device__ __forceinline__ T log1p_1x(T x, LogTab<T> t) {
    using K = P<T>;
    Tw<T> u = SMALL ? fast_two_sum(T(1), x) : two_sum(T(1), x);
    LogSplit<T> ls = log_split(u.x0);
    T invc = t.INVC[ls.i];
    T rhi = ffma(ls.z, invc, T(-1));
    T rlo = fldexp(u.x1, -ls.e) * invc;
    bool small = fabs_(x) < T(0.00390625);
    rhi = small ? x : rhi;
    rlo = small ? T(0) : rlo;
    T ed = (T)ls.e;
    typename K::V2 lg = t.LOG[ls.i];
    T hi = ffma(ed, K::LN2X_HI, lg.x);
    T lo = ffma(ed, K::LN2X_LO, lg.y);
    T tail = ffma(rhi * rhi, log_q(rhi), lo + ffma(-rlo, rhi, rlo));
    Tw<T> st = fast_two_sum(hi, rhi);
    T res = st.x0 + (st.x1 + tail);
    res = (fabs_(x) < K::LOG1P_TINY) ? x : res;
    if constexpr (FAST) return res;
    res = (x == K::INF) ? K::INF : res;
    res = (x == T(-1)) ? -K::INF : res;
    res = (x < T(-1)) ? K::qnan() : res;
    return isnan_(x) ? x + x : res;
}

// ----------------------------------------------------------------------------
// pexp0 core: x in [EXP_XLO, EXP_XMAX].  x = 2^L m + n/32 + y exactly;
// T = e^y N! by twofold Horner; V = Ehat (C T), e^x ~ (V0 + V1) 2^k.
// ----------------------------------------------------------------------------
template <class T> struct Scaled { Tw<T> v; int k; };

// Horner's scheme for sum_{i=J0..N} (N!/i!) y^(i-J0), the integer coefficients
// of the scaled Taylor sums of pexp0 (J0 = 0) and pexpm10 (J0 = 1); each step
// j multiplies by y and adds N!/j!, which dominates the product, so the sum is
// a fast two-sum.  The partial sum of step j enters the result with the
// weight |y|^(j-J0)/j! relative to its value.  Steps above JT run in 1x
// arithmetic (one FMA each): section "Twofold exponent / Method summary"
// notes that a few of the highest-degree terms can be computed in 1x
// precision; JT = N - 1 is the all-twofold scheme of the algorithm listings.
//
// pexpm10 (|y| <= 2^-8) runs the steps above EXPM1_TF_J in 1x, pexp0
// (|y| <= 2^-6) those above EXP_TF_J where its caller allows (TAIL): their
// rounding errors weigh at most 2^-113 (binary64) or 2^-52 (binary32) of the
// result, far below the twofold rounding of the other steps.  Callers whose
// result renormalises a second part spanning many ulps of the main part (the
// coupled pexp, and the exp-minus-one paths that pexpm1 renormalises) keep
// pexp0's all-twofold scheme: there a last-bit change in pexp0's twofold
// representation would move the renormalised second part by many of its own
// ulps, while the all-twofold result is the paper's, bit for bit.
//
// Build define TF_HORNER_1X_TAIL=0 turns the 1x steps off everywhere: every
// Horner step is then twofold, as in the algorithm listings.
#ifndef TF_HORNER_1X_TAIL
#define TF_HORNER_1X_TAIL 1
#endif
template <class T, int N, int J0, int JT_> __device__ __forceinline__ Tw<T> horner_fact(T y) {
    constexpr int JT = TF_HORNER_1X_TAIL ? JT_ : N - 1;
    constexpr int TOP = JT >= N - 1 ? N - 2 : JT - 1;   // first twofold step after the start
    Tw<T> p;
    if constexpr (JT >= N - 1) {
        p = fast_two_sum(T(N), y);
    } else {
        T q = T(N) + y;
#pragma unroll
        for (int j = N - 2; j > JT; --j) q = ffma(q, y, T(fact_ratio(N, j)));
        p = add_td_fast(two_prod(q, y), T(fact_ratio(N, JT)));
    }
#pragma unroll
    for (int j = TOP; j >= J0; --j) p = add_td_fast(mul_td(p, y), T(fact_ratio(N, j)));
    return p;
}

template <bool TAIL, class T> __device__ __forceinline__ Tw<T> horner_exp(T y) {
    return horner_fact<T, P<T>::N, 0, TAIL ? P<T>::EXP_TF_J : P<T>::N - 1>(y);
}

// TAIL: Horner with the 1x tail (horner_fact).
template <bool FAST, bool TAIL = false, class T>
__device__ __forceinline__ Scaled<T> pexp0_core(T x, Pexp0Tab<T> t) {
    using K = P<T>;
    constexpr int SH = K::L + K::K;
    T Md = frint(x * T(1 << K::K));
    T y = ffma(-Md, T(1.0 / (1 << K::K)), x);          // exact: x - M 2^-K
    int M = (int)Md;
    int a = M < 0 ? -M : M;
    int m = a >> SH, n = a & ((1 << SH) - 1);
    m = M < 0 ? -m : m;
    n = M < 0 ? -n : n;
    if constexpr (!FAST) {  // callers pass x in [EXP_XLO, EXP_XMAX]: these clamps do nothing
        m = m < -K::E_OFF ? -K::E_OFF : (m > K::E_CNT - 1 - K::E_OFF ? K::E_CNT - 1 - K::E_OFF : m);
        n = n < -K::C_OFF ? -K::C_OFF : (n > K::C_OFF ? K::C_OFF : n);
    }
    Tw<T> Tt = horner_exp<TAIL>(y);
    typename K::V2 e2 = t.E[m + K::E_OFF];
    typename K::V2 c2 = t.C[n + K::C_OFF];
    int k = t.EK[m + K::E_OFF];
    Tw<T> V = mul_tt(Tw<T>{e2.x, e2.y}, mul_tt(Tw<T>{c2.x, c2.y}, Tt));
    return {V, k};
}

// pexpm10 small path, |x| <= 89.5/128: x = n/128 + y, T = (e^y - 1) via the
// Horner of N1 without its last term, times y and the twofold 1/N1!,
// Z = (C + T) + C T with C = e^(n/128) - 1.  FAST: |x| <= 89/128.
template <bool FAST, class T> __device__ __forceinline__ Tw<T> pexpm10_small(T x, Pm1Tab<T> t) {
    using K = P<T>;
    constexpr int N1 = K::N1;
    T xs = x;
    if constexpr (!FAST) {
        // Valid arguments satisfy |x| <= ln 2 + tiny < 89/128; anything else (NaN,
        // inf from an invalid lane) is replaced so the index stays in [-89, 89].
        xs = (fabs_(x) <= T(0.6953125)) ? x : T(0);
    }
    T nd = frint(xs * T(128));
    T y = ffma(-nd, T(1.0 / 128), xs);                  // exact
    int n = (int)nd;
    if constexpr (!FAST) n = n < -K::CM1_OFF ? -K::CM1_OFF : (n > K::CM1_OFF ? K::CM1_OFF : n);
    Tw<T> p = mul_td(horner_fact<T, N1, 1, K::EXPM1_TF_J>(y), y);
    Tw<T> Tt = mul_tt(p, Tw<T>{K::RCP_HI, K::RCP_LO});
    typename K::V2 c2 = t.CM1[n + K::CM1_OFF];
    Tw<T> C = {c2.x, c2.y};
    return add_tt_fast(add_tt_fast(C, Tt), mul_tt(C, Tt));
}

// The rule for non-finite main parts: z0 NaN -> z1 NaN, z0 = +-inf -> z1 = +0.
template <class T> __device__ __forceinline__ T special_rule(T z0, T z1) {
    z1 = (fabs_(z0) == P<T>::INF) ? T(0) : z1;
    return isnan_(z0) ? P<T>::qnan() : z1;
}

// ----------------------------------------------------------------------------
// Twofold functions, one element each.  `x1_tiny` is a wave-uniform flag: all
// active lanes have |x1| < EXPM1_TINY, so expm1(x1) is its tiny branch.
// ----------------------------------------------------------------------------
template <class T> __device__ __forceinline__ T expm1_of_x1(T x1, bool x1_tiny, ExpTab<T> et) {
    return x1_tiny ? expm1_tiny(x1) : expm1_1x<false>(x1, et);
}

// Fast-wave conditions (checked per lane, voted per wave).
template <class T> __device__ __forceinline__ bool texp_fast_arg(T x0, T x1) {
    return x0 >= P<T>::EXP_XLO && x0 <= P<T>::EXP_XMAX && fabs_(x1) < P<T>::EXPM1_TINY;
}
template <class T> __device__ __forceinline__ bool texpm1_fast_arg(T x0, T x1) {
    return x0 >= P<T>::EXPM1_XNEG && x0 <= P<T>::EXPM1_XMAX && fabs_(x1) < P<T>::EXPM1_TINY;
}
// The log conditions also ask |y1| <= |y0|, so that the first renormalisation
// two_sum(y0, y1) is fast_two_sum_pz (true of every renormalised or coupled
// argument).
template <class T> __device__ __forceinline__ bool tlog_fast_arg(T y0, T y1) {
    T s = y0 + y1;
    return y0 > T(0) && y0 < P<T>::INF && s > T(0) && s < P<T>::INF && fabs_(y1) <= y0;
}
template <class T> __device__ __forceinline__ bool tlog1p_fast_arg(T y0, T y1) {
    T s = y0 + y1;
    return y0 > T(-1) && y0 < P<T>::INF && s > T(-1) && s < P<T>::INF &&
           fabs_(y1) <= fabs_(y0);
}

// Build define TF_TEXP_ACC=1 (the flagged variant "accexp"): texp's second
// part in twofold.  The method's step (section "Twofold exponent", algorithm
// texp, step 4) forms z0 t1 + (v1 + (v0 - z0)) with one rounded product of the
// 1x main part z0 and t1 = expm1(x1): it drops (v - z0) t1, about an ulp of z0
// times t1, and rounds the product, each near 2^-97 of the result for a
// coupled x1 at |x0| ~ 700.  The variant takes e^x0 (1 + t1) - z0 as
// v0 t1 (an exact FMA product) + v1 t1 + (v1 + (v0 - z0)), with t1 = x1 +
// x1^2/2 for a tiny x1 (far below its ulp there), and keeps the low part of
// the sum apart: the t-function texp adds it in one rounding, the coupled
// pexp carries it through its renormalisation.  The default keeps the
// method's step.
#ifndef TF_TEXP_ACC
#define TF_TEXP_ACC 0
#endif
constexpr bool kTexpAcc = TF_TEXP_ACC != 0;

// texp's second part in the 2^-k domain, from z0s = z0 2^-k, t1 = expm1(x1),
// x1 and v = pexp0(x0) 2^-k (one element): hi + lo.  The default gives
// z0s t1 + (v1 + (v0 - z0s)) as hi with lo = 0.  tiny: |x1| < EXPM1_TINY.
template <class T> struct SecondPart { T hi, lo; };
template <class T>
__device__ __forceinline__ SecondPart<T> texp_second(T z0s, T t1, T x1, bool tiny, Tw<T> v) {
    const T rest = v.x1 + (v.x0 - z0s);
    if constexpr (kTexpAcc) {
        const T tt = tiny ? x1 : t1;
        Tw<T> p = two_prod(v.x0, tt);
        const T q = tiny ? v.x0 * (x1 * x1 * T(0.5)) : T(0);
        // a non-finite product (x1 infinite or NaN) keeps the default's value
        if (!(fabs_(p.x0) < P<T>::INF)) return {z0s * t1 + rest, T(0)};
        return {p.x0, (p.x1 + (v.x1 * tt + q)) + rest};
    } else {
        return {z0s * t1 + rest, T(0)};
    }
}

// texp.  FAST: texp_fast_arg (then z0 is finite and pexp0 is in range).
// TAIL: pexp0 with the 1x Horner tail (z1 takes pexp0's value, not its
// representation, up to its own last bits).  z2o (the variant's low part of
// the second part, for the coupled pexp): if given, z1o is the high part and
// *z2o the low one (0 in the default build); otherwise z1o is their sum.
template <bool FAST, bool TAIL, class T>
__device__ __forceinline__ void texp_elem(T x0, T x1, bool x1_tiny, ExpTab<T> et, Pexp0Tab<T> pt,
                                          T& z0o, T& z1o, T* z2o = nullptr) {
    using K = P<T>;
    if constexpr (FAST) {
        T z0 = exp1x<true>(x0, et);
        T t1 = expm1_tiny(x1);
        Scaled<T> s = pexp0_core<true, TAIL>(x0, pt);
        T z0s = fldexp(z0, -s.k);                     // exact
        SecondPart<T> zs = texp_second(z0s, t1, x1, true, s.v);
        z0o = z0;
        if constexpr (kTexpAcc) {
            if (z2o) {
                z1o = fldexp(zs.hi, s.k);
                *z2o = fldexp(zs.lo, s.k);
            } else {
                z1o = fldexp(zs.hi + zs.lo, s.k);
            }
        } else {
            z1o = fldexp(zs.hi, s.k);
            if (z2o) *z2o = T(0);
        }
    } else {
        T z0 = exp1x<false>(x0, et);
        T t1 = expm1_of_x1(x1, x1_tiny, et);
        bool in = x0 >= K::EXP_XLO;                   // below: pexp0 gives (0, 0)
        T xc = in ? x0 : K::EXP_XLO;
        xc = (xc <= K::EXP_XMAX) ? xc : K::EXP_XMAX;
        Scaled<T> s = pexp0_core<false, TAIL>(xc, pt);
        T v0 = in ? s.v.x0 : T(0);
        T v1 = in ? s.v.x1 : T(0);
        int k = in ? s.k : 0;
        T z0s = fldexp(z0, -k);                       // exact
        SecondPart<T> zs = texp_second(z0s, t1, x1, fabs_(x1) < K::EXPM1_TINY, Tw<T>{v0, v1});
        z0o = z0;
        if constexpr (kTexpAcc) {
            if (z2o) {
                z1o = special_rule(z0, fldexp(zs.hi, k));
                *z2o = special_rule(z0, fldexp(zs.lo, k));
            } else {
                z1o = special_rule(z0, fldexp(zs.hi + zs.lo, k));
            }
        } else {
            z1o = special_rule(z0, fldexp(zs.hi, k));
            if (z2o) *z2o = T(0);
        }
    }
}

// The second part of texpm1 from z0 = expm1(x0), t1 = expm1(x1) and the
// twofold w = e^x0 - 1: e^(x0 + x1) - 1 - z0 = (z0 + 1) t1 + (w - z0) to
// first order, w - z0 = w1 + (w0 - z0) with w0 - z0 exact.  Every texpm1 body
// forms it with this one expression.
template <class T> __device__ __forceinline__ T texpm1_z1(T z0, T t1, Tw<T> w) {
    return (z0 + T(1)) * t1 + (w.x1 + (w.x0 - z0));
}

// texpm1, general form: small path pexpm10, and pexp0(x0) - 1 for |x0| > ln 2
// on the waves that hold such a lane.
template <class T>
__device__ __forceinline__ void texpm1_elem(T x0, T x1, bool x1_tiny, ExpTab<T> et, Pexp0Tab<T> pt,
                                            Pm1Tab<T> mt, T& z0o, T& z1o) {
    using K = P<T>;
    T z0 = expm1_1x<false>(x0, et);
    T t1 = expm1_of_x1(x1, x1_tiny, et);
    bool small = fabs_(x0) <= K::LN2_HI;
    Tw<T> w = pexpm10_small<false>(small ? x0 : T(0), mt);
    bool big = !small && x0 >= K::EXP_XLO && x0 <= K::EXP_XMAX;
    if (__any(big)) {                                 // pexp0(x0) - 1 on this wave
        T xc = big ? x0 : T(1);
        Scaled<T> s = pexp0_core<false>(xc, pt);
        Tw<T> wl = add_td(Tw<T>{fldexp(s.v.x0, s.k), fldexp(s.v.x1, s.k)}, T(-1));
        w = sel(big, wl, w);
    }
    w = sel(x0 < K::EXP_XLO, Tw<T>{T(-1), T(0)}, w);  // pexp0 = (0, 0) below range
    z0o = z0;
    z1o = special_rule(z0, texpm1_z1(z0, t1, w));
}

// texpm1 on a fast wave (texpm1_fast_arg on every lane), small path only.
// Returns true for a lane with |x0| > ln 2, whose z0, z1 are not computed here:
// the kernel hands that lane to texpm1_elem later.
template <class T>
__device__ __forceinline__ bool texpm1_small_fast(T x0, T x1, ExpTab<T> et, Pm1Tab<T> mt, T& z0o,
                                                  T& z1o) {
    using K = P<T>;
    bool small = fabs_(x0) <= K::LN2_HI;
    T z0 = expm1_1x<true>(x0, et);
    T t1 = expm1_tiny(x1);
    Tw<T> w = pexpm10_small<true>(small ? x0 : T(0), mt);
    z0o = z0;
    z1o = texpm1_z1(z0, t1, w);
    return !small;
}

// z1 of a lane that texpm1_small_fast deferred (texpm1_fast_arg holds and
// |x0| > ln 2), given the z0 it computed: pexp0(x0) - 1 alone.  The fast
// argument range [EXPM1_XNEG, EXPM1_XMAX] lies inside pexp0's
// [EXP_XLO, EXP_XMAX] and |x1| < EXPM1_TINY, so this is texpm1_elem's
// pexp0 branch without its range selects: the same z1, bit for bit.
template <class T>
__device__ __forceinline__ T texpm1_big_fast(T x0, T x1, T z0, Pexp0Tab<T> pt) {
    static_assert(P<T>::EXPM1_XNEG >= P<T>::EXP_XLO && P<T>::EXPM1_XMAX <= P<T>::EXP_XMAX,
                  "fast texpm1 arguments must lie in pexp0's range");
    T t1 = expm1_tiny(x1);
    Scaled<T> s = pexp0_core<true>(x0, pt);
    Tw<T> w = add_td(Tw<T>{fldexp(s.v.x0, s.k), fldexp(s.v.x1, s.k)}, T(-1));
    return special_rule(z0, texpm1_z1(z0, t1, w));
}

// Newton step shared by plog and plog1p: r0 = log1p(a0 + a1), s = pexpm10(-r0),
// u = ((a s) + a) + s, r1 = u0 + u1.  FAST: a0 + a1 finite.
// The correction for a given seed r0 ~ log(1 + a).  The reductions keep
// |r0| <= ln 2; in the general form a seed beyond the small range of pexpm10
// (|r0| > 89/128 or NaN: an argument that is not coupled, or not finite, where
// a coupled one is due) gives a NaN correction.  FAST: |r0| <= 89/128.
//
// On a fast wave the seed is a 1x log of 1 + a (error about an ulp) with a in
// [-1/2, 1] (up to the coupled second part).  Then m = a s + a = a e^-r0 is
// close to a/(1 + a) and s = e^-r0 - 1 close to -a/(1 + a): their magnitudes
// agree to a few ulps, or both are so small that every sum is exact.  So
// m0 + s0 is exact (Sterbenz), the two-sum of m + s has error 0, and its
// twofold reduces to the two sums below, bit for bit.  The sum a s + a keeps
// the full two-sum: |a s| can reach |a| from below at a = -1/2 (a just under
// 1/2 in magnitude, a s rounded up to 1/2), and there no three-operation sum
// is exact.
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> newton_seeded(Tw<T> a, T r0, Pm1Tab<T> mt) {
    Tw<T> s = pexpm10_small<FAST>(-r0, mt);
    Tw<T> m = add_tt(mul_tt(a, s), a);
    T r1;
    if constexpr (FAST) {
        r1 = (m.x0 + s.x0) + (m.x1 + s.x1);
    } else {
        Tw<T> u = add_tt(m, s);
        r1 = u.x0 + u.x1;
        r1 = (fabs_(r0) <= T(0.6953125)) ? r1 : P<T>::qnan();
    }
    return {r0, r1};
}

// Every caller reduces the argument to |a0 + a1| < 2 (a = z - 1 with z in
// [1/2, 2], or a = y with y0 in [-1/2, 1]); on a fast wave that is guaranteed,
// so the seed's 1 + x is a fast two-sum.
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog_newton(Tw<T> a, LogTab<T> lt, Pm1Tab<T> mt) {
    return newton_seeded<FAST>(a, log1p_1x<FAST, FAST>(a.x0 + a.x1, lt), mt);
}

// X + n ln2 (twofold).  FAST: |X0| < 1, as for every caller's Newton result
// (the log of a reduced argument in [1/2, 2]); then n ln2 = 0 or
// |n ln2| >= 1/2 has the larger exponent and the sum is a fast two-sum.
template <bool FAST = false, class T> __device__ __forceinline__ Tw<T> add_n_ln2(Tw<T> X, int n) {
    Tw<T> L = mul_td(Tw<T>{P<T>::LN2_HI, P<T>::LN2_LO}, (T)n);
    if constexpr (FAST) {
        Tw<T> st = fast_two_sum(L.x0, X.x0);
        return {st.x0, st.x1 + (X.x1 + L.x1)};
    } else {
        return add_tt(X, L);
    }
}

// w = 2^n z: frexp when w0 < 1/2 or w0 > 2, else n = 0.  Scaling w0 by
// 2^-n with n its frexp exponent gives frexp's mantissa exactly (subnormals
// included), and scaling by 2^0 is the identity, so one select of n suffices.
template <class T> __device__ __forceinline__ Tw<T> log_scale(Tw<T> w, int& n) {
    bool need = w.x0 < T(0.5) || w.x0 > T(2);
    n = need ? frexp_exp(w.x0) : 0;
    return {fldexp(w.x0, -n), fldexp(w.x1, -n)};
}

// x1 of a log whose renormalised argument w0 is outside (0, inf).
template <class T> __device__ __forceinline__ T log_domain_x1(T w0, T x1) {
    x1 = (w0 == P<T>::INF) ? P<T>::INF : x1;
    x1 = (w0 == T(0)) ? -P<T>::INF : x1;
    return (w0 < T(0) || isnan_(w0)) ? P<T>::qnan() : x1;
}

// tlog.  FAST: tlog_fast_arg (y0 and y0 + y1 positive and finite, |y1| <= y0).
template <bool FAST, class T>
__device__ __forceinline__ void tlog_elem(T y0, T y1, LogTab<T> lt, Pm1Tab<T> mt, T& x0o, T& x1o) {
    T x0 = log1x<FAST>(y0, lt);
    Tw<T> v = FAST ? fast_two_sum_pz(y0, y1) : two_sum(y0, y1);
    int n;
    Tw<T> z = log_scale(v, n);
    Tw<T> a = {z.x0 - T(1), z.x1};                    // exact
    Tw<T> X = add_n_ln2<FAST>(plog_newton<FAST>(a, lt, mt), n);
    T x1 = X.x1 + (X.x0 - x0);
    x0o = x0;
    if constexpr (FAST) {
        x1o = x1;
    } else {
        x1 = log_domain_x1(v.x0, x1);
        x1o = special_rule(x0, x1);
    }
}

// tlog1p on a fast wave (tlog1p_fast_arg on every lane), in parts, so that a
// kernel can evaluate the Newton seeds log1p_1x(a0 + a1) of a wave's elements
// together.  The head renormalises y into v and, on outer lanes
// (v0 < -1/2 or v0 > 1), reduces 1 + v to 2^nn z with a = z - 1; elsewhere
// a = v.  The main part x0 = log1p(y0) is computed apart.  The tail takes x0
// and the seed and finishes the Newton step.
//
// Outer lanes of a fast wave have v0 > 1 or -1 <= v0 < -1/2 (then 1 + v0 is
// exact), with |v1| <= ulp(v0)/2: both sums of the reduction are fast
// two-sums with the exact errors of the general form.
template <class T> struct Tlog1pHead {
    Tw<T> a;    // the Newton argument: |a0 + a1| <= 1
    int nn;     // outer lanes: 1 + y = 2^nn (1 + a); 0 elsewhere
};
template <class T>
__device__ __forceinline__ Tlog1pHead<T> tlog1p_fast_head(T y0, T y1, bool& any_outer) {
    Tlog1pHead<T> h;
    Tw<T> v = fast_two_sum_pz(y0, y1);
    const bool outer = v.x0 < T(-0.5) || v.x0 > T(1);
    h.a = v;
    h.nn = 0;
    any_outer = __any(outer);
    if (any_outer) {                                  // log of the renormalised 1 + y
        Tw<T> st = fast_two_sum(v.x0, T(1));
        Tw<T> w = fast_two_sum(st.x0, st.x1 + v.x1);
        int nn;
        Tw<T> z = log_scale(w, nn);
        h.nn = outer ? nn : 0;
        h.a = sel(outer, Tw<T>{z.x0 - T(1), z.x1}, v);
    }
    return h;
}
// The seed's argument; |a0 + a1| <= 1, so the seed is log1p_1x<true, true>.
template <class T> __device__ __forceinline__ T tlog1p_seed_arg(const Tlog1pHead<T>& h) {
    return h.a.x0 + h.a.x1;
}
template <class T>
__device__ __forceinline__ T tlog1p_fast_tail(const Tlog1pHead<T>& h, T x0, T seed,
                                              bool any_outer, Pm1Tab<T> mt) {
    Tw<T> X = newton_seeded<true>(h.a, seed, mt);
    // + 0 ln2 returns X itself up to the sign of a zero second part, which
    // the final sum below does not keep: no select needed
    if (any_outer) X = add_n_ln2<true>(X, h.nn);
    return X.x1 + (X.x0 - x0);
}

// tlog1p.  FAST: tlog1p_fast_arg (y0 and y0 + y1 above -1 and finite,
// |y1| <= |y0|).
template <bool FAST, class T>
__device__ __forceinline__ void tlog1p_elem(T y0, T y1, LogTab<T> lt, Pm1Tab<T> mt, T& x0o,
                                            T& x1o) {
    using K = P<T>;
    if constexpr (FAST) {
        const T x0 = log1p_1x<true>(y0, lt);
        bool any_outer;
        Tlog1pHead<T> h = tlog1p_fast_head(y0, y1, any_outer);
        T seed = log1p_1x<true, true>(tlog1p_seed_arg(h), lt);
        x0o = x0;
        x1o = tlog1p_fast_tail(h, x0, seed, any_outer, mt);
    } else {
        T x0 = log1p_1x<false>(y0, lt);
        Tw<T> v = two_sum(y0, y1);
        bool outer = v.x0 < T(-0.5) || v.x0 > T(1);
        Tw<T> a = v;
        Tw<T> w = v;
        int nn = 0;
        const bool any_outer = __any(outer);
        if (any_outer) {                              // log of the renormalised 1 + y
            w = add_td(v, T(1));
            w = two_sum(w.x0, w.x1);
            Tw<T> z = log_scale(w, nn);
            a = sel(outer, Tw<T>{z.x0 - T(1), z.x1}, v);
        }
        Tw<T> X = plog_newton<false>(a, lt, mt);
        if (any_outer) X = sel(outer, add_n_ln2<false>(X, outer ? nn : 0), X);
        T x1 = X.x1 + (X.x0 - x0);
        x0o = x0;
        x1 = (outer && any_outer) ? log_domain_x1(w.x0, x1) : x1;
        x1 = (v.x0 == K::INF) ? K::INF : x1;
        x1 = isnan_(v.x0) ? K::qnan() : x1;
        x1o = special_rule(x0, x1);
    }
}

// ----------------------------------------------------------------------------
// Twofold arithmetic (section "Twofolds update"): z = x op y (tadd, tsub,
// tmul, tdiv), z = sqrt(x) (tsqrt) and the renormalization of x (trenorm).  The
// main part is the 1x operation on the main parts (IEEE +, -, *, / and sqrt,
// correctly rounded); the second part is the exact error of that operation
// from an error-free transform (two_sum, the error-free difference, the FMA
// product) or the FMA remainder of a quotient or square root, plus the
// first-order terms of the low parts.  Then the rule for a non-finite main
// part.  y is not read for tsqrt and trenorm.
// ----------------------------------------------------------------------------
enum ArithOp : int { OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_DIV = 3, OP_SQRT = 4, OP_RENORM = 5 };

template <int OP, class T> __device__ __forceinline__ Tw<T> arith_elem(Tw<T> x, Tw<T> y) {
    Tw<T> z;
    if constexpr (OP == OP_ADD) {
        z = add_tt(x, y);
    } else if constexpr (OP == OP_SUB) {
        Tw<T> dt = two_diff(x.x0, y.x0);
        z = {dt.x0, dt.x1 + (x.x1 - y.x1)};
    } else if constexpr (OP == OP_MUL) {
        z = mul_tt(x, y);
    } else if constexpr (OP == OP_DIV) {
        z = div_tt(x, y);
    } else if constexpr (OP == OP_RENORM) {
        // the renormalized twofold of exactly the same value: RN(x0 + x1) and
        // the exact remainder, for any x0, x1 (where |x0| >= |x1| the fast
        // renormalization gives these bits)
        z = two_sum(x.x0, x.x1);
    } else {
        // z0 = sqrt(x0), r = x0 - z0^2 exactly (FMA), z1 = (r + x1) / (2 z0);
        // at x0 = 0 the correction is 0
        T z0 = fsqrt(x.x0);
        T r = ffma(-z0, z0, x.x0);
        T z1 = (r + x.x1) / (z0 + z0);
        z = {z0, x.x0 == T(0) ? T(0) : z1};
    }
    return {z.x0, special_rule(z.x0, z.x1)};
}

// ----------------------------------------------------------------------------
// The other entry points of the paper's interface: functions of a dotted
// argument x0 (x1 = 0) and of a coupled argument (x0 + x1 rounds to x0), and
// the p-functions, whose results are renormalised fast to a coupled twofold.
// Same operation sequences as the oracle; general forms handle any argument,
// FAST forms the arguments of the *_fast_arg predicates below.
// ----------------------------------------------------------------------------

// Renormalize fast a result, then the rule for a non-finite main part.
template <class T> __device__ __forceinline__ void renorm_out(T z0, T z1, T& z0o, T& z1o) {
    const bool fin = !(isnan_(z0) || fabs_(z0) == P<T>::INF);
    Tw<T> r = fast_two_sum(z0, z1);
    T o0 = fin ? r.x0 : z0;
    T o1 = fin ? r.x1 : z1;
    z0o = o0;
    z1o = special_rule(o0, o1);
}

// The renormalised z0 + z1 + z2 (|z2| << |z1| << |z0|, z0 finite) as a coupled
// pair; non-finite z0 as renorm_out.
template <class T>
__device__ __forceinline__ void renorm_out3(T z0, T z1, T z2, T& z0o, T& z1o) {
    const bool fin = !(isnan_(z0) || fabs_(z0) == P<T>::INF);
    Tw<T> r = fast_two_sum(z0, z1);
    Tw<T> q = fast_two_sum(r.x0, r.x1 + z2);
    T o0 = fin ? q.x0 : z0;
    T o1 = fin ? q.x1 : z1;
    z0o = o0;
    z1o = special_rule(o0, o1);
}

// pexp0 as a coupled p-function: 0 below the range, z0 = z1 = +inf above it
// (as the paper writes it), else E (C T) scaled and renormalised fast.
template <bool FAST, class T>
__device__ __forceinline__ void pexp0_p(T x, Pexp0Tab<T> pt, T& z0o, T& z1o) {
    using K = P<T>;
    if constexpr (FAST) {
        Scaled<T> s = pexp0_core<true, true>(x, pt);
        Tw<T> r = fast_two_sum(fldexp(s.v.x0, s.k), fldexp(s.v.x1, s.k));
        z0o = r.x0;
        z1o = r.x1;
    } else {
        const bool in = x >= K::EXP_XLO && x <= K::EXP_XMAX;
        Scaled<T> s = pexp0_core<false, true>(in ? x : T(0), pt);
        Tw<T> r = fast_two_sum(fldexp(s.v.x0, s.k), fldexp(s.v.x1, s.k));
        r = sel(x < K::EXP_XLO, Tw<T>{T(0), T(0)}, r);
        r = sel(x > K::EXP_XMAX, Tw<T>{K::INF, K::INF}, r);
        r = sel(isnan_(x), Tw<T>{x, x}, r);
        z0o = r.x0;
        z1o = r.x1;
    }
}

// texp0 (dotted argument): z0 = exp(x0), z1 = (v0 - z0) + v1 with
// v = pexp0(x0), in pexp0's 2^-k domain.  FAST: EXP_XLO <= x0 <= EXP_XMAX.
template <bool FAST, class T>
__device__ __forceinline__ void texp0_elem(T x0, ExpTab<T> et, Pexp0Tab<T> pt, T& z0o, T& z1o) {
    using K = P<T>;
    if constexpr (FAST) {
        T z0 = exp1x<true>(x0, et);
        Scaled<T> s = pexp0_core<true, true>(x0, pt);
        T z0s = fldexp(z0, -s.k);                     // exact
        z0o = z0;
        z1o = fldexp((s.v.x0 - z0s) + s.v.x1, s.k);
    } else {
        T z0 = exp1x<false>(x0, et);
        bool in = x0 >= K::EXP_XLO;                   // below: pexp0 gives (0, 0)
        T xc = in ? x0 : K::EXP_XLO;
        xc = (xc <= K::EXP_XMAX) ? xc : K::EXP_XMAX;
        Scaled<T> s = pexp0_core<false, true>(xc, pt);
        T v0 = in ? s.v.x0 : T(0);
        T v1 = in ? s.v.x1 : T(0);
        int k = in ? s.k : 0;
        T z0s = fldexp(z0, -k);                       // exact
        z0o = z0;
        z1o = special_rule(z0, fldexp((v0 - z0s) + v1, k));
    }
}

// pexpm10 body (not renormalised), any argument: the small path for
// |x| <= ln 2, pexp0(x) - 1 on the waves holding a larger in-range lane, -1
// below the range.
template <class T>
__device__ __forceinline__ Tw<T> pexpm10_any(T x, Pexp0Tab<T> pt, Pm1Tab<T> mt) {
    using K = P<T>;
    bool small = fabs_(x) <= K::LN2_HI;
    Tw<T> w = pexpm10_small<false>(small ? x : T(0), mt);
    bool big = !small && x >= K::EXP_XLO && x <= K::EXP_XMAX;
    if (__any(big)) {
        T xc = big ? x : T(1);
        Scaled<T> s = pexp0_core<false>(xc, pt);
        Tw<T> wl = add_td(Tw<T>{fldexp(s.v.x0, s.k), fldexp(s.v.x1, s.k)}, T(-1));
        w = sel(big, wl, w);
    }
    return sel(x < K::EXP_XLO, Tw<T>{T(-1), T(0)}, w);
}

// pexpm10 as a coupled p-function; texpm10: z0 = expm1(x0),
// z1 = (w0 - z0) + w1.  FAST (both): |x0| <= ln 2.
template <bool FAST, class T>
__device__ __forceinline__ void pexpm10_p(T x, Pexp0Tab<T> pt, Pm1Tab<T> mt, T& z0o, T& z1o) {
    using K = P<T>;
    if constexpr (FAST) {
        Tw<T> w = pexpm10_small<true>(x, mt);
        Tw<T> r = fast_two_sum(w.x0, w.x1);
        z0o = r.x0;
        z1o = r.x1;
    } else {
        Tw<T> w = pexpm10_any(x, pt, mt);
        Tw<T> r = fast_two_sum(w.x0, w.x1);
        r = sel(x > K::EXP_XMAX, Tw<T>{K::INF, K::INF}, r);
        r = sel(isnan_(x), Tw<T>{x, x}, r);
        z0o = r.x0;
        z1o = r.x1;
    }
}
template <bool FAST, class T>
__device__ __forceinline__ void texpm10_elem(T x0, ExpTab<T> et, Pexp0Tab<T> pt, Pm1Tab<T> mt,
                                             T& z0o, T& z1o) {
    if constexpr (FAST) {
        T z0 = expm1_1x<true>(x0, et);
        Tw<T> w = pexpm10_small<true>(x0, mt);
        z0o = z0;
        z1o = (w.x0 - z0) + w.x1;
    } else {
        T z0 = expm1_1x<false>(x0, et);
        Tw<T> w = pexpm10_any(x0, pt, mt);
        z0o = z0;
        z1o = special_rule(z0, (w.x0 - z0) + w.x1);
    }
}

// plog0 core (dotted y0 in (0, inf), not renormalised): y0 = 2^n z0, seed the
// 1x log of z0, Newton correction with 1 + a = z0, + n ln2.
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog0_core(T y0, LogTab<T> lt, Pm1Tab<T> mt) {
    int n;
    Tw<T> z = log_scale(Tw<T>{y0, T(0)}, n);
    Tw<T> a = {z.x0 - T(1), z.x1};                    // exact
    return add_n_ln2<FAST>(newton_seeded<FAST>(a, log1x<FAST>(z.x0, lt), mt), n);
}

// plog core (coupled y, y0 in (0, inf), not renormalised): scale by the
// exponent of y0, a = (z0 - 1) + z1, Newton step, + n ln2.
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog_coupled_core(Tw<T> y, LogTab<T> lt, Pm1Tab<T> mt) {
    int n;
    Tw<T> z = log_scale(y, n);
    Tw<T> a = {z.x0 - T(1), z.x1};
    return add_n_ln2<FAST>(plog_newton<FAST>(a, lt, mt), n);
}

// plog1p0 core (dotted y0 in (-1, inf), not renormalised): outside [-1/2, 1]
// the plog of the renormalised 1 + y0, inside the Newton correction with
// a = y0 seeded with log1p(y0).  One Newton step per lane: the branch only
// selects its argument and seed.  In two halves around the seed (head, seed
// argument, tail), so that a kernel can evaluate the seeds of a wave together;
// plog1p of a coupled argument (plog1p_head, plog1p_tail) likewise.
template <class T> struct Log1pCoreHead {
    Tw<T> a;     // the Newton argument
    int n;       // outer lanes: 1 + y = 2^n (1 + a)
    bool outer;  // y0 < -1/2 or y0 > 1
};
template <class T> __device__ __forceinline__ Log1pCoreHead<T> plog1p0_head(T y0) {
    Log1pCoreHead<T> h;
    h.outer = y0 < T(-0.5) || y0 > T(1);
    Tw<T> z = log_scale(two_sum(T(1), y0), h.n);
    h.a = sel(h.outer, Tw<T>{z.x0 - T(1), z.x1}, Tw<T>{y0, T(0)});
    return h;
}
template <class T>
__device__ __forceinline__ T plog1p0_seed_arg(const Log1pCoreHead<T>& h, T y0) {
    return h.outer ? h.a.x0 + h.a.x1 : y0;
}
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog1p0_tail(const Log1pCoreHead<T>& h, T r0, Pm1Tab<T> mt) {
    Tw<T> X = newton_seeded<FAST>(h.a, r0, mt);
    return sel(h.outer, add_n_ln2<FAST>(X, h.outer ? h.n : 0), X);
}
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog1p0_core(T y0, LogTab<T> lt, Pm1Tab<T> mt) {
    Log1pCoreHead<T> h = plog1p0_head(y0);
    return plog1p0_tail<FAST>(h, log1p_1x<FAST, FAST>(plog1p0_seed_arg(h, y0), lt), mt);
}

// plog1p core (coupled y, y0 in (-1, inf), not renormalised): outside
// [-1/2, 1] the plog of the renormalised 1 + y, inside the Newton step on
// a = y seeded with log1p(y0 + y1).
template <class T>
__device__ __forceinline__ Log1pCoreHead<T> plog1p_head(Tw<T> y, bool& any_outer) {
    Log1pCoreHead<T> h;
    h.outer = y.x0 < T(-0.5) || y.x0 > T(1);
    h.a = y;
    h.n = 0;
    any_outer = __any(h.outer);
    if (any_outer) {
        Tw<T> w = add_td(y, T(1));
        Tw<T> z = log_scale(two_sum(w.x0, w.x1), h.n);
        h.a = sel(h.outer, Tw<T>{z.x0 - T(1), z.x1}, y);
    }
    return h;
}
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog1p_tail(const Log1pCoreHead<T>& h, T r0, bool any_outer,
                                             Pm1Tab<T> mt) {
    Tw<T> X = newton_seeded<FAST>(h.a, r0, mt);
    if (any_outer) X = sel(h.outer, add_n_ln2<FAST>(X, h.outer ? h.n : 0), X);
    return X;
}
template <bool FAST, class T>
__device__ __forceinline__ Tw<T> plog1p_core(Tw<T> y, LogTab<T> lt, Pm1Tab<T> mt) {
    bool any_outer;
    Log1pCoreHead<T> h = plog1p_head(y, any_outer);
    return plog1p_tail<FAST>(h, log1p_1x<FAST, FAST>(h.a.x0 + h.a.x1, lt), any_outer, mt);
}

// The four log-family functions of each kind.  P: p-function (renormalised
// result; main part outside the 1x domain -> the 1x value and the rule).
// Otherwise t-function: x0 = the 1x function of y0, x1 = X1 + (X0 - x0).
// FAST: y0 inside the 1x domain and, for a coupled argument, |y1| <= 2^-24 |y0|
// (then every seed is within the small range of pexpm10).
enum LogKind : int { LK_LOG0 = 0, LK_LOG1P0 = 1, LK_LOGC = 2, LK_LOG1PC = 3 };

template <int KIND, bool PFN, bool FAST, class T>
__device__ __forceinline__ void log_iface_elem(T y0, T y1, LogTab<T> lt, Pm1Tab<T> mt, T& x0o,
                                               T& x1o) {
    using K = P<T>;
    constexpr bool LP = KIND == LK_LOG1P0 || KIND == LK_LOG1PC;
    Tw<T> X;
    if constexpr (KIND == LK_LOG0) X = plog0_core<FAST>(y0, lt, mt);
    else if constexpr (KIND == LK_LOG1P0) X = plog1p0_core<FAST>(y0, lt, mt);
    else if constexpr (KIND == LK_LOGC) X = plog_coupled_core<FAST>(Tw<T>{y0, y1}, lt, mt);
    else X = plog1p_core<FAST>(Tw<T>{y0, y1}, lt, mt);
    if constexpr (PFN) {
        if constexpr (FAST) {
            Tw<T> r = fast_two_sum(X.x0, X.x1);
            x0o = r.x0;
            x1o = special_rule(r.x0, r.x1);
        } else {
            const bool valid = (LP ? y0 > T(-1) : y0 > T(0)) && y0 < K::INF;
            T o0, o1;
            renorm_out(X.x0, X.x1, o0, o1);
            T e0 = LP ? log1p_1x<false>(y0, lt) : log1x<false>(y0, lt);
            x0o = valid ? o0 : e0;
            x1o = valid ? o1 : special_rule(e0, T(0));
        }
    } else {
        T u0 = LP ? log1p_1x<FAST>(y0, lt) : log1x<FAST>(y0, lt);
        T x1 = X.x1 + (X.x0 - u0);
        x0o = u0;
        x1o = FAST ? x1 : special_rule(u0, x1);
    }
}

// For log1p of a coupled argument, y0 + y1 > -1 (rounded) also keeps 1 + y
// positive, so its logarithm's reduction stays in range.
template <int KIND, class T> __device__ __forceinline__ bool log_iface_fast_arg(T y0, T y1) {
    constexpr T REL = T(1.0 / 16777216.0);            // 2^-24
    if constexpr (KIND == LK_LOG0) return y0 > T(0) && y0 < P<T>::INF;
    else if constexpr (KIND == LK_LOG1P0) return y0 > T(-1) && y0 < P<T>::INF;
    else if constexpr (KIND == LK_LOGC)
        return y0 > T(0) && y0 < P<T>::INF && fabs_(y1) <= y0 * REL;
    else
        return y0 > T(-1) && y0 < P<T>::INF && y0 + y1 > T(-1) && fabs_(y1) <= fabs_(y0) * REL;
}

// ----------------------------------------------------------------------------
// Backward: twofold adjoints of the four functions.  With x = x0 + x1, the
// saved forward value s (z for texp/texpm1, the argument y for tlog/tlog1p)
// and the twofold upstream gradient g, the gradient with respect to x is
//   texp g z,  texpm1 g (z + 1),  tlog g / y,  tlog1p g / (1 + y),
// each evaluated in twofold arithmetic.
// ----------------------------------------------------------------------------
template <int FN, class T> __device__ __forceinline__ Tw<T> bwd_elem(Tw<T> s, Tw<T> g) {
    if constexpr (FN == 0) return mul_tt(g, s);
    else if constexpr (FN == 1) return mul_tt(g, add_td(s, T(1)));
    else if constexpr (FN == 2) return div_tt(g, s);
    else return div_tt(g, add_td(s, T(1)));
}

}  // namespace tfh
