/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar CPU implementation of the twofold functions
 *     z0 + z1 = texp(x0 + x1), texpm1(x0 + x1), tlog(y0 + y1), tlog1p(y0 + y1)
 * of E. Latkin, "Twofold exp and log" (2015), for IEEE binary64 and binary32.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * it.  It shares no code, header or table generator with the GPU library: its
 * constants come from oracle/gen_tables.py (mpmath).
 *
 * Every function follows the paper's steps in the paper's order; the section
 * each one implements is named above it.  Where the paper is silent (the
 * twofold-arithmetic formulas of its reference [1], the C library's 1x
 * functions) the reading used here is written next to the code.
 *
 * Build (see oracle/__init__.py):
 *   g++ -O2 -mfma -ffp-contract=off -fno-fast-math -frounding-math -fopenmp
 *       -shared -fPIC oracle/tfo.cpp -o oracle/libtfo.so
 * -ffp-contract=off matters: every fused multiply-add below is an explicit fma().
 */
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <limits>

#include "tfo_tables.h"

namespace {

/* ------------------------------------------------------------------------ */
/* Op-counting scalar.  The oracle templates are instantiated with Cnt<T> only */
/* to count the floating-point operations the algorithm performs per element  */
/* (add/sub, mul, fma; rint/ldexp/frexp/conversions as "other").              */
/* ------------------------------------------------------------------------ */
struct OpCount {
    unsigned long long add, mul, fma, other;
};
OpCount g_cnt;

template <class U> struct Cnt {
    U v;
    Cnt() : v(0) {}
    Cnt(U x) : v(x) {}
    explicit operator U() const { return v; }
};
template <class U> Cnt<U> operator+(Cnt<U> a, Cnt<U> b) { g_cnt.add++; return Cnt<U>(a.v + b.v); }
template <class U> Cnt<U> operator-(Cnt<U> a, Cnt<U> b) { g_cnt.add++; return Cnt<U>(a.v - b.v); }
template <class U> Cnt<U> operator*(Cnt<U> a, Cnt<U> b) { g_cnt.mul++; return Cnt<U>(a.v * b.v); }
template <class U> Cnt<U> operator/(Cnt<U> a, Cnt<U> b) { g_cnt.other++; return Cnt<U>(a.v / b.v); }
template <class U> Cnt<U> operator-(Cnt<U> a) { return Cnt<U>(-a.v); }
template <class U> bool operator<(Cnt<U> a, Cnt<U> b) { return a.v < b.v; }
template <class U> bool operator>(Cnt<U> a, Cnt<U> b) { return a.v > b.v; }
template <class U> bool operator<=(Cnt<U> a, Cnt<U> b) { return a.v <= b.v; }
template <class U> bool operator>=(Cnt<U> a, Cnt<U> b) { return a.v >= b.v; }
template <class U> bool operator==(Cnt<U> a, Cnt<U> b) { return a.v == b.v; }
template <class U> Cnt<U> fma(Cnt<U> a, Cnt<U> b, Cnt<U> c) { g_cnt.fma++; return Cnt<U>(std::fma(a.v, b.v, c.v)); }
template <class U> Cnt<U> rint(Cnt<U> a) { g_cnt.other++; return Cnt<U>(std::rint(a.v)); }
template <class U> Cnt<U> ldexp(Cnt<U> a, int k) { g_cnt.other++; return Cnt<U>(std::ldexp(a.v, k)); }
template <class U> Cnt<U> frexp(Cnt<U> a, int* e) { g_cnt.other++; return Cnt<U>(std::frexp(a.v, e)); }
template <class U> Cnt<U> fabs(Cnt<U> a) { return Cnt<U>(std::fabs(a.v)); }
template <class U> Cnt<U> sqrt(Cnt<U> a) { g_cnt.other++; return Cnt<U>(std::sqrt(a.v)); }
template <class U> bool isnan(Cnt<U> a) { return std::isnan(a.v); }
template <class U> bool isinf(Cnt<U> a) { return std::isinf(a.v); }

using std::fabs;
using std::fma;
using std::frexp;
using std::isinf;
using std::isnan;
using std::ldexp;
using std::rint;
using std::sqrt;

template <class T> struct Base { using type = T; };
template <class U> struct Base<Cnt<U>> { using type = U; };
template <class T> using base_t = typename Base<T>::type;

template <class U> U value_of(U x) { return x; }
template <class U> U value_of(Cnt<U> x) { return x.v; }
template <class T> int to_int(T x) { return (int)value_of(x); }
template <class T> T from_int(int i) { return T((base_t<T>)i); }

/* ------------------------------------------------------------------------ */
/* Parameters per format (values: oracle/tfo_tables.h)                       */
/* ------------------------------------------------------------------------ */
template <class B> struct Par;

#define TFO_PAR_FIELDS(PFX, TYPE, BITS, MINNORM)                                       \
    using U = TYPE;                                                                  \
    static constexpr int L = PFX##L, K = PFX##K, N = PFX##N, N1 = PFX##N1;           \
    static constexpr int E_OFF = PFX##E_OFF, C_OFF = PFX##C_OFF, CM1_OFF = PFX##CM1_OFF; \
    static constexpr int E_CNT = PFX##E_CNT, C_CNT = PFX##C_CNT, CM1_CNT = PFX##CM1_CNT; \
    static constexpr int P = BITS; /* significand bits */                            \
    static constexpr int EXP_NC = (int)(sizeof(PFX##EXP_C) / sizeof(TYPE));          \
    static constexpr int LOG_NC = (int)(sizeof(PFX##LOG_C) / sizeof(TYPE));          \
    static U min_normal() { return MINNORM; }                                        \
    static const U* E_HI() { return PFX##E_HI; }                                     \
    static const U* E_LO() { return PFX##E_LO; }                                     \
    static const int* E_K() { return PFX##E_K; }                                     \
    static const U* C_HI() { return PFX##C_HI; }                                     \
    static const U* C_LO() { return PFX##C_LO; }                                     \
    static const U* CM1_HI() { return PFX##CM1_HI; }                                 \
    static const U* CM1_LO() { return PFX##CM1_LO; }                                 \
    static const U* HORNER() { return PFX##HORNER; }                                 \
    static const U* HORNER1() { return PFX##HORNER1; }                               \
    static const U* S_HI() { return PFX##S_HI; }                                     \
    static const U* S_LO() { return PFX##S_LO; }                                     \
    static const U* EXP_C() { return PFX##EXP_C; }                                   \
    static const U* LOG_C() { return PFX##LOG_C; }                                   \
    static const U* LOG_INVC() { return PFX##LOG_INVC; }                             \
    static const U* LOG_HI() { return PFX##LOG_HI; }                                 \
    static const U* LOG_LO() { return PFX##LOG_LO; }                                 \
    static U LN2_HI() { return PFX##LN2_HI; }                                        \
    static U LN2_LO() { return PFX##LN2_LO; }                                        \
    static U RCP_HI() { return PFX##RCP_HI; }                                        \
    static U RCP_LO() { return PFX##RCP_LO; }                                        \
    static U INV_L() { return PFX##INV_L; }                                          \
    static U L1() { return PFX##L1; }                                                \
    static U L2() { return PFX##L2; }                                                \
    static U LN2X_HI() { return PFX##LN2X_HI; }                                      \
    static U LN2X_LO() { return PFX##LN2X_LO; }                                      \
    static U EXP_XMAX() { return PFX##EXP_XMAX; }                                    \
    static U EXPM1_XMAX() { return PFX##EXPM1_XMAX; }                                \
    static U EXP_XLO() { return PFX##EXP_XLO; }                                      \
    static U EXPM1_XNEG() { return PFX##EXPM1_XNEG; }                                \
    static U EXPM1_TINY() { return PFX##EXPM1_TINY; }                                \
    static U LOG1P_TINY() { return PFX##LOG1P_TINY; }                                \
    static U LN2_RN() { return PFX##LN2_RN; }

template <> struct Par<double> { TFO_PAR_FIELDS(TFO_D_, double, 53, 0x1p-1022) };
template <> struct Par<float> { TFO_PAR_FIELDS(TFO_F_, float, 24, 0x1p-126f) };

template <class T> using K_ = Par<base_t<T>>;

template <class T> T qnan() { return T(std::numeric_limits<base_t<T>>::quiet_NaN()); }
template <class T> T pinf() { return T(std::numeric_limits<base_t<T>>::infinity()); }

/* Top 7 significand bits of a finite positive z (the 1x log table index). */
template <class T> int top7(T z) {
    base_t<T> b = value_of(z);
    if (sizeof(b) == 8) {
        uint64_t u; std::memcpy(&u, &b, 8);
        return (int)((u >> 45) & 127);
    }
    uint32_t u; std::memcpy(&u, &b, 4);
    return (int)((u >> 16) & 127);
}

/* ------------------------------------------------------------------------ */
/* Twofold arithmetic.  The paper takes these from its reference [1], whose   */
/* text is not available; these are the published error-free transforms      */
/* (Dekker 1971, Knuth's TwoSum) with the FMA exact product.  The outputs of  */
/* fast_two_sum / two_sum / two_prod are unique (the exact rounding error),   */
/* so fast_two_sum is used wherever |a| >= |b| (or a = 0) holds provably.     */
/* ------------------------------------------------------------------------ */
template <class T> struct Tw { T x0, x1; };

/* s + t = a + b exactly; needs |a| >= |b| or a == 0 ("renormalize fast"). */
template <class T> Tw<T> fast_two_sum(T a, T b) {
    T s = a + b;
    T t = b - (s - a);
    return {s, t};
}
/* s + t = a + b exactly, any a, b (Knuth's six-operation TwoSum: the sum,
 * the parts of it attributed to b and to a, and their rounding errors). */
template <class T> Tw<T> two_sum(T a, T b) {
    T s = a + b;
    T bp = s - a;
    T ap = s - bp;
    T db = b - bp;
    T da = a - ap;
    return {s, da + db};
}
/* p + e = a * b exactly (FMA remainder). */
template <class T> Tw<T> two_prod(T a, T b) {
    T p = a * b;
    T e = fma(a, b, -p);
    return {p, e};
}
/* twofold x dotted, as the paper counts it (section "Twofold exponent:
 * Method summary": 2 multiplications, 1 FMA and 1 summation): the exact
 * product of the main parts, then the low product A1 c rounded on its own and
 * added to the product's error. */
template <class T> Tw<T> mul_td(Tw<T> A, T c) {
    Tw<T> pe = two_prod(A.x0, c);
    return {pe.x0, pe.x1 + A.x1 * c};
}
/* twofold + dotted when |c| >= |A0| (the Horner coefficients dominate). */
template <class T> Tw<T> add_td_fast(Tw<T> A, T c) {
    Tw<T> st = fast_two_sum(c, A.x0);
    return {st.x0, st.x1 + A.x1};
}
/* twofold + dotted, any magnitudes. */
template <class T> Tw<T> add_td(Tw<T> A, T c) {
    Tw<T> st = two_sum(A.x0, c);
    return {st.x0, st.x1 + A.x1};
}
/* twofold x twofold. */
template <class T> Tw<T> mul_tt(Tw<T> A, Tw<T> B) {
    Tw<T> pe = two_prod(A.x0, B.x0);
    return {pe.x0, fma(A.x0, B.x1, fma(A.x1, B.x0, pe.x1))};
}
/* twofold + twofold, any magnitudes. */
template <class T> Tw<T> add_tt(Tw<T> A, Tw<T> B) {
    Tw<T> st = two_sum(A.x0, B.x0);
    return {st.x0, st.x1 + (A.x1 + B.x1)};
}
/* twofold + twofold when |A0| >= |B0| or A0 == 0. */
template <class T> Tw<T> add_tt_fast(Tw<T> A, Tw<T> B) {
    Tw<T> st = fast_two_sum(A.x0, B.x0);
    return {st.x0, st.x1 + (A.x1 + B.x1)};
}
/* twofold / twofold (Dekker's division with the FMA remainder
 * r = fma(-q, b, a) named in the section "Older CPUs"). */
template <class T> Tw<T> div_tt(Tw<T> A, Tw<T> B) {
    T q0 = A.x0 / B.x0;
    T r = fma(-q0, B.x0, A.x0);
    T q1 = ((r + A.x1) - q0 * B.x1) / B.x0;
    return {q0, q1};
}

/* ------------------------------------------------------------------------ */
/* The 1x functions: the "standard library" exp, expm1, log, log1p whose      */
/* results z0 the twofold functions reproduce bitwise (section "Twofold       */
/* exponent: Method summary").  The paper leaves them to the C library; here  */
/* they are table-driven algorithms after P.T.P. Tang (ACM TOMS 1989, 1990,   */
/* 1992), written for this project: accurate to within one ulp, built from    */
/* + - * fma rint ldexp frexp only, so the same steps give the same bits on   */
/* any IEEE machine.                                                          */
/* ------------------------------------------------------------------------ */

/* e^r - 1 ~ r + r^2 q(r): q = 1/2! + r/3! + ... (Taylor, |r| <= ln2/64). */
template <class T> T exp_q(T r) {
    using K = K_<T>;
    const auto* c = K::EXP_C();
    T q = T(c[K::EXP_NC - 1]);
    for (int i = K::EXP_NC - 2; i >= 0; --i) q = fma(r, q, T(c[i]));
    return q;
}

/* exp(x): x = (32m + j) ln2/32 + r; e^x = 2^m 2^(j/32) e^r. */
template <class T> T exp1x(T x) {
    using K = K_<T>;
    if (isnan(x)) return x + x;
    if (x > T(K::EXP_XMAX())) return pinf<T>();
    if (x < T(K::EXP_XLO())) return T(0);
    T kd = rint(x * T(K::INV_L()));
    int k = to_int(kd);
    T r = fma(-kd, T(K::L1()), x);           /* exact */
    r = fma(-kd, T(K::L2()), r);
    T p = fma(r * r, exp_q(r), r);           /* e^r - 1 */
    int j = k & 31, m = (k - j) / 32;
    T s = T(K::S_HI()[j]);
    T y = s + fma(s, p, T(K::S_LO()[j]));
    return ldexp(y, m);
}

/* expm1(x): same reduction with r carried as r_hi + r_lo; the -1 enters in the
 * 2^-m scaled domain through exact transforms, so there is no cancellation. */
template <class T> T expm1_1x(T x) {
    using K = K_<T>;
    if (isnan(x)) return x + x;
    if (x > T(K::EXPM1_XMAX())) return pinf<T>();
    if (x < T(K::EXPM1_XNEG())) return T(-1);
    if (fabs(x) < T(K::EXPM1_TINY())) return (x == T(0)) ? x : fma(x, x * T(0.5), x);
    T kd = rint(x * T(K::INV_L()));
    int k = to_int(kd);
    T rhi = fma(-kd, T(K::L1()), x);         /* exact */
    T rlo = -kd * T(K::L2());
    T r = rhi + rlo;
    T plo = fma(r * r, exp_q(r), rlo);       /* e^r - 1 ~ rhi + plo */
    int j = k & 31, m = (k - j) / 32;
    T shi = T(K::S_HI()[j]), slo = T(K::S_LO()[j]);
    Tw<T> A = two_sum(shi, -ldexp(T(1), -m));
    Tw<T> Bp = two_prod(shi, rhi);
    T c = fma(shi, plo, fma(slo, rhi, slo));
    Tw<T> H = two_sum(A.x0, Bp.x0);
    T tail = H.x1 + ((A.x1 + Bp.x1) + c);
    return ldexp(H.x0 + tail, m);
}

/* log1p(r) - r ~ r^2 q(r): q = -1/2 + r/3 - r^2/4 + ...  (|r| < 2^-7). */
template <class T> T log_q(T r) {
    using K = K_<T>;
    const auto* c = K::LOG_C();
    T q = T(c[K::LOG_NC - 1]);
    for (int i = K::LOG_NC - 2; i >= 0; --i) q = fma(r, q, T(c[i]));
    return q;
}

/* Split a finite positive normal u as u = z 2^e with z in [3/4, 3/2) and the
 * cell index i of z (top 7 significand bits of the [1,2) mantissa). */
template <class T> void log_split(T u, T* z, int* e, int* i) {
    int ee;
    T f = frexp(u, &ee);                      /* [1/2, 1) */
    T z2 = ldexp(f, 1);                       /* [1, 2)   */
    int ii = top7(z2);
    ee -= 1;
    if (ii >= 64) { z2 = ldexp(z2, -1); ee += 1; }
    *z = z2; *e = ee; *i = ii;
}

/* log(x) = e ln2 - log(invc) + log1p(z invc - 1), z invc - 1 exact. */
template <class T> T log1x(T x) {
    using K = K_<T>;
    if (isnan(x)) return x + x;
    if (x < T(0)) return qnan<T>();
    if (x == T(0)) return -pinf<T>();
    if (isinf(x)) return x;
    int eadj = 0;
    if (x < T(K::min_normal())) { x = ldexp(x, K::P + 1); eadj = -(K::P + 1); }
    T z; int e, i;
    log_split(x, &z, &e, &i);
    e += eadj;
    T r = fma(z, T(K::LOG_INVC()[i]), T(-1)); /* exact */
    T ed = from_int<T>(e);
    T hi = fma(ed, T(K::LN2X_HI()), T(K::LOG_HI()[i]));  /* exact */
    T lo = fma(ed, T(K::LN2X_LO()), T(K::LOG_LO()[i]));
    T tail = fma(r * r, log_q(r), lo);
    Tw<T> st = fast_two_sum(hi, r);
    return st.x0 + (st.x1 + tail);
}

/* log1p(x): u + c = 1 + x exactly, then log(u) with c folded in as r_lo. */
template <class T> T log1p_1x(T x) {
    using K = K_<T>;
    if (isnan(x)) return x + x;
    if (x < T(-1)) return qnan<T>();
    if (x == T(-1)) return -pinf<T>();
    if (isinf(x)) return x;
    if (fabs(x) < T(K::LOG1P_TINY())) return x;
    Tw<T> u = two_sum(T(1), x);
    T z; int e, i;
    log_split(u.x0, &z, &e, &i);
    T invc = T(K::LOG_INVC()[i]);
    T rhi = fma(z, invc, T(-1));              /* exact */
    T rlo = ldexp(u.x1, -e) * invc;
    if (fabs(x) < T(0.00390625)) {            /* |x| < 2^-8: e = 0, invc = 1; */
        rhi = x;                              /* r = x itself, unsplit       */
        rlo = T(0);
    }
    T ed = from_int<T>(e);
    T hi = fma(ed, T(K::LN2X_HI()), T(K::LOG_HI()[i]));
    T lo = fma(ed, T(K::LN2X_LO()), T(K::LOG_LO()[i]));
    T tail = fma(rhi * rhi, log_q(rhi), lo + fma(-rlo, rhi, rlo));
    Tw<T> st = fast_two_sum(hi, rhi);
    return st.x0 + (st.x1 + tail);
}

/* ------------------------------------------------------------------------ */
/* pexp0 (section "Function pexp0()", "Exponent: Algorithm summary").         */
/* Core for EXP_XLO <= x <= EXP_XMAX.  E = e^(2^L m) is stored as Ehat 2^k    */
/* with Ehat in [1,2), so V = Ehat (C T) is returned with the exponent k and  */
/* e^x ~ (V0 + V1) 2^k.  Not renormalised (internal use).                     */
/* ------------------------------------------------------------------------ */
template <class T> struct Scaled { Tw<T> v; int k; };

template <class T> Scaled<T> pexp0_core(T x) {
    using K = K_<T>;
    /* (a) decompose exactly x = 2^L m + 2^-K n + y */
    T Md = rint(x * T((base_t<T>)(1 << K::K)));        /* M = round(x 2^K) */
    T y = x - Md * T((base_t<T>)1 / (1 << K::K));      /* exact */
    int M = to_int(Md);
    int a = M < 0 ? -M : M, sg = M < 0 ? -1 : 1;
    int m = sg * (a >> (K::L + K::K));
    int n = sg * (a & ((1 << (K::L + K::K)) - 1));
    /* (b) table values E and C */
    Tw<T> E = {T(K::E_HI()[m + K::E_OFF]), T(K::E_LO()[m + K::E_OFF])};
    Tw<T> C = {T(K::C_HI()[n + K::C_OFF]), T(K::C_LO()[n + K::C_OFF])};
    /* (c) T = e^y N! by Horner: (...((y + N) y + N!/(N-2)!) y + ...) y + N!/0! */
    Tw<T> P = fast_two_sum(T((base_t<T>)K::N), y);
    for (int j = K::N - 2; j >= 0; --j) P = add_td_fast(mul_td(P, y), T(K::HORNER()[j]));
    /* (d) E (C T) */
    Tw<T> V = mul_tt(E, mul_tt(C, P));
    return {V, K::E_K()[m + K::E_OFF]};
}

/* pexp0 as a coupled p-function: range cases, E (C T), renormalize fast. */
template <class T> Tw<T> pexp0(T x) {
    using K = K_<T>;
    if (isnan(x)) return {x, x};
    if (x < T(K::EXP_XLO())) return {T(0), T(0)};
    if (x > T(K::EXP_XMAX())) return {pinf<T>(), pinf<T>()};
    Scaled<T> s = pexp0_core(x);
    return fast_two_sum(ldexp(s.v.x0, s.k), ldexp(s.v.x1, s.k));
}

/* pexpm10 small path (|x| <= 89.5/128): x = n/128 + y, C = e^(n/128) - 1,
 * T = e^y - 1 = (Horner without the last + N!) * y * (1/N!), Z = CT + (C + T).
 * Not renormalised. */
template <class T> Tw<T> pexpm10_small(T x) {
    using K = K_<T>;
    T nd = rint(x * T(128));
    T y = x - nd * T((base_t<T>)1 / 128);                /* exact */
    int n = to_int(nd);
    Tw<T> P = fast_two_sum(T((base_t<T>)K::N1), y);
    for (int j = K::N1 - 2; j >= 1; --j) P = add_td_fast(mul_td(P, y), T(K::HORNER1()[j]));
    P = mul_td(P, y);
    Tw<T> Tt = mul_tt(P, Tw<T>{T(K::RCP_HI()), T(K::RCP_LO())});
    Tw<T> C = {T(K::CM1_HI()[n + K::CM1_OFF]), T(K::CM1_LO()[n + K::CM1_OFF])};
    /* |C0| >= |T0| or C0 = 0, and |C + T| >= |C T|: fast sums are exact here */
    return add_tt_fast(add_tt_fast(C, Tt), mul_tt(C, Tt));
}

/* pexpm10 body: small path for |x| <= ln2, else pexp0(x) - 1. Not renormalised. */
template <class T> Tw<T> pexpm10_body(T x) {
    using K = K_<T>;
    if (fabs(x) <= T(K::LN2_RN())) return pexpm10_small(x);
    if (x < T(K::EXP_XLO())) return add_td(Tw<T>{T(0), T(0)}, T(-1));
    Scaled<T> s = pexp0_core(x);
    Tw<T> v = {ldexp(s.v.x0, s.k), ldexp(s.v.x1, s.k)};
    return add_td(v, T(-1));
}

/* pexpm10 as a coupled p-function (renormalize fast at the end). */
template <class T> Tw<T> pexpm10(T x) {
    using K = K_<T>;
    if (isnan(x)) return {x, x};
    if (x > T(K::EXP_XMAX())) return {pinf<T>(), pinf<T>()};
    Tw<T> w = pexpm10_body(x);
    return fast_two_sum(w.x0, w.x1);
}

/* The rule for non-finite main parts: z0 NaN -> z1 NaN; z0 = +-inf -> z1 = +0. */
template <class T> T special_rule(T z0, T z1) {
    if (isnan(z0)) return qnan<T>();
    if (isinf(z0)) return T(0);
    return z1;
}

/* ------------------------------------------------------------------------ */
/* texp (section "Exponent: Algorithm summary", twofold argument):            */
/*   v = pexp0(x0), z0 = exp(x0), t1 = expm1(x1), z1 = z0 t1 + (v1 + (v0 - z0)) */
/* evaluated in the 2^-k domain of pexp0's normalised table (exact scaling).  */
/* ------------------------------------------------------------------------ */
template <class T> T texp(T x0, T x1, T* z1out) {
    using K = K_<T>;
    T z0 = exp1x(x0);
    T t1 = expm1_1x(x1);
    T z1;
    if (isnan(z0) || isinf(z0)) {
        z1 = T(0);                                     /* replaced by the rule */
    } else if (x0 < T(K::EXP_XLO())) {
        Tw<T> v = {T(0), T(0)};                        /* pexp0 gives 0 below range */
        z1 = z0 * t1 + (v.x1 + (v.x0 - z0));
    } else {
        Scaled<T> s = pexp0_core(x0);
        T z0s = ldexp(z0, -s.k);                       /* exact */
        T z1s = z0s * t1 + (s.v.x1 + (s.v.x0 - z0s));
        z1 = ldexp(z1s, s.k);
    }
    *z1out = special_rule(z0, z1);
    return z0;
}

/* texpm1: w = pexpm10(x0), z0 = expm1(x0), t1 = expm1(x1),
 *         z1 = (z0 + 1) t1 + (w1 + (w0 - z0)). */
template <class T> T texpm1(T x0, T x1, T* z1out) {
    T z0 = expm1_1x(x0);
    T t1 = expm1_1x(x1);
    T z1 = T(0);
    if (!(isnan(z0) || isinf(z0))) {
        Tw<T> w = pexpm10_body(x0);
        z1 = (z0 + T(1)) * t1 + (w.x1 + (w.x0 - z0));
    }
    *z1out = special_rule(z0, z1);
    return z0;
}

/* The x1 that a log gives when its renormalised argument w0 leaves (0, inf):
 * NaN below 0 or NaN, -inf at 0, +inf at +inf.  Returns false if w0 is inside. */
template <class T> bool log_domain(T w0, T* x1) {
    if (isnan(w0) || w0 < T(0)) { *x1 = qnan<T>(); return true; }
    if (w0 == T(0)) { *x1 = -pinf<T>(); return true; }
    if (isinf(w0)) { *x1 = pinf<T>(); return true; }
    return false;
}

/* Decompose a renormalised twofold w = 2^n z (section "Logarithm: Algorithm
 * summary", plog step 1): frexp when w0 < 1/2 or w0 > 2, else n = 0. */
template <class T> Tw<T> log_scale(Tw<T> w, int* n) {
    *n = 0;
    if (w.x0 < T(0.5) || w.x0 > T(2)) {
        T f = frexp(w.x0, n);
        return {f, ldexp(w.x1, -*n)};
    }
    return w;
}

/* Newton correction (section "Twofold logarithm: Newton inversion"): for the
 * reduced argument 1 + a and a seed r0 ~ log(1 + a),
 *   s = pexpm10(-r0), u = (1+a)(1+s) - 1 = ((a s) + a) + s, r1 = u0 + u1.
 * The reduction keeps |r0| <= ln 2; a seed beyond the small path of pexpm10
 * (|r0| > 89/128, or not a number) arises only from an argument that is not
 * coupled (or not finite) where the paper asks for a coupled one, and gives a
 * NaN correction r1. */
template <class T> Tw<T> newton_log(Tw<T> a, T r0) {
    if (!(fabs(r0) <= T(0.6953125))) return {r0, qnan<T>()};
    Tw<T> s = pexpm10_small(-r0);
    Tw<T> u = add_tt(add_tt(mul_tt(a, s), a), s);
    T r1 = u.x0 + u.x1;
    return {r0, r1};
}

/* (r0 + r1) + n ln2, with n ln2 the twofold product of ln 2 and n. */
template <class T> Tw<T> add_n_ln2(Tw<T> X, int n) {
    using K = K_<T>;
    return add_tt(X, mul_td(Tw<T>{T(K::LN2_HI()), T(K::LN2_LO())}, from_int<T>(n)));
}

/* Newton step shared by plog and plog1p: seed r0 = log1p(a0 + a1), the
 * correction above, and, when add_n, (r0 + r1) + n ln2. */
template <class T> Tw<T> plog_core(Tw<T> a, int n, bool add_n) {
    Tw<T> X = newton_log(a, log1p_1x(a.x0 + a.x1));
    if (add_n) X = add_n_ln2(X, n);
    return X;
}

/* tlog (twofold argument): v = renormalised y, u = plog(v) (not renormalised),
 * x0 = log(y0), x1 = u1 + (u0 - x0). */
template <class T> T tlog(T y0, T y1, T* x1out) {
    T x0 = log1x(y0);
    T x1 = T(0);
    if (!(isnan(x0) || isinf(x0))) {
        Tw<T> v = two_sum(y0, y1);
        if (!log_domain(v.x0, &x1)) {
            int n;
            Tw<T> z = log_scale(v, &n);
            Tw<T> a = {z.x0 - T(1), z.x1};               /* exact (Sterbenz) */
            Tw<T> X = plog_core(a, n, true);
            x1 = X.x1 + (X.x0 - x0);
        }
    }
    *x1out = special_rule(x0, x1);
    return x0;
}

/* tlog1p (twofold argument): v = renormalised y; plog1p(v): for v0 < -1/2 or
 * v0 > 1 the log of the renormalised 1 + v (plog), else the Newton step on
 * a = v directly; x0 = log1p(y0), x1 = u1 + (u0 - x0). */
template <class T> T tlog1p(T y0, T y1, T* x1out) {
    T x0 = log1p_1x(y0);
    T x1 = T(0);
    if (!(isnan(x0) || isinf(x0))) {
        Tw<T> v = two_sum(y0, y1);
        if (isnan(v.x0)) {
            x1 = qnan<T>();
        } else if (isinf(v.x0) && v.x0 > T(0)) {
            x1 = pinf<T>();
        } else if (v.x0 < T(-0.5) || v.x0 > T(1)) {
            Tw<T> w = add_td(v, T(1));
            w = two_sum(w.x0, w.x1);                    /* renormalise 1 + y */
            if (!log_domain(w.x0, &x1)) {
                int n;
                Tw<T> z = log_scale(w, &n);
                Tw<T> a = {z.x0 - T(1), z.x1};
                Tw<T> X = plog_core(a, n, true);
                x1 = X.x1 + (X.x0 - x0);
            }
        } else {
            Tw<T> X = plog_core(v, 0, false);
            x1 = X.x1 + (X.x0 - x0);
        }
    }
    *x1out = special_rule(x0, x1);
    return x0;
}

/* ------------------------------------------------------------------------ */
/* The other entry points of the paper's interface (sections "Twofold         */
/* exponent: Algorithm summary", "Twofold logarithm: Algorithm summary" and   */
/* "C/C++ interface"): functions of a dotted argument x0 (x1 = 0), of a       */
/* coupled argument, and p-functions whose result is coupled.  Every          */
/* p-function ends with "renormalize fast"; inside a t-function that step is  */
/* omitted, as the paper allows.                                              */
/* ------------------------------------------------------------------------ */

/* Renormalize fast a result (|z0| >= |z1|), then the rule for a non-finite
 * main part. */
template <class T> T renorm_result(T z0, T z1, T* z1out) {
    if (isnan(z0) || isinf(z0)) {
        *z1out = special_rule(z0, z1);
        return z0;
    }
    Tw<T> r = fast_two_sum(z0, z1);
    *z1out = special_rule(r.x0, r.x1);
    return r.x0;
}

/* pexp0 and pexpm10 in the scalar form of the interface. */
template <class T> T pexp0_s(T x0, T* z1) { Tw<T> r = pexp0(x0); *z1 = r.x1; return r.x0; }
template <class T> T pexpm10_s(T x0, T* z1) { Tw<T> r = pexpm10(x0); *z1 = r.x1; return r.x0; }

/* texp0 (dotted argument): v = pexp0(x0) not renormalised, z0 = exp(x0),
 * z1 = (v0 - z0) + v1, in pexp0's 2^-k domain as texp. */
template <class T> T texp0(T x0, T* z1out) {
    using K = K_<T>;
    T z0 = exp1x(x0);
    T z1;
    if (isnan(z0) || isinf(z0)) {
        z1 = T(0);                                     /* replaced by the rule */
    } else if (x0 < T(K::EXP_XLO())) {
        Tw<T> v = {T(0), T(0)};                        /* pexp0 gives 0 below range */
        z1 = (v.x0 - z0) + v.x1;
    } else {
        Scaled<T> s = pexp0_core(x0);
        T z0s = ldexp(z0, -s.k);                       /* exact */
        z1 = ldexp((s.v.x0 - z0s) + s.v.x1, s.k);
    }
    *z1out = special_rule(z0, z1);
    return z0;
}

/* texpm10 (dotted argument): w = pexpm10(x0) not renormalised,
 * z0 = expm1(x0), z1 = (w0 - z0) + w1. */
template <class T> T texpm10(T x0, T* z1out) {
    T z0 = expm1_1x(x0);
    T z1 = T(0);
    if (!(isnan(z0) || isinf(z0))) {
        Tw<T> w = pexpm10_body(x0);
        z1 = (w.x0 - z0) + w.x1;
    }
    *z1out = special_rule(z0, z1);
    return z0;
}

/* texpp and texpm1p (coupled argument): the paper gives no special algorithm
 * for a coupled argument; they are texp and texpm1. */
template <class T> T texpp(T x0, T x1, T* z1) { return texp(x0, x1, z1); }
template <class T> T texpm1p(T x0, T x1, T* z1) { return texpm1(x0, x1, z1); }

/* pexp and pexpm1 (coupled argument, coupled result): texpp and texpm1p,
 * then renormalize fast. */
template <class T> T pexp(T x0, T x1, T* z1out) {
    T z1;
    T z0 = texpp(x0, x1, &z1);
    return renorm_result(z0, z1, z1out);
}
template <class T> T pexpm1(T x0, T x1, T* z1out) {
    T z1;
    T z0 = texpm1p(x0, x1, &z1);
    return renorm_result(z0, z1, z1out);
}

/* plog0 steps (1)-(3), dotted y0 in (0, inf), not renormalised:
 * y0 = 2^n z0, r0 = log(z0) (the 1x log), the Newton correction with
 * 1 + a = z0, then + n ln2. */
template <class T> Tw<T> plog0_core(T y0) {
    int n;
    Tw<T> z = log_scale(Tw<T>{y0, T(0)}, &n);
    Tw<T> a = {z.x0 - T(1), z.x1};                     /* exact (Sterbenz) */
    return add_n_ln2(newton_log(a, log1x(z.x0)), n);
}

/* plog (coupled argument) steps (1)-(3), y0 in (0, inf), not renormalised:
 * y = 2^n (z0 + z1) scaled by the exponent of y0, a = (z0 - 1) + z1, the
 * Newton step seeded with log1p(a0 + a1), then + n ln2. */
template <class T> Tw<T> plog_coupled_core(Tw<T> y) {
    int n;
    Tw<T> z = log_scale(y, &n);
    Tw<T> a = {z.x0 - T(1), z.x1};
    return plog_core(a, n, true);
}

/* plog1p0 steps (1)-(2), dotted y0 in (-1, inf), not renormalised: outside
 * [-1/2, 1] the plog of the renormalised 1 + y0; inside, x0 = log1p(y0) and
 * the Newton correction with a = y0 (the text's "pexpm10(-r0)" is read as
 * pexpm10(-x0), the seed just computed). */
template <class T> Tw<T> plog1p0_core(T y0) {
    if (y0 < T(-0.5) || y0 > T(1)) return plog_coupled_core(two_sum(T(1), y0));
    return newton_log(Tw<T>{y0, T(0)}, log1p_1x(y0));
}

/* plog1p (coupled argument) steps (1)-(2), y0 in (-1, inf), not
 * renormalised: outside [-1/2, 1] the plog of the renormalised 1 + y (the
 * text's tlogp(1 + y) differs from plog only in an x0 correction that the
 * p-function does not want); inside, the Newton step on a = y, seeded with
 * log1p(y0 + y1), which is log1p(y0) for a coupled y. */
template <class T> Tw<T> plog1p_core(Tw<T> y) {
    if (y.x0 < T(-0.5) || y.x0 > T(1)) {
        Tw<T> w = add_td(y, T(1));
        return plog_coupled_core(two_sum(w.x0, w.x1));
    }
    return plog_core(y, 0, false);
}

/* The p-functions of the logarithm: main part outside the domain of the 1x
 * function -> that function's value (-inf, +inf or NaN) and the rule;
 * otherwise the core, renormalised fast. */
template <class T> T plog0(T y0, T* x1out) {
    if (!(y0 > T(0) && y0 < pinf<T>())) {
        T x0 = log1x(y0);
        *x1out = special_rule(x0, T(0));
        return x0;
    }
    Tw<T> X = plog0_core(y0);
    return renorm_result(X.x0, X.x1, x1out);
}
template <class T> T plog(T y0, T y1, T* x1out) {
    if (!(y0 > T(0) && y0 < pinf<T>())) {
        T x0 = log1x(y0);
        *x1out = special_rule(x0, T(0));
        return x0;
    }
    Tw<T> X = plog_coupled_core(Tw<T>{y0, y1});
    return renorm_result(X.x0, X.x1, x1out);
}
template <class T> T plog1p0(T y0, T* x1out) {
    if (!(y0 > T(-1) && y0 < pinf<T>())) {
        T x0 = log1p_1x(y0);
        *x1out = special_rule(x0, T(0));
        return x0;
    }
    Tw<T> X = plog1p0_core(y0);
    return renorm_result(X.x0, X.x1, x1out);
}
template <class T> T plog1p(T y0, T y1, T* x1out) {
    if (!(y0 > T(-1) && y0 < pinf<T>())) {
        T x0 = log1p_1x(y0);
        *x1out = special_rule(x0, T(0));
        return x0;
    }
    Tw<T> X = plog1p_core(Tw<T>{y0, y1});
    return renorm_result(X.x0, X.x1, x1out);
}

/* The t-functions: the core not renormalised, then the correction that makes
 * the main part the 1x function bitwise: u0 = log(y0) (or log1p(y0)),
 * x1 = X1 + (X0 - u0), x0 = u0.  (The text writes the correction of tlog0 and
 * tlog1p0 as x1 + (u0 - x0); the sign that keeps x0 + x1 is X0 - u0, as in
 * tlog's own last step.) */
template <class T> T tlog0(T y0, T* x1out) {
    T u0 = log1x(y0);
    T x1 = T(0);
    if (!(isnan(u0) || isinf(u0))) {
        Tw<T> X = plog0_core(y0);
        x1 = X.x1 + (X.x0 - u0);
    }
    *x1out = special_rule(u0, x1);
    return u0;
}
template <class T> T tlogp(T y0, T y1, T* x1out) {
    T u0 = log1x(y0);
    T x1 = T(0);
    if (!(isnan(u0) || isinf(u0))) {
        Tw<T> X = plog_coupled_core(Tw<T>{y0, y1});
        x1 = X.x1 + (X.x0 - u0);
    }
    *x1out = special_rule(u0, x1);
    return u0;
}
template <class T> T tlog1p0(T y0, T* x1out) {
    T u0 = log1p_1x(y0);
    T x1 = T(0);
    if (!(isnan(u0) || isinf(u0))) {
        Tw<T> X = plog1p0_core(y0);
        x1 = X.x1 + (X.x0 - u0);
    }
    *x1out = special_rule(u0, x1);
    return u0;
}
template <class T> T tlog1pp(T y0, T y1, T* x1out) {
    T u0 = log1p_1x(y0);
    T x1 = T(0);
    if (!(isnan(u0) || isinf(u0))) {
        Tw<T> X = plog1p_core(Tw<T>{y0, y1});
        x1 = X.x1 + (X.x0 - u0);
    }
    *x1out = special_rule(u0, x1);
    return u0;
}

/* ------------------------------------------------------------------------ */
/* Twofold arithmetic over arrays (the paper's second measured workload,      */
/* section "Twofolds update", table of tadd/tmul/tdiv/tsqrt with FMA):        */
/* z = x op y for twofolds x = x0 + x1, y = y0 + y1.  The main part is the    */
/* 1x operation on the main parts; z1 carries the twofold error term.  The    */
/* definitions are those of the twofold primitives above; subtraction is the  */
/* exact difference of the corrected subtraction of section "Twofold bugs".   */
/* After the operation, the rule for a non-finite main part.                  */
/* ------------------------------------------------------------------------ */
/* d + t = a - b exactly: negation is exact, so the two-sum of a and -b is an
 * error-free difference; its operations are those of the corrected
 * subtraction of section "Twofold bugs", with the same results (x + (-y) and
 * x - y are the same IEEE operation). */
template <class T> Tw<T> two_diff(T a, T b) { return two_sum(a, -b); }

template <class T> Tw<T> rule_tw(Tw<T> z) { return {z.x0, special_rule(z.x0, z.x1)}; }

template <class T> Tw<T> tadd(Tw<T> x, Tw<T> y) { return rule_tw(add_tt(x, y)); }
template <class T> Tw<T> tsub(Tw<T> x, Tw<T> y) {
    Tw<T> dt = two_diff(x.x0, y.x0);
    return rule_tw(Tw<T>{dt.x0, dt.x1 + (x.x1 - y.x1)});
}
template <class T> Tw<T> tmul(Tw<T> x, Tw<T> y) { return rule_tw(mul_tt(x, y)); }
template <class T> Tw<T> tdiv(Tw<T> x, Tw<T> y) { return rule_tw(div_tt(x, y)); }
/* sqrt with the FMA remainder r = fma(-q, q, x0) (section "Older CPUs" names
 * this remainder for square roots): z0 = sqrt(x0), z1 = (r + x1) / (2 z0).
 * At x0 = 0 the correction is taken as 0 (the linearisation has no term
 * there). */
template <class T> Tw<T> tsqrt_tw(Tw<T> x) {
    T z0 = sqrt(x.x0);
    T r = fma(-z0, z0, x.x0);
    T z1 = (r + x.x1) / (z0 + z0);
    if (x.x0 == T(0)) z1 = T(0);
    return rule_tw(Tw<T>{z0, z1});
}
template <class T> T tsqrt(T x0, T x1, T* z1) {
    Tw<T> r = tsqrt_tw(Tw<T>{x0, x1});
    *z1 = r.x1;
    return r.x0;
}
/* Renormalization of an arbitrary twofold (section "Twofold logarithm": the
 * renormalized twofold with exactly the same value, as the general tlog takes
 * it from its argument): z0 = RN(x0 + x1) and z1 the exact remainder, by the
 * corrected two-sum.  Where |x0| >= |x1| this is the paper's "renormalize
 * fast" (three operations), bit for bit.  Then the rule. */
template <class T> T trenorm(T x0, T x1, T* z1) {
    Tw<T> r = rule_tw(two_sum(x0, x1));
    *z1 = r.x1;
    return r.x0;
}

/* Backward (twofold adjoints, not in the paper): for x = x0 + x1 and the saved
 * forward value s (z for texp/texpm1, y for tlog/tlog1p), given the twofold
 * upstream gradient g:  texp g*z, texpm1 g*(z + 1), tlog g/y, tlog1p g/(1 + y). */
template <class T> Tw<T> bwd_texp(Tw<T> s, Tw<T> g) { return mul_tt(g, s); }
template <class T> Tw<T> bwd_texpm1(Tw<T> s, Tw<T> g) { return mul_tt(g, add_td(s, T(1))); }
template <class T> Tw<T> bwd_tlog(Tw<T> s, Tw<T> g) { return div_tt(g, s); }
template <class T> Tw<T> bwd_tlog1p(Tw<T> s, Tw<T> g) { return div_tt(g, add_td(s, T(1))); }

/* ------------------------------------------------------------------------ */
/* Array drivers                                                             */
/* ------------------------------------------------------------------------ */
template <class T, T (*F)(T, T, T*)>
void run_tw(const T* x0, const T* x1, T* z0, T* z1, size_t n, int threads) {
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads)
    for (long long i = 0; i < (long long)n; ++i) z0[i] = F(x0[i], x1[i], &z1[i]);
}

template <class T, T (*F)(T)>
void run_1x(const T* x, T* z, size_t n, int threads) {
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads)
    for (long long i = 0; i < (long long)n; ++i) z[i] = F(x[i]);
}

template <class T, T (*F)(T, T*)>
void run_d(const T* x, T* z0, T* z1, size_t n, int threads) {
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads)
    for (long long i = 0; i < (long long)n; ++i) z0[i] = F(x[i], &z1[i]);
}

template <class T, Tw<T> (*F)(Tw<T>, Tw<T>)>
void run_bwd(const T* s0, const T* s1, const T* g0, const T* g1, T* gx0, T* gx1, size_t n,
             int threads) {
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads)
    for (long long i = 0; i < (long long)n; ++i) {
        Tw<T> r = F(Tw<T>{s0[i], s1[i]}, Tw<T>{g0[i], g1[i]});
        gx0[i] = r.x0; gx1[i] = r.x1;
    }
}

/* Op count of F over n elements (single thread): {add, mul, fma, other}. */
template <class U, Cnt<U> (*F)(Cnt<U>, Cnt<U>, Cnt<U>*)>
void count_tw(const U* x0, const U* x1, size_t n, unsigned long long* out) {
    g_cnt = OpCount{0, 0, 0, 0};
    for (size_t i = 0; i < n; ++i) {
        Cnt<U> z1;
        (void)F(Cnt<U>(x0[i]), Cnt<U>(x1[i]), &z1);
    }
    out[0] = g_cnt.add; out[1] = g_cnt.mul; out[2] = g_cnt.fma; out[3] = g_cnt.other;
}

template <class U, Cnt<U> (*F)(Cnt<U>, Cnt<U>*)>
void count_d(const U* x, size_t n, unsigned long long* out) {
    g_cnt = OpCount{0, 0, 0, 0};
    for (size_t i = 0; i < n; ++i) {
        Cnt<U> z1;
        (void)F(Cnt<U>(x[i]), &z1);
    }
    out[0] = g_cnt.add; out[1] = g_cnt.mul; out[2] = g_cnt.fma; out[3] = g_cnt.other;
}

template <class U, Tw<Cnt<U>> (*F)(Tw<Cnt<U>>, Tw<Cnt<U>>)>
void count_bwd(const U* s0, const U* s1, const U* g0, const U* g1, size_t n,
               unsigned long long* out) {
    g_cnt = OpCount{0, 0, 0, 0};
    for (size_t i = 0; i < n; ++i)
        (void)F(Tw<Cnt<U>>{Cnt<U>(s0[i]), Cnt<U>(s1[i])}, Tw<Cnt<U>>{Cnt<U>(g0[i]), Cnt<U>(g1[i])});
    out[0] = g_cnt.add; out[1] = g_cnt.mul; out[2] = g_cnt.fma; out[3] = g_cnt.other;
}

}  // namespace

/* ------------------------------------------------------------------------ */
/* C ABI (loaded with ctypes by oracle/__init__.py)                          */
/* ------------------------------------------------------------------------ */
extern "C" {

#define TFO_TW(NAME, T, FN)                                                                    \
    T tfo_##NAME(T x0, T x1, T* z1) { return FN<T>(x0, x1, z1); }                             \
    void tfo_##NAME##_n(const T* x0, const T* x1, T* z0, T* z1, size_t n, int threads) {     \
        run_tw<T, FN<T>>(x0, x1, z0, z1, n, threads);                                          \
    }                                                                                          \
    void tfo_count_##NAME##_n(const T* x0, const T* x1, size_t n, unsigned long long* out) { \
        count_tw<T, FN<Cnt<T>>>(x0, x1, n, out);                                               \
    }

TFO_TW(texp, double, texp)
TFO_TW(texpm1, double, texpm1)
TFO_TW(tlog, double, tlog)
TFO_TW(tlog1p, double, tlog1p)
TFO_TW(texpf, float, texp)
TFO_TW(texpm1f, float, texpm1)
TFO_TW(tlogf, float, tlog)
TFO_TW(tlog1pf, float, tlog1p)

TFO_TW(texpp, double, texpp)
TFO_TW(pexp, double, pexp)
TFO_TW(texpm1p, double, texpm1p)
TFO_TW(pexpm1, double, pexpm1)
TFO_TW(tlogp, double, tlogp)
TFO_TW(plog, double, plog)
TFO_TW(tlog1pp, double, tlog1pp)
TFO_TW(plog1p, double, plog1p)
TFO_TW(texppf, float, texpp)
TFO_TW(pexpf, float, pexp)
TFO_TW(texpm1pf, float, texpm1p)
TFO_TW(pexpm1f, float, pexpm1)
TFO_TW(tlogpf, float, tlogp)
TFO_TW(plogf, float, plog)
TFO_TW(tlog1ppf, float, tlog1pp)
TFO_TW(plog1pf, float, plog1p)

#define TFO_1X(NAME, T, FN)                                                                  \
    T tfo_##NAME(T x) { return FN<T>(x); }                                                  \
    void tfo_##NAME##_n(const T* x, T* z, size_t n, int threads) { run_1x<T, FN<T>>(x, z, n, threads); }

TFO_1X(exp1x, double, exp1x)
TFO_1X(expm1_1x, double, expm1_1x)
TFO_1X(log1x, double, log1x)
TFO_1X(log1p_1x, double, log1p_1x)
TFO_1X(exp1xf, float, exp1x)
TFO_1X(expm1_1xf, float, expm1_1x)
TFO_1X(log1xf, float, log1x)
TFO_1X(log1p_1xf, float, log1p_1x)

#define TFO_D(NAME, T, FN)                                                                \
    T tfo_##NAME(T x, T* z1) { return FN<T>(x, z1); }                                        \
    void tfo_##NAME##_n(const T* x, T* z0, T* z1, size_t n, int threads) {                  \
        run_d<T, FN<T>>(x, z0, z1, n, threads);                                               \
    }                                                                                         \
    void tfo_count_##NAME##_n(const T* x, size_t n, unsigned long long* out) {              \
        count_d<T, FN<Cnt<T>>>(x, n, out);                                                    \
    }

TFO_D(pexp0, double, pexp0_s)
TFO_D(texp0, double, texp0)
TFO_D(pexpm10, double, pexpm10_s)
TFO_D(texpm10, double, texpm10)
TFO_D(plog0, double, plog0)
TFO_D(tlog0, double, tlog0)
TFO_D(plog1p0, double, plog1p0)
TFO_D(tlog1p0, double, tlog1p0)
TFO_D(pexp0f, float, pexp0_s)
TFO_D(texp0f, float, texp0)
TFO_D(pexpm10f, float, pexpm10_s)
TFO_D(texpm10f, float, texpm10)
TFO_D(plog0f, float, plog0)
TFO_D(tlog0f, float, tlog0)
TFO_D(plog1p0f, float, plog1p0)
TFO_D(tlog1p0f, float, tlog1p0)

#define TFO_BWD(NAME, T, FN)                                                                   \
    void tfo_##NAME##_n(const T* s0, const T* s1, const T* g0, const T* g1, T* gx0, T* gx1,   \
                        size_t n, int threads) {                                               \
        run_bwd<T, FN<T>>(s0, s1, g0, g1, gx0, gx1, n, threads);                               \
    }                                                                                          \
    void tfo_count_##NAME##_n(const T* s0, const T* s1, const T* g0, const T* g1, size_t n,   \
                              unsigned long long* out) {                                       \
        count_bwd<T, FN<Cnt<T>>>(s0, s1, g0, g1, n, out);                                      \
    }

TFO_BWD(texp_bwd, double, bwd_texp)
TFO_BWD(texpm1_bwd, double, bwd_texpm1)
TFO_BWD(tlog_bwd, double, bwd_tlog)
TFO_BWD(tlog1p_bwd, double, bwd_tlog1p)
TFO_BWD(texpf_bwd, float, bwd_texp)
TFO_BWD(texpm1f_bwd, float, bwd_texpm1)
TFO_BWD(tlogf_bwd, float, bwd_tlog)
TFO_BWD(tlog1pf_bwd, float, bwd_tlog1p)

/* Twofold arithmetic: binary operations take (x0, x1, y0, y1). */
#define TFO_ARITH(NAME, T, FN) TFO_BWD(NAME, T, FN)
TFO_ARITH(tadd, double, tadd)
TFO_ARITH(tsub, double, tsub)
TFO_ARITH(tmul, double, tmul)
TFO_ARITH(tdiv, double, tdiv)
TFO_ARITH(taddf, float, tadd)
TFO_ARITH(tsubf, float, tsub)
TFO_ARITH(tmulf, float, tmul)
TFO_ARITH(tdivf, float, tdiv)
TFO_TW(tsqrt, double, tsqrt)
TFO_TW(tsqrtf, float, tsqrt)
TFO_TW(trenorm, double, trenorm)
TFO_TW(trenormf, float, trenorm)

/* Error-free transforms, exported for their exactness pins. */
void tfo_eft_n(int which, const double* a, const double* b, double* s, double* t, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        Tw<double> r = which == 0 ? two_sum(a[i], b[i])
                     : which == 1 ? fast_two_sum(a[i], b[i])
                                  : two_prod(a[i], b[i]);
        s[i] = r.x0; t[i] = r.x1;
    }
}

int tfo_abi_version(void) { return 1; }

}  // extern "C"
