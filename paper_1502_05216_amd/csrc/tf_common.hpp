// Shared pieces of the library's translation units: the LDS images of the
// tables, vector loads/stores of a thread's elements, the packed Newton seeds
// of the log1p kernels' fast waves, and host-side launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "../../include/twofold_hip.h"
#include "tf_device.hpp"

namespace tfk {

using namespace tfh;

constexpr int kBlock = 256;

enum Fn : int { FN_TEXP = 0, FN_TEXPM1 = 1, FN_TLOG = 2, FN_TLOG1P = 3 };
enum Fn1 : int { F1_EXP = 0, F1_EXPM1 = 1, F1_LOG = 2, F1_LOG1P = 3 };

// Global copies of the tables (tf_tables.inc), per format.
template <class T> struct G;
template <> struct G<double> {
    __device__ static const double2* E() { return TFH_D_E; }
    __device__ static const int* EK() { return TFH_D_EK; }
    __device__ static const double2* C() { return pexp0_c_table(0.0); }
    __device__ static const double2* CM1() { return TFH_D_CM1; }
    __device__ static const double2* S() { return TFH_D_S; }
    __device__ static const double2* LOG() { return TFH_D_LOG; }
    __device__ static const double* INVC() { return TFH_D_LOG_INVC; }
};
template <> struct G<float> {
    __device__ static const float2* E() { return TFH_F_E; }
    __device__ static const int* EK() { return TFH_F_EK; }
    __device__ static const float2* C() { return pexp0_c_table(0.0f); }
    __device__ static const float2* CM1() { return TFH_F_CM1; }
    __device__ static const float2* S() { return TFH_F_S; }
    __device__ static const float2* LOG() { return TFH_F_LOG; }
    __device__ static const float* INVC() { return TFH_F_LOG_INVC; }
};

template <class T, class U>
__device__ __forceinline__ void stage(U* dst, const U* src, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
}

// LDS image of the tables one kernel needs.
template <class T, bool EXP, bool PEXP0, bool PM1, bool LOG> struct Lds {
    using V2 = typename P<T>::V2;
    V2 S[EXP ? 32 : 1];
    V2 E[PEXP0 ? P<T>::E_CNT : 1];
    int EK[PEXP0 ? P<T>::E_CNT : 1];
    V2 C[PEXP0 ? P<T>::C_CNT : 1];
    V2 CM1[PM1 ? P<T>::CM1_CNT : 1];
    V2 LG[LOG ? 128 : 1];
    T INVC[LOG ? 128 : 1];

    __device__ void load() {
        if (EXP) stage<T>(S, G<T>::S(), 32);
        if (PEXP0) {
            stage<T>(E, G<T>::E(), P<T>::E_CNT);
            stage<T>(EK, G<T>::EK(), P<T>::E_CNT);
            stage<T>(C, G<T>::C(), P<T>::C_CNT);
        }
        if (PM1) stage<T>(CM1, G<T>::CM1(), P<T>::CM1_CNT);
        if (LOG) {
            stage<T>(LG, G<T>::LOG(), 128);
            stage<T>(INVC, G<T>::INVC(), 128);
        }
    }
    __device__ ExpTab<T> et() const { return {S}; }
    // Without the pexp0 tables in LDS (texpm1, which needs them only for its
    // rare |x0| > ln 2 lanes) they are read from global memory (L1/L2 hits).
    __device__ Pexp0Tab<T> pt() const {
        if constexpr (PEXP0) return {E, EK, C};
        else return {G<T>::E(), G<T>::EK(), G<T>::C()};
    }
    __device__ Pm1Tab<T> mt() const { return {CM1}; }
    __device__ LogTab<T> lt() const { return {INVC, LG}; }
};

// The same accessors over the tables in global memory (read in place, L1/L2
// hits), for launches where a workgroup has about one tile to evaluate and the
// LDS copy would be the larger part of its time.
template <class T> struct GlobalTabs {
    __device__ void load() {}
    __device__ ExpTab<T> et() const { return {G<T>::S()}; }
    __device__ Pexp0Tab<T> pt() const { return {G<T>::E(), G<T>::EK(), G<T>::C()}; }
    __device__ Pm1Tab<T> mt() const { return {G<T>::CM1()}; }
    __device__ LogTab<T> lt() const { return {G<T>::INVC(), G<T>::LOG()}; }
};

template <class T, int FN> struct LdsFor;
template <class T> struct LdsFor<T, FN_TEXP> { using type = Lds<T, true, true, false, false>; };
template <class T> struct LdsFor<T, FN_TEXPM1> { using type = Lds<T, true, false, true, false>; };
template <class T> struct LdsFor<T, FN_TLOG> { using type = Lds<T, false, false, true, true>; };
template <class T> struct LdsFor<T, FN_TLOG1P> { using type = Lds<T, false, false, true, true>; };

// Argument used for lanes past the end of the array: inside the main range of
// every function, so tail lanes never pull a wave onto a slow path.
template <class T> __device__ __forceinline__ T pad_arg() { return T(0.5); }

// EPT consecutive elements of one thread.
template <class T, int EPT> struct Vec { T v[EPT]; };

// 16-byte vector load/store of a thread's EPT consecutive elements (the
// pointer is 16-byte aligned: the host checks the base pointers).  NT: the
// access is non-temporal (streamed data that is not reused).  Measured at
// 2^26 elements, non-temporal streams are 4-8% faster for the purely
// streaming kernels (backward, twofold arithmetic, the 1x functions) and 1-9%
// faster for the twofold-function kernels.  For binary64 texp (one element
// per thread) they save 9% of its time, of which texpm1 in the same
// four-function step gives back two thirds.  TF_STREAM_NT,
// TF_COMPUTE_NT and TF_EXP64_NT (build defines, default 1) switch the
// streaming kernels, the function kernels and, within those, the binary64
// exp family.
#ifndef TF_STREAM_NT
#define TF_STREAM_NT 1
#endif
#ifndef TF_COMPUTE_NT
#define TF_COMPUTE_NT 1
#endif
constexpr bool kStreamNT = TF_STREAM_NT != 0;
#ifndef TF_EXP64_NT
#define TF_EXP64_NT 1
#endif
template <class T, bool EXP_FAMILY> constexpr bool compute_nt() {
    return TF_COMPUTE_NT != 0 && (TF_EXP64_NT != 0 || !(sizeof(T) == 8 && EXP_FAMILY));
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT, class T, int EPT>
__device__ __forceinline__ void vload(Vec<T, EPT>& r, const T* p) {
    if constexpr ((sizeof(T) * EPT) % 16 == 0) {
        constexpr int Q = sizeof(T) * EPT / 16, PER = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const u32x4* src = reinterpret_cast<const u32x4*>(p) + k;
            u32x4 q;
            if constexpr (NT) q = __builtin_nontemporal_load(src);
            else q = *src;
            __builtin_memcpy(&r.v[k * PER], &q, 16);
        }
    } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if constexpr (NT) r.v[e] = __builtin_nontemporal_load(p + e);
            else r.v[e] = p[e];
        }
    }
}
template <bool NT, class T, int EPT>
__device__ __forceinline__ void vstore(T* p, const Vec<T, EPT>& r) {
    if constexpr ((sizeof(T) * EPT) % 16 == 0) {
        constexpr int Q = sizeof(T) * EPT / 16, PER = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            u32x4 q;
            __builtin_memcpy(&q, &r.v[k * PER], 16);
            u32x4* dst = reinterpret_cast<u32x4*>(p) + k;
            if constexpr (NT) __builtin_nontemporal_store(q, dst);
            else *dst = q;
        }
    } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if constexpr (NT) __builtin_nontemporal_store(r.v[e], p + e);
            else p[e] = r.v[e];
        }
    }
}

// Per-wave LDS slots of the packed Newton seeds of the log1p kernels (up to 4
// per lane: 256 binary64 values per wave, reused as binary32).
constexpr int kSeedSlots = 256;
struct SeedSlots {
    double v[kBlock / 64][kSeedSlots];
};
template <class T> __device__ __forceinline__ T* seed_slots(SeedSlots& ss) {
    return reinterpret_cast<T*>(ss.v[threadIdx.x / 64]);
}

// Orders this wave's LDS accesses before and after it (compiler and memory).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The Newton seeds log1p_1x(arg) of the 64 x EPT elements of a fast wave of a
// log1p kernel (every lane active), together with their main parts
// x0 = log1p_1x(y0), which main(e) computes.  Where arg equals y0 bit for bit
// (an inner lane whose argument is already coupled) the seed is x0: both are
// the 1x log1p of the same value in [-1/2, 1], where its steps do not depend
// on the SMALL premise.  The other arguments (|arg| <= 1) are packed into the
// wave's LDS slots by a ballot prefix count and evaluated one per lane, so the
// wave runs one 1x log1p per 64 such elements instead of one per element
// slot.  The main parts are computed between the LDS writes and reads, in the
// same basic block, so that they cover the LDS latency.
template <class T, int EPT, class Main>
__device__ __forceinline__ void wave_log1p_seeds(const T (&arg)[EPT], const T (&y0)[EPT],
                                                 T (&x0)[EPT], T (&seed)[EPT], T* slot,
                                                 LogTab<T> lt, Main&& main) {
    static_assert(64 * EPT <= kSeedSlots, "seed slots");
    const int lane = threadIdx.x & 63;
    bool need[EPT];
    int rank[EPT];
    int total = 0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        need[e] = P<T>::bits(arg[e]) != P<T>::bits(y0[e]);
        const unsigned long long m = __ballot(need[e]);
        rank[e] = total + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        total += __popcll(m);
        if (need[e]) slot[rank[e]] = arg[e];
    }
    wave_sync();
    // first pass: lanes 0..63 take the first 64 packed arguments, beside the
    // main parts of the first half of the elements
    constexpr int H = (EPT + 1) / 2;
    T u = slot[lane];
    u = lane < total ? u : T(0);
#pragma unroll
    for (int e = 0; e < H; ++e) x0[e] = main(e);
    slot[lane] = log1p_1x<true, true>(u, lt);
#pragma unroll
    for (int p = 1; p < EPT; ++p) {
        if (64 * p < total) {                         // wave-uniform
            T w = slot[64 * p + lane];
            w = 64 * p + lane < total ? w : T(0);
            slot[64 * p + lane] = log1p_1x<true, true>(w, lt);
        }
    }
    wave_sync();
#pragma unroll
    for (int e = H; e < EPT; ++e) x0[e] = main(e);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        // an unconditional LDS read, then a select of the value (a select of
        // the two sources would put x0 on the stack)
        const T packed = slot[need[e] ? rank[e] : 0];
        seed[e] = need[e] ? packed : x0[e];
    }
    wave_sync();
}

// ----------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------
// Workgroups per compute unit of the purely streaming kernels (backward,
// twofold arithmetic).  Measured at 2^26 elements: 2 per CU streams at
// 5.3-5.4 TB/s, 4 at 4.7-5.2 and 8 or 16 at 3.9-4.8 (more concurrent streams
// than HBM serves well).
#ifndef TF_STREAM_BPC
#define TF_STREAM_BPC 2
#endif
constexpr int kStreamBpc = TF_STREAM_BPC;

// Compute units of the current device (cached per device).
tf_status device_cus(int* cus);

// Launch configuration per (function, format): elements per thread,
// workgroups per compute unit (0 = as many as fit, from the occupancy API) and
// prefetch depth.
struct LaunchCfg { int ept; int bpc; int pd; };

// The current configuration of twofold function fn (0..3) in format dtype.
LaunchCfg twofold_launch_config(int fn, int dtype);

template <class K> inline int blocks_per_cu(K kernel) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, kBlock, 0) != hipSuccess ||
        b <= 0) {
        (void)hipGetLastError();
        b = 2;
    }
    return b;
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace tfk
