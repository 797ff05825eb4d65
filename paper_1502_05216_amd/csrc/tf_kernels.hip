// HIP kernels and the C ABI (include/twofold_hip.h) of the twofold exp/log
// library for gfx950.
//
// Each twofold kernel streams the four split arrays x0, x1 -> z0, z1 through
// HBM once (32 B per element in binary64, 16 B in binary32) and evaluates the
// element on the vector ALUs.  The range-reduction tables of the method are
// copied once per workgroup into LDS; the kernels are grid-stride loops with a
// grid of a few workgroups per compute unit, so that copy is amortised over
// many tiles.  The per-element code is branch-free except for two wave-uniform
// switches taken with wave votes: the tiny-x1 shortcut of expm1(x1) (the
// common case of a coupled argument) and the pexp0(x0) - 1 path of texpm1
// (|x0| > ln 2), which runs only on waves that hold such a lane.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>

#include "../../include/twofold_hip.h"
#include "tf_device.hpp"

using namespace tfh;

namespace {

constexpr int kBlock = 256;

enum Fn : int { FN_TEXP = 0, FN_TEXPM1 = 1, FN_TLOG = 2, FN_TLOG1P = 3 };
enum Fn1 : int { F1_EXP = 0, F1_EXPM1 = 1, F1_LOG = 2, F1_LOG1P = 3 };

// Global copies of the tables (tf_tables.inc), per format.
template <class T> struct G;
template <> struct G<double> {
    __device__ static const double2* E() { return TFH_D_E; }
    __device__ static const int* EK() { return TFH_D_EK; }
    __device__ static const double2* C() { return TFH_D_C; }
    __device__ static const double2* CM1() { return TFH_D_CM1; }
    __device__ static const double2* S() { return TFH_D_S; }
    __device__ static const double2* LOG() { return TFH_D_LOG; }
    __device__ static const double* INVC() { return TFH_D_LOG_INVC; }
};
template <> struct G<float> {
    __device__ static const float2* E() { return TFH_F_E; }
    __device__ static const int* EK() { return TFH_F_EK; }
    __device__ static const float2* C() { return TFH_F_C; }
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
    __device__ Pexp0Tab<T> pt() const { return {E, EK, C}; }
    __device__ Pm1Tab<T> mt() const { return {CM1}; }
    __device__ LogTab<T> lt() const { return {INVC, LG}; }
};

template <class T, int FN> struct LdsFor;
template <class T> struct LdsFor<T, FN_TEXP> { using type = Lds<T, true, true, false, false>; };
template <class T> struct LdsFor<T, FN_TEXPM1> { using type = Lds<T, true, true, true, false>; };
template <class T> struct LdsFor<T, FN_TLOG> { using type = Lds<T, false, false, true, true>; };
template <class T> struct LdsFor<T, FN_TLOG1P> { using type = Lds<T, false, false, true, true>; };

// Argument used for lanes past the end of the array: inside the main range of
// every function, so tail lanes never pull a wave onto a slow path.
template <class T> __device__ __forceinline__ T pad_arg() { return T(0.5); }

template <class T, int FN, class L>
__device__ __forceinline__ void eval(const L& lds, T a, T b, bool x1_tiny, T& r0, T& r1) {
    if constexpr (FN == FN_TEXP) {
        texp_elem(a, b, x1_tiny, lds.et(), lds.pt(), r0, r1);
    } else if constexpr (FN == FN_TEXPM1) {
        texpm1_elem(a, b, x1_tiny, lds.et(), lds.pt(), lds.mt(), r0, r1);
    } else if constexpr (FN == FN_TLOG) {
        tlog_elem(a, b, lds.lt(), lds.mt(), r0, r1);
    } else {
        tlog1p_elem(a, b, lds.lt(), lds.mt(), r0, r1);
    }
}

// Twofold kernel: EPT elements per thread per tile, element index
// tile + e*blockDim + tid so each load/store instruction is coalesced.
template <class T, int FN, int EPT>
__global__ __launch_bounds__(kBlock) void k_twofold(const T* x0, const T* x1, T* z0, T* z1,
                                                    size_t n) {
    __shared__ typename LdsFor<T, FN>::type lds;
    lds.load();
    __syncthreads();
    const size_t tile = (size_t)blockDim.x * EPT;
    for (size_t base = (size_t)blockIdx.x * tile; base < n; base += (size_t)gridDim.x * tile) {
        T a[EPT], b[EPT], r0[EPT], r1[EPT];
        bool tiny = true;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            size_t i = base + (size_t)e * blockDim.x + threadIdx.x;
            a[e] = i < n ? x0[i] : pad_arg<T>();
            b[e] = i < n ? x1[i] : T(0);
            tiny = tiny && (fabs_(b[e]) < P<T>::EXPM1_TINY);
        }
        bool x1_tiny = __all(tiny);
#pragma unroll
        for (int e = 0; e < EPT; ++e) eval<T, FN>(lds, a[e], b[e], x1_tiny, r0[e], r1[e]);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            size_t i = base + (size_t)e * blockDim.x + threadIdx.x;
            if (i < n) {
                z0[i] = r0[e];
                z1[i] = r1[e];
            }
        }
    }
}

template <class T, int F1, int EPT>
__global__ __launch_bounds__(kBlock) void k_onex(const T* x, T* z, size_t n) {
    __shared__ Lds<T, true, false, false, true> lds;
    lds.load();
    __syncthreads();
    const size_t tile = (size_t)blockDim.x * EPT;
    for (size_t base = (size_t)blockIdx.x * tile; base < n; base += (size_t)gridDim.x * tile) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            size_t i = base + (size_t)e * blockDim.x + threadIdx.x;
            T a = i < n ? x[i] : pad_arg<T>();
            T r;
            if constexpr (F1 == F1_EXP) r = exp1x(a, lds.et());
            else if constexpr (F1 == F1_EXPM1) r = expm1_1x(a, lds.et());
            else if constexpr (F1 == F1_LOG) r = log1x(a, lds.lt());
            else r = log1p_1x(a, lds.lt());
            if (i < n) z[i] = r;
        }
    }
}

// ----------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------
constexpr int kMaxDev = 64;
std::atomic<int> g_cu[kMaxDev];   // compute units per device (0 = not queried)

tf_status device_cus(int* cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return TF_ENODEV;
    }
    if (dev < 0 || dev >= kMaxDev) return TF_EUNSUPPORTED;
    int c = g_cu[dev].load(std::memory_order_relaxed);
    if (c == 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0) {
            (void)hipGetLastError();
            return TF_ENODEV;
        }
        g_cu[dev].store(c, std::memory_order_relaxed);
    }
    *cus = c;
    return TF_OK;
}

// Grid: enough workgroups to cover n, capped at a few per compute unit
// (the kernels loop over tiles).
unsigned grid_for(size_t n, int ept, int cus, int per_cu) {
    size_t tiles = (n + (size_t)kBlock * ept - 1) / ((size_t)kBlock * ept);
    size_t cap = (size_t)cus * per_cu;
    return (unsigned)(tiles < cap ? tiles : cap);
}

template <class T, int FN>
tf_status launch_twofold(const T* x0, const T* x1, T* z0, T* z1, size_t n, void* stream) {
    if (n == 0) return TF_OK;
    if (!x0 || !x1 || !z0 || !z1) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    constexpr int EPT = 2;
    unsigned grid = grid_for(n, EPT, cus, 8);
    hipLaunchKernelGGL((k_twofold<T, FN, EPT>), dim3(grid), dim3(kBlock), 0,
                       (hipStream_t)stream, x0, x1, z0, z1, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

template <class T, int F1>
tf_status launch_onex(const T* x, T* z, size_t n, void* stream) {
    if (n == 0) return TF_OK;
    if (!x || !z) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    constexpr int EPT = 2;
    unsigned grid = grid_for(n, EPT, cus, 8);
    hipLaunchKernelGGL((k_onex<T, F1, EPT>), dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       x, z, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

}  // namespace

extern "C" {

#define TF_TWOFOLD_ENTRY(NAME, T, FN)                                                   \
    tf_status NAME(const T* x0, const T* x1, T* z0, T* z1, size_t n, void* stream) {    \
        return launch_twofold<T, FN>(x0, x1, z0, z1, n, stream);                        \
    }

TF_TWOFOLD_ENTRY(tf_texp, double, FN_TEXP)
TF_TWOFOLD_ENTRY(tf_texpm1, double, FN_TEXPM1)
TF_TWOFOLD_ENTRY(tf_tlog, double, FN_TLOG)
TF_TWOFOLD_ENTRY(tf_tlog1p, double, FN_TLOG1P)
TF_TWOFOLD_ENTRY(tf_texpf, float, FN_TEXP)
TF_TWOFOLD_ENTRY(tf_texpm1f, float, FN_TEXPM1)
TF_TWOFOLD_ENTRY(tf_tlogf, float, FN_TLOG)
TF_TWOFOLD_ENTRY(tf_tlog1pf, float, FN_TLOG1P)

#define TF_ONEX_ENTRY(NAME, T, F1)                                       \
    tf_status NAME(const T* x, T* z, size_t n, void* stream) {           \
        return launch_onex<T, F1>(x, z, n, stream);                      \
    }

TF_ONEX_ENTRY(tf_exp1x, double, F1_EXP)
TF_ONEX_ENTRY(tf_expm1_1x, double, F1_EXPM1)
TF_ONEX_ENTRY(tf_log1x, double, F1_LOG)
TF_ONEX_ENTRY(tf_log1p_1x, double, F1_LOG1P)
TF_ONEX_ENTRY(tf_exp1xf, float, F1_EXP)
TF_ONEX_ENTRY(tf_expm1_1xf, float, F1_EXPM1)
TF_ONEX_ENTRY(tf_log1xf, float, F1_LOG)
TF_ONEX_ENTRY(tf_log1p_1xf, float, F1_LOG1P)

const char* tf_status_string(tf_status s) {
    switch (s) {
        case TF_OK: return "ok";
        case TF_EINVAL: return "invalid argument";
        case TF_ELAUNCH: return "kernel launch failed";
        case TF_ENOMEM: return "device allocation failed";
        case TF_EUNSUPPORTED: return "unsupported";
        case TF_ENODEV: return "no HIP device";
    }
    return "unknown status";
}

const char* tf_version(void) { return "twofold_hip 0.1 (gfx950)"; }

int tf_abi_version(void) { return 1; }

}  // extern "C"
