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

// EPT consecutive elements of one thread.
template <class T, int EPT> struct Vec { T v[EPT]; };

// 16-byte vector load/store of a thread's EPT consecutive elements (the
// pointer is 16-byte aligned: the host checks the base pointers).  Built with
// -DTF_NONTEMPORAL=1 the streams use non-temporal accesses (no reuse).
#ifndef TF_NONTEMPORAL
#define TF_NONTEMPORAL 0
#endif
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T, int EPT> __device__ __forceinline__ void vload(Vec<T, EPT>& r, const T* p) {
    if constexpr ((sizeof(T) * EPT) % 16 == 0) {
        constexpr int Q = sizeof(T) * EPT / 16, PER = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const u32x4* src = reinterpret_cast<const u32x4*>(p) + k;
            u32x4 q = TF_NONTEMPORAL ? __builtin_nontemporal_load(src) : *src;
            __builtin_memcpy(&r.v[k * PER], &q, 16);
        }
    } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) r.v[e] = p[e];
    }
}
template <class T, int EPT> __device__ __forceinline__ void vstore(T* p, const Vec<T, EPT>& r) {
    if constexpr ((sizeof(T) * EPT) % 16 == 0) {
        constexpr int Q = sizeof(T) * EPT / 16, PER = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            u32x4 q;
            __builtin_memcpy(&q, &r.v[k * PER], 16);
            u32x4* dst = reinterpret_cast<u32x4*>(p) + k;
            if (TF_NONTEMPORAL) __builtin_nontemporal_store(q, dst);
            else *dst = q;
        }
    } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) p[e] = r.v[e];
    }
}

template <class T, int FN> __device__ __forceinline__ bool fast_arg(T a, T b) {
    if constexpr (FN == FN_TEXP) return texp_fast_arg(a, b);
    else if constexpr (FN == FN_TEXPM1) return texpm1_fast_arg(a, b);
    else if constexpr (FN == FN_TLOG) return tlog_fast_arg(a, b);
    else return tlog1p_fast_arg(a, b);
}

// General form of one element (any argument).
template <class T, int FN, class L>
__device__ __forceinline__ void eval_general(const L& lds, T a, T b, bool x1_tiny, T& r0, T& r1) {
    if constexpr (FN == FN_TEXP) texp_elem<false>(a, b, x1_tiny, lds.et(), lds.pt(), r0, r1);
    else if constexpr (FN == FN_TEXPM1) texpm1_elem(a, b, x1_tiny, lds.et(), lds.pt(), lds.mt(), r0, r1);
    else if constexpr (FN == FN_TLOG) tlog_elem<false>(a, b, lds.lt(), lds.mt(), r0, r1);
    else tlog1p_elem<false>(a, b, lds.lt(), lds.mt(), r0, r1);
}

// Evaluates a thread's EPT elements.  Returns true when the wave took the fast
// form; for texpm1 the fast form leaves the |x0| > ln 2 lanes to the caller
// (bit e of *deferred set for such an element).
template <class T, int FN, int EPT, class L>
__device__ __forceinline__ bool eval_tile(const L& lds, const Vec<T, EPT>& a, const Vec<T, EPT>& b,
                                          Vec<T, EPT>& r0, Vec<T, EPT>& r1, unsigned* deferred) {
    bool fast = true, tiny = true;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        fast = fast && fast_arg<T, FN>(a.v[e], b.v[e]);
        tiny = tiny && (fabs_(b.v[e]) < P<T>::EXPM1_TINY);
    }
    *deferred = 0;
    if (__all(fast)) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if constexpr (FN == FN_TEXP) {
                texp_elem<true>(a.v[e], b.v[e], true, lds.et(), lds.pt(), r0.v[e], r1.v[e]);
            } else if constexpr (FN == FN_TEXPM1) {
                if (texpm1_small_fast(a.v[e], b.v[e], lds.et(), lds.mt(), r0.v[e], r1.v[e]))
                    *deferred |= 1u << e;
            } else if constexpr (FN == FN_TLOG) {
                tlog_elem<true>(a.v[e], b.v[e], lds.lt(), lds.mt(), r0.v[e], r1.v[e]);
            } else {
                tlog1p_elem<true>(a.v[e], b.v[e], lds.lt(), lds.mt(), r0.v[e], r1.v[e]);
            }
        }
        return true;
    }
    const bool x1_tiny = __all(tiny);
#pragma unroll
    for (int e = 0; e < EPT; ++e) eval_general<T, FN>(lds, a.v[e], b.v[e], x1_tiny, r0.v[e], r1.v[e]);
    return false;
}

// Per-wave queue of deferred elements (texpm1 with |x0| > ln 2): the element
// index and its two argument parts in LDS, appended with a ballot prefix count
// and drained 64 at a time with one element per lane, so pexp0 runs on full
// waves and the drain reads no global memory.
template <class T, int CAP> struct WaveQueue {
    size_t* qi;   // this wave's slots: index, x0, x1
    T* qa;
    T* qb;
    int n;        // entries in use (wave-uniform)

    __device__ void push(bool on, size_t idx, T a, T b) {
        const unsigned long long m = __ballot(on);
        const int lane_off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (on) {
            qi[n + lane_off] = idx;
            qa[n + lane_off] = a;
            qb[n + lane_off] = b;
        }
        n += __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // Takes min(n, 64) entries: lane l gets entry l (valid if l < taken).
    __device__ int pop64(int lane, size_t* idx, T* a, T* b) {
        const int taken = n < 64 ? n : 64;
        if (lane < taken) {
            *idx = qi[lane];
            *a = qa[lane];
            *b = qb[lane];
        }
#pragma unroll
        for (int k = 1; k * 64 < CAP; ++k) {
            const int src = k * 64 + lane;
            if (src < n) {
                qi[src - 64] = qi[src];
                qa[src - 64] = qa[src];
                qb[src - 64] = qb[src];
            }
        }
        n -= taken;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return taken;
    }
};

// Drains up to 64 deferred texpm1 elements with the general form; their z0
// was already stored by the fast pass, only z1 is written here.
template <class T, class L, int CAP>
__device__ __forceinline__ void drain_texpm1(const L& lds, WaveQueue<T, CAP>& wq, int lane,
                                             T* z1) {
    size_t i = 0;
    T a = T(1), b = T(0);
    const int taken = wq.pop64(lane, &i, &a, &b);
    if (lane < taken) {
        const bool tiny = __all(fabs_(b) < P<T>::EXPM1_TINY);
        T r0, r1;
        texpm1_elem(a, b, tiny, lds.et(), lds.pt(), lds.mt(), r0, r1);
        z1[i] = r1;
    }
}

// Twofold kernel.  A tile is kBlock*EPT consecutive elements, thread t owning
// elements t*EPT .. t*EPT+EPT-1 (16-byte loads and stores, each wave touching
// one contiguous 64*EPT*sizeof(T) span).  Workgroups walk the full tiles with a
// grid stride and keep the next PD tiles in flight (loaded into registers
// before the current tile is evaluated), so HBM latency overlaps arithmetic.
// The ragged remainder (< one tile) is done by one workgroup with per-element
// guards and the general form.
template <class T, int FN, int EPT, int PD>
__global__ __launch_bounds__(kBlock) void k_twofold(const T* x0, const T* x1, T* z0, T* z1,
                                                    size_t n) {
    constexpr bool QUEUE = FN == FN_TEXPM1;
    constexpr int QCAP = 64 + 64 * EPT;   // < 64 left after a drain, + one tile
    constexpr int QW = QUEUE ? kBlock / 64 : 1, QC = QUEUE ? QCAP : 1;
    __shared__ typename LdsFor<T, FN>::type lds;
    __shared__ size_t q_idx[QW][QC];
    __shared__ T q_x0[QW][QC];
    __shared__ T q_x1[QW][QC];
    lds.load();
    __syncthreads();
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    const size_t stride = gridDim.x;
    const size_t off = (size_t)threadIdx.x * EPT;
    const int lane = threadIdx.x & 63;
    const int w = QUEUE ? threadIdx.x / 64 : 0;
    WaveQueue<T, QCAP> wq{q_idx[w], q_x0[w], q_x1[w], 0};
    Vec<T, EPT> a[PD + 1], b[PD + 1], r0, r1;
#pragma unroll
    for (int s = 0; s <= PD; ++s) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            a[s].v[e] = pad_arg<T>();
            b[s].v[e] = T(0);
        }
    }
    size_t t = blockIdx.x;
#pragma unroll
    for (int s = 0; s < PD; ++s) {
        const size_t ts = t + (size_t)s * stride;
        if (ts < nfull) {
            vload(a[s], x0 + ts * TILE + off);
            vload(b[s], x1 + ts * TILE + off);
        }
    }
    for (; t < nfull; t += stride) {
        const size_t tn = t + (size_t)PD * stride;
        if (tn < nfull) {
            vload(a[PD], x0 + tn * TILE + off);
            vload(b[PD], x1 + tn * TILE + off);
        }
        unsigned deferred;
        eval_tile<T, FN, EPT>(lds, a[0], b[0], r0, r1, &deferred);
        const size_t base = t * TILE + off;
        vstore(z0 + base, r0);
        if (QUEUE && __any(deferred != 0)) {
            // z1 of deferred elements is written by the drain, not here
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool d = (deferred >> e) & 1u;
                if (!d) z1[base + e] = r1.v[e];
                wq.push(d, base + e, a[0].v[e], b[0].v[e]);
            }
            while (wq.n >= 64) drain_texpm1<T>(lds, wq, lane, z1);
        } else {
            vstore(z1 + base, r1);
        }
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            a[s] = a[s + 1];
            b[s] = b[s + 1];
        }
    }
    if constexpr (QUEUE) {
        while (wq.n > 0) drain_texpm1<T>(lds, wq, lane, z1);
    }
    const size_t rbase = nfull * TILE;
    if (rbase < n && blockIdx.x == nfull % stride) {
        bool tiny = true;
        Vec<T, EPT> ra, rb;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            size_t i = rbase + off + e;
            ra.v[e] = i < n ? x0[i] : pad_arg<T>();
            rb.v[e] = i < n ? x1[i] : T(0);
            tiny = tiny && (fabs_(rb.v[e]) < P<T>::EXPM1_TINY);
        }
        const bool x1_tiny = __all(tiny);
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            eval_general<T, FN>(lds, ra.v[e], rb.v[e], x1_tiny, r0.v[e], r1.v[e]);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            size_t i = rbase + off + e;
            if (i < n) {
                z0[i] = r0.v[e];
                z1[i] = r1.v[e];
            }
        }
    }
}

template <class T, int F1>
__device__ __forceinline__ T eval1(const Lds<T, true, false, false, true>& lds, T a) {
    if constexpr (F1 == F1_EXP) return exp1x<false>(a, lds.et());
    else if constexpr (F1 == F1_EXPM1) return expm1_1x<false>(a, lds.et());
    else if constexpr (F1 == F1_LOG) return log1x<false>(a, lds.lt());
    else return log1p_1x<false>(a, lds.lt());
}

template <class T, int F1, int EPT>
__global__ __launch_bounds__(kBlock) void k_onex(const T* x, T* z, size_t n) {
    __shared__ Lds<T, true, false, false, true> lds;
    lds.load();
    __syncthreads();
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    const size_t off = (size_t)threadIdx.x * EPT;
    for (size_t t = blockIdx.x; t < nfull; t += gridDim.x) {
        Vec<T, EPT> a, r;
        vload(a, x + t * TILE + off);
#pragma unroll
        for (int e = 0; e < EPT; ++e) r.v[e] = eval1<T, F1>(lds, a.v[e]);
        vstore(z + t * TILE + off, r);
    }
    const size_t rbase = nfull * TILE;
    if (rbase < n && blockIdx.x == nfull % gridDim.x) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            size_t i = rbase + off + e;
            T r = eval1<T, F1>(lds, i < n ? x[i] : pad_arg<T>());
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

// Launch configuration per (function, format): elements per thread and
// workgroups per compute unit (0 = as many as fit, from the occupancy API).
struct LaunchCfg { int ept; int bpc; int pd; };
// Defaults measured on MI355X (256 CUs) with paper_1502_05216_amd.tune on
// 2^26-element arrays (beyond the last-level cache); the landscape is flat,
// the best few configurations being within a few percent of each other.
LaunchCfg g_cfg[4][2] = {
    {{4, 0, 1}, {4, 2, 1}},   // texp     {binary64, binary32}
    {{1, 4, 1}, {2, 3, 1}},   // texpm1
    {{2, 8, 1}, {4, 6, 2}},   // tlog
    {{2, 8, 1}, {2, 0, 1}},   // tlog1p
};
LaunchCfg g_cfg1[4][2] = {
    {{2, 4, 1}, {4, 4, 1}},   // exp1x
    {{2, 4, 1}, {4, 8, 1}},   // expm1_1x
    {{2, 4, 1}, {4, 4, 1}},   // log1x
    {{2, 8, 1}, {4, 8, 1}},   // log1p_1x
};

template <class K> int blocks_per_cu(K kernel) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, kBlock, 0) != hipSuccess ||
        b <= 0) {
        (void)hipGetLastError();
        b = 2;
    }
    return b;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <class T, int FN, int EPT, int PD>
tf_status launch_twofold_ept(const T* x0, const T* x1, T* z0, T* z1, size_t n, int cus, int bpc,
                             hipStream_t stream) {
    auto kern = k_twofold<T, FN, EPT, PD>;
    static int occ = 0;            // per instantiation; benign race (same value)
    if (occ == 0) occ = blocks_per_cu(kern);
    const size_t tile = (size_t)kBlock * EPT;
    size_t tiles = n / tile;
    size_t cap = (size_t)cus * (bpc > 0 ? bpc : occ);
    unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, stream, x0, x1, z0, z1, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

template <class T, int FN>
tf_status launch_twofold(const T* x0, const T* x1, T* z0, T* z1, size_t n, void* stream) {
    if (n == 0) return TF_OK;
    if (!x0 || !x1 || !z0 || !z1) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    LaunchCfg c = g_cfg[FN][sizeof(T) == 8 ? 0 : 1];
    // vector loads need 16-byte aligned arrays; otherwise one element per thread
    if (!(aligned16(x0) && aligned16(x1) && aligned16(z0) && aligned16(z1))) c.ept = 1;
    hipStream_t s = (hipStream_t)stream;
    const int key = c.ept * 10 + (c.pd == 2 ? 2 : 1);
    switch (key) {
        case 11: return launch_twofold_ept<T, FN, 1, 1>(x0, x1, z0, z1, n, cus, c.bpc, s);
        case 12: return launch_twofold_ept<T, FN, 1, 2>(x0, x1, z0, z1, n, cus, c.bpc, s);
        case 41: return launch_twofold_ept<T, FN, 4, 1>(x0, x1, z0, z1, n, cus, c.bpc, s);
        case 42: return launch_twofold_ept<T, FN, 4, 2>(x0, x1, z0, z1, n, cus, c.bpc, s);
        case 22: return launch_twofold_ept<T, FN, 2, 2>(x0, x1, z0, z1, n, cus, c.bpc, s);
        default: return launch_twofold_ept<T, FN, 2, 1>(x0, x1, z0, z1, n, cus, c.bpc, s);
    }
}

template <class T, int F1, int EPT>
tf_status launch_onex_ept(const T* x, T* z, size_t n, int cus, int bpc, hipStream_t stream) {
    auto kern = k_onex<T, F1, EPT>;
    static int occ = 0;
    if (occ == 0) occ = blocks_per_cu(kern);
    const size_t tile = (size_t)kBlock * EPT;
    size_t tiles = n / tile;
    size_t cap = (size_t)cus * (bpc > 0 ? bpc : occ);
    unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, stream, x, z, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

template <class T, int F1>
tf_status launch_onex(const T* x, T* z, size_t n, void* stream) {
    if (n == 0) return TF_OK;
    if (!x || !z) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    LaunchCfg c = g_cfg1[F1][sizeof(T) == 8 ? 0 : 1];
    if (!(aligned16(x) && aligned16(z))) c.ept = 1;
    hipStream_t s = (hipStream_t)stream;
    switch (c.ept) {
        case 1: return launch_onex_ept<T, F1, 1>(x, z, n, cus, c.bpc, s);
        case 4: return launch_onex_ept<T, F1, 4>(x, z, n, cus, c.bpc, s);
        default: return launch_onex_ept<T, F1, 2>(x, z, n, cus, c.bpc, s);
    }
}

// Backward kernel: streams s0, s1, g0, g1 -> gx0, gx1 (48 B per binary64
// element), grid-stride over tiles of kBlock*EPT elements.
template <class T, int FN, int EPT>
__global__ __launch_bounds__(kBlock) void k_backward(const T* s0, const T* s1, const T* g0,
                                                     const T* g1, T* gx0, T* gx1, size_t n) {
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    const size_t off = (size_t)threadIdx.x * EPT;
    for (size_t t = blockIdx.x; t < nfull; t += gridDim.x) {
        const size_t base = t * TILE + off;
        Vec<T, EPT> a, b, c, d, r0, r1;
        vload(a, s0 + base);
        vload(b, s1 + base);
        vload(c, g0 + base);
        vload(d, g1 + base);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            Tw<T> r = bwd_elem<FN>(Tw<T>{a.v[e], b.v[e]}, Tw<T>{c.v[e], d.v[e]});
            r0.v[e] = r.x0;
            r1.v[e] = r.x1;
        }
        vstore(gx0 + base, r0);
        vstore(gx1 + base, r1);
    }
    const size_t rbase = nfull * TILE;
    if (rbase < n && blockIdx.x == nfull % gridDim.x) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const size_t i = rbase + off + e;
            if (i < n) {
                Tw<T> r = bwd_elem<FN>(Tw<T>{s0[i], s1[i]}, Tw<T>{g0[i], g1[i]});
                gx0[i] = r.x0;
                gx1[i] = r.x1;
            }
        }
    }
}

template <class T, int FN>
tf_status launch_backward(const T* s0, const T* s1, const T* g0, const T* g1, T* gx0, T* gx1,
                          size_t n, void* stream) {
    if (n == 0) return TF_OK;
    if (!s0 || !s1 || !g0 || !g1 || !gx0 || !gx1) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    const bool al = aligned16(s0) && aligned16(s1) && aligned16(g0) && aligned16(g1) &&
                    aligned16(gx0) && aligned16(gx1);
    constexpr int EPT = 16 / sizeof(T);
    const size_t tile = (size_t)kBlock * (al ? EPT : 1);
    size_t tiles = n / tile, cap = (size_t)cus * 4;
    unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    if (al)
        hipLaunchKernelGGL((k_backward<T, FN, EPT>), dim3(grid), dim3(kBlock), 0,
                           (hipStream_t)stream, s0, s1, g0, g1, gx0, gx1, n);
    else
        hipLaunchKernelGGL((k_backward<T, FN, 1>), dim3(grid), dim3(kBlock), 0,
                           (hipStream_t)stream, s0, s1, g0, g1, gx0, gx1, n);
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

#define TF_BWD_ENTRY(NAME, T, FN)                                                            \
    tf_status NAME(const T* s0, const T* s1, const T* g0, const T* g1, T* gx0, T* gx1,       \
                   size_t n, void* stream) {                                                 \
        return launch_backward<T, FN>(s0, s1, g0, g1, gx0, gx1, n, stream);                  \
    }

TF_BWD_ENTRY(tf_texp_bwd, double, 0)
TF_BWD_ENTRY(tf_texpm1_bwd, double, 1)
TF_BWD_ENTRY(tf_tlog_bwd, double, 2)
TF_BWD_ENTRY(tf_tlog1p_bwd, double, 3)
TF_BWD_ENTRY(tf_texpf_bwd, float, 0)
TF_BWD_ENTRY(tf_texpm1f_bwd, float, 1)
TF_BWD_ENTRY(tf_tlogf_bwd, float, 2)
TF_BWD_ENTRY(tf_tlog1pf_bwd, float, 3)

tf_status tf_set_launch_config(int fn, int dtype, int ept, int blocks_per_cu, int prefetch) {
    if (fn < 0 || fn > 7 || dtype < 0 || dtype > 1 || (ept != 1 && ept != 2 && ept != 4) ||
        blocks_per_cu < 0 || blocks_per_cu > 64 || prefetch < 1 || prefetch > 2)
        return TF_EINVAL;
    LaunchCfg& c = fn < 4 ? g_cfg[fn][dtype] : g_cfg1[fn - 4][dtype];
    c.ept = ept;
    c.bpc = blocks_per_cu;
    c.pd = prefetch;
    return TF_OK;
}

tf_status tf_get_launch_config(int fn, int dtype, int* ept, int* blocks_per_cu, int* prefetch) {
    if (fn < 0 || fn > 7 || dtype < 0 || dtype > 1 || !ept || !blocks_per_cu || !prefetch)
        return TF_EINVAL;
    LaunchCfg c = fn < 4 ? g_cfg[fn][dtype] : g_cfg1[fn - 4][dtype];
    *ept = c.ept;
    *blocks_per_cu = c.bpc;
    *prefetch = c.pd;
    return TF_OK;
}

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
