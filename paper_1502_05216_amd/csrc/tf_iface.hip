// The other entry points of the paper's interface (sections "Twofold exponent:
// Algorithm summary", "Twofold logarithm: Algorithm summary", "C/C++
// interface"), as array functions for gfx950:
//
//   dotted argument x0 (x1 = 0):  pexp0 texp0 pexpm10 texpm10
//                                 plog0 tlog0 plog1p0 tlog1p0
//   coupled argument x0 + x1:     texpp pexp texpm1p pexpm1
//                                 tlogp plog tlog1pp plog1p
//
// texpp and texpm1p are texp and texpm1 (the paper gives no special algorithm
// for a coupled argument) and run their kernels.  The others stream x0 (and
// x1) -> z0, z1 once, with the element functions of tf_device.hpp: a wave
// whose lanes all hold an ordinary argument takes the FAST form, any other
// wave the general form (tlog1p0 and tlog1pp share their Newton seeds with the
// main parts on fast waves, as tlog1p does).  There is no deferred-lane queue
// here: on the waves of pexpm10 / texpm10 / pexpm1 that hold a lane with
// |x0| > ln 2 every lane runs pexp0 - 1 as well.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../../include/twofold_hip.h"
#include "tf_common.hpp"

using namespace tfk;

namespace {

enum Vf : int {
    V_PEXP0 = 0, V_TEXP0, V_PEXPM10, V_TEXPM10, V_PLOG0, V_TLOG0, V_PLOG1P0, V_TLOG1P0,
    V_PEXP, V_PEXPM1, V_TLOGP, V_PLOG, V_TLOG1PP, V_PLOG1P
};

template <int VF> struct VfInfo {
    static constexpr bool DOTTED = VF <= V_TLOG1P0;
    static constexpr bool EXP1 = VF == V_PEXP0 || VF == V_TEXP0 || VF == V_PEXP;
    static constexpr bool EXPM1 = VF == V_PEXPM10 || VF == V_TEXPM10 || VF == V_PEXPM1;
    // the twofold function whose launch shape (workgroups per CU) it takes
    static constexpr int BASE = EXP1 ? FN_TEXP
                              : EXPM1 ? FN_TEXPM1
                              : (VF == V_PLOG0 || VF == V_TLOG0 || VF == V_TLOGP || VF == V_PLOG)
                                    ? FN_TLOG
                                    : FN_TLOG1P;
};

// Tables: exp family with the pexp0 tables in LDS (no queue here, so waves
// with large expm1 arguments use them directly), log family as tlog.
template <class T, int VF> struct VfLds {
    using type = typename std::conditional<
        VfInfo<VF>::EXP1, Lds<T, true, true, false, false>,
        typename std::conditional<VfInfo<VF>::EXPM1, Lds<T, true, true, true, false>,
                                  Lds<T, false, false, true, true>>::type>::type;
};

template <class T, int VF> __device__ __forceinline__ bool iface_fast_arg(T a, T b) {
    using K = P<T>;
    if constexpr (VF == V_PEXP0 || VF == V_TEXP0) return a >= K::EXP_XLO && a <= K::EXP_XMAX;
    else if constexpr (VF == V_PEXPM10 || VF == V_TEXPM10) return fabs_(a) <= K::LN2_HI;
    else if constexpr (VF == V_PLOG0 || VF == V_TLOG0) return log_iface_fast_arg<LK_LOG0>(a, b);
    else if constexpr (VF == V_PLOG1P0 || VF == V_TLOG1P0)
        return log_iface_fast_arg<LK_LOG1P0>(a, b);
    else if constexpr (VF == V_PEXP) return texp_fast_arg(a, b);
    else if constexpr (VF == V_PEXPM1) return texpm1_fast_arg(a, b) && fabs_(a) <= K::LN2_HI;
    else if constexpr (VF == V_TLOGP || VF == V_PLOG) return log_iface_fast_arg<LK_LOGC>(a, b);
    else return log_iface_fast_arg<LK_LOG1PC>(a, b);
}

// One element.  x1_tiny: wave-uniform, every lane has |x1| < EXPM1_TINY.
template <class T, int VF, bool FAST, class L>
__device__ __forceinline__ void eval_iface(const L& lds, T a, T b, bool x1_tiny, T& r0, T& r1) {
    if constexpr (VF == V_PEXP0) {
        pexp0_p<FAST>(a, lds.pt(), r0, r1);
    } else if constexpr (VF == V_TEXP0) {
        texp0_elem<FAST>(a, lds.et(), lds.pt(), r0, r1);
    } else if constexpr (VF == V_PEXPM10) {
        pexpm10_p<FAST>(a, lds.pt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_TEXPM10) {
        texpm10_elem<FAST>(a, lds.et(), lds.pt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_PLOG0) {
        log_iface_elem<LK_LOG0, true, FAST>(a, T(0), lds.lt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_TLOG0) {
        log_iface_elem<LK_LOG0, false, FAST>(a, T(0), lds.lt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_PLOG1P0) {
        log_iface_elem<LK_LOG1P0, true, FAST>(a, T(0), lds.lt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_TLOG1P0) {
        log_iface_elem<LK_LOG1P0, false, FAST>(a, T(0), lds.lt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_PEXP) {
        T z0, z1, z2;
        texp_elem<FAST, false>(a, b, FAST || x1_tiny, lds.et(), lds.pt(), z0, z1, &z2);
        if constexpr (kTexpAcc) renorm_out3(z0, z1, z2, r0, r1);
        else renorm_out(z0, z1, r0, r1);
    } else if constexpr (VF == V_PEXPM1) {
        T z0, z1;
        if constexpr (FAST) (void)texpm1_small_fast(a, b, lds.et(), lds.mt(), z0, z1);
        else texpm1_elem(a, b, x1_tiny, lds.et(), lds.pt(), lds.mt(), z0, z1);
        renorm_out(z0, z1, r0, r1);
    } else if constexpr (VF == V_TLOGP) {
        log_iface_elem<LK_LOGC, false, FAST>(a, b, lds.lt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_PLOG) {
        log_iface_elem<LK_LOGC, true, FAST>(a, b, lds.lt(), lds.mt(), r0, r1);
    } else if constexpr (VF == V_TLOG1PP) {
        log_iface_elem<LK_LOG1PC, false, FAST>(a, b, lds.lt(), lds.mt(), r0, r1);
    } else {
        log_iface_elem<LK_LOG1PC, true, FAST>(a, b, lds.lt(), lds.mt(), r0, r1);
    }
}

// tlog1p0 and tlog1pp on a fast wave: the heads, the Newton seeds shared with
// the main parts log1p(y0) (every inner lane of tlog1p0, and of tlog1pp where
// the argument is coupled) or packed (wave_log1p_seeds), the tails.  The same
// values as log_iface_elem, bit for bit.
template <class T, int VF, int EPT, class L>
__device__ __forceinline__ void log1p_iface_fast_tile(const L& lds, const Vec<T, EPT>& a,
                                                      const Vec<T, EPT>& b, Vec<T, EPT>& r0,
                                                      Vec<T, EPT>& r1, T* slot) {
    Log1pCoreHead<T> h[EPT];
    bool any_outer[EPT];
    T arg[EPT], y[EPT], x0[EPT], seed[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        if constexpr (VF == V_TLOG1P0) {
            h[e] = plog1p0_head(a.v[e]);
            arg[e] = plog1p0_seed_arg(h[e], a.v[e]);
            any_outer[e] = true;
        } else {
            h[e] = plog1p_head(Tw<T>{a.v[e], b.v[e]}, any_outer[e]);
            arg[e] = h[e].a.x0 + h[e].a.x1;
        }
        y[e] = a.v[e];
    }
    const LogTab<T> lt = lds.lt();
    wave_log1p_seeds<T, EPT>(arg, y, x0, seed, slot, lt,
                             [&](int e) { return log1p_1x<true>(a.v[e], lt); });
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        Tw<T> X;
        if constexpr (VF == V_TLOG1P0) X = plog1p0_tail<true>(h[e], seed[e], lds.mt());
        else X = plog1p_tail<true>(h[e], seed[e], any_outer[e], lds.mt());
        r0.v[e] = x0[e];
        r1.v[e] = X.x1 + (X.x0 - x0[e]);
    }
}

template <class T, int VF, int EPT, class L>
__device__ __forceinline__ void iface_tile(const L& lds, const Vec<T, EPT>& a, const Vec<T, EPT>& b,
                                           Vec<T, EPT>& r0, Vec<T, EPT>& r1, T* slot) {
    bool fast = true, tiny = true;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        fast = fast && iface_fast_arg<T, VF>(a.v[e], b.v[e]);
        tiny = tiny && (fabs_(b.v[e]) < P<T>::EXPM1_TINY);
    }
    if (__all(fast)) {
        if constexpr (VF == V_TLOG1P0 || VF == V_TLOG1PP) {
            log1p_iface_fast_tile<T, VF, EPT>(lds, a, b, r0, r1, slot);
            return;
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            eval_iface<T, VF, true>(lds, a.v[e], b.v[e], true, r0.v[e], r1.v[e]);
    } else {
        const bool x1_tiny = __all(tiny);
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            eval_iface<T, VF, false>(lds, a.v[e], b.v[e], x1_tiny, r0.v[e], r1.v[e]);
    }
}

// x1 is not read for a dotted-argument function (it may be null).
template <class T, int VF, int EPT>
__global__ __launch_bounds__(kBlock) void k_iface(const T* x0, const T* x1, T* z0, T* z1,
                                                  size_t n) {
    constexpr bool DOT = VfInfo<VF>::DOTTED;
    constexpr bool NT = compute_nt<T, VfInfo<VF>::EXP1>();
    __shared__ typename VfLds<T, VF>::type lds;
    __shared__ SeedSlots ss;                         // tlog1p0 and tlog1pp only
    lds.load();
    __syncthreads();
    T* const slot = seed_slots<T>(ss);
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    const size_t off = (size_t)threadIdx.x * EPT;
    Vec<T, EPT> a[2], b[2], r0, r1;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            a[s].v[e] = pad_arg<T>();
            b[s].v[e] = T(0);
        }
    size_t t = blockIdx.x;
    if (t < nfull) {
        vload<NT>(a[0], x0 + t * TILE + off);
        if constexpr (!DOT) vload<NT>(b[0], x1 + t * TILE + off);
    }
    for (; t < nfull; t += gridDim.x) {
        const size_t tn = t + gridDim.x;                 // next tile, loaded ahead
        if (tn < nfull) {
            vload<NT>(a[1], x0 + tn * TILE + off);
            if constexpr (!DOT) vload<NT>(b[1], x1 + tn * TILE + off);
        }
        iface_tile<T, VF, EPT>(lds, a[0], b[0], r0, r1, slot);
        vstore<NT>(z0 + t * TILE + off, r0);
        vstore<NT>(z1 + t * TILE + off, r1);
        a[0] = a[1];
        b[0] = b[1];
    }
    // ragged remainder (< one tile): one workgroup, per-element guards
    const size_t rbase = nfull * TILE;
    if (rbase < n && blockIdx.x == nfull % gridDim.x) {
        Vec<T, EPT> ra, rb;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const size_t i = rbase + off + e;
            ra.v[e] = i < n ? x0[i] : pad_arg<T>();
            rb.v[e] = (!DOT && i < n) ? x1[i] : T(0);
        }
        iface_tile<T, VF, EPT>(lds, ra, rb, r0, r1, slot);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const size_t i = rbase + off + e;
            if (i < n) {
                z0[i] = r0.v[e];
                z1[i] = r1.v[e];
            }
        }
    }
}

template <class T, int VF, int EPT>
tf_status launch_iface_ept(const T* x0, const T* x1, T* z0, T* z1, size_t n, int cus, int bpc,
                           hipStream_t stream) {
    auto kern = k_iface<T, VF, EPT>;
    static int occ = 0;            // per instantiation; benign race (same value)
    if (occ == 0) occ = blocks_per_cu(kern);
    const size_t tile = (size_t)kBlock * EPT;
    const size_t tiles = n / tile;
    const size_t cap = (size_t)cus * (bpc > 0 ? bpc : occ);
    const unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, stream, x0, x1, z0, z1, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

template <class T, int VF>
tf_status launch_iface(const T* x0, const T* x1, T* z0, T* z1, size_t n, void* stream) {
    constexpr bool DOT = VfInfo<VF>::DOTTED;
    if (n == 0) return TF_OK;
    if (!x0 || (!DOT && !x1) || !z0 || !z1) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    const int bpc = twofold_launch_config(VfInfo<VF>::BASE, sizeof(T) == 8 ? 0 : 1).bpc;
    const bool al = aligned16(x0) && (DOT || aligned16(x1)) && aligned16(z0) && aligned16(z1);
    hipStream_t s = (hipStream_t)stream;
    constexpr int EPT = 16 / sizeof(T);
    if (al) return launch_iface_ept<T, VF, EPT>(x0, x1, z0, z1, n, cus, bpc, s);
    return launch_iface_ept<T, VF, 1>(x0, x1, z0, z1, n, cus, bpc, s);
}

}  // namespace

extern "C" {

#define TF_DOTTED_ENTRY(NAME, T, VF)                                                \
    tf_status NAME(const T* x0, T* z0, T* z1, size_t n, void* stream) {             \
        return launch_iface<T, VF>(x0, nullptr, z0, z1, n, stream);                 \
    }
#define TF_COUPLED_ENTRY(NAME, T, VF)                                                       \
    tf_status NAME(const T* x0, const T* x1, T* z0, T* z1, size_t n, void* stream) {        \
        return launch_iface<T, VF>(x0, x1, z0, z1, n, stream);                              \
    }

TF_DOTTED_ENTRY(tf_pexp0, double, V_PEXP0)
TF_DOTTED_ENTRY(tf_texp0, double, V_TEXP0)
TF_DOTTED_ENTRY(tf_pexpm10, double, V_PEXPM10)
TF_DOTTED_ENTRY(tf_texpm10, double, V_TEXPM10)
TF_DOTTED_ENTRY(tf_plog0, double, V_PLOG0)
TF_DOTTED_ENTRY(tf_tlog0, double, V_TLOG0)
TF_DOTTED_ENTRY(tf_plog1p0, double, V_PLOG1P0)
TF_DOTTED_ENTRY(tf_tlog1p0, double, V_TLOG1P0)
TF_DOTTED_ENTRY(tf_pexp0f, float, V_PEXP0)
TF_DOTTED_ENTRY(tf_texp0f, float, V_TEXP0)
TF_DOTTED_ENTRY(tf_pexpm10f, float, V_PEXPM10)
TF_DOTTED_ENTRY(tf_texpm10f, float, V_TEXPM10)
TF_DOTTED_ENTRY(tf_plog0f, float, V_PLOG0)
TF_DOTTED_ENTRY(tf_tlog0f, float, V_TLOG0)
TF_DOTTED_ENTRY(tf_plog1p0f, float, V_PLOG1P0)
TF_DOTTED_ENTRY(tf_tlog1p0f, float, V_TLOG1P0)

TF_COUPLED_ENTRY(tf_pexp, double, V_PEXP)
TF_COUPLED_ENTRY(tf_pexpm1, double, V_PEXPM1)
TF_COUPLED_ENTRY(tf_tlogp, double, V_TLOGP)
TF_COUPLED_ENTRY(tf_plog, double, V_PLOG)
TF_COUPLED_ENTRY(tf_tlog1pp, double, V_TLOG1PP)
TF_COUPLED_ENTRY(tf_plog1p, double, V_PLOG1P)
TF_COUPLED_ENTRY(tf_pexpf, float, V_PEXP)
TF_COUPLED_ENTRY(tf_pexpm1f, float, V_PEXPM1)
TF_COUPLED_ENTRY(tf_tlogpf, float, V_TLOGP)
TF_COUPLED_ENTRY(tf_plogf, float, V_PLOG)
TF_COUPLED_ENTRY(tf_tlog1ppf, float, V_TLOG1PP)
TF_COUPLED_ENTRY(tf_plog1pf, float, V_PLOG1P)

// texpp / texpm1p: texp / texpm1 (same kernels, same results).
tf_status tf_texpp(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                   void* stream) {
    return tf_texp(x0, x1, z0, z1, n, stream);
}
tf_status tf_texpm1p(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                     void* stream) {
    return tf_texpm1(x0, x1, z0, z1, n, stream);
}
tf_status tf_texppf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                    void* stream) {
    return tf_texpf(x0, x1, z0, z1, n, stream);
}
tf_status tf_texpm1pf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                      void* stream) {
    return tf_texpm1f(x0, x1, z0, z1, n, stream);
}

}  // extern "C"
