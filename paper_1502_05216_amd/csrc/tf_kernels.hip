// HIP kernels and the C ABI (include/twofold_hip.h) of the twofold exp/log
// library for gfx950.
//
// Each twofold kernel streams the four split arrays x0, x1 -> z0, z1 through
// HBM once (32 B per element in binary64, 16 B in binary32) and evaluates the
// element on the vector ALUs.  The range-reduction tables of the method are
// copied once per workgroup into LDS; the kernels are grid-stride loops with a
// grid of a few workgroups per compute unit, so that copy is amortised over
// many tiles.  A wave whose lanes all hold ordinary arguments runs a
// straight-line fast body; any other wave runs the general body with the edge
// handling.  The rare branch of texpm1 (|x0| > ln 2: pexp0(x0) - 1) does not
// hold the fast body back: such lanes go to a per-wave LDS queue that is
// drained with full waves.  tlog1p's outer branch (the log of 1 + y) runs
// under a wave vote inside the fast body, and its fast waves evaluate only the
// Newton seeds that differ from the main part, packed 64 to a pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/twofold_hip.h"
#include "tf_common.hpp"

using namespace tfk;

// Compute units per device, shared with the other translation unit.
namespace tfk {
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
}  // namespace tfk

namespace {

template <class T, int FN> __device__ __forceinline__ bool fast_arg(T a, T b) {
    if constexpr (FN == FN_TEXP) return texp_fast_arg(a, b);
    else if constexpr (FN == FN_TEXPM1) return texpm1_fast_arg(a, b);
    else if constexpr (FN == FN_TLOG) return tlog_fast_arg(a, b);
    else return tlog1p_fast_arg(a, b);
}

// General form of one element (any argument).
template <class T, int FN, class L>
__device__ __forceinline__ void eval_general(const L& lds, T a, T b, bool x1_tiny, T& r0, T& r1) {
    if constexpr (FN == FN_TEXP) texp_elem<false, true>(a, b, x1_tiny, lds.et(), lds.pt(), r0, r1);
    else if constexpr (FN == FN_TEXPM1) texpm1_elem(a, b, x1_tiny, lds.et(), lds.pt(), lds.mt(), r0, r1);
    else if constexpr (FN == FN_TLOG) tlog_elem<false>(a, b, lds.lt(), lds.mt(), r0, r1);
    else tlog1p_elem<false>(a, b, lds.lt(), lds.mt(), r0, r1);
}

// A fast tlog1p wave's 64 x EPT elements: the heads, the seeds shared with the
// main parts or packed (wave_log1p_seeds), the tails.
template <class T, int EPT>
__device__ __forceinline__ void tlog1p_fast_tile(const Vec<T, EPT>& y0, const Vec<T, EPT>& y1,
                                                 Vec<T, EPT>& r0, Vec<T, EPT>& r1, T* slot,
                                                 LogTab<T> lt, Pm1Tab<T> mt) {
    Tlog1pHead<T> h[EPT];
    bool any_outer[EPT];
    T arg[EPT], y[EPT], x0[EPT], seed[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        h[e] = tlog1p_fast_head(y0.v[e], y1.v[e], any_outer[e]);
        arg[e] = tlog1p_seed_arg(h[e]);
        y[e] = y0.v[e];
    }
    wave_log1p_seeds<T, EPT>(arg, y, x0, seed, slot, lt,
                             [&](int e) { return log1p_1x<true>(y0.v[e], lt); });
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        r0.v[e] = x0[e];
        r1.v[e] = tlog1p_fast_tail(h[e], x0[e], seed[e], any_outer[e], mt);
    }
}

// Evaluates a thread's EPT elements.  Returns true when the wave took the fast
// form; for texpm1 the fast form leaves the |x0| > ln 2 lanes to the caller
// (bit e of *deferred set for such an element).
template <class T, int FN, int EPT, class L>
__device__ __forceinline__ bool eval_tile(const L& lds, const Vec<T, EPT>& a, const Vec<T, EPT>& b,
                                          Vec<T, EPT>& r0, Vec<T, EPT>& r1, unsigned* deferred,
                                          T* slot) {
    bool fast = true, tiny = true;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        fast = fast && fast_arg<T, FN>(a.v[e], b.v[e]);
        tiny = tiny && (fabs_(b.v[e]) < P<T>::EXPM1_TINY);
    }
    *deferred = 0;
    if (__all(fast)) {
        if constexpr (FN == FN_TLOG1P) {
            tlog1p_fast_tile<T, EPT>(a, b, r0, r1, slot, lds.lt(), lds.mt());
            return true;
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if constexpr (FN == FN_TEXP) {
                texp_elem<true, true>(a.v[e], b.v[e], true, lds.et(), lds.pt(), r0.v[e], r1.v[e]);
            } else if constexpr (FN == FN_TEXPM1) {
                if (texpm1_small_fast(a.v[e], b.v[e], lds.et(), lds.mt(), r0.v[e], r1.v[e]))
                    *deferred |= 1u << e;
            } else {
                tlog_elem<true>(a.v[e], b.v[e], lds.lt(), lds.mt(), r0.v[e], r1.v[e]);
            }
        }
        return true;
    }
    const bool x1_tiny = __all(tiny);
#pragma unroll
    for (int e = 0; e < EPT; ++e) eval_general<T, FN>(lds, a.v[e], b.v[e], x1_tiny, r0.v[e], r1.v[e]);
    return false;
}

// Per-wave queue of deferred elements (texpm1 with |x0| > ln 2): the
// destination of z1, the two argument parts and z0, in LDS, appended with a
// ballot prefix count and drained 64 at a time with one element per lane, so
// pexp0 runs on full waves and the drain reads no argument from HBM.  Entries carry
// their destination pointer, so one queue serves any array.  CAP = 128: the
// caller drains after every push that brings n to 64 or more.
template <class T> struct WaveQueue {
    static constexpr int CAP = 128;
    T** qd;       // this wave's slots: z1 destination, x0, x1, z0
    T* qa;
    T* qb;
    T* qz;
    int n;        // entries in use (wave-uniform)

    __device__ void push(bool on, T* dst, T a, T b, T z) {
        const unsigned long long m = __ballot(on);
        const int lane_off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (on) {
            qd[n + lane_off] = dst;
            qa[n + lane_off] = a;
            qb[n + lane_off] = b;
            qz[n + lane_off] = z;
        }
        n += __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // Takes min(n, 64) entries: lane l gets entry l (valid if l < taken).
    __device__ int pop64(int lane, T** dst, T* a, T* b, T* z) {
        const int taken = n < 64 ? n : 64;
        if (lane < taken) {
            *dst = qd[lane];
            *a = qa[lane];
            *b = qb[lane];
            *z = qz[lane];
        }
        const int src = 64 + lane;
        if (src < n) {
            qd[lane] = qd[src];
            qa[lane] = qa[src];
            qb[lane] = qb[src];
            qz[lane] = qz[src];
        }
        n -= taken;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return taken;
    }
};

// LDS slots of the four per-wave queues of a workgroup (sized for binary64,
// reused as binary32).
struct QueueSlots {
    unsigned char raw[kBlock / 64][WaveQueue<double>::CAP * (sizeof(void*) + 3 * sizeof(double))];
};

template <class T> __device__ __forceinline__ WaveQueue<T> wave_queue(QueueSlots& qs) {
    constexpr int C = WaveQueue<T>::CAP;
    unsigned char* base = qs.raw[threadIdx.x / 64];
    return {reinterpret_cast<T**>(base), reinterpret_cast<T*>(base + C * sizeof(void*)),
            reinterpret_cast<T*>(base + C * (sizeof(void*) + sizeof(T))),
            reinterpret_cast<T*>(base + C * (sizeof(void*) + 2 * sizeof(T))), 0};
}

// Functions whose fast waves defer their rare lanes to the queue: texpm1
// (|x0| > ln 2: pexp0 - 1).  tlog1p's outer branch stays under a wave vote:
// it costs 8% of tlog1p on the benchmark's arguments (2.5% of lanes), about
// what the deferral itself costs texpm1 (13% for 4.1% of lanes).
template <int FN> constexpr bool kDefers = FN == FN_TEXPM1;

// Drains up to 64 deferred elements: pexp0(x0) - 1 alone (texpm1_big_fast),
// with the z0 the fast pass computed and stored; only z1 is written here.
// Against the general form (texpm1_elem), this skips a second expm1(x0), the
// pexpm10 small path and the range selects of every drained element.
template <class T, int FN, class L>
__device__ __forceinline__ void drain_deferred(const L& lds, WaveQueue<T>& wq, int lane) {
    T* dst = nullptr;
    T a = T(1), b = T(0), z = T(0);
    const int taken = wq.pop64(lane, &dst, &a, &b, &z);
    if (lane < taken) {
        // dst points to device memory: a global (not flat) store
        *(__attribute__((address_space(1))) T*)dst = texpm1_big_fast(a, b, z, lds.pt());
    }
}

// Whether run_tiles peels its first tile off the loop (the loop then starts in
// its steady state, see below).  Both forms compute the same values; the
// choice only changes where the compiler places its memory-counter waits.
// Measured inside the binary64 step at 2^26 elements per function, peeled:
// texpm1 and tlog ran about 1% faster, texp 0.5-2% slower, tlog1p the same.
// Unpeeled, texpm1 with the pexp0-only drain below ran 3% slower than with a
// drain through the general form: its loop waited on the loads it had just
// issued.
template <int FN> constexpr bool kPeel = FN == FN_TEXPM1 || FN == FN_TLOG;

// Full tiles t = t0, t0 + step, ... < t_end of one array (a tile is kBlock*EPT
// consecutive elements, thread t owning elements t*EPT .. t*EPT+EPT-1, so loads
// and stores are 16 bytes per lane and each wave touches one contiguous span).
// The next PD tiles are kept in flight (loaded into registers before the
// current tile is evaluated), so HBM latency overlaps arithmetic.  Deferred
// texpm1 lanes go to the wave queue, which the caller drains at the end.
template <class T, int FN, int EPT, int PD, class L>
__device__ __forceinline__ void run_tiles(const L& lds, WaveQueue<T>& wq, T* slot, const T* x0,
                                          const T* x1, T* z0, T* z1, size_t t0, size_t t_end,
                                          size_t step) {
    constexpr bool QUEUE = kDefers<FN>;
    constexpr bool NT = compute_nt<T, FN == FN_TEXP>();
    // binary32 texpm1 stores z1 through the caches: a line holds 16 elements,
    // so half of the lines get a drained lane's second write, which can then
    // merge in the caches.  texpm1 at 2^26 elements: binary32 0.231 ms cached
    // against 0.260 ms streamed; binary64 0.476 ms streamed against 0.502 ms
    // cached and 0.502 ms with only the lines that hold a deferred lane cached.
    constexpr bool NT_Z1 = NT && !(QUEUE && sizeof(T) == 4);
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t off = (size_t)threadIdx.x * EPT;
    const int lane = threadIdx.x & 63;
    Vec<T, EPT> a[PD + 1], b[PD + 1], r0, r1;
#pragma unroll
    for (int s = 0; s <= PD; ++s) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            a[s].v[e] = pad_arg<T>();
            b[s].v[e] = T(0);
        }
    }
#pragma unroll
    for (int s = 0; s < PD; ++s) {
        const size_t ts = t0 + (size_t)s * step;
        if (ts < t_end) {
            vload<NT>(a[s], x0 + ts * TILE + off);
            vload<NT>(b[s], x1 + ts * TILE + off);
        }
    }
    // one tile: issue the loads of tile t + PD*step, evaluate and store tile
    // t, rotate the register sets
    auto tile_step = [&](size_t t) __attribute__((always_inline)) {
        const size_t tn = t + (size_t)PD * step;
        if (tn < t_end) {
            vload<NT>(a[PD], x0 + tn * TILE + off);
            vload<NT>(b[PD], x1 + tn * TILE + off);
        }
        unsigned deferred;
        eval_tile<T, FN, EPT>(lds, a[0], b[0], r0, r1, &deferred, slot);
        const size_t base = t * TILE + off;
        vstore<NT>(z0 + base, r0);
        // Every lane stores z1, so each store covers whole lines; a deferred
        // lane's z1 is a placeholder that the drain overwrites later.  Both
        // stores come from this wave, the drain's after the push's release
        // and the pop's acquire fence (wavefront scope), so it lands last.
        // Leaving the deferred lanes out, as masked stores, made 28% of the
        // binary64 z1 lines partial writes (4% of lanes deferred), and texpm1
        // 10% slower at 2^26 elements.
        vstore<NT_Z1>(z1 + base, r1);
        if (QUEUE && __any(deferred != 0)) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool d = (deferred >> e) & 1u;
                wq.push(d, z1 + base + e, a[0].v[e], b[0].v[e], r0.v[e]);
                if (wq.n >= 64) drain_deferred<T, FN>(lds, wq, lane);
            }
        }
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            a[s] = a[s + 1];
            b[s] = b[s + 1];
        }
    };
    if constexpr (kPeel<FN>) {
        // The first tile is peeled off the loop, so the loop is entered in
        // its steady state (stores of the previous tile in flight after the
        // loads of the current one) from both sides: the memory-counter waits
        // the compiler places at the loop head then cover the loads alone,
        // not the stores.
        if (t0 < t_end) tile_step(t0);
        for (size_t t = t0 + step; t < t_end; t += step) tile_step(t);
    } else {
        for (size_t t = t0; t < t_end; t += step) tile_step(t);
    }
}

// Elements [base, end) of one array, fewer than one tile's worth per call
// step: per-element guards and the general form (ragged remainders, and whole
// arrays that are not 16-byte aligned).
template <class T, int FN, int EPT, class L>
__device__ __forceinline__ void run_guarded(const L& lds, const T* x0, const T* x1, T* z0, T* z1,
                                            size_t base, size_t end) {
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t off = (size_t)threadIdx.x * EPT;
    for (size_t b0 = base; b0 < end; b0 += TILE) {
        Vec<T, EPT> ra, rb, r0, r1;
        bool tiny = true;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const size_t i = b0 + off + e;
            ra.v[e] = i < end ? x0[i] : pad_arg<T>();
            rb.v[e] = i < end ? x1[i] : T(0);
            tiny = tiny && (fabs_(rb.v[e]) < P<T>::EXPM1_TINY);
        }
        const bool x1_tiny = __all(tiny);
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            eval_general<T, FN>(lds, ra.v[e], rb.v[e], x1_tiny, r0.v[e], r1.v[e]);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const size_t i = b0 + off + e;
            if (i < end) {
                z0[i] = r0.v[e];
                z1[i] = r1.v[e];
            }
        }
    }
}

// Plain twofold kernel over one array: workgroups walk the full tiles with a
// grid stride; the ragged remainder (< one tile) is done by one workgroup.
// GT: the tables are read from global memory (GlobalTabs), for arrays of a few
// tiles per compute unit; otherwise each workgroup copies them to LDS.
template <class T, int FN, int EPT, int PD, bool GT = false>
__global__ __launch_bounds__(kBlock) void k_twofold(const T* x0, const T* x1, T* z0, T* z1,
                                                    size_t n) {
    using L = typename std::conditional<GT, GlobalTabs<T>, typename LdsFor<T, FN>::type>::type;
    __shared__ L lds;
    __shared__ QueueSlots qs;
    __shared__ SeedSlots ss;
    if constexpr (!GT) {
        lds.load();
        __syncthreads();
    }
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    WaveQueue<T> wq = wave_queue<T>(qs);
    run_tiles<T, FN, EPT, PD>(lds, wq, seed_slots<T>(ss), x0, x1, z0, z1, blockIdx.x, nfull,
                              gridDim.x);
    if constexpr (kDefers<FN>) {
        while (wq.n > 0) drain_deferred<T, FN>(lds, wq, threadIdx.x & 63);
    }
    if (nfull * TILE < n && blockIdx.x == nfull % gridDim.x)
        run_guarded<T, FN, EPT>(lds, x0, x1, z0, z1, nfull * TILE, n);
}

// ----------------------------------------------------------------------------
// Batched ragged launch: many arrays of any length, function and format in one
// persistent launch.  The host cuts every array into chunks of chunk_tiles
// tiles and orders the chunks by estimated cost (dearest first); workgroups
// pull chunks from a device counter and run them with the same tile loop as
// the plain kernels.  The LDS tables are restaged only when the (function,
// format) of the next chunk differs from the current one; with the cost order
// that happens a handful of times per workgroup.
// ----------------------------------------------------------------------------
struct BatchDesc {       // device copy of one tf_batch_desc
    int func, dtype, aligned, pad;
    size_t n;
    const void* x0;
    const void* x1;
    void* z0;
    void* z1;
};
struct BatchChunk {
    unsigned desc, chunk;
};

union BatchLds {
    Lds<double, true, true, false, false> d_exp;
    Lds<double, true, false, true, false> d_expm1;
    Lds<double, false, false, true, true> d_log;
    Lds<float, true, true, false, false> f_exp;
    Lds<float, true, false, true, false> f_expm1;
    Lds<float, false, false, true, true> f_log;
};

__device__ __forceinline__ void batch_stage(BatchLds& lds, int key) {
    switch (key) {
        case 0: lds.d_exp.load(); break;
        case 2: lds.d_expm1.load(); break;
        case 4: case 6: lds.d_log.load(); break;
        case 1: lds.f_exp.load(); break;
        case 3: lds.f_expm1.load(); break;
        default: lds.f_log.load(); break;
    }
}

template <class T, int FN, int EPT, class L>
__device__ __forceinline__ void batch_chunk(const L& lds, WaveQueue<T>& wq, T* slot,
                                            const BatchDesc& d, unsigned chunk,
                                            unsigned chunk_tiles) {
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t start = (size_t)chunk * chunk_tiles * TILE;
    const size_t lim = start + (size_t)chunk_tiles * TILE;
    const size_t end = lim < d.n ? lim : d.n;
    const T* x0 = static_cast<const T*>(d.x0);
    const T* x1 = static_cast<const T*>(d.x1);
    T* z0 = static_cast<T*>(d.z0);
    T* z1 = static_cast<T*>(d.z1);
    size_t g0 = start;
    if (d.aligned) {
        const size_t t0 = start / TILE, t1 = end / TILE;
        run_tiles<T, FN, EPT, 1>(lds, wq, slot, x0, x1, z0, z1, t0, t1, 1);
        g0 = t1 * TILE;
    }
    if (g0 < end) run_guarded<T, FN, EPT>(lds, x0, x1, z0, z1, g0, end);
}

template <int EPT64, int EPT32>
__device__ __forceinline__ void batch_dispatch(BatchLds& lds, WaveQueue<double>& q64,
                                               WaveQueue<float>& q32, SeedSlots& ss,
                                               const BatchDesc& d, int key, unsigned chunk,
                                               unsigned ct) {
    double* s64 = seed_slots<double>(ss);
    float* s32 = seed_slots<float>(ss);
    switch (key) {
        case 0: batch_chunk<double, FN_TEXP, EPT64>(lds.d_exp, q64, s64, d, chunk, ct); break;
        case 2: batch_chunk<double, FN_TEXPM1, EPT64>(lds.d_expm1, q64, s64, d, chunk, ct); break;
        case 4: batch_chunk<double, FN_TLOG, EPT64>(lds.d_log, q64, s64, d, chunk, ct); break;
        case 6: batch_chunk<double, FN_TLOG1P, EPT64>(lds.d_log, q64, s64, d, chunk, ct); break;
        case 1: batch_chunk<float, FN_TEXP, EPT32>(lds.f_exp, q32, s32, d, chunk, ct); break;
        case 3: batch_chunk<float, FN_TEXPM1, EPT32>(lds.f_expm1, q32, s32, d, chunk, ct); break;
        case 5: batch_chunk<float, FN_TLOG, EPT32>(lds.f_log, q32, s32, d, chunk, ct); break;
        default: batch_chunk<float, FN_TLOG1P, EPT32>(lds.f_log, q32, s32, d, chunk, ct); break;
    }
}

// Empties the deferred-lane queue of the (function, format) being left.
__device__ __forceinline__ void batch_drain(BatchLds& lds, WaveQueue<double>& q64,
                                            WaveQueue<float>& q32, int key) {
    const int lane = threadIdx.x & 63;
    if (key == 2) {
        while (q64.n > 0) drain_deferred<double, FN_TEXPM1>(lds.d_expm1, q64, lane);
    } else if (key == 3) {
        while (q32.n > 0) drain_deferred<float, FN_TEXPM1>(lds.f_expm1, q32, lane);
    }
}

__global__ void k_batch_reset(unsigned* counter) { *counter = 0u; }

// Waves per SIMD asked of the register allocator for the fused batch kernel,
// which holds the code of all eight (function, format) pairs.  Measured on the
// 4096-array batch (elements per thread 2/4, 32-tile chunks): 3 waves per SIMD
// 152 Gelem/s, 4 waves 148, 5 waves 142 (more waves, more spills).
#ifndef TF_BATCH_WPE
#define TF_BATCH_WPE 3
#endif

template <int EPT64, int EPT32>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(TF_BATCH_WPE))) void k_batch(const BatchDesc* descs,
                                                  const BatchChunk* chunks, unsigned nchunks,
                                                  unsigned* counter, unsigned chunk_tiles) {
    __shared__ BatchLds lds;
    __shared__ QueueSlots qs;
    __shared__ SeedSlots ss;
    __shared__ unsigned s_chunk;
    WaveQueue<double> q64 = wave_queue<double>(qs);
    WaveQueue<float> q32 = wave_queue<float>(qs);
    int cur = -1;
    for (;;) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(counter, 1u);
        __syncthreads();
        // uniform across the workgroup: keep it (and the descriptor) scalar
        const unsigned c = __builtin_amdgcn_readfirstlane(s_chunk);
        __syncthreads();
        if (c >= nchunks) break;
        const BatchChunk ch = chunks[c];
        const BatchDesc d = descs[ch.desc];
        const int key = d.func * 2 + d.dtype;
        if (key != cur) {
            if (cur >= 0) batch_drain(lds, q64, q32, cur);
            __syncthreads();
            batch_stage(lds, key);
            __syncthreads();
            cur = key;
        }
        batch_dispatch<EPT64, EPT32>(lds, q64, q32, ss, d, key, ch.chunk, chunk_tiles);
    }
    if (cur >= 0) batch_drain(lds, q64, q32, cur);
}

// ----------------------------------------------------------------------------
// Batched launch without allocation (tf_batch_run_noalloc): the plan's device
// tables (descriptors, chunk list, work counter) live in one static device
// array, `scratch`, of fixed size.  The host copies the caller's descriptors
// into it; a one-workgroup planner kernel converts them and writes the chunk
// list, and k_batch runs over it exactly as over a plan's tables.
// ----------------------------------------------------------------------------
constexpr size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaMaxArrays = TF_BATCH_NOALLOC_MAX_ARRAYS;
constexpr size_t kNaMaxChunks = TF_BATCH_NOALLOC_MAX_CHUNKS;
constexpr size_t kNaOffRaw = 256;  // [0, 256): the work counter
constexpr size_t kNaOffDesc = kNaOffRaw + round256(kNaMaxArrays * sizeof(tf_batch_desc));
constexpr size_t kNaOffChunk = kNaOffDesc + round256(kNaMaxArrays * sizeof(BatchDesc));
constexpr size_t kNaBytes = kNaOffChunk + round256(kNaMaxChunks * sizeof(BatchChunk));
static_assert(kNaBytes == TF_BATCH_NOALLOC_SCRATCH_BYTES, "scratch size stated in the header");

// One copy per GPU; host code reaches it only through the address that
// hipGetSymbolAddress returns on that GPU (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct NaPlanArgs {
    unsigned count;             // descriptors in scratch (<= kNaMaxArrays)
    unsigned chunk_elems[2];    // elements per chunk: binary64, binary32
    unsigned class_base[8];     // first chunk slot of each key func*2 + dtype
};

// Converts the raw descriptors and writes the chunk list: the chunks of each
// key in descriptor order, from that key's first slot (the host orders the
// keys dearest first and checked every bound: count, and the chunk total
// that class_base partitions).  Thread t owns a contiguous run of
// descriptors; an exclusive scan over the threads' per-key chunk counts gives
// each run its slots.  Also clears the work counter.
__global__ __launch_bounds__(kBlock) void k_batch_plan_noalloc(unsigned char* scr, NaPlanArgs a) {
    const tf_batch_desc* raw = reinterpret_cast<const tf_batch_desc*>(scr + kNaOffRaw);
    BatchDesc* descs = reinterpret_cast<BatchDesc*>(scr + kNaOffDesc);
    BatchChunk* chunks = reinterpret_cast<BatchChunk*>(scr + kNaOffChunk);
    __shared__ unsigned run[kBlock][8];
    const unsigned t = threadIdx.x;
    const unsigned seg = (a.count + kBlock - 1) / kBlock;
    const unsigned i0 = t * seg < a.count ? t * seg : a.count;
    const unsigned i1 = i0 + seg < a.count ? i0 + seg : a.count;
#pragma unroll
    for (int k = 0; k < 8; ++k) run[t][k] = 0u;
    for (unsigned i = i0; i < i1; ++i) {
        const tf_batch_desc d = raw[i];
        const uintptr_t bits = (uintptr_t)d.x0 | (uintptr_t)d.x1 | (uintptr_t)d.z0 |
                               (uintptr_t)d.z1;
        descs[i] = BatchDesc{d.func, d.dtype, (bits & 15u) == 0 ? 1 : 0, 0, d.n, d.x0, d.x1,
                             d.z0, d.z1};
        const size_t ce = a.chunk_elems[d.dtype];
        run[t][d.func * 2 + d.dtype] += (unsigned)((d.n + ce - 1) / ce);
    }
    __syncthreads();
    if (t < 8) {
        unsigned next = a.class_base[t];
        for (unsigned u = 0; u < kBlock; ++u) {
            const unsigned c = run[u][t];
            run[u][t] = next;
            next += c;
        }
    }
    __syncthreads();
    for (unsigned i = i0; i < i1; ++i) {
        const tf_batch_desc d = raw[i];
        const size_t ce = a.chunk_elems[d.dtype];
        const unsigned nch = (unsigned)((d.n + ce - 1) / ce);
        const int key = d.func * 2 + d.dtype;
        const unsigned off = run[t][key];
        run[t][key] = off + nch;
        for (unsigned k = 0; k < nch; ++k) chunks[off + k] = BatchChunk{i, k};
    }
    if (t == 0) *reinterpret_cast<unsigned*>(scr) = 0u;
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
        vload<kStreamNT>(a, x + t * TILE + off);
#pragma unroll
        for (int e = 0; e < EPT; ++e) r.v[e] = eval1<T, F1>(lds, a.v[e]);
        vstore<kStreamNT>(z + t * TILE + off, r);
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
// Launch configuration per (function, format): elements per thread and
// workgroups per compute unit (0 = as many as fit, from the occupancy API).
// Defaults measured on MI355X (256 CUs) with paper_1502_05216_amd.tune on
// 2^26-element arrays (beyond the last-level cache), then checked inside the
// four-function binary64 step; the landscape is flat, the best few
// configurations being within a few percent of each other.  More workgroups
// than fit at once (bpc 12) shorten the tail of the grid-stride loop for the
// ALU-bound tlog1p.
LaunchCfg g_cfg[4][2] = {
    {{1, 4, 2}, {4, 4, 1}},   // texp     {binary64, binary32}
    {{1, 4, 1}, {2, 12, 1}},  // texpm1
    {{2, 6, 2}, {4, 12, 2}},  // tlog
    {{2, 12, 1}, {4, 12, 1}}, // tlog1p
};
LaunchCfg g_cfg1[4][2] = {
    {{2, 4, 1}, {4, 4, 1}},   // exp1x
    {{2, 4, 1}, {4, 8, 1}},   // expm1_1x
    {{2, 4, 1}, {4, 4, 1}},   // log1x
    {{2, 8, 1}, {4, 8, 1}},   // log1p_1x
};

// Table placement of the twofold-function kernels (tf_set_table_placement).
std::atomic<int> g_tables{TF_TABLES_AUTO};

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
    // A few tiles per compute unit: the LDS copy of the tables would not pay
    // for itself, so they are read from global memory (one prefetch stage).
    // Timed from replayed graphs at 2^17..2^21 elements against the LDS form,
    // the break-even lies beyond 8 tiles per CU in binary64 (e.g. texp at
    // 2^19: 5.4 against 6.2 us) and at 2-4 in binary32 (texp at 2^20: 4.7
    // against 5.2 us with global tables at 4 tiles per CU).
    const int tm = g_tables.load(std::memory_order_relaxed);
    if (tm == TF_TABLES_GLOBAL ||
        (tm == TF_TABLES_AUTO && tiles <= (size_t)cus * (sizeof(T) == 8 ? 8 : 2)))
        kern = k_twofold<T, FN, EPT, 1, true>;
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
        vload<kStreamNT>(a, s0 + base);
        vload<kStreamNT>(b, s1 + base);
        vload<kStreamNT>(c, g0 + base);
        vload<kStreamNT>(d, g1 + base);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            Tw<T> r = bwd_elem<FN>(Tw<T>{a.v[e], b.v[e]}, Tw<T>{c.v[e], d.v[e]});
            r0.v[e] = r.x0;
            r1.v[e] = r.x1;
        }
        vstore<kStreamNT>(gx0 + base, r0);
        vstore<kStreamNT>(gx1 + base, r1);
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
    size_t tiles = n / tile, cap = (size_t)cus * kStreamBpc;
    unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    if (al)
        hipLaunchKernelGGL((k_backward<T, FN, EPT>), dim3(grid), dim3(kBlock), 0,
                           (hipStream_t)stream, s0, s1, g0, g1, gx0, gx1, n);
    else
        hipLaunchKernelGGL((k_backward<T, FN, 1>), dim3(grid), dim3(kBlock), 0,
                           (hipStream_t)stream, s0, s1, g0, g1, gx0, gx1, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

// Backward of a chain of twofold functions in one pass (tf_chain_bwd).  The
// stage adjoints of k_backward are applied on registers from the last stage
// to the first, so the gradient equals that of the chained single-stage
// calls bit for bit, while every saved array is read once (a stage that
// saved the same arrays as the next one reuses its registers) and the
// intermediate gradients never reach HBM.  Up to TF_CHAIN_MAX stages; the
// stage count and functions are kernel arguments, uniform across the grid.
constexpr int kChainMax = TF_CHAIN_MAX;

template <class T> struct ChainArgs {
    int k;
    int fn[kChainMax];
    int reuse[kChainMax];            // stage j saved the same arrays as stage j + 1
    const T* s0[kChainMax];
    const T* s1[kChainMax];
};

template <class T, int EPT>
__device__ __forceinline__ void chain_stage(int fn, const Vec<T, EPT>& sa, const Vec<T, EPT>& sb,
                                            Vec<T, EPT>& ga, Vec<T, EPT>& gb) {
#define TF_STAGE(F)                                                                          \
    _Pragma("unroll") for (int e = 0; e < EPT; ++e) {                                        \
        Tw<T> r = bwd_elem<F>(Tw<T>{sa.v[e], sb.v[e]}, Tw<T>{ga.v[e], gb.v[e]});            \
        ga.v[e] = r.x0;                                                                      \
        gb.v[e] = r.x1;                                                                      \
    }
    switch (fn) {                    // wave-uniform: a scalar branch
        case 0: TF_STAGE(0) break;
        case 1: TF_STAGE(1) break;
        case 2: TF_STAGE(2) break;
        default: TF_STAGE(3) break;
    }
#undef TF_STAGE
}

template <class T, int EPT>
__global__ __launch_bounds__(kBlock) void k_chain_bwd(ChainArgs<T> a, const T* g0, const T* g1,
                                                      T* gx0, T* gx1, size_t n) {
    constexpr size_t TILE = (size_t)kBlock * EPT;
    const size_t nfull = n / TILE;
    const size_t off = (size_t)threadIdx.x * EPT;
    for (size_t t = blockIdx.x; t < nfull; t += gridDim.x) {
        const size_t base = t * TILE + off;
        Vec<T, EPT> sa[kChainMax], sb[kChainMax], ga, gb;
        // every load of the element group is issued before the first stage
#pragma unroll
        for (int j = kChainMax - 1; j >= 0; --j) {
            if (j < a.k) {
                if (j + 1 < a.k && a.reuse[j]) {
                    sa[j] = sa[j + 1];
                    sb[j] = sb[j + 1];
                } else {
                    vload<kStreamNT>(sa[j], a.s0[j] + base);
                    vload<kStreamNT>(sb[j], a.s1[j] + base);
                }
            }
        }
        vload<kStreamNT>(ga, g0 + base);
        vload<kStreamNT>(gb, g1 + base);
#pragma unroll
        for (int j = kChainMax - 1; j >= 0; --j)
            if (j < a.k) chain_stage<T, EPT>(a.fn[j], sa[j], sb[j], ga, gb);
        vstore<kStreamNT>(gx0 + base, ga);
        vstore<kStreamNT>(gx1 + base, gb);
    }
    const size_t rbase = nfull * TILE;
    if (rbase < n && blockIdx.x == nfull % gridDim.x) {
        for (int e = 0; e < EPT; ++e) {
            const size_t i = rbase + off + e;
            if (i < n) {
                Vec<T, 1> ra, rb;
                ra.v[0] = g0[i];
                rb.v[0] = g1[i];
                for (int j = a.k - 1; j >= 0; --j) {
                    Vec<T, 1> qa, qb;
                    qa.v[0] = a.s0[j][i];
                    qb.v[0] = a.s1[j][i];
                    chain_stage<T, 1>(a.fn[j], qa, qb, ra, rb);
                }
                gx0[i] = ra.v[0];
                gx1[i] = rb.v[0];
            }
        }
    }
}

template <class T>
tf_status launch_chain_bwd(int k, const int* fns, const T* const* s0, const T* const* s1,
                           const T* g0, const T* g1, T* gx0, T* gx1, size_t n, void* stream) {
    if (k < 1 || k > kChainMax || !fns || !s0 || !s1) return TF_EINVAL;
    ChainArgs<T> a{};
    a.k = k;
    bool al = aligned16(g0) && aligned16(g1) && aligned16(gx0) && aligned16(gx1);
    for (int j = 0; j < k; ++j) {
        if (fns[j] < 0 || fns[j] > 3) return TF_EINVAL;
        if (n > 0 && (!s0[j] || !s1[j])) return TF_EINVAL;
        a.fn[j] = fns[j];
        a.s0[j] = s0[j];
        a.s1[j] = s1[j];
        a.reuse[j] = j + 1 < k && s0[j] == s0[j + 1] && s1[j] == s1[j + 1];
        al = al && aligned16(s0[j]) && aligned16(s1[j]);
    }
    if (n == 0) return TF_OK;
    if (!g0 || !g1 || !gx0 || !gx1) return TF_EINVAL;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    constexpr int EPT = 16 / sizeof(T);
    const size_t tile = (size_t)kBlock * (al ? EPT : 1);
    size_t tiles = n / tile, cap = (size_t)cus * kStreamBpc;
    unsigned grid = (unsigned)(tiles == 0 ? 1 : (tiles < cap ? tiles : cap));
    if (al)
        hipLaunchKernelGGL((k_chain_bwd<T, EPT>), dim3(grid), dim3(kBlock), 0,
                           (hipStream_t)stream, a, g0, g1, gx0, gx1, n);
    else
        hipLaunchKernelGGL((k_chain_bwd<T, 1>), dim3(grid), dim3(kBlock), 0,
                           (hipStream_t)stream, a, g0, g1, gx0, gx1, n);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_ELAUNCH;
}

// Relative cost per element of each (function, format), used to order the
// chunks of a batch (measured plain-kernel times on 2^26 elements).
constexpr double kCost[4][2] = {{1.00, 0.46}, {1.25, 0.64}, {1.28, 0.61}, {1.35, 0.60}};

}  // namespace

LaunchCfg tfk::twofold_launch_config(int fn, int dtype) { return g_cfg[fn][dtype]; }

struct tf_batch_plan {
    BatchDesc* d_descs = nullptr;
    BatchChunk* d_chunks = nullptr;
    unsigned* d_counter = nullptr;
    unsigned nchunks = 0;
    size_t elements = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace {

void plan_free(tf_batch_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_descs) (void)hipFree(p->d_descs);
    if (p->d_chunks) (void)hipFree(p->d_chunks);
    if (p->d_counter) (void)hipFree(p->d_counter);
    delete p;
}

template <int E64, int E32>
tf_status batch_capture(tf_batch_plan* p, int cus, int bpc, unsigned chunk_tiles) {
    auto kern = k_batch<E64, E32>;
    int occ = blocks_per_cu(kern);
    unsigned grid = (unsigned)cus * (unsigned)(bpc > 0 ? bpc : occ);
    if (grid > p->nchunks) grid = p->nchunks > 0 ? p->nchunks : 1;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return TF_ELAUNCH;
    tf_status st = TF_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
        st = TF_ELAUNCH;
    } else {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, p->d_counter);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, p->d_descs, p->d_chunks,
                           p->nchunks, p->d_counter, chunk_tiles);
        if (hipStreamEndCapture(s, &p->graph) != hipSuccess ||
            hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
            st = TF_ELAUNCH;
    }
    (void)hipStreamDestroy(s);
    (void)hipGetLastError();
    return st;
}

// This GPU's address of `scratch`, taken once per device with that device
// current (each GPU holds its own copy of the array).
std::atomic<unsigned char*> g_scratch[kMaxDev];

tf_status noalloc_scratch(unsigned char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return TF_ENODEV;
    }
    if (dev < 0 || dev >= kMaxDev) return TF_EUNSUPPORTED;
    unsigned char* p = g_scratch[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || q == nullptr) {
            (void)hipGetLastError();
            return TF_ELAUNCH;
        }
        p = static_cast<unsigned char*>(q);
        g_scratch[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return TF_OK;
}

template <int E64, int E32>
tf_status noalloc_batch(unsigned char* scr, unsigned nchunks, int cus, int bpc,
                        unsigned chunk_tiles, hipStream_t s) {
    auto kern = k_batch<E64, E32>;
    static int occ = 0;            // per instantiation; benign race (same value)
    if (occ == 0) occ = blocks_per_cu(kern);
    unsigned grid = (unsigned)cus * (unsigned)(bpc > 0 ? bpc : occ);
    if (grid > nchunks) grid = nchunks;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s,
                       reinterpret_cast<const BatchDesc*>(scr + kNaOffDesc),
                       reinterpret_cast<const BatchChunk*>(scr + kNaOffChunk), nchunks,
                       reinterpret_cast<unsigned*>(scr), chunk_tiles);
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

tf_status tf_chain_bwd(int k, const int* fns, const double* const* s0, const double* const* s1,
                       const double* g0, const double* g1, double* gx0, double* gx1, size_t n,
                       void* stream) {
    return launch_chain_bwd<double>(k, fns, s0, s1, g0, g1, gx0, gx1, n, stream);
}
tf_status tf_chain_bwdf(int k, const int* fns, const float* const* s0, const float* const* s1,
                        const float* g0, const float* g1, float* gx0, float* gx1, size_t n,
                        void* stream) {
    return launch_chain_bwd<float>(k, fns, s0, s1, g0, g1, gx0, gx1, n, stream);
}

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

tf_status tf_set_table_placement(int mode) {
    if (mode != TF_TABLES_AUTO && mode != TF_TABLES_LDS && mode != TF_TABLES_GLOBAL)
        return TF_EINVAL;
    g_tables.store(mode, std::memory_order_relaxed);
    return TF_OK;
}

int tf_get_table_placement(void) { return g_tables.load(std::memory_order_relaxed); }

tf_status tf_batch_plan_create(const tf_batch_desc* descs, size_t count,
                               const tf_batch_config* config, tf_batch_plan** out) {
    if (!out || (count > 0 && !descs)) return TF_EINVAL;
    *out = nullptr;
    tf_batch_config c = {2, 4, 32, 0};
    if (config) c = *config;
    if (!((c.ept64 == 2 && c.ept32 == 4) || (c.ept64 == 4 && c.ept32 == 4) ||
          (c.ept64 == 1 && c.ept32 == 2)) ||
        c.chunk_tiles < 1 || c.chunk_tiles > 4096 || c.blocks_per_cu < 0 || c.blocks_per_cu > 64)
        return TF_EINVAL;
    if (count > 0xffffffffu) return TF_EINVAL;
    for (size_t i = 0; i < count; ++i) {
        const tf_batch_desc& d = descs[i];
        if (d.func < 0 || d.func > 3 || d.dtype < 0 || d.dtype > 1) return TF_EINVAL;
        if (d.n > 0 && (!d.x0 || !d.x1 || !d.z0 || !d.z1)) return TF_EINVAL;
    }
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    std::vector<BatchDesc> hd(count);
    struct Item { double cost; BatchChunk ch; };
    std::vector<Item> items;
    size_t total = 0;
    for (size_t i = 0; i < count; ++i) {
        const tf_batch_desc& d = descs[i];
        const bool al = aligned16(d.x0) && aligned16(d.x1) && aligned16(d.z0) && aligned16(d.z1);
        hd[i] = BatchDesc{d.func, d.dtype, al ? 1 : 0, 0, d.n, d.x0, d.x1, d.z0, d.z1};
        const size_t chunk = (size_t)c.chunk_tiles * kBlock * (d.dtype == 0 ? c.ept64 : c.ept32);
        const size_t nch = (d.n + chunk - 1) / chunk;
        if (nch > 0xffffffffull) return TF_EINVAL;
        for (size_t k = 0; k < nch; ++k) {
            const size_t len = (k + 1 < nch) ? chunk : d.n - k * chunk;
            items.push_back({(double)len * kCost[d.func][d.dtype], {(unsigned)i, (unsigned)k}});
        }
        total += d.n;
    }
    if (items.size() > 0xffffffffull) return TF_EINVAL;
    // dearest chunks first; equal costs keep descriptor order
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<BatchChunk> hc(items.size());
    for (size_t k = 0; k < items.size(); ++k) hc[k] = items[k].ch;

    tf_batch_plan* p = new (std::nothrow) tf_batch_plan();
    if (!p) return TF_ENOMEM;
    p->nchunks = (unsigned)hc.size();
    p->elements = total;
    (void)hipGetDevice(&p->device);
    const size_t dbytes = hd.size() * sizeof(BatchDesc), cbytes = hc.size() * sizeof(BatchChunk);
    if (hipMalloc(&p->d_descs, dbytes > 0 ? dbytes : 16) != hipSuccess ||
        hipMalloc(&p->d_chunks, cbytes > 0 ? cbytes : 16) != hipSuccess ||
        hipMalloc(&p->d_counter, sizeof(unsigned)) != hipSuccess) {
        (void)hipGetLastError();
        plan_free(p);
        return TF_ENOMEM;
    }
    if ((dbytes && hipMemcpy(p->d_descs, hd.data(), dbytes, hipMemcpyHostToDevice) != hipSuccess) ||
        (cbytes && hipMemcpy(p->d_chunks, hc.data(), cbytes, hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipGetLastError();
        plan_free(p);
        return TF_ELAUNCH;
    }
    if (p->nchunks > 0) {
        if (c.ept64 == 2) st = batch_capture<2, 4>(p, cus, c.blocks_per_cu, c.chunk_tiles);
        else if (c.ept64 == 4) st = batch_capture<4, 4>(p, cus, c.blocks_per_cu, c.chunk_tiles);
        else st = batch_capture<1, 2>(p, cus, c.blocks_per_cu, c.chunk_tiles);
        if (st != TF_OK) {
            plan_free(p);
            return st;
        }
    }
    *out = p;
    return TF_OK;
}

tf_status tf_batch_launch(tf_batch_plan* plan, void* stream) {
    if (!plan) return TF_EINVAL;
    if (plan->nchunks == 0) return TF_OK;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? TF_OK : TF_ELAUNCH;
}

tf_status tf_batch_plan_destroy(tf_batch_plan* plan) {
    if (!plan) return TF_EINVAL;
    plan_free(plan);
    return TF_OK;
}

tf_status tf_batch_plan_info(const tf_batch_plan* plan, size_t* chunks, size_t* elements) {
    if (!plan) return TF_EINVAL;
    if (chunks) *chunks = plan->nchunks;
    if (elements) *elements = plan->elements;
    return TF_OK;
}

tf_status tf_batch_run_noalloc(const tf_batch_desc* descs, size_t count,
                               const tf_batch_config* config, void* stream) {
    if (count > 0 && !descs) return TF_EINVAL;
    tf_batch_config c = {2, 4, 32, 0};
    if (config) c = *config;
    if (!((c.ept64 == 2 && c.ept32 == 4) || (c.ept64 == 4 && c.ept32 == 4) ||
          (c.ept64 == 1 && c.ept32 == 2)) ||
        c.chunk_tiles < 1 || c.chunk_tiles > 4096 || c.blocks_per_cu < 0 || c.blocks_per_cu > 64)
        return TF_EINVAL;
    if (count > kNaMaxArrays) return TF_ECAPACITY;
    // validate and count the chunks per key (no buffer: a pass over descs)
    const size_t ce[2] = {(size_t)c.chunk_tiles * kBlock * c.ept64,
                          (size_t)c.chunk_tiles * kBlock * c.ept32};
    size_t per_key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    size_t total = 0;
    for (size_t i = 0; i < count; ++i) {
        const tf_batch_desc& d = descs[i];
        if (d.func < 0 || d.func > 3 || d.dtype < 0 || d.dtype > 1) return TF_EINVAL;
        if (d.n > 0 && (!d.x0 || !d.x1 || !d.z0 || !d.z1)) return TF_EINVAL;
        const size_t nch = d.n / ce[d.dtype] + (d.n % ce[d.dtype] != 0);
        if (nch > kNaMaxChunks) return TF_ECAPACITY;
        per_key[d.func * 2 + d.dtype] += nch;
        total += nch;
        if (total > kNaMaxChunks) return TF_ECAPACITY;
    }
    if (total == 0) return TF_OK;
    int cus = 0;
    tf_status st = device_cus(&cus);
    if (st != TF_OK) return st;
    unsigned char* scr = nullptr;
    st = noalloc_scratch(&scr);
    if (st != TF_OK) return st;
    // keys dearest first by the cost of a full chunk, as the plan orders
    // its chunks (ties: lower key first)
    int order[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    auto full_cost = [&](int key) { return (double)ce[key & 1] * kCost[key >> 1][key & 1]; };
    std::stable_sort(order, order + 8, [&](int a, int b) { return full_cost(a) > full_cost(b); });
    NaPlanArgs a{};
    a.count = (unsigned)count;
    a.chunk_elems[0] = (unsigned)ce[0];
    a.chunk_elems[1] = (unsigned)ce[1];
    unsigned base = 0;
    for (int j = 0; j < 8; ++j) {
        a.class_base[order[j]] = base;
        base += (unsigned)per_key[order[j]];
    }
    hipStream_t s = (hipStream_t)stream;
    // the descriptors are read from host memory before this call returns
    if (hipMemcpyAsync(scr + kNaOffRaw, descs, count * sizeof(tf_batch_desc),
                       hipMemcpyHostToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        return TF_ELAUNCH;
    }
    hipLaunchKernelGGL(k_batch_plan_noalloc, dim3(1), dim3(kBlock), 0, s, scr, a);
    if (hipGetLastError() != hipSuccess) return TF_ELAUNCH;
    const unsigned nch = (unsigned)total;
    if (c.ept64 == 2) return noalloc_batch<2, 4>(scr, nch, cus, c.blocks_per_cu, c.chunk_tiles, s);
    if (c.ept64 == 4) return noalloc_batch<4, 4>(scr, nch, cus, c.blocks_per_cu, c.chunk_tiles, s);
    return noalloc_batch<1, 2>(scr, nch, cus, c.blocks_per_cu, c.chunk_tiles, s);
}

const char* tf_status_string(tf_status s) {
    switch (s) {
        case TF_OK: return "ok";
        case TF_EINVAL: return "invalid argument";
        case TF_ELAUNCH: return "kernel launch failed";
        case TF_ENOMEM: return "device allocation failed";
        case TF_EUNSUPPORTED: return "unsupported";
        case TF_ENODEV: return "no HIP device";
        case TF_ECAPACITY: return "beyond the static capacity of tf_batch_run_noalloc";
    }
    return "unknown status";
}

const char* tf_version(void) {
#if TF_HORNER_1X_TAIL && TF_PEXP0_K == 6
    return "twofold_hip 0.2 (gfx950; Horner with 1x tails; pexp0 K=6)";
#elif TF_HORNER_1X_TAIL && TF_TEXP_ACC
    return "twofold_hip 0.2 (gfx950; Horner with 1x tails; texp exact z0 t1)";
#elif TF_HORNER_1X_TAIL
    return "twofold_hip 0.2 (gfx950; Horner with 1x tails)";
#else
    return "twofold_hip 0.2 (gfx950; all-twofold Horner)";
#endif
}

int tf_abi_version(void) { return 1; }

}  // extern "C"
