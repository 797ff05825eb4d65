/*
 * twofold_hip.h -- C ABI of the MI355X twofold exp/log library
 * (libtwofold_hip.so, HIP kernels for gfx950).
 *
 * A twofold x0 + x1 is a pair of IEEE numbers whose sum carries nearly twice
 * the working precision.  The twofold functions of E. Latkin, "Twofold exp and
 * log" (2015), return z0 + z1 ~ f(x0 + x1) where z0 is, bit for bit, the 1x
 * function of x0 and z1 estimates the deviation f(x0 + x1) - z0 (sections
 * "Twofold exponent: Method summary" and "Twofold logarithm: Newton
 * inversion"; the plain C interface z0 = texp(x0, x1, &z1) of the section
 * "C/C++ interface" becomes an elementwise call over arrays here).
 *
 * Conventions shared by every entry point:
 *  - Arrays are split: x0[i], x1[i] are the two parts of element i (SoA),
 *    contiguous, n elements each.  All array pointers are DEVICE pointers
 *    owned by the caller; the library keeps no reference after the call.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous: they enqueue work on `stream` and return.  Results are
 *    visible after the stream is synchronised.  Execution faults surface at
 *    that synchronisation, as usual for HIP.
 *  - n == 0 returns TF_OK and enqueues nothing.  A NULL array pointer with
 *    n > 0 returns TF_EINVAL and enqueues nothing (checked before any HIP
 *    call).  No HIP device -> TF_ENODEV.  A failed launch -> TF_ELAUNCH.
 *  - In-place use (z0 == x0 and z1 == x1) is allowed; any other overlap of
 *    outputs with inputs is undefined.
 *  - Numeric domain problems are not errors: they give NaN or infinities.
 *    When z0 is NaN, z1 is NaN; when z0 is +-inf, z1 is +0.  A log whose
 *    main part y0 is inside the domain while y0 + y1 is not returns a number
 *    x0 and x1 = NaN (x1 = -inf when y0 + y1 is exactly the pole, +inf when it
 *    is +inf) -- section "Logarithm: Algorithm summary".
 *  - The functions are reentrant; the library holds no mutable state except
 *    a per-device cache of the compute-unit count.
 */
#ifndef TWOFOLD_HIP_H
#define TWOFOLD_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TF_OK = 0,
    TF_EINVAL = 1,      /* invalid argument (NULL pointer with n > 0, bad descriptor) */
    TF_ELAUNCH = 2,     /* kernel launch or HIP runtime call failed */
    TF_ENOMEM = 3,      /* device allocation failed (batch plans only) */
    TF_EUNSUPPORTED = 4,
    TF_ENODEV = 5,      /* no HIP device visible */
    TF_ECAPACITY = 6    /* beyond the static capacity of tf_batch_run_noalloc */
} tf_status;

/* --- twofold functions, binary64 --------------------------------------- */
/* texp: z0 = exp(x0) (1x), z1 ~ e^(x0+x1) - z0.  Section "Exponent:
 * Algorithm summary", algorithm texp(x0 + x1): v = pexp0(x0) (table E (C T)
 * with a degree-12 Taylor-Horner T in twofold arithmetic), t1 = expm1(x1),
 * z1 = z0 t1 + (v1 + (v0 - z0)). */
tf_status tf_texp(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                  void* stream);
/* texpm1: z0 = expm1(x0), z1 ~ (e^(x0+x1) - 1) - z0; w = pexpm10(x0),
 * z1 = (z0 + 1) t1 + (w1 + (w0 - z0)).  Same section, algorithm texpm1. */
tf_status tf_texpm1(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                    void* stream);
/* tlog: z0 = log(x0), z1 ~ log(x0 + x1) - z0 by one Newton step on pexpm10
 * seeded with a 1x log1p (section "Logarithm: Algorithm summary", tlog/plog). */
tf_status tf_tlog(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                  void* stream);
/* tlog1p: z0 = log1p(x0), z1 ~ log1p(x0 + x1) - z0 (tlog1p/plog1p). */
tf_status tf_tlog1p(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                    void* stream);

/* --- twofold functions, binary32 (same algorithms, float parameters:
 *     pexp0 L = 1, N = 6; pexpm10 N = 5) ---------------------------------- */
tf_status tf_texpf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                   void* stream);
tf_status tf_texpm1f(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                     void* stream);
tf_status tf_tlogf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                   void* stream);
tf_status tf_tlog1pf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                     void* stream);

/* --- the 1x functions that define the main parts z0 --------------------
 * z[i] = f(x[i]); the same values the twofold functions return as z0. */
tf_status tf_exp1x(const double* x, double* z, size_t n, void* stream);
tf_status tf_expm1_1x(const double* x, double* z, size_t n, void* stream);
tf_status tf_log1x(const double* x, double* z, size_t n, void* stream);
tf_status tf_log1p_1x(const double* x, double* z, size_t n, void* stream);
tf_status tf_exp1xf(const float* x, float* z, size_t n, void* stream);
tf_status tf_expm1_1xf(const float* x, float* z, size_t n, void* stream);
tf_status tf_log1xf(const float* x, float* z, size_t n, void* stream);
tf_status tf_log1p_1xf(const float* x, float* z, size_t n, void* stream);

/* --- the other entry points of the paper's interface --------------------
 * Section "C/C++ interface" lists, besides texp/texpm1/tlog/tlog1p, the
 * functions below (algorithms: sections "Twofold exponent: Algorithm
 * summary" and "Twofold logarithm: Algorithm summary").  Conventions as
 * above; add "f" for binary32 (same signature with float).
 *
 * Dotted argument (an ordinary number x0; x1 = 0), one input array:
 *   pexp0    coupled e^x0: 0 below ln 2^min, z0 = z1 = +inf above ln 2^max,
 *            else E (C T) renormalised fast (z0 + z1 rounds to z0)
 *   texp0    z0 = exp(x0) bitwise, z1 = (v0 - z0) + v1 with v = pexp0(x0)
 *   pexpm10  coupled e^x0 - 1 (small-path table for |x0| <= ln 2, else
 *            pexp0(x0) - 1); +inf above ln 2^max
 *   texpm10  z0 = expm1(x0) bitwise, z1 = (w0 - z0) + w1, w = pexpm10(x0)
 *   plog0    coupled log y0: y0 = 2^n z0, seed log(z0), one Newton step on
 *            pexpm10, + n ln2, renormalised fast
 *   tlog0    z0 = log(y0) bitwise, z1 = X1 + (X0 - z0) with X = plog0(y0)
 *            (not renormalised)
 *   plog1p0  coupled log(1 + y0): for y0 outside [-1/2, 1] plog of the
 *            renormalised 1 + y0, else the Newton step seeded with log1p(y0)
 *   tlog1p0  z0 = log1p(y0) bitwise, z1 = X1 + (X0 - z0), X = plog1p0(y0)
 * The p-functions of the logarithm return, for y0 outside the domain of the
 * 1x function (y0 <= 0, resp. y0 <= -1, +inf, NaN), that function's value
 * and the rule for z1.
 *
 * Coupled argument (x0 + x1 rounds to x0), two input arrays:
 *   texpp, texpm1p   texp and texpm1 (no special algorithm for a coupled
 *                    argument; they run the same kernels)
 *   pexp, pexpm1     texpp, texpm1p renormalised fast (coupled result)
 *   plog             coupled log: scaled by the exponent of y0 (no
 *                    renormalisation of y first), Newton step, + n ln2,
 *                    renormalised fast
 *   tlogp            z0 = log(y0) bitwise, z1 = X1 + (X0 - z0), X = plog(y)
 *   plog1p           coupled log(1 + y): plog of the renormalised 1 + y
 *                    outside [-1/2, 1], else the Newton step on a = y
 *   tlog1pp          z0 = log1p(y0) bitwise, z1 = X1 + (X0 - z0)
 * An argument that is not coupled where a coupled one is due (or a non-finite
 * y1) gives z1 = NaN when the Newton step's seed leaves its range.
 */
tf_status tf_pexp0(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_texp0(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_pexpm10(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_texpm10(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_plog0(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_tlog0(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_plog1p0(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_tlog1p0(const double* x0, double* z0, double* z1, size_t n, void* stream);
tf_status tf_pexp0f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_texp0f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_pexpm10f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_texpm10f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_plog0f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_tlog0f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_plog1p0f(const float* x0, float* z0, float* z1, size_t n, void* stream);
tf_status tf_tlog1p0f(const float* x0, float* z0, float* z1, size_t n, void* stream);

tf_status tf_texpp(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                   void* stream);
tf_status tf_pexp(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                  void* stream);
tf_status tf_texpm1p(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                     void* stream);
tf_status tf_pexpm1(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                    void* stream);
tf_status tf_tlogp(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                   void* stream);
tf_status tf_plog(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                  void* stream);
tf_status tf_tlog1pp(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                     void* stream);
tf_status tf_plog1p(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                    void* stream);
tf_status tf_texppf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                    void* stream);
tf_status tf_pexpf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                   void* stream);
tf_status tf_texpm1pf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                      void* stream);
tf_status tf_pexpm1f(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                     void* stream);
tf_status tf_tlogpf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                    void* stream);
tf_status tf_plogf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                   void* stream);
tf_status tf_tlog1ppf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                      void* stream);
tf_status tf_plog1pf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                     void* stream);

/* --- twofold arithmetic ------------------------------------------------
 * The paper's second measured workload (section "Twofolds update": tadd,
 * tmul, tdiv, tsqrt with FMA).  z = x op y for twofolds x = x0 + x1,
 * y = y0 + y1; the main part z0 is the 1x operation on the main parts
 * (IEEE, correctly rounded), z1 the twofold error term:
 *   tadd   (s, t) = two_sum(x0, y0),  z1 = t + (x1 + y1)
 *   tsub   (d, t) = the corrected subtraction of section "Twofold bugs",
 *          z1 = t + (x1 - y1)
 *   tmul   z1 = fma(x0, y1, fma(x1, y0, e)),  e = fma(x0, y0, -z0)
 *   tdiv   r = fma(-z0, y0, x0),  z1 = ((r + x1) - z0 y1) / y0
 *   tsqrt  r = fma(-z0, z0, x0),  z1 = (r + x1) / (2 z0)  (0 when x0 = 0)
 *   trenorm  (z0, z1) = two_sum(x0, x1): the renormalized twofold of exactly
 *          the same value (section "Twofold logarithm", general case), for
 *          any x0, x1; where |x0| >= |x1| it is the paper's three-operation
 *          fast renormalization, bit for bit
 * Then the rule for non-finite main parts.  Arrays as above; tsqrt and
 * trenorm read x0, x1 only. */
tf_status tf_tadd(const double* x0, const double* x1, const double* y0, const double* y1,
                  double* z0, double* z1, size_t n, void* stream);
tf_status tf_tsub(const double* x0, const double* x1, const double* y0, const double* y1,
                  double* z0, double* z1, size_t n, void* stream);
tf_status tf_tmul(const double* x0, const double* x1, const double* y0, const double* y1,
                  double* z0, double* z1, size_t n, void* stream);
tf_status tf_tdiv(const double* x0, const double* x1, const double* y0, const double* y1,
                  double* z0, double* z1, size_t n, void* stream);
tf_status tf_tsqrt(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                   void* stream);
tf_status tf_taddf(const float* x0, const float* x1, const float* y0, const float* y1, float* z0,
                   float* z1, size_t n, void* stream);
tf_status tf_tsubf(const float* x0, const float* x1, const float* y0, const float* y1, float* z0,
                   float* z1, size_t n, void* stream);
tf_status tf_tmulf(const float* x0, const float* x1, const float* y0, const float* y1, float* z0,
                   float* z1, size_t n, void* stream);
tf_status tf_tdivf(const float* x0, const float* x1, const float* y0, const float* y1, float* z0,
                   float* z1, size_t n, void* stream);
tf_status tf_tsqrtf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                    void* stream);
tf_status tf_trenorm(const double* x0, const double* x1, double* z0, double* z1, size_t n,
                     void* stream);
tf_status tf_trenormf(const float* x0, const float* x1, float* z0, float* z1, size_t n,
                      void* stream);

/* --- backward (twofold adjoints; not part of the paper) ----------------
 * Gradient of a twofold function with respect to its twofold argument
 * x = x0 + x1, given the twofold upstream gradient g = g0 + g1 and the saved
 * forward value s = s0 + s1:
 *   tf_texp_bwd    gx = g * z          (s = z = texp(x))
 *   tf_texpm1_bwd  gx = g * (z + 1)    (s = z = texpm1(x))
 *   tf_tlog_bwd    gx = g / y          (s = y, the argument of tlog)
 *   tf_tlog1p_bwd  gx = g / (1 + y)    (s = y, the argument of tlog1p)
 * in twofold arithmetic: gx0 is the 1x product/quotient of the main parts,
 * gx1 its correction (division: Dekker's quotient with the FMA remainder
 * fma(-q, b, a) of the section "Older CPUs").  All six arrays have n elements;
 * same conventions as above (gx may alias s or g element for element). */
tf_status tf_texp_bwd(const double* s0, const double* s1, const double* g0, const double* g1, double* gx0,
                      double* gx1, size_t n, void* stream);
tf_status tf_texpm1_bwd(const double* s0, const double* s1, const double* g0, const double* g1, double* gx0,
                        double* gx1, size_t n, void* stream);
tf_status tf_tlog_bwd(const double* s0, const double* s1, const double* g0, const double* g1, double* gx0,
                      double* gx1, size_t n, void* stream);
tf_status tf_tlog1p_bwd(const double* s0, const double* s1, const double* g0, const double* g1, double* gx0,
                        double* gx1, size_t n, void* stream);
tf_status tf_texpf_bwd(const float* s0, const float* s1, const float* g0, const float* g1, float* gx0,
                       float* gx1, size_t n, void* stream);
tf_status tf_texpm1f_bwd(const float* s0, const float* s1, const float* g0, const float* g1, float* gx0,
                         float* gx1, size_t n, void* stream);
tf_status tf_tlogf_bwd(const float* s0, const float* s1, const float* g0, const float* g1, float* gx0,
                       float* gx1, size_t n, void* stream);
tf_status tf_tlog1pf_bwd(const float* s0, const float* s1, const float* g0, const float* g1, float* gx0,
                         float* gx1, size_t n, void* stream);

/* Backward of a chain y = f[k-1](... f[1](f[0](x))) of k twofold functions
 * (1 <= k <= TF_CHAIN_MAX), in one pass over the arrays.  fns[j] is stage j's
 * function (0 texp, 1 texpm1, 2 tlog, 3 tlog1p; stage 0 is applied first in
 * the forward pass) and (s0[j], s1[j]) its saved forward value, as for
 * tf_*_bwd.  fns, s0 and s1 are host arrays of k entries (read during the
 * call); the s0[j], s1[j], g and gx are device arrays of n elements.  With
 * the upstream gradient g of y, gx is the chain's gradient with respect to
 * x: the stage adjoints applied from stage k-1 down to stage 0, the same
 * twofold operations as k calls of tf_*_bwd, so the result equals theirs bit
 * for bit.  A stage whose saved arrays are those of the next stage (as when
 * texpm1's output is tlog1p's argument) reads them once.  gx may alias g or a
 * saved array element for element.  Errors: TF_EINVAL for k outside
 * [1, TF_CHAIN_MAX], an unknown function id, a NULL host array, or a NULL
 * device pointer with n > 0 (all checked before any GPU work). */
#define TF_CHAIN_MAX 8
tf_status tf_chain_bwd(int k, const int* fns, const double* const* s0, const double* const* s1,
                       const double* g0, const double* g1, double* gx0, double* gx1, size_t n,
                       void* stream);
tf_status tf_chain_bwdf(int k, const int* fns, const float* const* s0, const float* const* s1,
                        const float* g0, const float* g1, float* gx0, float* gx1, size_t n,
                        void* stream);

/* --- batched ragged launch --------------------------------------------
 * Many arrays of uneven lengths, each with its own function and format, in
 * one persistent launch captured once into a hipGraph.  The plan copies the
 * descriptors (host memory, read during tf_batch_plan_create only), cuts every
 * array into chunks of chunk_tiles * 256 * ept elements ordered dearest first,
 * and owns a small device allocation (descriptors, chunk list, a work
 * counter) until tf_batch_plan_destroy.  Results equal the plain calls bit
 * for bit.  Errors: TF_EINVAL for a bad descriptor (func or dtype out of
 * range, NULL array with n > 0) or configuration, TF_ENOMEM when the device
 * allocation fails, TF_ELAUNCH when capture fails.  A plan must not be
 * launched on two streams at once (it owns one work counter); launches on
 * one stream run in order.  Arrays need not be 16-byte aligned (unaligned
 * ones take a slower element-wise path). */
typedef struct {
    int32_t func;       /* 0 texp, 1 texpm1, 2 tlog, 3 tlog1p */
    int32_t dtype;      /* 0 binary64, 1 binary32 */
    size_t n;           /* elements (0 allowed) */
    const void* x0;     /* device arrays of n elements of the dtype */
    const void* x1;
    void* z0;
    void* z1;
} tf_batch_desc;

typedef struct {
    int32_t ept64;          /* elements per thread, binary64 arrays: 1, 2 or 4 */
    int32_t ept32;          /* binary32 arrays: 2 (with ept64 1) or 4 */
    int32_t chunk_tiles;    /* tiles of 256*ept elements per chunk, 1..4096 */
    int32_t blocks_per_cu;  /* workgroups per compute unit, 0 = all resident */
} tf_batch_config;          /* NULL in tf_batch_plan_create = {2, 4, 32, 0} */

typedef struct tf_batch_plan tf_batch_plan;

tf_status tf_batch_plan_create(const tf_batch_desc* descs, size_t count,
                               const tf_batch_config* config, tf_batch_plan** plan);
tf_status tf_batch_launch(tf_batch_plan* plan, void* stream);
tf_status tf_batch_plan_destroy(tf_batch_plan* plan);
tf_status tf_batch_plan_info(const tf_batch_plan* plan, size_t* chunks, size_t* elements);

/* --- batched ragged launch that allocates nothing -----------------------
 * For callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  One call does what
 * tf_batch_plan_create + tf_batch_launch + tf_batch_plan_destroy do, with the
 * same kernels and the same results bit for bit, but calls no hipMalloc,
 * hipFree or other allocating routine: the descriptor table, chunk list and
 * work counter live in a static device array of the library,
 * TF_BATCH_NOALLOC_SCRATCH_BYTES on each GPU it runs on, held until the
 * process ends.  descs (host memory, count entries) are validated as for
 * tf_batch_plan_create, then copied into that array on `stream` and read
 * before the call returns; config as for tf_batch_plan_create (NULL = the
 * defaults).  The chunks run dearest (function, format) first.
 * Limits: count <= TF_BATCH_NOALLOC_MAX_ARRAYS and at most
 * TF_BATCH_NOALLOC_MAX_CHUNKS chunks of chunk_tiles * 256 * ept elements in
 * all (about 10^9 binary64 elements at the default configuration); beyond
 * them TF_ECAPACITY, with nothing enqueued.  Errors otherwise as for the
 * plan: TF_EINVAL for a bad descriptor or configuration, TF_ELAUNCH when a
 * copy or launch fails.  Every call on one GPU uses that GPU's one array and
 * leaves the last call's contents in it: calls on one stream run in order,
 * calls that overlap on one GPU (other streams, other threads) race. */
#define TF_BATCH_NOALLOC_MAX_ARRAYS 8192
#define TF_BATCH_NOALLOC_MAX_CHUNKS 65536
#define TF_BATCH_NOALLOC_SCRATCH_BYTES 1376512
tf_status tf_batch_run_noalloc(const tf_batch_desc* descs, size_t count,
                               const tf_batch_config* config, void* stream);

/* --- launch configuration (used by the autotuner) ----------------------
 * fn: 0 texp, 1 texpm1, 2 tlog, 3 tlog1p, 4 exp1x, 5 expm1_1x, 6 log1x,
 * 7 log1p_1x; dtype: 0 binary64, 1 binary32.  ept: elements per thread
 * (1, 2 or 4; arrays that are not 16-byte aligned always use 1);
 * blocks_per_cu: workgroups of 256 threads per compute unit in the grid
 * (0 = as many as are resident at once); prefetch: tiles kept in flight
 * ahead of the one being evaluated (1 or 2; the 1x kernels ignore it).
 * Process-wide setting, not thread-safe against concurrent launches;
 * TF_EINVAL for out-of-range values. */
tf_status tf_set_launch_config(int fn, int dtype, int ept, int blocks_per_cu, int prefetch);
tf_status tf_get_launch_config(int fn, int dtype, int* ept, int* blocks_per_cu, int* prefetch);

/* Where the twofold-function kernels (tf_texp ... tf_tlog1pf) read their
 * range-reduction tables: TF_TABLES_AUTO from global memory, read in place,
 * when an array has at most 8 tiles per compute unit in binary64 or 2 in
 * binary32 (there the per-workgroup copy to LDS would not pay for itself),
 * and from that LDS copy otherwise; TF_TABLES_LDS always the LDS copy;
 * TF_TABLES_GLOBAL always global memory.  The results are the same bit for
 * bit.  Process-wide setting (tests and tuning), not thread-safe against
 * concurrent launches; TF_EINVAL for other values.  The default is
 * TF_TABLES_AUTO. */
#define TF_TABLES_AUTO 0
#define TF_TABLES_LDS 1
#define TF_TABLES_GLOBAL 2
tf_status tf_set_table_placement(int mode);
int tf_get_table_placement(void);

/* --- library information ---------------------------------------------- */
const char* tf_status_string(tf_status s);
const char* tf_version(void);
int tf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TWOFOLD_HIP_H */
