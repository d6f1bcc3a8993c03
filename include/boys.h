/*
 * boys.h -- C-ABI of the MI355X (gfx950) Boys-function library libboys.so.
 *
 * Evaluates the Boys functions
 *
 *     F_k(x) = integral_0^1 t^(2k) exp(-x t^2) dt,   x >= 0, k = 0, 1, ...
 *
 * (Vikhamar-Sandberg and Repisky, "Efficient Boys function evaluation using
 * minimax approximation", arXiv 2512.10059, Sec. I eq. 3) with the paper's
 * method (Sec. II F, Algorithm 1): the axis is split into A = [0, x0),
 * B = [x0, x1] and C = (x1, inf).  (The paper's region equation leaves the
 * end at x1 open to reading; here x = x1 is evaluated in B, on whose closed
 * interval r_B was fitted.)  On A a rational minimax approximant
 * r_{A,k} gives F_k and the downward recurrence the lower orders; on B the
 * approximant r_B gives F_0 and the upward recurrence the higher orders; on C
 * the asymptotic form sqrt(pi)/(2 sqrt x) and its upward recurrence are used.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller (for
 *    example the storage of a torch tensor).  The library never frees it.
 *  - Every call is asynchronous: it only enqueues kernels on `stream` (0 is
 *    the null stream) and returns.  Results are ready when the stream has
 *    executed them.
 *  - Return value: BOYS_OK (0) or a negative status.  Argument errors
 *    (BOYS_EINVAL) are detected on the host before anything is enqueued;
 *    BOYS_EHIP reports a failed HIP runtime call (the HIP error is kept for
 *    boys_last_hip_error()).  n == 0 is valid and enqueues nothing.
 *  - Domain: x must be >= 0.  Negative x and NaN give NaN in every output
 *    they feed; x = +inf gives 0.
 *  - Accuracy: FP64 results are within 5e-14 absolute of the exact function
 *    for 0 <= k <= 32 (the paper's appendix tables, eps_tol = 5e-14) and,
 *    where an entry point accepts them (boys_eval_f64(_tol),
 *    boys_backward(_tol), boys_pairsum(_tol)), for orders 33..40 (a table set built the same
 *    way); the _tol entry points trade this for 1e-10 at lower cost; FP32
 *    results are within 1e-6.
 *  - The library keeps lazily created workspaces per device (the batched
 *    entry points' prefix arrays and cached graphs, the pair sums' sort
 *    buffers); boys_finalize() releases them.  A workspace that has to grow
 *    is replaced by a larger one and the old one is kept until
 *    boys_finalize(), since work already enqueued may still read it: no
 *    call waits on the device.  The entry points that keep such state
 *    (boys_weighted_sum(_tol), boys_tune_weighted_sum, boys_pairsum(_tol))
 *    return BOYS_ECAPTURE, enqueueing nothing, when `stream` is under graph
 *    capture; boys_weighted_sum_noalloc is the batched entry point for
 *    captured streams.
 *  - Calls are thread-safe with respect to each other except that two
 *    concurrent batched calls (boys_weighted_sum, boys_weighted_sum_tol), or
 *    two concurrent pair-sum calls, on one device share a workspace and must
 *    be ordered by the caller (same stream, or synchronised).
 */
#ifndef BOYS_H
#define BOYS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#if defined(__GNUC__)
#define BOYS_API __attribute__((visibility("default")))
#else
#define BOYS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BOYS_OK = 0,
    BOYS_EINVAL = -1,   /* bad argument: null pointer, size, order or stride */
    BOYS_EHIP = -2,     /* a HIP runtime call failed */
    BOYS_ENOTSUP = -3,  /* the current device is not supported (needs gfx950) */
    BOYS_ENOMEM = -4,   /* the workspace could not be allocated */
    BOYS_ECAPTURE = -5  /* a call that keeps a cached workspace or graph was made
                           on a stream under graph capture (nothing enqueued) */
};

/* Highest order of the paper's FP64 tables (every FP64 entry point), of the
 * high-order FP64 tables (boys_eval_f64 and boys_eval_f64_tol), the highest
 * kmax of boys_backward (which recomputes order kmax+1 <= 40), and the
 * highest order of the FP32 tables. */
#define BOYS_F64_KMAX_LIMIT 32
#define BOYS_F64_EVAL_KMAX_LIMIT 40
#define BOYS_F64_BACKWARD_KMAX_LIMIT 39
#define BOYS_F32_KMAX_LIMIT 16

/*
 * Which tables serve the paper's accuracy (5e-14) at orders 0..32, for every
 * call with tol < 1e-10 (all entry points without _tol, and the _tol ones
 * below 1e-10) except boys_backward(_tol), which always takes the paper's:
 *
 *   BOYS_TABLES_PAPER     the paper's appendix: x0 = 11.899848152108484 and
 *                         x1 = 28.98933773882074, the regions of kmax = 32,
 *                         for every kmax (the default).
 *   BOYS_TABLES_PER_KMAX  the regions of the call's own kmax (Sec. II C: x0
 *                         and x1 depend on the highest order evaluated):
 *                         x0(K) = max{1, (prod_{n<K} (n+1/2))^(1/K)}, x1(K)
 *                         the root of the asymptote-error equation at 5e-14
 *                         for F_K (rounded up to a double), and r_B on
 *                         [x0(K), x1(K)] and r_{A,K} on [0, x0(K)] computed
 *                         with the library's Remez tool and the Walsh-table
 *                         degree choice; kmax = 32 is the paper's set.  The
 *                         batched consumer applies each batch's own kmax.
 *   BOYS_TABLES_CENTRE    the paper's x0 and x1, with r_B and every r_{A,k}
 *                         refitted at the Walsh-table entry nearest the
 *                         centre of the first feasible anti-diagonal
 *                         (n close to m; Sec. II D's alternative choice).
 *
 * Every variant keeps |error| <= 5e-14.  The setting is process-wide (all
 * devices and threads) and applies to calls made after it returns; work
 * already enqueued is not affected.  boys_set_tables returns BOYS_EINVAL for
 * an unknown variant (and changes nothing); boys_get_tables returns the
 * current one.
 */
#define BOYS_TABLES_PAPER 0
#define BOYS_TABLES_PER_KMAX 1
#define BOYS_TABLES_CENTRE 2
BOYS_API int boys_set_tables(int variant);
BOYS_API int boys_get_tables(void);

/* Text for a status code (static storage, never NULL). */
BOYS_API const char *boys_strerror(int status);

/* The hipError_t of the last failed HIP call made by this thread. */
BOYS_API int boys_last_hip_error(void);

/*
 * F_0..F_kmax in FP64 (Algorithm 1, Sec. II F).
 *
 *   x      [n] FP64 arguments.
 *   out    row-major n x ld_out FP64: out[i*ld_out + k] = F_k(x[i]) for
 *          k = 0..kmax; columns kmax+1..ld_out-1 are left untouched.
 *   kmax   0 <= kmax <= 40.  Up to 32 the paper's tables, or the variant
 *          chosen with boys_set_tables (r_{A,kmax} is the
 *          region-A approximant used); 33..40 a table set built the same way
 *          for kmax = 40 at the same 5e-14 (x0 = 14.842842360917231, x1 and
 *          every rational from the library's Remez tool), whose guarantee
 *          is the same |error| <= 5e-14.
 *   ld_out row stride in elements, ld_out >= kmax + 1.
 * Errors: BOYS_EINVAL for n < 0, kmax out of range, ld_out too small, a null
 * pointer with n > 0, or x and out overlapping.
 */
BOYS_API int boys_eval_f64(const double *x, int64_t n, int kmax, double *out, int64_t ld_out,
                  hipStream_t stream);

/*
 * boys_eval_f64 at a caller-chosen accuracy (the method at another eps_tol,
 * Sec. II C-D).  The library holds two table sets and uses the cheaper one
 * whose guarantee is at most tol:
 *   tol >= 1e-10   "screening" set: the same x0 (it depends only on kmax),
 *                  x1 = 23.149988540679747 (the asymptote-error equation at
 *                  1e-10, root rounded up), r_B and r_{A,k} computed with the
 *                  library's Remez tool (Walsh-table degree choice, lower
 *                  degrees than the paper's); |error| <= 1e-10.
 *   tol >= 5e-14   the paper's tables or the boys_set_tables variant
 *                  (identical to boys_eval_f64).
 * Orders 33..40 exist only at 5e-14 (the high-order tables) and take them
 * for any tol >= 5e-14.  Arguments and layout as boys_eval_f64.  Errors: as
 * boys_eval_f64, and BOYS_EINVAL for tol < 5e-14 or NaN.
 */
BOYS_API int boys_eval_f64_tol(const double *x, int64_t n, int kmax, double tol, double *out,
                               int64_t ld_out, hipStream_t stream);

/*
 * F_0..F_kmax in FP32 storage (mixed precision; the FP32 variant of
 * Algorithm 1 with the library's own minimax coefficients, regions
 * A' = [0, x0'), B' = [x0', x1'), C' = [x1', inf) for kmax <= 16).
 * FP32 rational and downward recurrence on A'; FP64 rational and FP64 upward
 * recurrence on B', where upward recurrence cancels; FP32 asymptote on C'.
 * Results are within 1e-6 absolute of the exact function at the FP32 x.
 *
 *   x      [n] FP32 arguments.
 *   out    row-major n x ld_out FP32, out[i*ld_out + k] = F_k(x[i]).
 *   kmax   0 <= kmax <= 16.   ld_out >= kmax + 1.
 * Errors as boys_eval_f64.
 */
BOYS_API int boys_eval_f32(const float *x, int64_t n, int kmax, float *out, int64_t ld_out,
                  hipStream_t stream);

/*
 * Batched fused consumer: for every batch b and every argument i of it
 *
 *     out[i] = sum_{l=0..kmax_b} w[w_off[b] + l] * F_l(x[i]),
 *
 * the weighted sum the paper's benchmark accumulates inside the recurrence
 * (Sec. III, Algorithm 2), here with one order and one weight vector per
 * batch.  Batch b covers x[batch_off[b] .. batch_off[b] + batch_n[b]).
 * One persistent kernel serves every batch; the library launches it through
 * a cached hipGraph (rebuilt when an argument changes).
 *
 *   x, out     FP64 arrays indexed by batch_off; only batch elements of out
 *              are written.
 *   batch_off  [nbatch] int64 first argument of each batch (>= 0).
 *   batch_n    [nbatch] int32 size of each batch (>= 0).
 *   batch_kmax [nbatch] int32 order of each batch, 0..32.
 *   w          FP64 weights; batch b uses w[w_off[b] .. w_off[b] + kmax_b].
 *   w_off      [nbatch] int64.
 *   nbatch     number of batches, 0 <= nbatch <= 2^24.
 * The batch table lives in device memory and is not validated element by
 * element: out-of-range orders are clamped to 0..32 in the kernel, and
 * batches must not overlap in out.
 * Errors: BOYS_EINVAL for a null pointer with nbatch > 0 or nbatch out of
 * range; BOYS_ENOMEM if the workspace cannot grow; BOYS_ECAPTURE on a
 * stream under graph capture.
 */
BOYS_API int boys_weighted_sum(const double *x, const int64_t *batch_off, const int32_t *batch_n,
                      const int32_t *batch_kmax, const double *w, const int64_t *w_off,
                      int32_t nbatch, double *out, hipStream_t stream);

/*
 * boys_weighted_sum for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, same kernels and the same result, bit for bit,
 * as boys_weighted_sum (the 5e-14 tables of the variant set by
 * boys_set_tables, the configuration chosen for boys_weighted_sum).  The scan's prefix arrays live in a fixed device array
 * of 2 (BOYS_NOALLOC_MAX_BATCHES + 1) int64 (1 MiB), one copy per device,
 * held until the process ends; the two kernels are launched directly on
 * `stream` (no cached graph), so the call enqueues only kernel launches and
 * may be captured.  Calls that overlap on one device share that array and
 * race: order them (same stream, or synchronised).  The first call on a
 * device looks up the array's address and the kernels' occupancy; make it
 * outside a capture.
 * Errors: as boys_weighted_sum, and BOYS_EINVAL for
 * nbatch > BOYS_NOALLOC_MAX_BATCHES.
 */
#define BOYS_NOALLOC_MAX_BATCHES 65536
BOYS_API int boys_weighted_sum_noalloc(const double *x, const int64_t *batch_off,
                                       const int32_t *batch_n, const int32_t *batch_kmax,
                                       const double *w, const int64_t *w_off, int32_t nbatch,
                                       double *out, hipStream_t stream);

/*
 * boys_weighted_sum with the table set chosen by tol as in boys_eval_f64_tol:
 * tol >= 1e-10 takes the screening set (per argument |error| <= 1e-10
 * sum_l |w_l| plus rounding), 5e-14 <= tol < 1e-10 the 5e-14 tables of the
 * variant set by boys_set_tables (the same result as boys_weighted_sum, bit
 * for bit).  The configuration chosen by boys_tune_weighted_sum serves every
 * set.  Errors: as boys_weighted_sum,
 * and BOYS_EINVAL for tol < 5e-14 or NaN.
 */
BOYS_API int boys_weighted_sum_tol(const double *x, const int64_t *batch_off,
                                   const int32_t *batch_n, const int32_t *batch_kmax,
                                   const double *w, const int64_t *w_off, int32_t nbatch,
                                   double tol, double *out, hipStream_t stream);

/*
 * Times every configuration of the persistent kernel (tile length, region
 * binning on or off, sweep chunk, register prefetch of the next tile, grid
 * of 2 to 4 rounds of resident workgroups, equal or tapered per-wave
 * shares) on these arguments (each run
 * writes out) with the 5e-14 tables of the current boys_set_tables variant,
 * keeps the fastest for later boys_weighted_sum calls on this device, and
 * reports it.  Synchronises `stream`.  best_config (may be NULL)
 * receives the configuration index, best_ms (may be NULL) its time in
 * milliseconds.
 *
 * If the environment variable BOYS_TUNE_CACHE names a file, the result is
 * appended to it as "weighted_sum <arch> <set> <bucket> <name>" (device
 * architecture, table set: 0 the paper's, 2 per-kmax, 3 centre, then
 * floor(log2 nbatch) and the configuration name), and the
 * first boys_weighted_sum(_tol) call on a device that has not chosen a
 * configuration takes the last matching entry; without a match (no
 * variable, no file, another device or build, malformed lines) it takes the
 * default.  boys_weighted_sum_noalloc reads no file: it uses the configuration
 * already chosen on the device, else the default.
 */
BOYS_API int boys_tune_weighted_sum(const double *x, const int64_t *batch_off, const int32_t *batch_n,
                           const int32_t *batch_kmax, const double *w, const int64_t *w_off,
                           int32_t nbatch, double *out, hipStream_t stream,
                           int *best_config, float *best_ms);

/* Number of persistent-kernel configurations, their description, and the one
 * boys_weighted_sum uses now on the current device (set_config: -1 = auto). */
BOYS_API int boys_weighted_sum_num_configs(void);
BOYS_API const char *boys_weighted_sum_config_name(int config);
BOYS_API int boys_weighted_sum_get_config(void);
BOYS_API int boys_weighted_sum_set_config(int config);

/*
 * Backward pass of F_0..F_kmax with respect to x, from dF_k/dx = -F_{k+1}
 * (differentiate eq. 3 under the integral sign):
 *
 *     grad_x[i] = - sum_{k=0..kmax} grad_f[i*ld_g + k] * F_{k+1}(x[i]).
 *
 * F_1..F_{kmax+1} are recomputed from x with the FP64 method at order
 * kmax+1 (nothing is saved by the forward pass): the paper's tables up to
 * order 32, the high-order tables (as boys_eval_f64) for orders 33..40.
 *
 *   x       [n] FP64.   grad_f  row-major n x ld_g FP64, ld_g >= kmax + 1.
 *   kmax    0 <= kmax <= 39.   grad_x [n] FP64 output.
 * Errors as boys_eval_f64.
 */
BOYS_API int boys_backward(const double *x, const double *grad_f, int64_t n, int kmax, int64_t ld_g,
                  double *grad_x, hipStream_t stream);

/*
 * boys_backward with the table set of the recomputation (order kmax+1)
 * chosen by tol as in boys_eval_f64_tol: tol >= 1e-10 takes the screening
 * set for kmax <= 31 (each F_{k+1} within 1e-10, so |error| <= 1e-10
 * sum_k |grad_f[i, k]| plus rounding); 5e-14 <= tol < 1e-10 gives
 * boys_backward's result bit for bit; kmax 32..39 take the high-order set
 * for any tol >= 5e-14.  Errors: as boys_backward, and BOYS_EINVAL for
 * tol < 5e-14 or NaN.
 */
BOYS_API int boys_backward_tol(const double *x, const double *grad_f, int64_t n, int kmax,
                               int64_t ld_g, double tol, double *grad_x, hipStream_t stream);

/*
 * The paper's benchmark workload (Sec. III, Algorithm 2), n^2 Boys
 * evaluations on arguments formed on the fly:
 *
 *     z[i] = sum_{l=0..kmax} c[l] sum_{j=0..n-1} F_l(x[i] + x[j]) y[j].
 *
 *   x, y, z  device arrays [n] (FP64); z must not overlap x or y.
 *   c        HOST array of kmax+1 FP64 weights, read during the call.
 *   n        0 <= n <= 2^31 - 1.   kmax 0..40 (up to 32 the paper's tables
 *            or the boys_set_tables variant; orders above 32 take the
 *            high-order tables, as boys_eval_f64).
 * Each z[i] is summed over j in chunks of 512 terms (chunk sums added in
 * order), so its rounding is about (512 + n/512) ulps of sum_j |y_j w_ij|
 * on top of the method's 5e-14 sum_l |c_l| per term.  The arguments are
 * sorted on the device first (rows evaluated in sorted order, results
 * scattered back), which needs a per-device workspace of 12 N + 24 n bytes,
 * N the power of two at or above n (at most 48 n bytes), allocated on first
 * use and grown when n grows.
 * Errors: BOYS_EINVAL for bad sizes, orders, null or overlapping pointers;
 * BOYS_ENOMEM if the workspace cannot grow; BOYS_ECAPTURE on a stream under
 * graph capture.
 */
BOYS_API int boys_pairsum(const double *x, const double *y, int64_t n, const double *c, int kmax,
                          double *z, hipStream_t stream);

/*
 * boys_pairsum with the table set chosen by tol as in boys_eval_f64_tol
 * (tol >= 1e-10: screening set, per-term bound 1e-10 sum_l |c_l|; tol >=
 * 5e-14: the paper's or the boys_set_tables variant; orders above 32 take
 * the high-order tables for any
 * tol >= 5e-14).  Errors: as boys_pairsum, and BOYS_EINVAL for
 * tol < 5e-14 or NaN.
 */
BOYS_API int boys_pairsum_tol(const double *x, const double *y, int64_t n, const double *c,
                              int kmax, double tol, double *z, hipStream_t stream);

/* Releases the per-device workspaces and cached graphs of every device. */
BOYS_API void boys_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* BOYS_H */
