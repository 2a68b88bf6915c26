/*
 * lbessel: log I_v(x) and log K_v(x) of the modified Bessel functions over
 * device arrays, on AMD Instinct MI355X (gfx950).
 *
 * Method: Plesner, Sorensen, Hauberg, "Accurate Computation of the Logarithm
 * of Modified Bessel Functions on GPUs" (arXiv 2409.08729).  Each element is
 * evaluated by one of three branches chosen from (v, x) alone (Sec.
 * "Algorithms", Table 1 and Algorithm 1 in its GPU form): the Hankel
 * expansion with 20 correction terms (eqs. log Iv mu k / log Kv mu k), the
 * Debye expansion with 13 terms (eqs. log Iv u k / log Kv u k), or, for small
 * arguments, the power series of I_v (eqs. Iv infinite series, log Iv) or an
 * integral of K_v.  The paper integrates its own representation (eq. log Kv
 * integral, 600 nodes); this library's K fallback instead applies the
 * trapezoid rule to K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt (DLMF
 * 10.32.9) for x >= 1e-10, and the leading terms of DLMF 10.27.4 below; the
 * paper's integral stays available as lbessel_log_kv_integral_f64.  All
 * intermediate quantities stay on a log scale, so results are finite
 * wherever log I_v(x) and log K_v(x) are.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named v, x, gout, kappa, out, gx are DEVICE pointers owned by
 *    the caller, each to n contiguous elements (kappa: n, v/x: n).  Outputs
 *    must not overlap inputs.  The library allocates nothing and keeps no
 *    state between calls; calls are safe from several host threads (the vMF
 *    column sum takes a caller-provided workspace).
 *  - stream is a hipStream_t passed as void*; NULL means the null stream.
 *    Every call only enqueues work on that stream and returns; the caller
 *    synchronises before reading out.
 *  - n may be 0 (nothing is launched).  n < 0, or a NULL pointer with n > 0,
 *    is an API error.
 *  - Return value: LBESSEL_OK (0), or a negative LBESSEL_E* code; nothing is
 *    enqueued when an error is returned.
 *  - Domain problems are per-element values, never error codes:
 *      log I_v(x): v < 0 or x < 0 -> NaN;  x = 0 -> 0 if v = 0 else -inf;
 *                  x = +inf -> +inf;  v = +inf -> -inf;  NaN -> NaN.
 *      log K_v(x): evaluated at |v| (K_{-v} = K_v);  x < 0 -> NaN;
 *                  x = 0 -> +inf;  x = +inf -> -inf;  |v| = inf -> +inf;
 *                  NaN -> NaN.
 *    (The paper states the domains v >= 0, x >= 0 for I and real v for K;
 *    the boundary values are the limits of the functions.)
 *  - f64 entry points compute in binary64 throughout; f32 entry points take
 *    and return binary32 and compute in binary32 except where stated.
 */
#ifndef LBESSEL_H
#define LBESSEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBESSEL_OK 0
#define LBESSEL_EINVAL (-1)   /* NULL pointer with n > 0, n < 0, bad scalar   */
#define LBESSEL_EHIP (-2)     /* the HIP runtime rejected a launch          */
#define LBESSEL_ENODEV (-3)   /* no usable gfx950 device is current         */
#define LBESSEL_ENOSPACE (-7) /* request needs more than the static buffer  */

#define LBESSEL_ABI_VERSION 1

/* ---------------------------------------------------------------------- */
/* Forward evaluation                                                      */
/* ---------------------------------------------------------------------- */

/*
 * out[i] = log I_{v[i]}(x[i]).
 * Algorithm 1 of the paper in its three-branch GPU form, with re-fitted
 * branch thresholds (Table 1 shapes).  Elements are grouped by branch inside
 * each workgroup so a wavefront runs one branch; results do not depend on
 * neighbouring elements.
 */
int lbessel_log_iv_f64(const double *v, const double *x, double *out,
                       int64_t n, void *stream);
int lbessel_log_iv_f32(const float *v, const float *x, float *out,
                       int64_t n, void *stream);

/*
 * out[i] = log K_{v[i]}(x[i]); same structure.  Small-argument branch (the
 * paper's fallback of Algorithm 1), for x >= 1e-10: integer orders 0..14
 * take the integer-order path of lbessel_log_kv_order_f64 (the order-0/1
 * expansions, then the recurrence K_{j+1} = K_{j-1} + (2j/x) K_j); other
 * orders at x <= 1.25 Temme's series for K_mu and K_{mu+1} at the
 * fractional part mu = v - rint(v) followed by the same recurrence up to v
 * (N. M. Temme, J. Comput. Phys. 19, 1975); above x = 1.25 the trapezoid
 * rule on
 * K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt (DLMF 10.32.9), summed in
 * log scale over the nodes within a fixed drop of the integrand's peak.  For
 * x < 1e-10 the two leading terms of K_v = pi (I_{-v} - I_v) / (2 sin v pi)
 * (DLMF 10.27.4), rearranged for v < 0.3.  This replaces the paper's
 * 600-node rule on its own integral (eq. log Kv integral), which
 * lbessel_log_kv_integral_f64 and lbessel_eval_variant (LBESSEL_VAR_U_INTEGRAL
 * / _SIMPSON / _PAPER) keep.
 */
int lbessel_log_kv_f64(const double *v, const double *x, double *out,
                       int64_t n, void *stream);
int lbessel_log_kv_f32(const float *v, const float *x, float *out,
                       int64_t n, void *stream);

/*
 * out[i] = log K_{v[i]}(x[i]) by the paper's own small-argument method for K
 * (Sec. "Theory", eq. (log Kv integral) with n = 8, the composite rule after
 * it and the maxima of "Finding heuristics for maximums"): the integral of
 * g + h over u in (0, 1] on the paper's 600 nodes u_k = k/600, each term
 * exponentiated relative to the heuristic maximum of its part.  Weights:
 * trapezoid with an order-8 Gregory end correction (the paper's composite
 * Simpson rule misses the binary64 target by orders of magnitude; it stays
 * available as LBESSEL_VAR_SIMPSON).  The Hankel and Debye branches and the
 * special values are those of lbessel_log_kv_f64.  Same results as
 * lbessel_eval_variant(1, LBESSEL_VAR_U_INTEGRAL, LBESSEL_LAYOUT_GROUPED, ..),
 * within the same accuracy bar as lbessel_log_kv_f64; it runs 600 integrand
 * evaluations per fallback element where lbessel_log_kv_f64 runs 10-150.
 * Binary64 only.
 */
int lbessel_log_kv_integral_f64(const double *v, const double *x, double *out,
                                int64_t n, void *stream);

/*
 * One order for the whole array: out[i] = log I_v(x[i]) / log K_v(x[i]).
 * v is a host scalar, x and out device arrays of n elements.  Orders 0 and 1
 * (for K, |v| in {0, 1}) take a fast path whose expansions reduce to
 * polynomials with constant coefficients (power series of I_0, I_1, DLMF
 * 10.25.2; small-argument series of K_0, K_1, DLMF 10.31.1; a Chebyshev
 * expansion of log K_v(x) + x + log(2x/pi)/2 in 1/x on 2 < x <= 17.5; the
 * Hankel expansion above the thresholds of the general path; in binary32,
 * order 1 between the Debye and Hankel bounds of x, the Debye branch as in
 * the general path), the orders of the paper's v = 0, 1 comparisons (Sec.
 * "Precision", Tables 5 and 7).
 * Integer orders 2..14 of I take an integer-order path: where the general
 * path would sum the I series, a polynomial with the exact constant
 * coefficients n!/(k!(k+n)!) (DLMF 10.25.2); elsewhere the general path's
 * Hankel / Debye code, with the same bits.  Every other order, and every
 * other order of K, runs the general path with v broadcast, bit-identical to
 * lbessel_log_{iv,kv}_{f64,f32} on an array filled with v (for the integer
 * orders 2..14 of K its fallback runs the forward recurrence
 * K_{j+1} = K_{j-1} + (2j/x) K_j, DLMF 10.29.1, from K_0 and K_1 of the
 * order-0/1 path: every term positive, stable).  Special values follow the
 * general conventions.
 */
int lbessel_log_iv_order_f64(double v, const double *x, double *out, int64_t n,
                             void *stream);
int lbessel_log_kv_order_f64(double v, const double *x, double *out, int64_t n,
                             void *stream);
int lbessel_log_iv_order_f32(float v, const float *x, float *out, int64_t n,
                             void *stream);
int lbessel_log_kv_order_f32(float v, const float *x, float *out, int64_t n,
                             void *stream);

/* ---------------------------------------------------------------------- */
/* Derivatives in x (the paper names derivatives as future work)            */
/* ---------------------------------------------------------------------- */

/*
 * gx[i] = gout[i] * d/dx log I_v(x) at (v[i], x[i]), using
 * I_v'(x) = I_{v+1}(x) + (v/x) I_v(x) (DLMF 10.29.2):
 *   d/dx log I_v(x) = exp(log I_{v+1}(x) - log I_v(x)) + v/x.
 * Both log-values come from the forward algorithm above.  At x = 0 the
 * derivative is 0 for v = 0 and +inf for v > 0; at x = +inf it is 1.
 */
int lbessel_log_iv_grad_x_f64(const double *v, const double *x,
                              const double *gout, double *gx, int64_t n,
                              void *stream);
int lbessel_log_iv_grad_x_f32(const float *v, const float *x,
                              const float *gout, float *gx, int64_t n,
                              void *stream);

/*
 * gx[i] = gout[i] * d/dx log K_v(x), with K_v' = -K_{v+1} + (v/x) K_v:
 *   d/dx log K_v(x) = -exp(log K_{v+1}(x) - log K_v(x)) + v/x,  v -> |v|.
 * At x = 0 the derivative is -inf; at x = +inf it is -1.
 */
int lbessel_log_kv_grad_x_f64(const double *v, const double *x,
                              const double *gout, double *gx, int64_t n,
                              void *stream);
int lbessel_log_kv_grad_x_f32(const float *v, const float *x,
                              const float *gout, float *gx, int64_t n,
                              void *stream);

/* ---------------------------------------------------------------------- */
/* von Mises-Fisher log-normaliser (paper, Sec. "Metric learning")          */
/* ---------------------------------------------------------------------- */

/*
 * out[i] = log C_p(kappa[i]),
 *   C_p(k) = k^{p/2-1} / ((2 pi)^{p/2} I_{p/2-1}(k)),
 * the normalising constant of the vMF density on the unit sphere in R^p.
 * p is a host scalar, p >= 2 (LBESSEL_EINVAL otherwise, also for NaN/inf).
 * kappa = 0 gives the limit (p/2-1) log 2 + lgamma(p/2) - (p/2) log 2 pi
 * (the uniform density); kappa < 0 or NaN gives NaN; kappa = +inf -> NaN.
 */
int lbessel_vmf_log_norm_f64(const double *kappa, double p, double *out,
                             int64_t n, void *stream);
int lbessel_vmf_log_norm_f32(const float *kappa, float p, float *out,
                             int64_t n, void *stream);

/*
 * out[i] = d/dkappa log C_p(kappa[i]) = -I_{p/2}(kappa)/I_{p/2-1}(kappa)
 * = -A_p(kappa), the derivative used for maximum-likelihood fitting of kappa
 * (paper, eq. kappa estimates); computed as -exp(log I_{p/2} - log I_{p/2-1}).
 * kappa = 0 gives 0.
 */
int lbessel_vmf_log_norm_grad_f64(const double *kappa, double p, double *out,
                                  int64_t n, void *stream);

/*
 * Column sums of the L2-normalised rows of a feature matrix, the mean
 * resultant of the vMF fit (paper, Sec. "Metric learning", eq. mean direction
 * estimate: xbar = (1/N) sum_i x_i / ||x_i||, R = ||xbar||):
 *   colsum[j] = sum_{i < n} X[i, j] / ||X[i, :]||_2      (zero rows add 0)
 * X: device, row-major float32, n rows of p columns (n <= 2^31 - 1).
 * colsum: device, p doubles.  sumsq: device, 1 double receiving
 * sum_j colsum[j]^2 (so R = sqrt(sumsq) / n), or NULL.  Accumulation is
 * binary64 in a fixed order, so the results are the same on every call.
 * work: device workspace of at least lbessel_vmf_colsum_workspace(n, p)
 * bytes, owned by the caller (contents on return are unspecified).
 * lbessel_vmf_colsum_workspace returns that size in bytes, or a negative
 * status for negative n or p.
 */
int64_t lbessel_vmf_colsum_workspace(int64_t n, int64_t p);
int lbessel_vmf_colsum_f32(const float *X, int64_t n, int64_t p, double *colsum,
                           double *sumsq, void *work, int64_t work_bytes,
                           void *stream);

/*
 * Maximum-likelihood vMF concentration on the device (paper, Sec. "Metric
 * learning", eqs. kappa estimates and the Newton update): the column sums
 * above, then R = sqrt(sumsq)/n, kappa_0 = R (p - R^2) / (1 - R^2) and
 * Newton steps kappa <- kappa - (A_p - R) / (1 - A_p^2 - (p-1) A_p / kappa)
 * with A_p = I_{p/2}(kappa) / I_{p/2-1}(kappa) from the same evaluation code
 * as lbessel_log_iv_f64, until a step is below 1e-15 relative or no longer
 * shrinks (the noise floor: A_p has a relative error of ~kappa * 1e-16, so
 * kappa is defined to ~1e-11 relative at p ~ 1e4), at most 40 steps.
 * result: device, 4 doubles {kappa, R, kappa_0, Newton steps}; kappa is NaN
 * when R is 0 or 1 (all rows zero, or all rows parallel).
 * work: device workspace of lbessel_vmf_fit_workspace(n, p) bytes.
 */
int64_t lbessel_vmf_fit_workspace(int64_t n, int64_t p);
int lbessel_vmf_fit_f32(const float *X, int64_t n, int64_t p, double *result,
                        void *work, int64_t work_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fit as lbessel_vmf_fit_f32, bit for bit, with its workspace taken from a
 * static device buffer of LBESSEL_VMF_FIT_STATIC_BYTES bytes instead of a
 * caller argument.  The library holds one such buffer on each GPU it runs
 * on, until the process ends; the first call on a device (with that device
 * current) resolves the buffer's address, later calls allocate nothing.
 * X and result are caller-owned device pointers as for lbessel_vmf_fit_f32.
 * Returns LBESSEL_ENOSPACE when lbessel_vmf_fit_workspace(n, p) exceeds the
 * buffer (24 MiB holds p = 32768 with n up to about 10^6 rows, and p = 2048
 * with n up to about 2.6 * 10^6), LBESSEL_EINVAL for n < 1, p < 2 or a NULL
 * pointer, LBESSEL_EHIP if the buffer's address cannot be resolved.
 * Every call on one GPU uses that GPU's one buffer, which keeps the last
 * call's contents (every word a call reads it writes first): calls that
 * overlap in time on one GPU (several streams or host threads) race and
 * must be serialised by the caller.
 */
#define LBESSEL_VMF_FIT_STATIC_BYTES (24LL << 20)
int lbessel_vmf_fit_f32_noalloc(const float *X, int64_t n, int64_t p,
                                double *result, void *stream);

/* ---------------------------------------------------------------------- */
/* Segmented evaluation (many independent arrays in one launch)            */
/* ---------------------------------------------------------------------- */

/*
 * One array of a segmented launch: n pairs at v, x (device), results to out
 * (device), all of the launch's precision.  tile0 is the first workgroup
 * tile of the segment: the running sum of lbessel_segment_tiles(n) over the
 * segments before it (the first segment has tile0 = 0).
 */
typedef struct lbessel_segment {
    const void *v;
    const void *x;
    void *out;
    int64_t n;
    int64_t tile0;
} lbessel_segment_t;

/*
 * The same launch with the descriptor table in HOST memory, at most
 * LBESSEL_SEG_INLINE_MAX entries: the table is copied into the kernel's
 * arguments when the call enqueues the launch, so no device table and no
 * copy on the stream are needed (the serving runtime's small batches); segs
 * may be reused as soon as the call returns.  Results as for
 * lbessel_eval_segments.  nseg > LBESSEL_SEG_INLINE_MAX -> LBESSEL_EINVAL.
 */
#define LBESSEL_SEG_INLINE_MAX 32
int lbessel_eval_segments_inline(int kind, int precision,
                                 const lbessel_segment_t *segs, int nseg,
                                 int64_t tiles, void *stream);

/* Workgroup tiles covering n elements in a segmented launch (n >= 0). */
int64_t lbessel_segment_tiles(int64_t n);

/*
 * Forward log I (kind 0) or log K (kind 1) of every segment in one launch of
 * tiles workgroups; precision 64 or 32.  segs: DEVICE array of nseg
 * descriptors sorted by tile0; tiles: total tile count (tile0 of the last
 * segment plus its own tiles).  Each result equals what
 * lbessel_log_{iv,kv}_{f64,f32} gives for the segment alone, bit for bit.
 * This is the batching primitive of the serving runtime (lbessel_serve.h):
 * many small requests fill the chip in one launch.
 */
int lbessel_eval_segments(int kind, int precision, const lbessel_segment_t *segs,
                          int nseg, int64_t tiles, void *stream);

/* ---------------------------------------------------------------------- */
/* Diagnostics                                                             */
/* ---------------------------------------------------------------------- */

/*
 * Per-element branch selection, for tests and measurement: branch[i] is
 * 0 (Hankel, mu_20), 1 (Debye, U_13), 2 (series for I / integral for K) or
 * 3 (special value resolved without a branch).  kind: 0 = I, 1 = K.
 * precision: 64 or 32 (the f32 path has its own thresholds); v and x are
 * read as double or float accordingly.
 */
int lbessel_classify(int kind, int precision, const void *v, const void *x,
                     uint8_t *branch, int64_t n, void *stream);

/*
 * Integrand evaluations the log K fallback spends on each element (for the
 * op model of the benchmark): the node count of its integral rule, 0 for
 * elements of another branch or sub-case (integer orders 0..14, x < 1e-10
 * and the Temme series at x <= 1.25 run no integral).
 * precision 64 or 32.
 */
int lbessel_k_nodes(int precision, const void *v, const void *x, int32_t *nodes,
                    int64_t n, void *stream);

/*
 * Series terms the log K fallback's Temme branch (1e-10 <= x <= 1.25,
 * non-integer order) spends on each element, after its first term; 0 for
 * elements of another branch or sub-case (for the op model of the
 * benchmark, beside lbessel_k_nodes).  precision 64 or 32 (v and x read as
 * double or float); device arrays of n elements; n = 0 is a no-op;
 * LBESSEL_EINVAL for another precision, null pointers or n < 0.
 */
int lbessel_k_terms(int precision, const void *v, const void *x, int32_t *terms,
                    int64_t n, void *stream);

/*
 * The library's binary64 elementary functions on the device, for testing
 * their accuracy where the kernels run them: out[i] = f(a[i]) with op
 * 0 = 1/a (hardware estimate and two Newton steps), 1 = exp(a), 2 = exp(a)
 * for |a| < 1e9 (the form the branches use on bounded arguments),
 * 3 = log(a), 4 = log(1 + a), a >= 0, 5 = 1/sqrt(a) for normal a > 0
 * (hardware estimate and two Newton steps; the Debye branch's inverse square
 * root).  Device arrays of n elements; n = 0 is a no-op; LBESSEL_EINVAL for
 * another op, null pointers or n < 0.
 */
int lbessel_elementary_f64(int op, const double *a, double *out, int64_t n,
                           void *stream);

/*
 * Evaluate every element with one forced branch (0, 1 or 2 as above)
 * regardless of its regime.  Used to validate each branch
 * against the reference on its own; outside a branch's regime the result is
 * simply that expansion's value, which may be inaccurate.  The K fallback's
 * integration grid covers t < 32, which every element of its own region
 * (x >= 1e-10, v <= 16) stays inside; a forced fallback far outside it
 * (orders of thousands at x ~ 1e-10) is not meaningful.
 */
int lbessel_eval_branch_f64(int kind, int branch, const double *v,
                            const double *x, double *out, int64_t n,
                            void *stream);
/* The same in binary32 (the binary32 branches, thresholds not applied). */
int lbessel_eval_branch_f32(int kind, int branch, const float *v,
                            const float *x, float *out, int64_t n,
                            void *stream);

/*
 * The same forward evaluation as lbessel_log_{iv,kv}_{f64,f32} but one
 * element per thread with no regrouping by branch (kind 0 = I, 1 = K;
 * precision 64 or 32).  Results must equal the grouped kernels bit for bit;
 * tests use this to check the regrouping, the benchmark to price it.
 */
int lbessel_eval_ungrouped(int kind, int precision, const void *v,
                           const void *x, void *out, int64_t n, void *stream);

/*
 * Variants of the method and of the grouping, for measurement (binary64):
 * the same forward evaluation as lbessel_log_{iv,kv}_f64 with one of the
 * paper's own choices put back.  variant:
 *   LBESSEL_VAR_DEFAULT        this library's path
 *   LBESSEL_VAR_PAPER_REGIMES  Table 1 thresholds as printed (GPU subset:
 *                              mu_20, U_13, fallback)
 *   LBESSEL_VAR_U_INTEGRAL     K fallback by the paper's integral (eq. log Kv
 *                              integral) on its 600 nodes, trapezoid weights
 *                              with an order-8 Gregory end correction
 *   LBESSEL_VAR_SIMPSON        the same integral with the composite Simpson
 *                              1/3 rule of the paper (normalised by 1/(3N))
 *   LBESSEL_VAR_PAPER          Table 1 GPU subset + Simpson: the paper's GPU
 *                              method
 *   LBESSEL_VAR_SEVEN          Algorithm 1 as run on a CPU: mu_3, mu_20, U_4,
 *                              U_6, U_9, U_13 (Table 1), then the fallback
 * layout: how elements meet the branches:
 *   LBESSEL_LAYOUT_GROUPED  per-workgroup branch-sorted lists in LDS (this
 *                           library; not for LBESSEL_VAR_SEVEN)
 *   LBESSEL_LAYOUT_NAIVE    one element per thread, in input order
 *   LBESSEL_LAYOUT_SORTED   global radix sort of the elements by branch
 *                           first (the paper's GPU grouping); needs work
 * work: device workspace of lbessel_eval_variant_workspace(n) bytes for the
 * sorted layout (ignored otherwise).  n <= 2^31 - 1.  Variants other than
 * the default do not meet this library's accuracy bar everywhere; that is
 * what they are for.
 */
#define LBESSEL_VAR_DEFAULT 0
#define LBESSEL_VAR_PAPER_REGIMES 1
#define LBESSEL_VAR_U_INTEGRAL 2
#define LBESSEL_VAR_SIMPSON 3
#define LBESSEL_VAR_PAPER 4
#define LBESSEL_VAR_SEVEN 5
#define LBESSEL_LAYOUT_GROUPED 0
#define LBESSEL_LAYOUT_NAIVE 1
#define LBESSEL_LAYOUT_SORTED 2
int64_t lbessel_eval_variant_workspace(int64_t n);
int lbessel_eval_variant(int kind, int variant, int layout, const double *v,
                         const double *x, double *out, int64_t n, void *work,
                         int64_t work_bytes, void *stream);

/* Static description of a status code. */
const char *lbessel_status_string(int status);

/* LBESSEL_ABI_VERSION of the built library. */
int lbessel_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBESSEL_H */
