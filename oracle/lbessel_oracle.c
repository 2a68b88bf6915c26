/*
 * Reference oracle for log I_v(x), log K_v(x), their x-derivatives and the
 * von Mises-Fisher log-normaliser.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against plain
 * definitions evaluated in binary128 (__float128, libquadmath, ~34 digits).
 * It shares no code, header, table or constant with the GPU library.
 *
 * What is computed (paper sections cited; the paper is Plesner, Sorensen,
 * Hauberg, "Accurate Computation of the Logarithm of Modified Bessel
 * Functions on GPUs", arXiv 2409.08729):
 *
 *  log I_v(x)  Sec. "Modified Bessel function of the first kind", eqs.
 *              (Iv infinite series), (ak terms), (log Iv): the defining power
 *              series, summed with the logarithm-of-a-sum trick (eq. log sum
 *              trick) anchored at the largest term a_i, whose index follows
 *              from eq. (K).  Every later/earlier term is reached through the
 *              exact term ratio of eq. (ak recurrence), and the series is cut
 *              only when a geometric bound on the whole remaining tail falls
 *              below 2^-118 of the partial sum (rigorous truncation).
 *
 *  log K_v(x)  The integral K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt
 *              (DLMF 10.32.9).  This is deliberately NOT the integral the
 *              paper evaluates on the GPU (eq. log Kv integral, after
 *              Rothwell): an independent definition of the same function.
 *              The integrand is even and entire in t, so the trapezoid rule
 *              with a half weight at t = 0 converges geometrically; the step
 *              is set from the peak width and halved until two successive
 *              steps agree to 2^-105.
 *
 *  d/dx log I_v(x)  term-by-term derivative of the same power series:
 *              I_v'(x) = sum_k (2k+v)/x * (x/2)^v a_k.
 *  d/dx log K_v(x)  derivative under the integral sign:
 *              K_v'(x) = -int_0^inf cosh t exp(-x cosh t) cosh(v t) dt.
 *
 *  vMF log C_p(kappa) = (p/2-1) log kappa - (p/2) log 2pi - log I_{p/2-1}(kappa)
 *              (Sec. "Metric learning", density of the vMF distribution).
 *
 * Domain conventions for special inputs (the paper only states v >= 0,
 * x >= 0 for I and v real for K):
 *   I: NaN in -> NaN; v < 0 or x < 0 -> NaN; x = 0 -> 0 if v = 0 else -inf;
 *      x = +inf (v finite) -> +inf; v = +inf (x finite) -> -inf.
 *   K: evaluated at |v| (K_{-v} = K_v); NaN in -> NaN; x < 0 -> NaN;
 *      x = 0 -> +inf; x = +inf (v finite) -> -inf; |v| = inf (x finite,
 *      x > 0) -> +inf; both infinite -> NaN.
 * Results are returned as (hi, lo) double pairs with hi + lo == the binary128
 * value rounded twice (hi = RN(q), lo = RN(q - hi)).
 *
 * Range: the series needs O(sqrt(x)) terms, so I is not computed (NaN) for
 * x > 1e12; the trapezoid rule needs the log-integrand resolved to O(1) at
 * its peak, so K is not computed (NaN) for x > 1e15 or |v| > 1e15, where the
 * log-integrand exceeds 2^113 in size.  Tests use closed forms there.
 */
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <omp.h>

typedef __float128 qf;

#define Q_NAN (nanq(""))
#define Q_INF (HUGE_VALQ)

/* Largest arguments the oracle evaluates (see the header). */
static const qf MAX_X_SERIES = 1e12Q;
static const qf MAX_K_ARG = 1e15Q;

/* Truncation target of the series tail, relative to the partial sum. */
static const qf SERIES_TAIL = 3.00926553810505e-36Q; /* 2^-118 */
/* Agreement required between two successive trapezoid steps, on the log
   scale and relative to max(1, |log of the peak integrand|): nodes far from
   t = 0 carry log-integrand values whose own binary128 rounding is about
   |kphi| * 2^-113, so an absolute target would be unreachable there. */
static const qf TRAP_AGREE = 2.465190328815662e-32Q; /* 2^-105 */
/* Nodes are kept until the log-integrand is this far below its maximum. */
static const qf TRAP_DROP = 110.0Q;

/* ------------------------------------------------------------------ */
/* Power series of I_v                                                  */
/* ------------------------------------------------------------------ */

/*
 * Sum the series around its largest term.  With a_k = (x^2/4)^k /
 * (k! Gamma(k+v+1)) the ratio a_{k+1}/a_k = (x^2/4)/((k+1)(k+1+v)) is
 * decreasing in k and crosses 1 at K* = (sqrt(v^2+x^2) - v)/2 (the positive
 * root in eq. (K)); a_{floor(K*)} is therefore the largest term.
 * On return: *log_i = log I_v(x); *dlog = I_v'(x)/I_v(x) when dlog != NULL.
 */
static void series_iv(qf v, qf x, qf *log_i, qf *dlog)
{
    const qf half_x = x / 2;
    const qf lhx = logq(half_x);
    const qf r2 = half_x * half_x;                  /* x^2/4 */
    const qf kstar = (sqrtq(v * v + x * x) - v) / 2;
    const qf i0 = floorq(kstar);
    /* log a_{i0}, written out from the definition of a_k */
    const qf log_ai = 2 * i0 * lhx - lgammaq(i0 + 1) - lgammaq(i0 + v + 1);

    qf s0 = 1;               /* sum_k a_k / a_{i0}            */
    qf s1 = 2 * i0 + v;      /* sum_k (2k+v) a_k / a_{i0}      */

    /* upward from the peak */
    qf t = 1;
    for (qf k = i0;; k += 1) {
        t *= r2 / ((k + 1) * (k + 1 + v));          /* a_{k+1}/a_{i0} */
        s0 += t;
        s1 += (2 * (k + 1) + v) * t;
        /* every later ratio is at most rho; the (2k+v) weight grows by at
           most (2k+4+v)/(2k+2+v) per step from here on */
        const qf rho = r2 / ((k + 2) * (k + 2 + v));
        const qf q1 = rho * (2 * (k + 2) + v) / (2 * (k + 1) + v);
        if (q1 < 1) {
            const qf tail0 = t * rho / (1 - rho);
            const qf tail1 = (2 * (k + 1) + v) * t * q1 / (1 - q1);
            if (tail0 <= SERIES_TAIL * s0 && tail1 <= SERIES_TAIL * s1)
                break;
        }
    }
    /* downward from the peak to k = 0 */
    t = 1;
    for (qf k = i0; k >= 1; k -= 1) {
        t *= (k * (k + v)) / r2;                    /* a_{k-1}/a_{i0} */
        s0 += t;
        s1 += (2 * (k - 1) + v) * t;
        /* every earlier ratio a_{j-1}/a_j, j <= k-1, is at most rho */
        const qf rho = ((k - 1) * (k - 1 + v)) / r2;
        if (rho < 1) {
            const qf tail0 = t * rho / (1 - rho);
            const qf tail1 = (2 * (k - 1) + v) * tail0;
            if (tail0 <= SERIES_TAIL * s0 && tail1 <= SERIES_TAIL * s1)
                break;
        }
    }
    *log_i = v * lhx + log_ai + logq(s0);
    if (dlog)
        *dlog = s1 / (x * s0);
}

static qf log_iv_q(qf v, qf x)
{
    if (isnanq(v) || isnanq(x) || v < 0 || x < 0)
        return Q_NAN;
    if (isinfq(v))
        return isinfq(x) ? Q_NAN : -Q_INF;
    if (x == 0)
        return v == 0 ? 0 : -Q_INF;
    if (isinfq(x))
        return Q_INF;
    if (x > MAX_X_SERIES)
        return Q_NAN;
    qf li;
    series_iv(v, x, &li, NULL);
    return li;
}

static qf dlog_iv_q(qf v, qf x)
{
    if (isnanq(v) || isnanq(x) || v < 0 || x < 0 || isinfq(v))
        return Q_NAN;
    if (x == 0)
        return v == 0 ? 0 : Q_INF;
    if (isinfq(x))
        return 1;
    if (x > MAX_X_SERIES)
        return Q_NAN;
    qf li, d;
    series_iv(v, x, &li, &d);
    return d;
}

/* ------------------------------------------------------------------ */
/* Integral of K_v                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    qf v, x;     /* v >= 0, x > 0, both finite */
    int weight;  /* 0: integrand of K_v; 1: cosh(t) times it (for -K_v') */
} kint;

/* log cosh(a) for a >= 0, without overflow */
static qf log_cosh(qf a)
{
    return a + log1pq(expq(-2 * a)) - M_LN2q;
}

/* log of the integrand at t >= 0 */
static qf kphi(const kint *p, qf t)
{
    qf r = -p->x * coshq(t) + log_cosh(p->v * t);
    if (p->weight)
        r += log_cosh(t);
    return r;
}

/* derivative of kphi in t */
static qf kdphi(const kint *p, qf t)
{
    qf r = -p->x * sinhq(t) + p->v * tanhq(p->v * t);
    if (p->weight)
        r += tanhq(t);
    return r;
}

/*
 * Location of the maximum of kphi on t >= 0.  kdphi(t) ~ (v^2 + w - x) t
 * near 0 (w = weight), and x sinh t outgrows the bounded tanh terms, so the
 * maximum is at 0 when v^2 + w <= x and otherwise at the single sign change
 * of kdphi, found by bisection.
 */
static qf kpeak(const kint *p)
{
    const qf w = p->weight ? 1 : 0;
    if (p->v * p->v + w <= p->x)
        return 0;
    qf lo = 0;
    qf hi = asinhq((p->v + w) / p->x) + 1;   /* kdphi(hi) < 0 */
    for (int it = 0; it < 90; ++it) {
        const qf mid = (lo + hi) / 2;
        if (kdphi(p, mid) > 0)
            lo = mid;
        else
            hi = mid;
    }
    return (lo + hi) / 2;
}

/* distance from the peak at which kphi has dropped by 1 (smaller side) */
static qf kwidth(const kint *p, qf tpk, qf fmax)
{
    const qf target = fmax - 1;
    /* right side: kphi -> -inf, bracket by doubling */
    qf a = 0, b = 1e-3Q / sqrtq(1 + p->x + p->v);
    while (kphi(p, tpk + b) >= target)
        b *= 2;
    for (int it = 0; it < 60; ++it) {
        const qf m = (a + b) / 2;
        if (kphi(p, tpk + m) >= target)
            a = m;
        else
            b = m;
    }
    qf w = b;
    /* left side, only if the drop happens before t = 0 */
    if (tpk > 0 && kphi(p, 0) < target) {
        a = 0;
        b = tpk;
        for (int it = 0; it < 60; ++it) {
            const qf m = (a + b) / 2;
            if (kphi(p, tpk - m) >= target)
                a = m;
            else
                b = m;
        }
        if (b < w)
            w = b;
    }
    return w;
}

/*
 * log of the trapezoid sum h * [f(0)/2 + sum_{j>=1} f(j h)] minus ref, where
 * ref = kphi(tpk) is the value at the continuous maximum.  The walk goes out of
 * the peak in both directions until the log-integrand is TRAP_DROP below the
 * largest value seen and still decreasing (kphi is unimodal).  Keeping ref
 * outside the sum lets two step sizes be compared without the rounding of
 * the (possibly large) ref itself.
 */
static qf ktrap(const kint *p, qf h, qf tpk, qf ref)
{
    long cap = 1024, n = 0;
    qf *val = malloc(sizeof(qf) * cap);
    qf *wt = malloc(sizeof(qf) * cap);
    qf fmax = -Q_INF;
    const long j0 = (long)(tpk / h);

    /* right of (and including) j0 */
    qf prev = Q_INF;
    for (long j = j0;; ++j) {
        const qf f = kphi(p, j * h);
        if (n == cap) {
            cap *= 2;
            val = realloc(val, sizeof(qf) * cap);
            wt = realloc(wt, sizeof(qf) * cap);
        }
        val[n] = f;
        wt[n] = (j == 0) ? 0.5Q : 1;
        ++n;
        if (f > fmax)
            fmax = f;
        if (f < fmax - TRAP_DROP && f < prev)
            break;
        prev = f;
    }
    /* left of j0 down to 0 */
    prev = Q_INF;
    for (long j = j0 - 1; j >= 0; --j) {
        const qf f = kphi(p, j * h);
        if (n == cap) {
            cap *= 2;
            val = realloc(val, sizeof(qf) * cap);
            wt = realloc(wt, sizeof(qf) * cap);
        }
        val[n] = f;
        wt[n] = (j == 0) ? 0.5Q : 1;
        ++n;
        if (f > fmax)
            fmax = f;
        if (f < fmax - TRAP_DROP && f < prev)
            break;
        prev = f;
    }
    qf s = 0;
    for (long i = 0; i < n; ++i)
        s += wt[i] * expq(val[i] - ref);
    free(val);
    free(wt);
    return logq(h) + logq(s);
}

/* log of int_0^inf exp(kphi(t)) dt, or NaN if ten step halvings do not settle */
static qf klog_integral(const kint *p)
{
    const qf tpk = kpeak(p);
    const qf fmax = kphi(p, tpk);
    const qf w = kwidth(p, tpk, fmax);
    qf h = w / 8;
    if (h > 0.05Q)
        h = 0.05Q;
    qf prev = ktrap(p, h, tpk, fmax);
    for (int it = 0; it < 10; ++it) {       /* converges in one or two */
        h /= 2;
        const qf cur = ktrap(p, h, tpk, fmax);
        if (fabsq(cur - prev) <= TRAP_AGREE * fmaxq(1, fabsq(fmax)))
            return fmax + cur;
        prev = cur;
    }
    return Q_NAN;
}

static qf log_kv_q(qf v, qf x)
{
    if (isnanq(v) || isnanq(x) || x < 0)
        return Q_NAN;
    v = fabsq(v);
    if (isinfq(v))
        return (isinfq(x) || x == 0) ? Q_NAN : Q_INF;
    if (x == 0)
        return Q_INF;
    if (isinfq(x))
        return -Q_INF;
    if (x > MAX_K_ARG || v > MAX_K_ARG)
        return Q_NAN;
    kint p = {v, x, 0};
    return klog_integral(&p);
}

static qf dlog_kv_q(qf v, qf x)
{
    if (isnanq(v) || isnanq(x) || x < 0)
        return Q_NAN;
    v = fabsq(v);
    if (isinfq(v))
        return Q_NAN;
    if (x == 0)
        return -Q_INF;
    if (isinfq(x))
        return -1;
    if (x > MAX_K_ARG || v > MAX_K_ARG)
        return Q_NAN;
    kint p0 = {v, x, 0};
    kint p1 = {v, x, 1};
    return -expq(klog_integral(&p1) - klog_integral(&p0));
}

/* ------------------------------------------------------------------ */
/* von Mises-Fisher log-normaliser                                      */
/* ------------------------------------------------------------------ */

/*
 * log C_p(kappa), C_p(kappa) = kappa^{p/2-1} / ((2 pi)^{p/2} I_{p/2-1}(kappa)).
 * At kappa = 0 the limit I_v(k) ~ (k/2)^v / Gamma(v+1) gives
 * log C_p(0) = v log 2 + lgamma(v+1) - (p/2) log 2pi, v = p/2 - 1.
 */
static qf vmf_log_norm_q(qf kappa, qf p)
{
    const qf v = p / 2 - 1;
    const qf log2pi = logq(2 * M_PIq);
    if (isnanq(kappa) || isnanq(p) || kappa < 0 || v < 0)
        return Q_NAN;
    if (kappa == 0)
        return v * M_LN2q + lgammaq(v + 1) - (p / 2) * log2pi;
    if (isinfq(kappa))
        return Q_NAN;
    return v * logq(kappa) - (p / 2) * log2pi - log_iv_q(v, kappa);
}

/* ------------------------------------------------------------------ */
/* Exported array entry points (hi, lo pairs)                           */
/* ------------------------------------------------------------------ */

static void split(qf r, double *hi, double *lo)
{
    const double h = (double)r;
    *hi = h;
    *lo = (isinf(h) || isnan(h)) ? 0.0 : (double)(r - (qf)h);
}

#define ORACLE_MAP2(NAME, FN)                                                 \
    void NAME(const double *v, const double *x, double *hi, double *lo,       \
              int64_t n)                                                      \
    {                                                                         \
        _Pragma("omp parallel for schedule(dynamic, 8)")                      \
        for (int64_t i = 0; i < n; ++i)                                       \
            split(FN((qf)v[i], (qf)x[i]), &hi[i], &lo[i]);                    \
    }

ORACLE_MAP2(lbo_log_iv, log_iv_q)
ORACLE_MAP2(lbo_log_kv, log_kv_q)
ORACLE_MAP2(lbo_dlog_iv, dlog_iv_q)
ORACLE_MAP2(lbo_dlog_kv, dlog_kv_q)

void lbo_vmf_log_norm(const double *kappa, double p, double *hi, double *lo,
                      int64_t n)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i)
        split(vmf_log_norm_q((qf)kappa[i], (qf)p), &hi[i], &lo[i]);
}

int lbo_max_threads(void) { return omp_get_max_threads(); }
void lbo_set_threads(int n) { omp_set_num_threads(n); }
