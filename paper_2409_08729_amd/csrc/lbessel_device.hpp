// Device math for log I_v(x) and log K_v(x) on gfx950.
//
// Branches follow Plesner, Sorensen, Hauberg, arXiv 2409.08729:
//   mu_20 : Hankel expansion with 20 correction terms, eqs. (log Iv mu k),
//           (log Kv mu k);
//   U_13  : Debye expansion with 13 terms, eqs. (log Iv u k), (log Kv u k),
//           u_k(t) from eqs. (u0), (uk);
//   series: power series of I_v summed in log scale, eqs. (Iv infinite
//           series), (ak recurrence), (log Iv), truncated when the remaining
//           terms fall below the working precision (text after eq. K);
//   K fallback (the library's path): for x >= 1e-10 integer orders 0..14
//           by the order-0/1 expansions and the order recurrence
//           (order_int_fb); other orders at x <= 1.25 by Temme's series
//           and the same recurrence (br_k_temme); otherwise
//           the trapezoid rule on
//           K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt (DLMF 10.32.9)
//           over the nodes within a fixed drop of the log-integrand's peak
//           (br_k_cosh, br_k_cosh32); for x < 1e-10 the leading terms of
//           DLMF 10.27.4 (br_k_tiny_x, br_k_small_x);
//   quad  : the paper's own integral representation of K_v (eq. log Kv
//           integral, n = 8) on its N = 600 equispaced nodes, summed in log
//           scale with the heuristic maxima u* = 1 for g and u* = 1/2 or
//           1/(2v) for h (br_quad_k; the measurement variants only).
// Branch selection keeps the predicate shapes of Table 1 / Algorithm 1 (GPU
// form: mu_20, then U_13, else the fallback) with thresholds re-fitted so
// that each branch meets 1e-15 relative error on its region.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbessel_fastmath.hpp"
#include "lbessel_tables.h"

namespace lbessel {

enum : int { KIND_I = 0, KIND_K = 1 };
enum : int { BR_MU = 0, BR_U = 1, BR_FB = 2, BR_NONE = 3 };

// ---------------------------------------------------------------------------
// Constant tables
// ---------------------------------------------------------------------------
// Coefficient tables are read through a pointer the optimiser cannot see
// through, in the constant address space: the loads become scalar loads at
// their point of use instead of ~200 registers of constants hoisted out of
// the evaluation loop of the grouped kernel.
#define LB_CONST_AS __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const LB_CONST_AS T *opaque_const(const T *p) {
    const LB_CONST_AS T *q = (const LB_CONST_AS T *)p;
    asm volatile("" : "+s"(q));
    return q;
}

// ---------------------------------------------------------------------------
// Elementary functions: binary64 through the short sequences of
// lbessel_fastmath.hpp, binary32 through the device library (hardware
// v_exp_f32 / v_log_f32 based).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lexp(double a) { return fm::exp64(a); }
__device__ __forceinline__ double llog(double a) { return fm::log64(a); }
__device__ __forceinline__ float lexp(float a) { return expf(a); }
__device__ __forceinline__ float llog(float a) { return logf(a); }
// log(1 + a), a >= 0, to ~1 ulp relative also for a near 0: the log of the
// rounded sum u = 1 + a plus the rounding error of that sum over u
__device__ __forceinline__ double llog1p(double a) { return fm::log1p64(a); }
__device__ __forceinline__ float llog1p(float a) {
    const float u = 1.0f + a;
    return fmaf(a - (u - 1.0f), fm::rcp_hw(u), logf(u));
}
// exp of an argument known to satisfy |a| < 1e9
__device__ __forceinline__ double lexp_b(double a) { return fm::exp64_bounded(a); }
// reciprocal: the hardware estimate with two Newton steps in binary64
// (<= 1 ulp, fm::rcp64); the hardware v_rcp_f32 (1 ulp) in binary32, for
// normal arguments (the binary32 branches take it of x >= 7, v > 0.1, r >= 1
// and series denominators >= 1)
__device__ __forceinline__ double lrcp(double a) { return fm::rcp64(a); }
__device__ __forceinline__ float lrcp(float a) { return fm::rcp_hw(a); }
__device__ __forceinline__ double lrsq(double a) { return fm::rsq64(a); }
__device__ __forceinline__ float lrsq(float a) {   // v_rsq_f32 and one Newton step
    const float y = fm::rsqrt_hw(a);
    return fmaf(0.5f * y, fmaf(-a * y, y, 1.0f), y);
}
__device__ __forceinline__ float lexp_b(float a) { return expf(a); }

// ---------------------------------------------------------------------------
// Constants
// ---------------------------------------------------------------------------

template <typename T> struct Cst;
template <> struct Cst<double> {
    static constexpr double log_2pi = 0x1.d67f1c864beb5p+0;      // log(2 pi)
    static constexpr double log_pi_2 = 0x1.ce6bb25aa1316p-2;     // log(pi/2)
    static constexpr double half_log_pi = 0x1.250d048e7a1bdp-1;  // log(pi)/2
    static constexpr double log_n = 0x1.99674ba3fdd16p+2;        // log(600)
    static constexpr double ln2 = 0x1.62e42fefa39efp-1;
    static constexpr double log_pi = 0x1.250d048e7a1bdp+0;         // log(pi)
    static constexpr double series_eps = 0x1p-56;  // relative truncation
    static constexpr double big_z = 1e150;         // sqrt(1+z^2) == z beyond
    static constexpr double tiny_z = 1e-290;       // x/v may have lost bits below
    static constexpr double safe_big = 1e300;      // 1/a and products stay normal below
};
template <> struct Cst<float> {
    static constexpr float log_2pi = 0x1.d67f1cp+0f;
    static constexpr float log_pi_2 = 0x1.ce6bb2p-2f;
    static constexpr float half_log_pi = 0x1.250d04p-1f;
    static constexpr float log_n = 0x1.99674cp+2f;
    static constexpr float ln2 = 0x1.62e430p-1f;
    static constexpr float log_pi = 0x1.250d04p+0f;
    static constexpr float series_eps = 0x1p-27f;
    static constexpr float big_z = 1e18f;
    static constexpr float tiny_z = 1e-30f;
    static constexpr float safe_big = 1e36f;
};

// Regime thresholds.  Shapes of Table 1:
//   mu_20 : (x > x1 && v < v1) || (v^2 < c x && x > x2)
//   U_13  : (x > x3 && v > v3) || (v > v4)
// The second mu clause is the paper's (a log x + b > log v) with a = 1/2,
// written without logarithms: v^2 < e^{2b} x, here e^{2b} = e^{1.4}.
struct RegimeSet {
    double x1, v1, c, x2, x3, v3, v4;
};
// binary64 sets: every branch within 1e-15 (relative to max(|y|, 1 + |(v, x)|))
// of the reference on its region.
template <typename T, int KIND> struct Regime;
template <> struct Regime<double, KIND_I> {
    static constexpr RegimeSet r = {21.5, 8.5, 0x1.0388657115a47p+2, 24.0, 23.0, 0.1, 14.5};
};
template <> struct Regime<double, KIND_K> {
    static constexpr RegimeSet r = {17.5, 8.5, 0x1.0388657115a47p+2, 17.5, 20.0, 0.1, 14.5};
};
// binary32 sets (2e-6 target): the expansions reach further down in x, but
// two binary32 rounding effects bound them: the Debye polynomials P_k(t^2)
// cancel near t = 1 (coefficients up to ~1e12 against values ~1), which
// needs v > 9 for all x; and the alternating Hankel sum for I amplifies
// rounding by ~exp(v^2/x), which needs v^2 < 2x (and v < 4.5 on the box).
template <> struct Regime<float, KIND_I> {
    static constexpr RegimeSet r = {9.5, 4.5, 2.0, 9.5, 7.5, 0.1, 9.0};
};
template <> struct Regime<float, KIND_K> {
    static constexpr RegimeSet r = {7.5, 16.0, 0x1.d8e64b8d4ddaep+2, 7.5, 7.0, 0.1, 9.0};
};

// ---------------------------------------------------------------------------
// Special values and branch choice
// ---------------------------------------------------------------------------

// Returns true (and sets *y) when (v, x) is outside the region the branches
// handle: NaN, negative, zero or infinite arguments.  For K, v is |v|.
template <typename T, int KIND>
__device__ __forceinline__ bool special_value(T v, T x, T *y) {
    const T inf = __builtin_huge_val();
    const T nan = __builtin_nan("");
    if (KIND == KIND_I) {
        if (!(v >= T(0)) || !(x >= T(0))) { *y = nan; return true; }   // NaN or < 0
        if (v == inf) { *y = (x == inf) ? nan : -inf; return true; }
        if (x == T(0)) { *y = (v == T(0)) ? T(0) : -inf; return true; }
        if (x == inf) { *y = inf; return true; }
        return false;
    } else {
        if (!(x >= T(0)) || v != v) { *y = nan; return true; }
        if (v == inf) { *y = (x == inf || x == T(0)) ? nan : inf; return true; }
        if (x == T(0)) { *y = inf; return true; }
        if (x == inf) { *y = -inf; return true; }
        return false;
    }
}

template <typename T, int KIND>
__device__ __forceinline__ int classify(T v, T x) {
    constexpr RegimeSet r = Regime<T, KIND>::r;
    const bool mu = (x > T(r.x1) && v < T(r.v1)) || (v * v < T(r.c) * x && x > T(r.x2));
    const bool u = (x > T(r.x3) && v > T(r.v3)) || (v > T(r.v4));
    return mu ? BR_MU : (u ? BR_U : BR_FB);
}

// ---------------------------------------------------------------------------
// Variants of the method, for measurement (f64 only)
// ---------------------------------------------------------------------------
//   VAR_DEFAULT        the library's path
//   VAR_PAPER_REGIMES  Table 1 thresholds as printed (GPU subset: mu_20, U_13)
//   VAR_U_INTEGRAL     K fallback by the paper's u-integral on its 600 nodes,
//                      trapezoid + order-8 Gregory end weights
//   VAR_SIMPSON        the same integral with composite Simpson 1/3 weights
//   VAR_PAPER          Table 1 GPU subset + Simpson: the paper's GPU method
//   VAR_SEVEN          Algorithm 1's CPU ordering: mu_3, mu_20, U_4, U_6, U_9,
//                      U_13 with Table 1 thresholds, then the fallback
enum { VAR_DEFAULT = 0, VAR_PAPER_REGIMES = 1, VAR_U_INTEGRAL = 2, VAR_SIMPSON = 3,
       VAR_PAPER = 4, VAR_SEVEN = 5, VAR_COUNT = 6 };
// branch codes of VAR_SEVEN, in priority order
enum { B7_MU3 = 0, B7_MU20 = 1, B7_U4 = 2, B7_U6 = 3, B7_U9 = 4, B7_U13 = 5, B7_FB = 6 };

// Table 1 predicates (natural logarithms), both kinds.
__device__ __forceinline__ bool paper_mu3(double v, double x) {
    return (x > 1400.0 && v < 3.05) || (0.6229 * fm::log64(x) - 3.2318 > fm::log64(v) && v > 3.1);
}
__device__ __forceinline__ bool paper_mu20(double v, double x) {
    return (x > 30.0 && v < 15.3919) ||
           (0.5113 * fm::log64(x) + 0.7939 > fm::log64(v) && x > 59.6925);
}
__device__ __forceinline__ bool paper_u(double v, double x, double x0, double v0, double v1) {
    return (x > x0 && v > v0) || (v > v1);
}

template <typename T, int KIND, int VAR>
__device__ __forceinline__ int classify_var(T v, T x) {
    if (VAR == VAR_PAPER_REGIMES || VAR == VAR_PAPER) {
        const double dv = v, dx = x;
        return paper_mu20(dv, dx) ? BR_MU
                                  : (paper_u(dv, dx, 19.6931, 0.7, 12.6964) ? BR_U : BR_FB);
    }
    if (VAR == VAR_SEVEN) {
        const double dv = v, dx = x;
        if (paper_mu3(dv, dx)) return B7_MU3;
        if (paper_mu20(dv, dx)) return B7_MU20;
        if (paper_u(dv, dx, 274.2377, 0.3, 163.6993)) return B7_U4;
        if (paper_u(dv, dx, 84.4153, 0.46, 56.9971)) return B7_U6;
        if (paper_u(dv, dx, 35.9074, 0.6, 20.1534)) return B7_U9;
        if (paper_u(dv, dx, 19.6931, 0.7, 12.6964)) return B7_U13;
        return B7_FB;
    }
    return classify<T, KIND>(v, x);
}

// ---------------------------------------------------------------------------
// mu_20: Hankel expansion
// ---------------------------------------------------------------------------
// S = 1 + sum_{k=1}^{20} c_k,  c_k = c_{k-1} (mu - (2k-1)^2) s / (8 k x),
// s = -1 for I (alternating), +1 for K; mu = 4 v^2.
template <typename T> __device__ __forceinline__ const T (*hankel_table())[2];
template <> __device__ __forceinline__ const double (*hankel_table<double>())[2] {
    return tables::kHankel64;
}
template <> __device__ __forceinline__ const float (*hankel_table<float>())[2] {
    return tables::kHankel32;
}

// NT correction terms (mu_NT); the library uses NT = 20, the seven-branch
// variant of Algorithm 1 also mu_3.
// x at least safe_big: a division and two logarithms, every intermediate in range.
template <typename T, int KIND, int NT>
__device__ __forceinline__ T br_mu_wide(T v, T x) {
    const T mu = T(4) * v * v;
    const T q = (KIND == KIND_I ? T(-0.125) : T(0.125)) / x;
    const LB_CONST_AS T *hk = opaque_const<T>(&hankel_table<T>()[0][0]);
    T c = T(1);
    T s = T(0);
#pragma unroll
    for (int k = 1; k <= NT; ++k) {
        const T d = (mu - hk[2 * (k - 1) + 1]) * hk[2 * (k - 1)];
        c = c * d * q;
        s = s + c;
    }
    const T ls = llog(fabs(T(1) + s));
    if (KIND == KIND_I)
        return x - T(0.5) * (Cst<T>::log_2pi + llog(x)) + ls;
    else
        return T(0.5) * (Cst<T>::log_pi_2 - llog(x)) - x + ls;
}

// Below safe_big 1/x is a normal number: one reciprocal serves the series and
// the prefactor, and log|1 + s| - log(x)/2 is taken as one logarithm,
// log((1 + s)^2 / x) / 2.
template <typename T, int KIND, int NT = tables::kMuTerms>
__device__ __forceinline__ T br_mu(T v, T x) {
    if (!(x < Cst<T>::safe_big))
        return br_mu_wide<T, KIND, NT>(v, x);
    const T mu = T(4) * v * v;
    const T ix = lrcp(x);
    const T q = (KIND == KIND_I ? T(-0.125) : T(0.125)) * ix;
    const LB_CONST_AS T *hk = opaque_const<T>(&hankel_table<T>()[0][0]);
    // 1 + s = 1 + t_1 (1 + t_2 (1 + ... (1 + t_NT))), t_k = c_k / c_{k-1} =
    // (mu - (2k-1)^2) (1/k) q, by Horner from the last term (both constants are
    // scalar operands); mu - (2k-1)^2 is exact, so at a half-integer order the
    // vanishing factor still ends the sum exactly
    T acc = T(1);
#pragma unroll
    for (int k = NT; k >= 1; --k) {
        const T t = (mu - hk[2 * (k - 1) + 1]) * (hk[2 * (k - 1)] * q);
        acc = fma(t, acc, T(1));
    }
    const T s1 = fabs(acc);
    const T lq = llog(s1 * s1 * ix);
    if (KIND == KIND_I)
        return x - T(0.5) * Cst<T>::log_2pi + T(0.5) * lq;
    else
        return T(0.5) * (Cst<T>::log_pi_2 + lq) - x;
}

// ---------------------------------------------------------------------------
// U_13: Debye expansion
// ---------------------------------------------------------------------------
// z = x/v, r = sqrt(1+z^2), t = 1/r, eta = r + log(z/(1+r)),
// S = 1 + sum_k (+-1)^k u_k(t) / v^k = 1 + sum_k w^k P_k(t^2), w = +-t/v
// (u_k(t) = t^k P_k(t^2)).  The -1/2 log(2 pi v) - 1/4 log(1+z^2) terms are
// merged into -1/2 log(2 pi v r).
template <typename T> __device__ __forceinline__ const T (*debye_table())[14];
template <> __device__ __forceinline__ const double (*debye_table<double>())[14] {
    return tables::kDebyeP64;
}
template <> __device__ __forceinline__ const float (*debye_table<float>())[14] {
    return tables::kDebyeP32;
}

// NT Debye terms (U_NT); the library uses NT = 13, the seven-branch variant
// of Algorithm 1 also U_4, U_6 and U_9.
// Arguments up to the end of the range (v or x at least safe_big): divisions
// and three logarithms, every intermediate in range.
template <typename T, int KIND, int NT>
// nt (<= NT, runtime): terms actually summed.  Terms above nt are skipped
// per lane, so lanes of one wave with different nt cost the largest nt once,
// and a term count gives the same bits whichever way it is reached.
__device__ __forceinline__ T br_u_wide(T v, T x, int nt) {
    const T z = x / v;
    const T r = (z < Cst<T>::big_z) ? sqrt(fma(z, z, T(1))) : z;
    const T t = T(1) / r;
    const T p = t * t;
    const T w = (KIND == KIND_I ? t : -t) / v;
    const LB_CONST_AS T *P = opaque_const<T>(&debye_table<T>()[0][0]);
    T acc = T(0);
#pragma unroll
    for (int k = NT; k >= 1; --k) {
        if (k > nt)
            continue;
        const LB_CONST_AS T *row = P + 14 * (k - 1);
        T pk = fm::fma_c(row[k], p, row[k - 1]);
#pragma unroll
        for (int j = k - 2; j >= 0; --j)
            pk = fm::fma_c(pk, p, row[j]);
        acc = w * (pk + acc);
    }
    // z below the normal range (x/v < ~1e-290 in f64): log z from log x - log v
    T lz = llog(z / (T(1) + r));
    if (z < Cst<T>::tiny_z)
        lz = llog(x) - llog(v) - llog(T(1) + r);
    const T eta = r + lz;
    const T ls = llog(fabs(T(1) + acc));
    const T lvr = llog(v * r);
    if (KIND == KIND_I)
        return v * eta - T(0.5) * (Cst<T>::log_2pi + lvr) + ls;
    else
        return T(0.5) * (Cst<T>::log_pi_2 - lvr) - v * eta + ls;
}

// Below big_z (v^2 + x^2 stays finite) everything derives from one inverse
// square root: with q = sqrt(v^2 + x^2) = v r, 1/(v r) = 1/q is the
// expansion's step (w = t/v) and t = v/q, v eta = q + v log(x/(v + q))
// (z/(1 + r) = x/(v + q)), the quotient by a reciprocal and one correction
// step (~0.5 ulp: it enters v eta), and log|1 + acc| - log(v r)/2 as one
// logarithm, log((1 + acc)^2 / q) / 2.
template <typename T, int KIND, int NT = tables::kUTerms>
// nt (<= NT, runtime): terms actually summed.  Terms above nt are skipped
// per lane, so lanes of one wave with different nt cost the largest nt once,
// and a term count gives the same bits whichever way it is reached.
__device__ __forceinline__ T br_u(T v, T x, int nt = NT) {
    if (!(v < Cst<T>::big_z && x < Cst<T>::big_z))
        return br_u_wide<T, KIND, NT>(v, x, nt);
    const T s2 = fma(v, v, x * x);
    const T iq = lrsq(s2);                                   // 1/(v r)
    const T q = s2 * iq;                                     // v r
    const T t = v * iq;
    const T p = t * t;
    const T w = (KIND == KIND_I ? iq : -iq);
    const LB_CONST_AS T *P = opaque_const<T>(&debye_table<T>()[0][0]);
    T acc = T(0);
#pragma unroll
    for (int k = NT; k >= 1; --k) {
        if (k > nt)
            continue;
        const LB_CONST_AS T *row = P + 14 * (k - 1);
        T pk = fm::fma_c(row[k], p, row[k - 1]);
#pragma unroll
        for (int j = k - 2; j >= 0; --j)
            pk = fm::fma_c(pk, p, row[j]);
        acc = w * (pk + acc);
    }
    const T d = v + q;
    const T id = lrcp(d);
    T zq = x * id;
    zq = fma(fma(-zq, d, x), id, zq);
    // x/(v + q) below the normal range (x/v < ~1e-290 in f64): log x - log(v + q)
    T lz = llog(zq);
    if (x < Cst<T>::tiny_z * v)
        lz = llog(x) - llog(d);
    const T veta = fma(v, lz, q);                            // v eta
    const T s1 = fabs(T(1) + acc);
    const T lq = llog(s1 * s1 * iq);
    if (KIND == KIND_I)
        return veta - T(0.5) * Cst<T>::log_2pi + T(0.5) * lq;
    else
        return T(0.5) * (Cst<T>::log_pi_2 + lq) - veta;
}

// ---------------------------------------------------------------------------
// Series for I_v (fallback of I)
// ---------------------------------------------------------------------------
// log I = v log(x/2) - lgamma(v+1) + log sum_k a_k/a_0,
// a_k/a_{k-1} = (x/2)^2 / (k (k+v)).  On this branch's region (v < 14.5,
// x <= 23) every ratio a_k/a_0 stays below 1e16, so the log-sum shift by the
// first term cannot overflow.  The sum stops once the current ratio is below
// 1/2 (all later ones are smaller) and the term is below eps * sum, which
// bounds the dropped tail by 2 eps relative.
// log Gamma(1 + v) for 0 <= v <= 15 in binary64 (the prefactor of the I
// series): on v in [j/2, (j+1)/2] a degree-15 polynomial in u = 4v - 2j - 1
// (a truncated Chebyshev interpolant in monomial form, absolute error below
// ~2e-16), read from a table in LDS.  Branch-free, so the lanes of a wave
// run the same instructions whatever their orders; the library lgamma
// branches by argument range.  The table is copied into LDS by the kernel
// (lgtab_load) before any use.
struct LgTab {
    double c[tables::kLgIntervals][tables::kLgCoefs];
    float c32[tables::kLgIntervals][tables::kLgCoefs];   // rounded to binary32
};

// Cooperative copy of the table into LDS; every thread of the workgroup must
// call it, before any evaluation of the I series.
__device__ __forceinline__ void lgtab_load(LgTab *t) {
    constexpr int n = tables::kLgIntervals * tables::kLgCoefs;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double c = (&tables::kLgamma1p64[0][0])[i];
        (&t->c[0][0])[i] = c;
        (&t->c32[0][0])[i] = float(c);
    }
    __syncthreads();
}

__device__ __forceinline__ double lgamma1p_tab(double v, const LgTab *t) {
    const int j = min(int(2.0 * v), tables::kLgIntervals - 1);
    const double u = fma(4.0, v, -double(2 * j + 1));
    const double *c = t->c[j];
    double s = c[tables::kLgCoefs - 1];
#pragma unroll
    for (int i = tables::kLgCoefs - 2; i >= 0; --i)
        s = fma(s, u, c[i]);
    return s;
}

__device__ __forceinline__ float lgamma1p_tab(float v, const LgTab *t) {
    const int j = min(int(2.0f * v), tables::kLgIntervals - 1);
    const float u = fmaf(4.0f, v, -float(2 * j + 1));
    const float *c = t->c32[j];
    float s = c[tables::kLgCoefs - 1];
#pragma unroll
    for (int i = tables::kLgCoefs - 2; i >= 0; --i)
        s = fmaf(s, u, c[i]);
    return s;
}

template <typename T>
__device__ __forceinline__ T br_series_i(T v, T x, const LgTab *lt) {
    const T hx = T(0.5) * x;
    const T q = hx * hx;
    // four terms per step with one reciprocal: a_k/a_{k-1} = q / d_k,
    // d_k = k (k + v), so with R = 1/(d_k d_{k+1} d_{k+2} d_{k+3}) the pair
    // reciprocals are 1/(d_k d_{k+1}) = R d_{k+2} d_{k+3} and 1/(d_{k+2} d_{k+3})
    // = R d_k d_{k+1}; a_k = a_{k-1} q d_{k+1} / (d_k d_{k+1}) and
    // a_{k+1} = a_{k-1} q^2 / (d_k d_{k+1}), and likewise for the second pair.
    // The stop test runs on the last term of a step, so at most three terms
    // more than a per-term test are summed.
    // The sum is kept without its leading 1 (sum of a_k / a_0 over k >= 1)
    // and enters through log1p: where I_v(x) is close to (x/2)^v / Gamma(v+1)
    // (small x) its log stays accurate relative to the small correction.
    const T q2 = q * q;
    const T q_2 = T(2) * q;
    T term = T(1);
    T sum = T(0);
    T f0 = T(-3);
    for (int k = 1; k < 200; k += 4) {
        f0 += T(4);
        const T f1 = f0 + T(1), f2 = f0 + T(2), f3 = f0 + T(3);
        const T d0 = f0 * (f0 + v);
        const T d1 = f1 * (f1 + v);
        const T d2 = f2 * (f2 + v);
        const T d3 = f3 * (f3 + v);
        const T d01 = d0 * d1, d23 = d2 * d3;
        const T r = lrcp(d01 * d23);
        const T r01 = r * d23, r23 = r * d01;
        const T t0 = term * q * d1 * r01;
        const T t1 = term * q2 * r01;
        const T t2 = t1 * q * d3 * r23;
        term = t1 * q2 * r23;
        sum = sum + t0;
        sum = sum + t1;
        sum = sum + t2;
        sum = sum + term;
        if ((d3 > q_2) & (term < fma(Cst<T>::series_eps, sum, Cst<T>::series_eps)))
            break;
    }
    T lg;
    if (v <= T(15))
        lg = lgamma1p_tab(v, lt);
    else
        lg = lgamma(v + T(1));
    // log(x/2) as log x - log 2: x/2 can underflow for subnormal x
    return v * (llog(x) - Cst<T>::ln2) - lg + llog1p(sum);
}

// ---------------------------------------------------------------------------
// Integral for K_v (fallback of K)
// ---------------------------------------------------------------------------
// log K = 1/2 log pi - lgamma(v+1/2) - v log 2x - x + log int_0^1 (g + h) du,
//   g(u) = beta exp(-u^beta) (2x + u^beta)^{v-1/2} u^{n-1},  beta = 2n/(2v+1),
//   h(u) = exp(-1/u) u^{-2v-1} (2xu + 1)^{v-1/2},            n = 8.
// Nodes u_j = j/600 (g(0) = h(0) = 0); weights: trapezoid with a Gregory
// end correction of order 8 at u = 1.  Each term is exponentiated relative to
// the heuristic maximum of its function, log g(1) and log h(u*), written as
// log-ratios so that no large intermediate cancels:
//   log g(u) - log g(1)  = (1 - u^b) + (v - 1/2) log((2x + u^b)/(2x + 1)) + 7 log u
//   log h(u) - log h(u*) = (1/u* - 1/u) - (2v+1) log(u/u*)
//                          + (v - 1/2) log((2xu + 1)/(2xu* + 1)).
template <typename T> __device__ __forceinline__ const T (*quad_nodes())[3];
template <> __device__ __forceinline__ const double (*quad_nodes<double>())[3] {
    return tables::kQuadNode64;
}
template <> __device__ __forceinline__ const float (*quad_nodes<float>())[3] {
    return tables::kQuadNode32;
}
template <typename T> __device__ __forceinline__ const T *gregory_tail();
template <> __device__ __forceinline__ const double *gregory_tail<double>() {
    return tables::kGregoryTail64;
}
template <> __device__ __forceinline__ const float *gregory_tail<float>() {
    return tables::kGregoryTail32;
}

// ACC: type of the two 600-term sums (binary64 also for binary32 terms).
// SIMPSON: composite Simpson 1/3 weights instead (the paper's rule, with the
// normalisation 1/(3N) of h/3 for h = 1/N).
template <typename T, typename ACC, bool SIMPSON = false>
__device__ __forceinline__ T br_quad_k(T v, T x) {
    constexpr int N = tables::kQuadN;
    constexpr int NT = tables::kGregoryOrder + 1;   // nodes with weight != 1
    const T beta = T(16) / (T(2) * v + T(1));
    const T vm = v - T(0.5);
    const T tv1 = T(2) * v + T(1);
    const T x2 = T(2) * x;
    const T inv2x1 = T(1) / (x2 + T(1));
    const T us = (v < T(2)) ? T(0.5) : T(0.5) / v;
    const T ius = (v < T(2)) ? T(2) : T(2) * v;
    const T lus = llog(us);
    const T den_h = fma(x2, us, T(1));
    const T inv2xus1 = T(1) / den_h;
    const LB_CONST_AS T *node = opaque_const<T>(&quad_nodes<T>()[0][0]);
    const LB_CONST_AS T *wt = opaque_const<T>(gregory_tail<T>());
    // log g(u_j) - log g(1) and log h(u_j) - log h(u*) at node j
    auto terms = [&](int j, T &eg, T &eh) {
        const T u = node[3 * j], lu = node[3 * j + 1], iu = node[3 * j + 2];
        // arguments of the exponentials are bounded: beta log u in [-103, 0];
        // the log-ratios are finite sums of terms below ~1e5 in size
        const T ub = lexp_b(beta * lu);
        const T lg = (T(1) - ub) + vm * llog((x2 + ub) * inv2x1) + T(7) * lu;
        const T lh = (ius - iu) - tv1 * (lu - lus) + vm * llog(fma(x2, u, T(1)) * inv2xus1);
        eg = lexp_b(lg);
        eh = lexp_b(lh);
    };
    ACC G = ACC(0), H = ACC(0);
    if (SIMPSON) {
        // node j is u = (j+1)/N: weight 4/3 (j+1 odd), 2/3 (even), 1/3 at u = 1
        for (int j = 0; j < N; ++j) {
            T eg, eh;
            terms(j, eg, eh);
            const ACC w = (j == N - 1) ? ACC(1.0 / 3.0) : ((j & 1) ? ACC(2.0 / 3.0) : ACC(4.0 / 3.0));
            G = fma(w, ACC(eg), G);
            H = fma(w, ACC(eh), H);
        }
    } else {
        // interior nodes: unit weight
        for (int j = 0; j < N - NT; ++j) {
            T eg, eh;
            terms(j, eg, eh);
            G += ACC(eg);
            H += ACC(eh);
        }
        // last NT nodes: trapezoid + Gregory end weights
        for (int j = N - NT; j < N; ++j) {
            T eg, eh;
            terms(j, eg, eh);
            const ACC w = ACC(wt[j - (N - NT)]);
            G = fma(w, ACC(eg), G);
            H = fma(w, ACC(eh), H);
        }
    }
    const T mg = llog(beta) - T(1) + vm * llog(x2 + T(1));
    const T mh = -ius - tv1 * lus + vm * llog(den_h);
    const T m = fmax(mg, mh);
    const T li = -Cst<T>::log_n + m + llog(T(G * ACC(lexp(mg - m)) + H * ACC(lexp(mh - m))));
    return Cst<T>::half_log_pi - lgamma(v + T(0.5)) - v * llog(x2) - x + li;
}

// ---------------------------------------------------------------------------
// K_v at tiny x and small v (sub-case of the K fallback)
// ---------------------------------------------------------------------------
// For v < 0.3 the g part of the integrand behaves like u^a, a = 7 - 8(1-2v)/(1+2v)
// (a < 4.8), between u ~ (2x)^{1/beta} and 1; once x < ~1e-15 that scale falls
// below the node spacing 1/600 and the 600-node rule loses mass (at v = 0,
// x = 1e-300 the integral is off by a factor ~6).  Below x = 1e-10 the
// two-term small-argument form is exact to O(x^2) (DLMF 10.27.4 with the
// leading terms of the series of I_{+-v}):
//   K_v(x) = [Gamma(1+v) y^{-v} - Gamma(1-v) y^{v}] / (2v),  y = x/2
//          = Gamma(1+v) L sinhc(vL) - e^{-vL} D(v),  L = log(2/x),
//   D(v) = (Gamma(1-v) - Gamma(1+v)) / (2v) = e^{E(v)} q(v) sinhc(v q(v)),
// with log Gamma(1+v) = -gamma v + sum_{k>=2} (-1)^k zeta(k) v^k / k split into
// its even part E(v) and odd part -v q(v) (DLMF 5.7.3).  Both terms of K are
// positive-dominated (first >= L > 23, second < 0.6): no cancellation.
__device__ __forceinline__ double sinhc64(double t) {   // sinh(t)/t, t >= 0
    if (t < 0.5) {
        const double t2 = t * t;
        double s = fma(t2, 1.0 / 156.0, 1.0);
        s = fma(t2 * (1.0 / 110.0), s, 1.0);
        s = fma(t2 * (1.0 / 72.0), s, 1.0);
        s = fma(t2 * (1.0 / 42.0), s, 1.0);
        s = fma(t2 * (1.0 / 20.0), s, 1.0);
        return fma(t2 * (1.0 / 6.0), s, 1.0);
    }
    return (fm::exp64(t) - fm::exp64(-t)) / (2.0 * t);
}

__device__ __forceinline__ double br_k_tiny_x(double v, double x) {
    const double L = Cst<double>::ln2 - fm::log64(x);
    const double t = v * L;
    double d;
    if (v < 0.05) {
        const double v2 = v * v;
        // q = gamma + zeta(3) v^2/3 + zeta(5) v^4/5 + ... + zeta(11) v^10/11
        double q = fma(v2, 0x1.0020631be48b3p+0 / 11.0, 0x1.00839f3d816b5p+0 / 9.0);
        q = fma(v2, q, 0x1.02232da14cf39p+0 / 7.0);
        q = fma(v2, q, 0x1.097418eca7ccep+0 / 5.0);
        q = fma(v2, q, 0x1.33ba004f00621p+0 / 3.0);
        q = fma(v2, q, 0x1.2788cfc6fb619p-1);
        // E = zeta(2) v^2/2 + zeta(4) v^4/4 + ... + zeta(12) v^12/12
        double e = fma(v2, 0x1.001020a5b2cd3p+0 / 12.0, 0x1.00412e33a5bb9p+0 / 10.0);
        e = fma(v2, e, 0x1.010b36af86397p+0 / 8.0);
        e = fma(v2, e, 0x1.0470984c09245p+0 / 6.0);
        e = fma(v2, e, 0x1.151322ac7d848p+0 / 4.0);
        e = fma(v2, e, 0x1.a51a6625307d3p+0 / 2.0);
        e = e * v2;
        d = fm::exp64(e) * q * sinhc64(v * q);
    } else {
        d = (tgamma(1.0 - v) - tgamma(1.0 + v)) / (2.0 * v);
    }
    const double k = tgamma(1.0 + v) * L * sinhc64(t) - fm::exp64(-t) * d;
    return fm::log64(k);
}

// K_v at tiny x for v >= 0.3 (the rest of the fallback below x = 1e-10): the
// same two-term form, K_v(x) = [Gamma(1+v) y^{-v} - Gamma(1-v) y^{v}] / (2v),
// y = x/2 < 5e-11, in log form.  The second term, relative Gamma(1-v) /
// Gamma(1+v) y^{2v} <= ~1e-6, is kept for v < 0.9; from 0.9 up it is below
// 1e-17 except within ~1e-4 of the integers, where it and the O(y^2) term
// of the first series both grow like 1/(v - n) and cancel to O(y^2 log y)
// (the logarithmic terms of DLMF 10.31.1): both are dropped there.  Every
// other neglected term is O(y^2) relative.
__device__ __forceinline__ double br_k_small_x(double v, double x) {
    const double ly = fm::log64(x) - Cst<double>::ln2;          // log y, no underflow
    const double g1 = tgamma(1.0 + v);                          // v <= ~15: finite
    double lk = fm::log64(g1 / (2.0 * v)) - v * ly;
    if (v < 0.9) {
        const double r = tgamma(1.0 - v) / g1 * fm::exp64(2.0 * v * ly);
        lk += fm::log64(1.0 - r);
    }
    return lk;
}

// ---------------------------------------------------------------------------
// K_v by the trapezoid rule on the cosh integral (fallback for x >= 1e-10)
// ---------------------------------------------------------------------------
// K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt (DLMF 10.32.9).  The
// integrand is even in t and entire, and decays double-exponentially, so the
// trapezoid rule with step h converges geometrically: its error is the
// integrand's Fourier transform at 2 pi / h, ~ K_{v + 2 pi i / h}(x), and
// h = min(0.25 / (1 + v/20), 0.5 / sqrt(x cosh t*)) keeps it below ~3e-16
// relative on the whole fallback region (x <= 21, v <= 14.6; fitted against
// the binary128 oracle: the first constant binds, and 0.27 would already
// give 2.3e-15 near v = 3, x = 3.4).  Only nodes where the log-integrand is
// within kDrop of its value at the peak t* are summed, which takes 10 to ~150
// nodes instead of the 600 of the rule on the u-integral.  Node positions
// are multiples of 1/64, so every t_j is exact and the only rounding in a
// term is that of its own exponent.  The sum is kept relative to the
// log-integrand at the grid point nearest t* (log-sum shift).
// e^t and e^-t at the grid nodes of br_k_cosh (t = i/64, 0 <= i < 2048) as
// e^{+-(i>>6)} e^{+-(i&63)/64}, integer part clamped to the table; two
// correctly rounded table entries and one product each (<= 1.5 ulp), so a
// node needs no division.  Each entry holds the pair (e^+, e^-), read with
// one 16-byte LDS load.  No walk reaches t = 32: on the fallback region
// (x >= 1e-10, v <= 14.5) the log-integrand has dropped 40 below its peak by
// t ~ 29 (the peak is below t = 27), and each walk ends there.  The tables
// are copied into LDS by the kernel (ktab_load) before any use; the binary32
// rule reads the same entries rounded to binary32.
constexpr int kKTabInt = 32;
struct KTab {
    double2 eint[kKTabInt];   // (e^n, e^-n)
    double2 efrac[64];        // (e^{f/64}, e^{-f/64})
};
struct KTab32 {
    float2 eint[kKTabInt];
    float2 efrac[64];
};

// Cooperative copy of the tables into LDS; every thread of the workgroup
// must call it, before any evaluation of the K fallback.
template <typename Tab>
__device__ __forceinline__ void ktab_load(Tab *t) {
    using E = decltype(t->eint[0].x);
    for (int i = threadIdx.x; i < kKTabInt + 64; i += blockDim.x) {
        if (i < kKTabInt) {
            t->eint[i] = {E(tables::kExpInt64[i]), E(tables::kExpNegInt64[i])};
        } else {
            const int j = i - kKTabInt;
            t->efrac[j] = {E(tables::kExpFrac64[j]), E(tables::kExpNegFrac64[j])};
        }
    }
    __syncthreads();
}

// The fallback's LDS tables by kind and precision: e^{+-t} for K, log
// Gamma(1 + v) for I (both precisions' coefficients in one table).
template <int KIND, typename T> struct FbTabSel {
    using type = typename std::conditional<std::is_same<T, float>::value, KTab32, KTab>::type;
};
template <typename T> struct FbTabSel<KIND_I, T> { using type = LgTab; };
template <int KIND, typename T> using FbTab = typename FbTabSel<KIND, T>::type;

// Peak and step of the trapezoid rule on the cosh integral (both rules below).
// peak: root t* > 0 of psi(t) = x sinh t - v tanh(v t) (convex on t >= 0,
// psi(0) = 0, psi'(0) = x - v^2 < 0).  tanh(vt) <= 1 and tanh(vt) <= vt
// give t* <= asinh(v/x) and t* <= t_s, sinh(t_s)/t_s = v^2/x; two steps of
// t <- asinh(R t) from asinh(R), R = v^2/x, approach t_s from below.
// Newton starts at the smaller of asinh(v/x) and that estimate: from the
// right of t* it decreases monotonically, from the left (where psi' > 0)
// its first step lands right of t*; where psi' <= 0 it restarts from the
// bound asinh(v/x).  t0 is rounded to the 1/64 grid, so |dt| < 4e-3 ends it.
// step: h = min(cv / (1 + v/20), cs / sqrt(x cosh t*)), rounded down to a
// multiple of 1/64 (hq/64, at least 1/64).  The peak and the step only place
// the grid, so they are computed in binary32 with hardware approximations
// (x >= 1e-10 and v <= ~15 here, so every quantity is in range).
__device__ __forceinline__ void k_peak_step(float vf, float xf, bool interior, float cv, float cs,
                                            int &t0q, int &hq) {
    float t = 0.0f;
    if (interior) {
        const float q = vf * fm::rcp_hw(xf);
        const float R = vf * q;
        auto asinh_pos = [](float a) { return fm::log_hw(a + fm::sqrt_hw(fmaf(a, a, 1.0f))); };
        const float tu = asinh_pos(q);
        float ts = asinh_pos(R);
        ts = asinh_pos(R * ts);
        ts = asinh_pos(R * ts);
        t = fminf(tu, ts);
        for (int it = 0; it < 16; ++it) {
            const float e = fm::exp_hw(t), r = fm::rcp_hw(e);
            const float z = fm::exp_hw(-2.0f * vf * t);
            const float iz = fm::rcp_hw(1.0f + z);
            const float psi = fmaf(0.5f * xf, e - r, -vf * (1.0f - z) * iz);
            const float dpsi = fmaf(0.5f * xf, e + r, -4.0f * vf * vf * z * iz * iz);
            if (!(dpsi > 0.0f)) {   // left of psi's minimum
                t = tu;
                continue;
            }
            const float dt = psi * fm::rcp_hw(dpsi);
            t = fmaxf(t - dt, 0.0f);
            if (fabsf(dt) < 4e-3f)
                break;
        }
    }
    const float et = fm::exp_hw(t);
    const float ch = 0.5f * (et + fm::rcp_hw(et));
    const float hf = fminf(cv * fm::rcp_hw(fmaf(0.05f, vf, 1.0f)), cs * fm::rsqrt_hw(xf * ch));
    hq = max(int(floorf(hf * 64.0f)), 1);
    t0q = int(rintf(t * 64.0f));
}

// nodes (may be null): receives the number of integrand evaluations.
__device__ __forceinline__ double br_k_cosh(double v, double x, const KTab *kt,
                                            int *nodes = nullptr) {
    constexpr double kGrid = 1.0 / 64.0;
    constexpr double kDrop = 40.0;          // e^-40 ~ 4e-18 of the peak term
    constexpr int kMaxNodes = 1024;         // every walk ends (window <= ~40 / h)
    // the shift, every term, both sums and the result are binary64
    int t0q, hq;
    k_peak_step(float(v), float(x), v * v > x, 0.25f, 0.5f, t0q, hq);
    const double h = hq * kGrid;
    // shift M = log-integrand at t0 = t0q/64 in binary64 (log cosh(vt) =
    // vt + log1p(e^{-2vt}) - ln 2), e^{+-t0} from the node tables
    const double2 pi0 = kt->eint[min(t0q >> 6, kKTabInt - 1)];
    const double2 pf0 = kt->efrac[t0q & 63];
    const double vt0 = v * (t0q * kGrid);
    const double M = fma(-0.5 * x, pi0.x * pf0.x + pi0.y * pf0.y, vt0) +
                     fm::log64(1.0 + fm::exp64_bounded(-2.0 * vt0)) - Cst<double>::ln2;
    // One walk over nodes i = i0 + j*di (units of 1/64), j = j0, j0+1, ...:
    // F(t) = E+ + E-, E+ = exp(-x cosh t + v t - M), E- = E+ r with
    // r = e^{-2 v t} carried by a product with e^{-2 v di/64}, recomputed
    // every 16 nodes (its relative error stays below 16 ulp, and it only
    // enters through E-).  Stops after the first node with log E+ < -kDrop
    // (and, for a walk from 0, past t0).
    const double lead = fm::pin_v(fm::kExpLead);
    auto walk = [&](int i0, int di, int j0, double w0, bool past_t0, int &cnt) -> double {
        const double q2 = fm::exp64_bounded(-2.0 * v * (di * kGrid));
        double S = 0.0, r = 1.0;
        for (int j = j0; j < j0 + kMaxNodes; ++j) {
            const int iq = i0 + j * di;
            const double tj = iq * kGrid;
            if (((j - j0) & 15) == 0)
                r = fm::exp64_bounded(-2.0 * v * tj);
            // e^{|t|}: a walk from t0 may step past t = 0, where the even
            // integrand is evaluated at its mirror node
            const int aq = abs(iq);
            const double2 pi = kt->eint[min(aq >> 6, kKTabInt - 1)];
            const double2 pf = kt->efrac[aq & 63];
            const double a = fma(-0.5 * x, pi.x * pf.x + pi.y * pf.y, -M);
            const double ap = fma(v, tj, a);
            const double ep = fm::exp64_bounded_lc(ap, lead);
            const double f = fma(ep, r, ep);
            S = (j == j0) ? fma(w0, f, S) : S + f;
            r *= q2;
            ++cnt;
            if (ap < -kDrop && (!past_t0 || iq > t0q))
                break;
        }
        return S;
    };
    double S;
    int cnt = 0;
    if (-x - M >= -kDrop) {
        // the window reaches t = 0: grid j h, j >= 0, half weight at 0
        S = walk(0, hq, 0, 0.5, true, cnt);
    } else {
        // interior window: grid t0 + j h, walked right then left from t0
        S = walk(t0q, hq, 0, 1.0, false, cnt) + walk(t0q, -hq, 1, 1.0, false, cnt);
    }
    if (nodes != nullptr)
        *nodes = cnt;
    return M + fm::log64(0.5 * h * S);
}

// The same rule in binary32 for the binary32 path (2e-6 target): the window
// ends 18 below the peak (e^-18 ~ 1.5e-8 of the peak term) and the step
// doubles to min(0.44 / (1 + v/20), 1 / sqrt(x cosh t*)), which keeps the
// rule's own error below the binary32 rounding floor (largest error 2.3e-7
// against the oracle on 3,681 points of the binary32 fallback region, in a
// binary32 model of this code; ~25 nodes instead of ~50 for the binary64
// rule there).  Terms, sums and the shift are binary32; e^{+-t} comes from
// the binary32 copies of the node tables, each term's exponential from the
// hardware exp2 (its relative error grows with |exponent|, but so does the
// term's smallness) and the r resets from the library expf.
__device__ __forceinline__ float br_k_cosh32(float v, float x, const KTab32 *kt,
                                             int *nodes = nullptr) {
    constexpr float kGrid = 1.0f / 64.0f;
    constexpr float kDrop = 18.0f;
    constexpr int kMaxNodes = 1024;
    int t0q, hq;
    k_peak_step(v, x, v * v > x, 0.44f, 1.0f, t0q, hq);
    const float h = float(hq) * kGrid;
    const float2 pi0 = kt->eint[min(t0q >> 6, kKTabInt - 1)];
    const float2 pf0 = kt->efrac[t0q & 63];
    const float vt0 = v * (float(t0q) * kGrid);
    const float M = fmaf(-0.5f * x, pi0.x * pf0.x + pi0.y * pf0.y, vt0) +
                    logf(1.0f + expf(-2.0f * vt0)) - Cst<float>::ln2;
    auto walk = [&](int i0, int di, int j0, float w0, bool past_t0, int &cnt) -> float {
        const float q2 = expf(-2.0f * v * (float(di) * kGrid));
        float S = 0.0f, r = 1.0f;
        for (int j = j0; j < j0 + kMaxNodes; ++j) {
            const int iq = i0 + j * di;
            const float tj = float(iq) * kGrid;
            if (((j - j0) & 15) == 0)
                r = expf(-2.0f * v * tj);
            const int aq = abs(iq);
            const float2 pi = kt->eint[min(aq >> 6, kKTabInt - 1)];
            const float2 pf = kt->efrac[aq & 63];
            const float a = fmaf(-0.5f * x, pi.x * pf.x + pi.y * pf.y, -M);
            const float ap = fmaf(v, tj, a);
            const float ep = fm::exp_hw(ap);
            const float f = fmaf(ep, r, ep);
            S = (j == j0) ? fmaf(w0, f, S) : S + f;
            r *= q2;
            ++cnt;
            if (ap < -kDrop && (!past_t0 || iq > t0q))
                break;
        }
        return S;
    };
    float S;
    int cnt = 0;
    if (-x - M >= -kDrop)
        S = walk(0, hq, 0, 0.5f, true, cnt);
    else
        S = walk(t0q, hq, 0, 1.0f, false, cnt) + walk(t0q, -hq, 1, 1.0f, false, cnt);
    if (nodes != nullptr)
        *nodes = cnt;
    return M + logf(0.5f * h * S);
}

// Debye term-count tier of an order on the Debye branch: 0 = U_13, 1 = U_9,
// 2 = U_6, 3 = U_4.  U_K's truncation error, relative to max(|y|, 1 + |(v, x)|),
// is below 1e-15 for every x once v >= 14.2 (K = 13), 24 (9), 56 (6) and
// 176 (4) (error maps against the oracle, I and K); the cuts keep ~8% margin.
constexpr int kUTiers = 4;
template <typename T>
__device__ __forceinline__ int u_tier(T v) {
    return (v > T(190)) ? 3 : (v > T(60)) ? 2 : (v > T(26)) ? 1 : 0;
}

// Integer orders whose K fallback (x >= 1e-10) runs the integer-order path
// (order_int_fb) instead of the integral: 0 <= v <= 14, v integral.
template <typename T>
__device__ __forceinline__ bool int_order(T v) {
    return v <= T(tables::kIntOrderMax) && v == rint(v);
}

// Cost bucket 0..B-1 of an I series element: its term count grows with x
// (about 3 terms below x = 0.01, 8 at x = 1, 18 at x = 6, 33 at x = 20).
// Only used to order work inside a tile; any value is correct.
template <int B, typename T>
__device__ __forceinline__ int i_cost_bucket(T x) {
    static_assert(B == 4, "thresholds are set for four buckets");
    return (x < T(0.1)) ? 0 : (x < T(1)) ? 1 : (x < T(5)) ? 2 : 3;
}

// Cost bucket of a K fallback element: 0..5, a rough count of the nodes
// br_k_cosh will visit (window width / step) cut at fixed thresholds, or 6
// for an interior window (the peak estimate stands more than 40 above the
// integrand at t = 0), whose right and left walks would otherwise run one
// after the other in chunks shared with the single walk of windows that
// start at 0.  With TEMME (the default variant) buckets 0..3 hold the
// Temme-series elements (x <= 1.25) by term and order-step estimate, and
// the integer orders; bucket 4 every integral element (5 and 6 stay
// empty).  Only used to order work inside a tile; any value is correct.
template <int B, bool TEMME>
__device__ __forceinline__ int k_cost_bucket(double v, double x) {
    static_assert(B == 7, "six cost buckets and the interior-window class");
    if (x >= 1e-10 && int_order(v))   // integer-order path: no walk
        return 0;
    // binary32 hardware approximations: only an ordering key (x >= 1e-10 on
    // this branch keeps v/x and 45/x in binary32 range; smaller x only ever
    // lands in the last bucket)
    const float vf = float(v), xf = fmaxf(float(x), 1e-30f);
    if (TEMME && x <= tables::kTemmeX) {
        // Temme's series: ~4.7 order steps' worth per term (the term count
        // grows with x; measured 26.8 and 5.7 instructions) and one unit per
        // order step above mu + 1
        const float nt = (xf < 1e-4f) ? 2.0f : (xf < 1e-2f) ? 3.5f : (xf < 0.1f) ? 5.5f
                         : (xf < 0.4f) ? 7.5f : 10.0f;
        const float est = fmaf(4.7f, nt, fmaxf(rintf(vf) - 1.0f, 0.0f));
        return (est < 20.0f) ? 0 : (est < 30.0f) ? 1 : (est < 42.0f) ? 2 : 3;
    }
    // the integral's elements above the series bound (and x < 1e-10): one
    // bucket, the costliest in list order; the node-count estimate below
    // cost more than its ordering saved there (K stress grid f64 1.43-1.44
    // -> 1.39 ms, f32 0.91-0.92 -> 0.82 ms)
    if (TEMME)
        return 4;
    float w;
    if (v * v > x) {
        const float q = vf * fm::rcp_hw(xf);
        const float tu = fm::log_hw(q + fm::sqrt_hw(fmaf(q, q, 1.0f)));
        w = fminf(tu, 45.0f * fm::rcp_hw(vf)) + 4.0f;
        // interior window (both walks): the log-integrand at a peak estimate
        // stands more than 40 above its value -x at t = 0
        const float R = vf * q;
        auto asinh_pos = [](float a) { return fm::log_hw(a + fm::sqrt_hw(fmaf(a, a, 1.0f))); };
        float ts = asinh_pos(R);
        ts = asinh_pos(R * ts);
        ts = asinh_pos(R * ts);
        const float t = fminf(tu, ts);
        const float et = fm::exp_hw(t);
        const float phi = fmaf(-0.5f * xf, et + fm::rcp_hw(et), vf * t) + xf;
        if (phi > 40.7f)
            return 6;
    } else {
        const float a = 45.0f * fm::rcp_hw(xf);
        w = fm::log_hw(1.0f + a + fm::sqrt_hw(a * (2.0f + a)));   // acosh(1 + 45/x)
    }
    const float est = w * fmaf(0.05f, vf, 1.0f) * (1.0f / 0.25f);
    return (est < 19.0) ? 0 : (est < 29.0) ? 1 : (est < 37.0) ? 2 : (est < 45.0) ? 3
                                                                 : (est < 55.0) ? 4 : 5;
}

// ---------------------------------------------------------------------------
// Orders 0 and 1 (scalar-order fast path)
// ---------------------------------------------------------------------------
// With v fixed at 0 or 1 every expansion reduces to polynomials with constant
// coefficients (tables generated in exact or 100-digit arithmetic):
//   x > x1 (the Hankel region of both orders): br_mu, as on the general path;
//   I:  log I_v = v log(x/2) + log1p(sum_{k>=1} q^k/(k!(k+v)!)),  q = x^2/4
//       (DLMF 10.25.2; 48 terms cover x <= 21.5);
//   K, 2 < x <= x1: log K_v = g_v(1/x) - x - 1/2 log(2x/pi), g_v a degree-20
//       Chebyshev expansion in s = 1/x on [1/17.5, 1/2] (Clenshaw);
//   K, x <= 2: DLMF 10.31.1 with n = 0, 1 (18 terms):
//       K_0 = C(q) - (log(x/2) + gamma) S_0(q),
//       x K_1 = 1 + q (2 (log(x/2) + gamma) S_1(q) - A(q)),
//       C_k = H_k/(k!)^2, A_k = (H_k + H_{k+1})/(k!(k+1)!), S_v as for I.
template <typename T> struct Tab01;
template <> struct Tab01<double> {
    static __device__ __forceinline__ const double *iser() { return &tables::kI01Ser64[0][0]; }
    static __device__ __forceinline__ const double *k0() { return tables::kK0Ser64; }
    static __device__ __forceinline__ const double *k1() { return tables::kK1Ser64; }
    static __device__ __forceinline__ const double *cheb() { return &tables::kK01Cheb64[0][0]; }
    static constexpr double gamma = tables::kEulerGamma64;
};
template <> struct Tab01<float> {
    static __device__ __forceinline__ const float *iser() { return &tables::kI01Ser32[0][0]; }
    static __device__ __forceinline__ const float *k0() { return tables::kK0Ser32; }
    static __device__ __forceinline__ const float *k1() { return tables::kK1Ser32; }
    static __device__ __forceinline__ const float *cheb() { return &tables::kK01Cheb32[0][0]; }
    static constexpr float gamma = tables::kEulerGamma32;
};

template <typename T, int NT>
__device__ __forceinline__ T horner(const LB_CONST_AS T *c, T q) {
    T s = c[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k)
        s = fm::fma_c(s, q, c[k]);
    return s;
}

template <typename T, int KIND, int V>
__device__ __forceinline__ T order01(T x) {
    constexpr RegimeSet r = Regime<T, KIND>::r;
    if (x > T(r.x1))
        return br_mu<T, KIND>(T(V), x);
    const T lx2 = llog(x) - Cst<T>::ln2;                 // log(x/2), safe for subnormal x
    const T q = T(0.25) * x * x;
    const LB_CONST_AS T *ser = opaque_const<T>(Tab01<T>::iser()) + V * tables::kI01Terms;
    if (KIND == KIND_I) {
        // sum = 1 + q h(q): log1p of q h keeps log I_0 ~ x^2/4 accurate
        // relative to itself for small x
        const T qh = q * horner<T, tables::kI01Terms - 1>(ser + 1, q);
        return (V == 0) ? llog1p(qh) : lx2 + llog1p(qh);
    }
    if (x > T(2)) {
        // Clenshaw on u = (2s - (sa + sb)) / (sb - sa), s = 1/x
        constexpr T sa = T(1) / T(17.5), sb = T(0.5);
        const LB_CONST_AS T *c = opaque_const<T>(Tab01<T>::cheb()) + V * (tables::kCheb01Deg + 1);
        const T u = fma(T(2) / (sb - sa), T(1) / x, -(sa + sb) / (sb - sa));
        const T u2 = u + u;
        T b1 = T(0), b2 = T(0);
#pragma unroll
        for (int j = tables::kCheb01Deg; j >= 1; --j) {
            const T b0 = fma(u2, b1, c[j] - b2);
            b2 = b1;
            b1 = b0;
        }
        const T g = fma(u, b1, c[0] - b2);
        return g - x - T(0.5) * (llog(x) + Cst<T>::ln2 - Cst<T>::log_pi);
    }
    const T lg = lx2 + Tab01<T>::gamma;
    if (V == 0) {
        const T s0 = horner<T, tables::kK01Terms>(ser, q);
        const T c0 = horner<T, tables::kK01Terms>(opaque_const<T>(Tab01<T>::k0()), q);
        return llog(c0 - lg * s0);
    }
    const T s1 = horner<T, tables::kK01Terms>(ser, q);
    const T a1 = horner<T, tables::kK01Terms>(opaque_const<T>(Tab01<T>::k1()), q);
    return llog(fma(q, T(2) * lg * s1 - a1, T(1))) - llog(x);
}

// ---------------------------------------------------------------------------
// Integer orders 2..14 (scalar-order path)
// ---------------------------------------------------------------------------
// Outside the series / integral region of order n the general branches apply
// unchanged (same bits as the general path).  Inside it:
//   I: log I_n = n log(x/2) - log n! + log1p(q h_n(q)), q = x^2/4, h_n the
//      polynomial with the exact constant coefficients n!/(k!(k+n)!)
//      (DLMF 10.25.2): no divisions and one trip count for every argument;
//   K: the forward recurrence K_{j+1} = K_{j-1} + (2j/x) K_j (DLMF 10.29.1)
//      from K_0 and K_1 of the order-0/1 path (k_up: values scaled to
//      K_1 = 1, in binary64).  Both terms are positive, so nothing cancels:
//      about one rounding per step.  log K_n = log K_1 + log(K_n / K_1).
//      Below x = 1e-10 the small-argument form of the general path.
template <typename T> struct TabInt;
template <> struct TabInt<double> {
    static constexpr int terms = tables::kIIntTerms64;
    static __device__ __forceinline__ const double *ser() { return &tables::kIIntSer64[0][0]; }
    static __device__ __forceinline__ const double *logfact() { return tables::kLogFact64; }
};
template <> struct TabInt<float> {
    static constexpr int terms = tables::kIIntTerms32;
    static __device__ __forceinline__ const float *ser() { return &tables::kIIntSer32[0][0]; }
    static __device__ __forceinline__ const float *logfact() { return tables::kLogFact32; }
};

// K_{mu+n} (n >= 1) by the recurrence K_{nu+1} = K_{nu-1} + (2 nu / x) K_nu
// (DLMF 10.29.1), nu = mu + 1 .. mu + n - 1, from d = K_mu and k1 = K_{mu+1}
// (or both scaled by one factor), ix2 = 2/x: one fma per step, no
// reciprocal.  For mu >= -1/2 every term is positive (K grows with the
// order), so nothing cancels and each step adds about one rounding.  In
// binary64 for both precisions: K_{mu+n} / K_{mu+1} stays in [1, ~1e160] for
// n <= 15 and x >= 1e-10 (each step at most 1 + 2 (mu + 14) / x), so values
// with K_{mu+1} below 1e140 need no rescaling there.
__device__ __forceinline__ double k_up(double d, double k1, double mu, int n, double ix2) {
    const double a0 = mu * ix2;
    double kn = k1, jd = 0.0;
    int j = 1;
    // two steps per trip (no register shuffle between them), then the odd one
    for (; j + 1 < n; j += 2) {
        const double k1 = fma(fma(jd + 1.0, ix2, a0), kn, d);
        const double k2 = fma(fma(jd + 2.0, ix2, a0), k1, kn);
        jd += 2.0;
        d = k1;
        kn = k2;
    }
    if (j < n)
        kn = fma(fma(jd + 1.0, ix2, a0), kn, d);
    return kn;
}

// The fallback region's part for integer order n, 0 <= n <= 14 (orders 0 and
// 1 by their fast path, whose expansions cover the whole fallback region).
template <typename T, int KIND>
__device__ __forceinline__ T order_int_fb(int n, T x) {
    const T v = T(n);
    if (n == 0)
        return order01<T, KIND, 0>(x);
    if (n == 1)
        return order01<T, KIND, 1>(x);
    if (KIND == KIND_I) {
        const T q = T(0.25) * x * x;
        const LB_CONST_AS T *c =
            opaque_const<T>(TabInt<T>::ser()) + (n - tables::kIntOrderMin) * TabInt<T>::terms;
        const T qh = q * horner<T, TabInt<T>::terms>(c, q);
        const T lf = opaque_const<T>(TabInt<T>::logfact())[n];
        return v * (llog(x) - Cst<T>::ln2) - lf + llog1p(qh);
    }
    if (x < T(1e-10))
        return T(br_k_small_x(double(v), double(x)));
    const T l0 = order01<T, KIND_K, 0>(x);
    const T l1 = order01<T, KIND_K, 1>(x);
    return l1 + T(llog(k_up(double(lexp(l0 - l1)), 1.0, 0.0, n, 2.0 * lrcp(double(x)))));
}

// ---------------------------------------------------------------------------
// K fallback for small arguments: Temme's series
// ---------------------------------------------------------------------------
// For 1e-10 <= x <= kTemmeX = 1.25 and a non-integer order v the log K
// fallback takes K_mu and K_{mu+1} at the fractional part mu = v - n,
// n = rint(v), |mu| <= 1/2, from Temme's series (N. M. Temme, J. Comput.
// Phys. 19, 1975), with q = x^2/4, c_k = q^k / k!, s = mu ln(2/x):
//   K_mu     = sum_k c_k f_k,
//   K_{mu+1} = (2/x) sum_k c_k (p_k - k f_k),
//   f_0 = (mu pi / sin mu pi) (cosh(s) G1(mu) + (sinh(s)/s) ln(2/x) G2(mu)),
//   p_0 = (x/2)^-mu Gamma(1+mu) / 2,
//   q_0 = (x/2)^mu Gamma(1-mu) / 2,
//   f_k = (k f_{k-1} + p_{k-1} + q_{k-1}) / (k^2 - mu^2),
//   p_k = p_{k-1} / (k - mu),  q_k = q_{k-1} / (k + mu),
// (G1, G2, sin(pi mu)/(pi mu) as polynomials in mu^2, generated tables), the
// sum stopped once c_k (k |f_k| + |p_k|), which bounds both new terms, falls
// below 2^-56 of the smaller sum (the c_k fall faster than geometrically for
// x <= 1.25); then the upward recurrence
// K_{nu+1} = K_{nu-1} + (2 nu / x) K_nu (DLMF 10.29.1) from nu = mu + 1 to v
// (k_up), as in the integer-order path.  One reciprocal per term:
// 1/(k - mu) = (k + mu)/(k^2 - mu^2) and likewise; 1/k from a table (k is the
// same in every lane of a wave).
// Cost (VALU instructions, binary64) ~205 + ~27 per term (2..11 terms) + ~5
// per order step, against ~145 + ~41 per node (20..70 nodes there) for the
// integral; the series is
// independent of the integral representations (the paper's and DLMF 10.32.9).
// Binary32: the same with binary32 tables and stop rule (2^-27), the order
// recurrence in binary64.  nterms, if given, receives the number of series
// terms after f_0.
template <typename T> struct TabTm;
template <> struct TabTm<double> {
    static __device__ __forceinline__ const double *g() { return &tables::kTmG64[0][0]; }
    static __device__ __forceinline__ const double *sinc() { return tables::kTmSinc64; }
    static __device__ __forceinline__ const double *sinh() { return tables::kTmSinh64; }
    static __device__ __forceinline__ const double *invk() { return tables::kTmInvK64; }
};
template <> struct TabTm<float> {
    static __device__ __forceinline__ const float *g() { return &tables::kTmG32[0][0]; }
    static __device__ __forceinline__ const float *sinc() { return tables::kTmSinc32; }
    static __device__ __forceinline__ const float *sinh() { return tables::kTmSinh32; }
    static __device__ __forceinline__ const float *invk() { return tables::kTmInvK32; }
};

template <typename T>
__device__ __forceinline__ T br_k_temme(T v, T x, int *nterms = nullptr) {
    const T n = rint(v);
    const T mu = v - n;
    const T t = mu * mu;
    const T L = Cst<T>::ln2 - llog(x);                        // ln(2/x) > 0
    const T s = mu * L;
    const T e = lexp_b(s);                                    // (2/x)^mu
    const T ie = lrcp(e);
    const LB_CONST_AS T *G = opaque_const<T>(TabTm<T>::g());
    const T g1 = horner<T, tables::kTmGCoefs>(G, t);
    const T g2 = horner<T, tables::kTmGCoefs>(G + tables::kTmGCoefs, t);
    const T sinc = horner<T, tables::kTmSincTerms>(opaque_const<T>(TabTm<T>::sinc()), t);
    T shs;                                                    // sinh(s)/s
    if (fabs(s) < T(1))
        shs = horner<T, tables::kTmSinhTerms>(opaque_const<T>(TabTm<T>::sinh()), s * s);
    else
        shs = (e - ie) * (T(0.5) * lrcp(s));
    const T ch = T(0.5) * (e + ie);
    const T rs = lrcp(sinc);                                  // Gamma(1+mu) Gamma(1-mu)
    T f = fma(g1, ch, shs * L * g2) * rs;
    // 1/Gamma(1-mu) = G2 + mu G1 and 1/Gamma(1+mu) = G2 - mu G1, so by the
    // reflection formula Gamma(1+mu) = rs (G2 + mu G1), Gamma(1-mu) = rs (G2 - mu G1)
    const T hr = T(0.5) * rs;
    T p = hr * e * fma(mu, g1, g2);
    T q = hr * ie * fma(-mu, g1, g2);
    const T qx = T(0.25) * x * x;
    const LB_CONST_AS T *ik = opaque_const<T>(TabTm<T>::invk());
    T c = T(1), s0 = f, s1 = p, kk = T(0);
    int k = 0;
    while (k < tables::kTmMaxTerms) {
        ++k;
        kk += T(1);
        const T d = lrcp(fma(kk, kk, -t));
        f = fma(kk, f, p + q) * d;
        c = c * qx * ik[k];
        p = p * (kk + mu) * d;
        q = q * (kk - mu) * d;
        s0 = fma(c, f, s0);
        s1 = fma(c, fma(-kk, f, p), s1);
        // c (k |f| + |p|) bounds both new terms (k >= 1): one test against the
        // smaller sum
        if (c * fma(kk, fabs(f), fabs(p)) <= Cst<T>::series_eps * fmin(s0, s1))
            break;
    }
    if (nterms != nullptr)
        *nterms = k;
    // one logarithm for every order step count (lanes of one wave differ):
    // K_v = K_mu (n = 0), else the recurrence from K_mu, K_{mu+1} in binary64
    // (K_{mu+1} < 2e15 and K_v < 1e181 for x >= 1e-10, v < 15)
    const double ix2 = 2.0 * lrcp(double(x));
    const double kv = (n == T(0)) ? double(s0)
                                  : k_up(double(s0), double(s1) * ix2, double(mu), int(n), ix2);
    return T(llog(kv));
}

template <typename T, int KIND>
__device__ __forceinline__ T order_int(int n, T x) {
    const T v = T(n);
    const int b = classify<T, KIND>(v, x);
    if (b == BR_MU)
        return br_mu<T, KIND>(v, x);
    if (b == BR_U) {
        const int tr = u_tier(v);
        return br_u<T, KIND>(v, x, (tr == 3) ? 4 : (tr == 2) ? 6 : (tr == 1) ? 9 : 13);
    }
    return order_int_fb<T, KIND>(n, x);
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------

// Value of the given branch, in the precision T, except the K fallback below
// x = 1e-10 (binary64 for both precisions).  K fallback: the cosh-integral
// trapezoid for x >= 1e-10; below, the small-argument forms (br_k_tiny_x for
// v < 0.3, br_k_small_x above).  Integer orders 0..14 take the
// integer-order path for x >= 1e-10 instead: K_0, K_1 by their fast path and
// K_n by the recurrence from them.  The u-integral variants take the paper's
// 600-node rule for x >= 1e-10 and for x < 1e-10 with v >= 0.3.
template <typename T, int KIND, int VAR = VAR_DEFAULT>
__device__ __forceinline__ T eval_branch(int b, T v, T x, const FbTab<KIND, T> *kt) {
    if (VAR == VAR_SEVEN) {
        switch (b) {
        case B7_MU3: return br_mu<T, KIND, 3>(v, x);
        case B7_MU20: return br_mu<T, KIND, 20>(v, x);
        case B7_U4: return br_u<T, KIND, 4>(v, x);
        case B7_U6: return br_u<T, KIND, 6>(v, x);
        case B7_U9: return br_u<T, KIND, 9>(v, x);
        case B7_U13: return br_u<T, KIND, 13>(v, x);
        default: b = BR_FB;
        }
    }
    if (b == BR_MU)
        return br_mu<T, KIND>(v, x);
    if (b == BR_U) {
        if (VAR == VAR_DEFAULT) {
            const int tr = u_tier(v);
            return br_u<T, KIND>(v, x, (tr == 3) ? 4 : (tr == 2) ? 6 : (tr == 1) ? 9 : 13);
        }
        return br_u<T, KIND>(v, x);
    }
    if constexpr (KIND == KIND_I) {
        // (integer orders keep the series here: the unrolled constant-
        // coefficient polynomials of the scalar-order path need more
        // registers than the grouped I kernels hold at full occupancy)
        return br_series_i<T>(v, x, kt);
    } else {
    constexpr bool u_integral = (VAR == VAR_U_INTEGRAL || VAR == VAR_SIMPSON || VAR == VAR_PAPER);
    if (!u_integral && x >= T(1e-10)) {
        if (VAR == VAR_DEFAULT && int_order(v))
            return order_int_fb<T, KIND_K>(int(v), x);
        if (VAR == VAR_DEFAULT && x <= T(tables::kTemmeX))
            return br_k_temme<T>(v, x);
        if constexpr (std::is_same<T, float>::value)
            return br_k_cosh32(v, x, kt);
        else
            return br_k_cosh(v, x, kt);
    }
    if (x < T(1e-10) && v < T(0.3))
        return T(br_k_tiny_x(double(v), double(x)));
    if (!u_integral)   // x < 1e-10, v >= 0.3
        return T(br_k_small_x(double(v), double(x)));
    if (VAR == VAR_SIMPSON || VAR == VAR_PAPER)
        return br_quad_k<T, double, true>(v, x);
    return br_quad_k<T, double>(v, x);
    }
}



}  // namespace lbessel
