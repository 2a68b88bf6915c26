// binary64 exp and log for the hot loops.
//
// gfx950 has no FP64 transcendental unit, so every f64 exp/log is a software
// sequence.  The device library's versions cost ~36 (exp) and ~92 (log) VALU
// instructions; these cost ~19 and ~32 at <= ~1 ulp, which is all the
// log-scale sums need.  Coefficients: paper_2409_08729_amd/fit_elementary.py
// (Chebyshev interpolants computed in 60-digit arithmetic, rounded once).
//
// Standard math calls (rint, fma, frexp, ldexp) plus fma_c below; the host
// build of the same code is what the unit tests exercise.
#pragma once

#include <math.h>

namespace lbessel {
namespace fm {

// a * b + c for a wavefront-uniform c (a compile-time constant or a value
// read with a uniform address).  gfx950 has no literal operands in 3-operand
// VALU encodings, and the compiler otherwise copies each 64-bit constant into
// two VGPRs with two VALU moves to use the accumulating fma form; here the
// constant stays in SGPRs (written by the scalar unit) and the fma is one
// VALU instruction.  The host build (unit tests) uses the same IEEE fma.
// c must really be uniform: a lane-varying c would be read from lane 0.
__host__ __device__ __forceinline__ double fma_c(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
#else
    return fma(a, b, c);
#endif
}

__host__ __device__ __forceinline__ float fma_c(float a, float b, float c) {
#if defined(__HIP_DEVICE_COMPILE__)
    float d;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
#else
    return fmaf(a, b, c);
#endif
}

// 1/d from the hardware reciprocal (v_rcp_f64: ~2^-24 relative, measured up
// to 2.3e8 ulps) and one Newton step: ~2^-47 relative, up to ~9 ulps
// measured (the host build divides).  Only used where the quotient feeds a
// small correction term.
__host__ __device__ __forceinline__ double rcp_nr(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double q = __builtin_amdgcn_rcp(d);
    return fma(q, fma(-d, q, 1.0), q);
#else
    return 1.0 / d;
#endif
}

// 1/d to within one ulp: the hardware reciprocal and two Newton steps (the
// second squares the first one's ~2^-47 error away, leaving the rounding of
// its final fma), for normal d with 1/d normal (the host build divides).
__host__ __device__ __forceinline__ double rcp64(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    double q = __builtin_amdgcn_rcp(d);
    q = fma(q, fma(-d, q, 1.0), q);
    return fma(q, fma(-d, q, 1.0), q);
#else
    return 1.0 / d;
#endif
}

// 1/sqrt(a) to within about one ulp: the hardware estimate (v_rsq_f64) and
// two Newton steps y <- y + y (1 - a y^2) / 2, for normal a > 0 whose square
// root and its reciprocal are normal (the host build divides).
__host__ __device__ __forceinline__ double rsq64(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(a);
    y = fma(0.5 * y, fma(-a * y, y, 1.0), y);
    return fma(0.5 * y, fma(-a * y, y, 1.0), y);
#else
    return 1.0 / sqrt(a);
#endif
}

// ln 2 = kLn2Hi + kLn2Lo, kLn2Hi with 32 significant bits (k * kLn2Hi exact
// for |k| < 2^21).
constexpr double kLog2e = 0x1.71547652b82fep+0;
constexpr double kLn2Hi = 0x1.62e42ff000000p-1;
constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;

// 2^k e^r with k = rint(y log2 e), r = y - k ln 2 in [-ln2/2, ln2/2]; e^r by a
// degree-11 polynomial (relative error 3e-18).  Returns (e^r, k).
__host__ __device__ __forceinline__ double exp64_core(double y, double &k_out) {
    const double k = rint(y * kLog2e);
    double r = fma(-k, kLn2Hi, y);
    r = fma(-k, kLn2Lo, r);
    double p = fma_c(0x1.af631d0059becp-26, r, 0x1.28b4057f44145p-22);
    p = fma_c(p, r, 0x1.71ddf5749d126p-19);
    p = fma_c(p, r, 0x1.a01991ac8730ap-16);
    p = fma_c(p, r, 0x1.a01a01b14378fp-13);
    p = fma_c(p, r, 0x1.6c16c187fbe02p-10);
    p = fma_c(p, r, 0x1.111111110f225p-7);
    p = fma_c(p, r, 0x1.555555554f0cfp-5);
    p = fma_c(p, r, 0x1.555555555555ap-3);
    p = fma_c(p, r, 0x1.0000000000011p-1);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    k_out = k;
    return p;
}

// The leading coefficient of exp64_core's polynomial, held in a VGPR pair by
// a loop that calls exp64_bounded_lc many times: the first Horner step then
// reads one SGPR constant instead of copying both into VGPRs every call.
constexpr double kExpLead = 0x1.af631d0059becp-26;
__host__ __device__ __forceinline__ double pin_v(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(a));
#endif
    return a;
}

// exp64_bounded with the leading coefficient lead == kExpLead supplied by the
// caller (same result bits).
__host__ __device__ __forceinline__ double exp64_bounded_lc(double y, double lead) {
    const double k = rint(y * kLog2e);
    double r = fma(-k, kLn2Hi, y);
    r = fma(-k, kLn2Lo, r);
    double p = fma_c(lead, r, 0x1.28b4057f44145p-22);
    p = fma_c(p, r, 0x1.71ddf5749d126p-19);
    p = fma_c(p, r, 0x1.a01991ac8730ap-16);
    p = fma_c(p, r, 0x1.a01a01b14378fp-13);
    p = fma_c(p, r, 0x1.6c16c187fbe02p-10);
    p = fma_c(p, r, 0x1.111111110f225p-7);
    p = fma_c(p, r, 0x1.555555554f0cfp-5);
    p = fma_c(p, r, 0x1.555555555555ap-3);
    p = fma_c(p, r, 0x1.0000000000011p-1);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, int(k));
}

// exp(y) for finite y; below about -745 gives 0, above about 709.8 +inf.
__host__ __device__ __forceinline__ double exp64(double y) {
    double k;
    const double p = exp64_core(y, k);
    // clamp the exponent so the conversion is defined; beyond +-1100 the
    // scaling over/underflows to inf/0 exactly as the true value does
    const double kc = fmin(fmax(k, -1100.0), 1100.0);
    return ldexp(p, int(kc));
}

// exp(y) for |y| < 1e9 (the exponent fits an int without clamping); values
// below about -745 still underflow to 0 through the final scaling.
__host__ __device__ __forceinline__ double exp64_bounded(double y) {
    double k;
    const double p = exp64_core(y, k);
    return ldexp(p, int(k));
}

// log(a) for finite a > 0 (normal or subnormal).  a = m 2^e with m in
// [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f/(2+f), z = s^2:
// log(1+f) = f - f^2/2 + s (f^2/2 + z P(z)) (the first terms exact or
// nearly so, the polynomial only corrects), P of degree 6.
__host__ __device__ __forceinline__ double log64(double a) {
    int e;
    double m = frexp(a, &e);                     // [0.5, 1)
    const bool low = m < 0x1.6a09e667f3bcdp-1;   // sqrt(1/2)
    m = low ? m + m : m;
    e = low ? e - 1 : e;
    const double f = m - 1.0;
    const double s = f * rcp_nr(2.0 + f);
    const double z = s * s;
    double p = fma_c(0x1.2b584aae78a57p-3, z, 0x1.39fe606542ddep-3);
    p = fma_c(p, z, 0x1.7462b4ab2ef6bp-3);
    p = fma_c(p, z, 0x1.c71c62e5800a1p-3);
    p = fma_c(p, z, 0x1.2492492df148dp-2);
    p = fma_c(p, z, 0x1.99999999952e2p-2);
    p = fma_c(p, z, 0x1.5555555555558p-1);
    const double r = z * p;
    const double hfsq = 0.5 * f * f;
    const double de = double(e);
    return fma(de, kLn2Hi, -((hfsq - fma(s, hfsq + r, de * kLn2Lo)) - f));
}

// log(1 + t) for finite t >= 0.  u = 1 + t rounded; then
// log(1 + t) = log(u) + log(1 + d/u) with d = t - (u - 1) the rounding error
// of the sum (u - 1 and d are exact), and log(1 + d/u) = d/u to within
// (d/u)^2 <= 2^-106.  Relative error ~1 ulp for every t, where log64(1 + t)
// has an absolute error of ~2^-53 (large relative error for t near 0).
__host__ __device__ __forceinline__ double log1p64(double t) {
    const double u = 1.0 + t;
    return fma(t - (u - 1.0), rcp_nr(u), log64(u));
}

// binary32 hardware approximations (v_exp_f32, v_log_f32, v_rcp_f32,
// v_rsq_f32, v_sqrt_f32; about one binary32 ulp) for quantities that only
// steer an algorithm (a Newton start and iterate, a step size, a shift,
// a cost estimate) and never enter a result's arithmetic.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float exp_hw(float a) {
    return __builtin_amdgcn_exp2f(a * 1.44269504f);
}
__device__ __forceinline__ float log_hw(float a) {
    return __builtin_amdgcn_logf(a) * 0.693147181f;
}
__device__ __forceinline__ float rcp_hw(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ float rsqrt_hw(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ float sqrt_hw(float a) { return __builtin_sqrtf(a); }
#else
__host__ __device__ inline float exp_hw(float a) { return expf(a); }
__host__ __device__ inline float log_hw(float a) { return logf(a); }
__host__ __device__ inline float rcp_hw(float a) { return 1.0f / a; }
__host__ __device__ inline float rsqrt_hw(float a) { return 1.0f / sqrtf(a); }
__host__ __device__ inline float sqrt_hw(float a) { return sqrtf(a); }
#endif

}  // namespace fm
}  // namespace lbessel
