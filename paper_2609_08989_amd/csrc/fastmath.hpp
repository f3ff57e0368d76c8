// fastmath.hpp -- compact FP64 sine/cosine and reciprocal for the integrator's
// hot loop.  Written with explicit fma so that the host build (used by the CPU
// tests) and the device build round identically.
//
// sincos64: Cody & Waite argument reduction x = k pi/2 + r with pi/2 split in
// three doubles (each product k * P_i is fused, so the reduction is exact to
// well below an ulp of r for |k| < 2^20), then polynomials for sin r and cos r
// on |r| <= pi/4, and the quadrant swap.  The polynomials are the Taylor
// series economized on that interval (Chebyshev re-expansion, cut at degree
// 13 for sin and 14 for cos, truncation error below 4e-18; sincos_coeffs.py
// derives the coefficients).  Valid for |x| < 1e6; the polar angle of a ray
// stays within a few pi.
#pragma once

#include <cmath>
#include <cstring>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define TT_HD __host__ __device__
#else
#define TT_HD
#endif

namespace tartarus {

// Coefficients of sincos64 in the order it uses them: 2/pi; pi/2 = hi + mid +
// lo; the sine polynomial s6 .. s1 and the cosine polynomial c7 .. c2 (Horner
// order; cos r = 1 + r^2 (c1 + ...) with c1 = -1/2 exact).
constexpr double kSinCos64[16] = {
    0.6366197723675814,   1.5707963267948966,    6.123233995736766e-17,  -1.4973849048591698e-33,
    1.5894740706160615e-10, -2.5050717053109253e-08, 2.7557313376976021e-06, -0.0001984126982865223,
    0.0083333333333203662, -0.16666666666666616,
    -1.1353381481384318e-11, 2.0875582423297387e-09, -2.7557313098175798e-07, 2.4801587283882876e-05,
    -0.0013888888888861099, 0.041666666666666449};

// The coefficients as compile-time immediates.
struct SinCosImm {
    TT_HD double operator()(int i) const { return kSinCos64[i]; }
};

// Coefficients of the angle shift sin, cos(theta0 + d) from those of theta0
// for |d| <= 1/16: sin d = d + d^3 (s1 + z (s2 + z s3)) and cos d - 1 =
// z (-1/2 + z (c2 + z (c3 + z c4))), z = d^2, the Taylor series economized on
// that interval (truncation below 5e-18 relative and 5e-22; sincos_coeffs.py
// derives them).  Order: s3, s2, s1, c4, c3, c2.
constexpr double kShift64[6] = {-0.00019839117033214164, 0.0083333332807754186, -0.16666666666662561,
                                2.4798896288531483e-05,  -0.00138888887969124,   0.041666666666653834};

struct ShiftImm {
    TT_HD double operator()(int i) const { return kShift64[i]; }
};

// x with its sign bit XORed with bit 31 of hi_bit (the other bits of hi_bit
// must be zero).
TT_HD inline double flip_sign(double x, unsigned hi_bit)
{
#if defined(__HIP_DEVICE_COMPILE__)
    // one XOR on the high word (through a 64-bit integer the compiler split
    // the XOR into byte-wise masks, three instructions)
    return __hiloint2double(__double2hiint(x) ^ (int)hi_bit, __double2loint(x));
#else
    unsigned long long u;
    std::memcpy(&u, &x, sizeof u);
    u ^= (unsigned long long)hi_bit << 32;
    std::memcpy(&x, &u, sizeof u);
    return x;
#endif
}

// The reduced argument's sine and cosine (sr, cr) and the quadrant q: with
// odd q the two swap, and sin x = +-(q odd ? cr : sr) with the sign of bit 1 of
// q, cos x = +-(q odd ? sr : cr) with the sign of bit 1 of q + 1.
template <class Coef>
TT_HD inline void sincos64_parts(double x, double* srp, double* crp, int* qp, Coef coef)
{
    const double k = std::rint(x * coef(0));
    double r = std::fma(-k, coef(1), x);
    r = std::fma(-k, coef(2), r);
    r = std::fma(-k, coef(3), r);
    const double r2 = r * r;
    // sin r = r + r^3 (s1 + r^2 (s2 + ... + r^2 s6))
    double ps = coef(4);
#pragma unroll
    for (int i = 5; i <= 9; ++i) ps = std::fma(ps, r2, coef(i));
    const double sr = std::fma(ps * r2, r, r);
    // cos r = 1 + r^2 (c1 + r^2 (c2 + ... + r^2 c7))
    double pc = coef(10);
#pragma unroll
    for (int i = 11; i <= 15; ++i) pc = std::fma(pc, r2, coef(i));
    pc = std::fma(pc, r2, -0.5);
    *crp = std::fma(pc, r2, 1.0);
    *srp = sr;
    // quadrant: |k| < 2^20, so the int conversion is exact (one instruction,
    // where a 64-bit integer conversion of a double takes four)
    *qp = ((int)k) & 3;
}

// x y + z rounded twice (never fused): the shift polynomials' first steps,
// whose two coefficients, as operands of one fused instruction, would be more
// scalar registers than one instruction may read and cost a copy.
TT_HD inline double mul_then_add(double x, double y, double z)
{
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
    return x * y + z;
}

// sin and cos of theta0 + dt from s0 = sin(theta0), c0 = cos(theta0), for
// |dt| <= 1/16: the shift polynomials (kShift64 taken from coef(i)), then the
// angle-sum identities with the small terms added last (about one ulp each).
// The sine keeps its relative accuracy while |dt| stays well below |s0|; the
// caller checks both bounds.
template <class Coef>
TT_HD inline void sincos_shift(double s0, double c0, double dt, double& s, double& c, Coef coef)
{
    const double z = dt * dt;
    const double ps = std::fma(mul_then_add(z, coef(0), coef(1)), z, coef(2));
    const double sd = std::fma(dt * z, ps, dt);   // sin(dt)
    const double cm = z * std::fma(std::fma(mul_then_add(z, coef(3), coef(4)), z, coef(5)), z, -0.5);   // cos(dt) - 1
    s = std::fma(s0, cm, std::fma(c0, sd, s0));
    c = std::fma(c0, cm, std::fma(-s0, sd, c0));
}

// sincos64 with the coefficients taken from coef(i) (i indexes kSinCos64).
// The signs are applied by flipping the sign bit (same bits as negation).
template <class Coef>
TT_HD inline void sincos64_with(double x, double* sp, double* cp, Coef coef)
{
    double sr, cr;
    int q;
    sincos64_parts(x, &sr, &cr, &q, coef);
    const double s = (q & 1) ? cr : sr;
    const double c = (q & 1) ? sr : cr;
    *sp = flip_sign(s, (unsigned)(q & 2) << 30);
    *cp = flip_sign(c, (unsigned)((q + 1) & 2) << 30);
}

TT_HD inline void sincos64(double x, double* sp, double* cp)
{
    sincos64_with(x, sp, cp, SinCosImm{});
}

// sincos32: the single-precision counterpart for the FP32 far-field stages.
// Cody & Waite reduction with pi/2 in three floats (fused products), then the
// Taylor series economized on |r| <= pi/4 to degree 7 (sin) and 8 (cos)
// (truncation below 3e-9 and 5e-11, under 0.05 ulp of float; sincos_coeffs.py
// with the single-precision degrees).  Valid for |x| < 1e4, far beyond any
// polar angle a ray reaches; no large-argument branch.
TT_HD inline void sincos32(float x, float* sp, float* cp)
{
    const float k = std::rint(x * 0.63661975f);
    float r = std::fma(-k, 1.57079637f, x);
    r = std::fma(-k, -4.37113883e-08f, r);
    r = std::fma(-k, -1.77635684e-15f, r);
    const float r2 = r * r;
    float ps = -0.000195039582f;
    ps = std::fma(ps, r2, 0.00833203644f);
    ps = std::fma(ps, r2, -0.166666508f);
    const float sr = std::fma(ps * r2, r, r);
    float pc = 2.43798731e-05f;
    pc = std::fma(pc, r2, -0.00138866180f);
    pc = std::fma(pc, r2, 0.0416666158f);
    pc = std::fma(pc, r2, -0.5f);
    const float cr = std::fma(pc, r2, 1.0f);
    const int q = ((int)k) & 3;
    const float s = (q & 1) ? cr : sr;
    const float c = (q & 1) ? sr : cr;
    *sp = (q & 2) ? -s : s;
    *cp = ((q + 1) & 2) ? -c : c;
}

#if defined(__HIPCC__)
// 1/x from the hardware reciprocal estimate refined by two Newton-Raphson
// steps (r <- r + r (1 - x r)); within an ulp or two of the rounded quotient.
// (The host pass of hipcc only parses this device function.)
__device__ __forceinline__ double rcp64(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// 1/x with one Newton-Raphson step: the estimate's ~2^-24 relative error
// becomes ~2^-47.  For the error norm, whose value only steers the step size.
__device__ __forceinline__ double rcp64_coarse(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}
#endif

}  // namespace tartarus
