// fastmath.hpp -- compact FP64 sine/cosine and reciprocal for the integrator's
// hot loop.  Written with explicit fma so that the host build (used by the CPU
// tests) and the device build round identically.
//
// sincos64: Cody & Waite argument reduction x = k pi/2 + r with pi/2 split in
// three doubles (each product k * P_i is fused, so the reduction is exact to
// well below an ulp of r for |k| < 2^20), then the Taylor series of sin and
// cos on |r| <= pi/4 truncated after r^17 / 17! and r^16 / 16! (truncation
// error below 7e-17 relative), and the quadrant swap.  Valid for |x| < 1e6;
// the polar angle of a ray stays within a few pi.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define TT_HD __host__ __device__
#else
#define TT_HD
#endif

namespace tartarus {

constexpr double kPio2Hi = 1.5707963267948966;       // pi/2 = hi + mid + lo
constexpr double kPio2Mid = 6.123233995736766e-17;
constexpr double kPio2Lo = -1.4973849048591698e-33;
constexpr double kTwoOverPi = 0.6366197723675814;

TT_HD inline void sincos64(double x, double* sp, double* cp)
{
    const double k = std::rint(x * kTwoOverPi);
    double r = std::fma(-k, kPio2Hi, x);
    r = std::fma(-k, kPio2Mid, r);
    r = std::fma(-k, kPio2Lo, r);
    const double r2 = r * r;
    // sin r = r + r^3 * (-1/3! + r^2 (1/5! - r^2 (1/7! - ...)))
    double ps = 2.8114572543455206e-15;                 //  1/17!
    ps = std::fma(ps, r2, -7.647163731819816e-13);      // -1/15!
    ps = std::fma(ps, r2, 1.6059043836821613e-10);      //  1/13!
    ps = std::fma(ps, r2, -2.505210838544172e-08);      // -1/11!
    ps = std::fma(ps, r2, 2.7557319223985893e-06);      //  1/9!
    ps = std::fma(ps, r2, -0.0001984126984126984);      // -1/7!
    ps = std::fma(ps, r2, 0.008333333333333333);        //  1/5!
    ps = std::fma(ps, r2, -0.16666666666666666);        // -1/3!
    const double sr = std::fma(ps * r2, r, r);
    // cos r = 1 + r^2 * (-1/2 + r^2 (1/4! - ...))
    double pc = 4.779477332387385e-14;                  //  1/16!
    pc = std::fma(pc, r2, -1.1470745597729725e-11);     // -1/14!
    pc = std::fma(pc, r2, 2.08767569878681e-09);        //  1/12!
    pc = std::fma(pc, r2, -2.755731922398589e-07);      // -1/10!
    pc = std::fma(pc, r2, 2.48015873015873e-05);        //  1/8!
    pc = std::fma(pc, r2, -0.001388888888888889);       // -1/6!
    pc = std::fma(pc, r2, 0.041666666666666664);        //  1/4!
    pc = std::fma(pc, r2, -0.5);                        // -1/2
    const double cr = std::fma(pc, r2, 1.0);
    const int q = ((int)(long long)k) & 3;
    const double s = (q & 1) ? cr : sr;
    const double c = (q & 1) ? sr : cr;
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
#endif

}  // namespace tartarus
