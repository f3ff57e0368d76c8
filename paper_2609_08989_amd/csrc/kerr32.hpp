// kerr32.hpp -- FP32 far-field right-hand side of analytic Kerr, for the
// Runge-Kutta stages of the mixed-precision integrator.
//
// Two algebraic rearrangements keep FP32 accurate far from the hole, where
// the FP64 form of the equations loses digits to cancellation:
//   * dp_r/dlambda.  The off-shell form sums three O(r) terms to an O(1/r^2)
//     result.  On the constraint surface K = 2 Sigma H = 0 one may eliminate
//     p_r^2, which gives
//         dK/dr = 4 (P / Delta^2) [p_t (r^2 - a^2) + a p_phi (r - 1)]
//                 - 2 (r - 1) T / Delta,     T = p_theta^2 + W^2 / s^2,
//     free of cancellation; the K-proportional terms of Eq. (3) are dropped
//     (they vanish on the constraint, so the constraint stays invariant).
//   * dt/dlambda = -p_t + delta_t with delta_t = -2 r P / (Delta Sigma)
//     exactly; only delta_t (which is O(1/r)) is formed in FP32 and the
//     constant -p_t is added in FP64, so the error estimate of t is not
//     swamped by FP32 rounding of a nearly constant derivative.
// Outside these two, the formulas are those of kerr_rhs64.
#pragma once

#include <hip/hip_runtime.h>

#include "kerr.hpp"

namespace tartarus {

// Returns (delta_t, dr, dth, dph, dpr, dpth); delta_t excludes the constant -p_t.
__device__ __forceinline__ void kerr_rhs32(float a, float r, float th, float pr, float pth, float pt, float pph,
                                           Deriv<float>& d)
{
    float s, c;
    sincos32(th, &s, &c);
    const float a2 = a * a;
    const float r2 = r * r;
    const float s2 = s * s;
    const float sig = fmaf(a2, c * c, r2);
    const float del = fmaf(r, r - 2.0f, a2);
    const float iS = __builtin_amdgcn_rcpf(sig);
    const float iD = __builtin_amdgcn_rcpf(del);
    const float is2 = __builtin_amdgcn_rcpf(s2);
    const float ra = r2 + a2;
    const float P = fmaf(ra, pt, a * pph);
    const float W = fmaf(a * s2, pt, pph);
    const float Ws = W * is2;
    const float PiD = P * iD;
    d.r = del * pr * iS;
    d.th = pth * iS;
    d.ph = fmaf(-a, PiD, Ws) * iS;
    d.t = -2.0f * r * PiD * iS;
    const float T = fmaf(pth, pth, W * Ws);
    const float rm1 = r - 1.0f;
    const float dKr = fmaf(4.0f * PiD * iD, fmaf(pt, r2 - a2, a * pph * rm1), -2.0f * rm1 * T * iD);
    d.pr = -0.5f * iS * dKr;
    const float q = pph * is2;
    d.pth = -iS * s * c * fmaf(a2 * pt, pt, -q * q);
}

// FP64 Hamiltonian (Eq. (1), separated form) and cos(theta) at a point, for the
// constraint monitor of steps whose stages ran in FP32.
__device__ __forceinline__ double kerr_H64(double a, double r, double th, double pr, double pth, double pt,
                                           double pph, double& cth, double& sth)
{
    double s, c;
    sincos64(th, &s, &c);
    const double a2 = a * a, r2 = r * r, s2 = s * s;
    const double sig = fma(a2, c * c, r2);
    const double del = fma(r, r - 2.0, a2);
    const double P = fma(r2 + a2, pt, a * pph);
    const double W = fma(a * s2, pt, pph);
    const double K = fma(del * pr, pr, fma(pth, pth, fma(W * W, rcp64(s2), -(P * P * rcp64(del)))));
    cth = c;
    sth = s;
    return 0.5 * K * rcp64(sig);
}

}  // namespace tartarus
