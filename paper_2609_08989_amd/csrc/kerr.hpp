// kerr.hpp -- device functions for analytic Kerr: metric, Hamiltonian right-hand
// side, observer initial conditions and the Novikov-Thorne emitter.
//
// Boyer-Lindquist coordinates, G = c = M = 1.  With Sigma = r^2 + a^2 cos^2,
// Delta = r^2 - 2r + a^2, s = sin(theta), c = cos(theta), the Hamiltonian of
// Eq. (1) in Carter-separated form reads
//     2 Sigma H = K = Delta p_r^2 + p_th^2 + W^2 / s^2 - P^2 / Delta,
//     W = p_ph + a s^2 p_t,   P = (r^2 + a^2) p_t + a p_ph,
// which equals 1/2 g^{mu nu} p_mu p_nu of the Kerr metric identically.
// Hamilton's equations (Eqs. (2)-(3)) are its exact derivatives; the term
// proportional to K is kept, so the flow is Hamiltonian off the constraint too.
#pragma once

#include <hip/hip_runtime.h>

#include "fastmath.hpp"

namespace tartarus {

// The spin a and its square.  A trace of one metric takes both from the
// launch, wave-uniform in scalar registers, so a^2 is not formed again in every
// right-hand side; a ray of a serving epoch carries its own.
struct Spin {
    double a, a2;
};

__device__ __forceinline__ Spin spin_of(double a)
{
    return {a, a * a};
}

// d/dlambda of (t, r, theta, phi, p_r, p_theta); p_t and p_phi are constant.
template <typename T>
struct Deriv {
    T t, r, th, ph, pr, pth;
};

// FP64 right-hand side from sin^2(theta) s2, cos^2(theta) c2 and
// sin(theta) cos(theta) sc; also returns H (Eq. (1)).
__device__ __forceinline__ void kerr_rhs64_trig(Spin sp, double r, double s2, double c2, double sc, double pr,
                                                double pth, double pt, double pph, Deriv<double>& d, double& H)
{
    const double a = sp.a, a2 = sp.a2;
    const double r2 = r * r;
    const double sig = fma(a2, c2, r2);
    const double del = fma(r, r - 2.0, a2);
    // 1/Sigma, 1/Delta and 1/sin^2 from one reciprocal of their product (radii
    // are bounded by the escape radius, so the product stays in range)
    const double sd = sig * del;
    const double inv = rcp64(sd * s2);
    const double iS = (del * s2) * inv;
    const double iD = (sig * s2) * inv;
    const double is2 = sd * inv;
    const double ra = r2 + a2;
    const double P = fma(ra, pt, a * pph);
    const double W = fma(a * s2, pt, pph);
    const double Ws = W * is2;
    const double PiD = P * iD;
    const double dpr = del * pr;
    const double K = fma(dpr, pr, fma(pth, pth, fma(W, Ws, -P * PiD)));
    const double iSK = iS * K;   // K / Sigma = 2 H
    d.r = dpr * iS;
    d.th = pth * iS;
    d.ph = fma(-a, PiD, Ws) * iS;
    d.t = fma(a, W, -ra * PiD) * iS;
    // dp_r = -(1/2) d(K / Sigma)/dr with dK/dr = 2 (r - 1)(p_r^2 + (P/Delta)^2) - 4 r p_t P/Delta
    // and dSigma/dr = 2 r
    d.pr = iS * fma(r, fma(2.0 * pt, PiD, iSK), (1.0 - r) * fma(pr, pr, PiD * PiD));
    // dp_theta = -(1/2) d(K / Sigma)/dtheta with dK/dtheta = 2 sin cos (a^2 p_t^2 - (p_phi / sin^2)^2)
    // and dSigma/dtheta = -2 a^2 sin cos
    const double qp = pph * is2;
    d.pth = -(iS * sc) * fma(a2, fma(pt, pt, iSK), -(qp * qp));
    H = 0.5 * iSK;
}

// FP64 right-hand side at polar angle th.  Also returns H (Eq. (1)), cos(theta)
// and sin(theta) of the point.  coef supplies the sincos64 coefficients
// (compile-time immediates by default).
template <class Coef = SinCosImm>
__device__ __forceinline__ void kerr_rhs64(Spin a, double r, double th, double pr, double pth, double pt,
                                           double pph, Deriv<double>& d, double& H, double& cth, double& sth,
                                           Coef coef = {})
{
    // sin and cos from the reduced argument's (sr, cr) and the quadrant q: the
    // squares need only the swap of odd quadrants, sin cos is negative exactly
    // for odd q, and the signed values are formed only where they are used
    double sr, cr;
    int q;
    sincos64_parts(th, &sr, &cr, &q, coef);
    const bool odd = (q & 1) != 0;
    const double sr2 = sr * sr, cr2 = cr * cr;
    const double scr = sr * cr;
    kerr_rhs64_trig(a, r, odd ? cr2 : sr2, odd ? sr2 : cr2, odd ? -scr : scr, pr, pth, pt, pph, d, H);
    cth = flip_sign(odd ? sr : cr, (unsigned)((q + 1) & 2) << 30);
    sth = flip_sign(odd ? cr : sr, (unsigned)(q & 2) << 30);
}

// Covariant components (g_tt, g_tphi, g_rr, g_thth, g_phph) of Kerr at (r, theta).
__device__ __forceinline__ void kerr_metric64(double a, double r, double th, double g[5])
{
    double s, c;
    sincos64(th, &s, &c);
    const double a2 = a * a, r2 = r * r, s2 = s * s;
    const double sig = fma(a2, c * c, r2);
    const double del = fma(r, r - 2.0, a2);
    const double tr = 2.0 * r / sig;
    g[0] = tr - 1.0;
    g[1] = -a * tr * s2;
    g[2] = sig / del;
    g[3] = sig;
    g[4] = fma(a2 * tr, s2, r2 + a2) * s2;
}

// Observer initial conditions (Sec. 2.2): celestial coordinates -> local
// momentum (Eq. (4)) -> ZAMO tetrad (Eqs. (5), (7)-(10), e_(t)^phi = omega e_(t)^t)
// -> covariant momentum, negated for backward tracing.
__device__ __forceinline__ void observer_momentum(const double g[5], double D, double al, double be, double p[4])
{
    const double omega = -g[1] / g[4];
    const double ett = 1.0 / sqrt(fma(omega * omega, g[4], -g[0]));
    const double etp = omega * ett;
    const double err = 1.0 / sqrt(g[2]);
    const double ehh = 1.0 / sqrt(g[3]);
    const double epp = 1.0 / sqrt(g[4]);
    const double iD = 1.0 / D;
    const double plr = sqrt(1.0 - (al * al + be * be) * (iD * iD));
    const double put = ett;
    const double pur = err * plr;
    const double puh = ehh * (be * iD);
    const double pup = fma(epp, -al * iD, etp);
    p[0] = -fma(g[0], put, g[1] * pup);   // p_t
    p[1] = -(g[2] * pur);                 // p_r
    p[2] = -(g[3] * puh);                 // p_theta
    p[3] = -fma(g[1], put, g[4] * pup);   // p_phi
}

__device__ __forceinline__ double horizon_radius(double a) { return 1.0 + sqrt(1.0 - a * a); }

// Prograde ISCO (Bardeen, Press & Teukolsky 1972).
__device__ __forceinline__ double isco_radius(double a)
{
    const double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    const double z2 = sqrt(fma(3.0 * a, a, z1 * z1));
    return 3.0 + z2 - sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

// Roots of x^3 - 3x + 2a (Eq. (12)) and the coefficients of the logarithms in
// Eq. (11), 3 (x_i - a)^2 / (x_i prod_{j != i} (x_i - x_j)).  The root x_2
// vanishes at a = 0, where its term tends to zero: its coefficient is set to 0.
__device__ __forceinline__ void nt_flux_constants(double a, double xi[3], double coef[3])
{
    const double ac = acos(a);
    const double third = 1.0 / 3.0;
    xi[0] = 2.0 * cos((ac - M_PI) * third);
    xi[1] = 2.0 * cos((ac + M_PI) * third);
    xi[2] = -2.0 * cos(ac * third);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double xa = xi[i], xb = xi[(i + 1) % 3], xc = xi[(i + 2) % 3];
        coef[i] = fabs(xa) < 1e-12 ? 0.0 : 3.0 * (xa - a) * (xa - a) / (xa * (xa - xb) * (xa - xc));
    }
}

// Page-Thorne flux, Eq. (11), for r inside [r_in, r_out] (the caller checks),
// with x0 = sqrt(r_in) and the constants of nt_flux_constants.
__device__ __forceinline__ double nt_flux_pre(double a, double x0, const double xi[3], const double coef[3], double r)
{
    const double x = sqrt(r);
    double br = x - x0 - 1.5 * a * log(x / x0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (coef[i] != 0.0) br -= coef[i] * log((x - xi[i]) / (x0 - xi[i]));
    const double x2 = x * x;
    return 1.5 / (x2 * x2 * (x * (x2 - 3.0) + 2.0 * a)) * br;
}

// Redshift factor, Eq. (15), with u^t of Eq. (14) in the equatorial plane and
// the prograde Keplerian Omega = 1 / (r^{3/2} + a).
__device__ __forceinline__ double redshift(double a, double r, double pt, double pph)
{
    const double Om = 1.0 / (r * sqrt(r) + a);
    const double ir = 1.0 / r;
    const double gtt = 2.0 * ir - 1.0;
    const double gtp = -2.0 * a * ir;
    const double gpp = r * r + a * a + 2.0 * a * a * ir;
    const double ut = 1.0 / sqrt(-gtt - 2.0 * Om * gtp - Om * Om * gpp);
    return pt / (ut * fma(Om, pph, pt));
}

}  // namespace tartarus
