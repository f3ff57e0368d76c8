// order.hpp -- scheduling key of a ray: how close it passes to the spherical
// photon orbits of Kerr.
//
// The integrator's cost per ray is dominated by rays that wind around the hole
// before escaping or falling in: those whose radial potential (Carter's
// separation of the null geodesic equations in Boyer-Lindquist coordinates)
//
//   R(r) / E^2 = (r^2 + a^2 - a b)^2 - Delta(r) (q + (b - a)^2),
//   b = L / E,  q = Q / E^2,  Delta = r^2 - 2 r + a^2,
//
// has a (near) double root outside the horizon.  The key is the binary order of
// magnitude of min over r in [r_+, 5] of R(r) / r^4 (zero exactly on the
// critical curve; every spherical photon orbit of Kerr lies in 1 <= r <= 4),
// mapped to kOrderBuckets bins, larger = closer to critical = started earlier.
// The key only reorders the work queue: it never enters a ray's arithmetic, so
// traced results do not depend on it.
#pragma once

#include <cmath>

#include "fastmath.hpp"

namespace tartarus {

constexpr int kOrderBuckets = 32;

// R(r) / (E^2 r^4) with w = a^2 - a b and C = q + (b - a)^2.
TT_HD inline double potential_r4(double r, double a2, double w, double C)
{
    const double r2 = r * r;
    const double u = r2 + w;
    const double del = r2 - 2.0 * r + a2;
    return (u * u - del * C) / (r2 * r2);
}

// min over r in [rp, 5] of R(r) / r^4: a 16-point scan
// (quadratically spaced from r_+), then eight Newton steps
// on R'(r) = 0 from the best sample (clamped to the interval).
TT_HD inline double critical_distance(double a, double b, double q, double rp)
{
    const double a2 = a * a;
    const double w = a2 - a * b;
    const double C = q + (b - a) * (b - a);
    const double hi = 5.0;
    double rbest = rp, vbest = INFINITY;
    for (int k = 0; k < 16; ++k) {
        const double x = (double)k / 15.0;
        const double r = rp + (hi - rp) * x * x;   // denser next to the horizon
        const double v = potential_r4(r, a2, w, C);
        if (v < vbest) {
            vbest = v;
            rbest = r;
        }
    }
    double r = rbest;
    for (int it = 0; it < 8; ++it) {
        const double d1 = 4.0 * r * (r * r + w) - 2.0 * (r - 1.0) * C;
        const double d2 = 12.0 * r * r + 4.0 * w - 2.0 * C;
        if (d2 != 0.0) r -= d1 / d2;
        r = r < rp ? rp : (r > hi ? hi : r);
    }
    const double v = potential_r4(r, a2, w, C);
    return v < vbest ? v : vbest;
}

// Bucket in [0, kOrderBuckets): half-octaves of -log2 |D| from -8 upward.
TT_HD inline int cost_bucket(double a, double b, double q, double rp)
{
    const double d = std::fabs(critical_distance(a, b, q, rp));
    if (!(d == d)) return 0;
    const double x = -std::log2(d > 1e-300 ? d : 1e-300);
    const double k = std::floor((x + 8.0) * 2.0);
    return k < 0.0 ? 0 : (k > (double)(kOrderBuckets - 1) ? kOrderBuckets - 1 : (int)k);
}

}  // namespace tartarus
