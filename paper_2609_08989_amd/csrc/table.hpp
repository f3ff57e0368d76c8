// table.hpp -- tabulated stationary axisymmetric metric (the form of Eq. (6)):
// bicubic Hermite interpolation in (u = ln r, theta) and the generic
// Hamiltonian right-hand side of Eqs. (2)-(3).
//
// Table layout (caller-owned device memory): tab[c][k][l][4], c over
// (g_tt, g_tphi / sin^2, g_rr, g_thth, g_phph / sin^2), k over
// r_k = exp(ln r_min + k du), l over theta_l = l dth, dth = pi / (nth - 1),
// last index (f, df/dr, df/dth, d2f/dr dth).  The two azimuthal components are
// tabulated divided by sin^2(theta) so that they stay smooth at the axis.
//
// The integrator reads a copy the library interleaves by grid point,
// [k][l][c][4]: the five components of a node share 160 contiguous bytes, so
// the 2 x 2 nodes of a cell are two 320-byte runs instead of ten 64-byte pieces
// on five planes 4 MiB apart.  The values are the caller's, only reordered.
#pragma once

#include <hip/hip_runtime.h>

#include "kerr.hpp"

namespace tartarus {

struct TableView {
    const double* tab;       // [c][k][l][4] (the caller's layout)
    const double* inter;     // [k][l][c][4] (interleaved copy), or null
    int nr, nth;
    double u0, du, idu, dth, idth;
};

__host__ __device__ inline TableView make_table_view(const double* tab, int nr, int nth, double r_min, double r_max)
{
    TableView v;
    v.tab = tab;
    v.inter = nullptr;
    v.nr = nr;
    v.nth = nth;
    v.u0 = log(r_min);
    v.du = (log(r_max) - log(r_min)) / (double)(nr - 1);
    v.idu = 1.0 / v.du;
    v.dth = M_PI / (double)(nth - 1);
    v.idth = 1.0 / v.dth;
    return v;
}

// Cubic Hermite basis at x: value weights p0, p1 and slope weights m0, m1, and
// their derivatives.
struct Hb {
    double p0, p1, m0, m1, dp0, dp1, dm0, dm1;
};

__device__ __forceinline__ Hb hermite_basis(double x)
{
    Hb b;
    const double x2 = x * x, x3 = x2 * x;
    b.p1 = fma(-2.0, x3, 3.0 * x2);
    b.p0 = 1.0 - b.p1;
    b.m0 = fma(x2, x - 2.0, x);
    b.m1 = x3 - x2;
    b.dp1 = 6.0 * x * (1.0 - x);
    b.dp0 = -b.dp1;
    b.dm0 = fma(x, fma(3.0, x, -4.0), 1.0);
    b.dm1 = x * fma(3.0, x, -2.0);
    return b;
}

// Interpolated metric: g[5] covariant components, gr[5] = d/dr, gt[5] = d/dtheta.
// INTER: read the interleaved copy (T.inter), else the caller's layout.
template <bool WITH_DERIVS, bool INTER>
__device__ __forceinline__ void table_metric(const TableView& T, double r, double th, double g[5], double gr[5],
                                             double gt[5])
{
    const double u = log(r);
    int k = (int)floor((u - T.u0) * T.idu);
    k = k < 0 ? 0 : (k > T.nr - 2 ? T.nr - 2 : k);
    int l = (int)floor(th * T.idth);
    l = l < 0 ? 0 : (l > T.nth - 2 ? T.nth - 2 : l);
    const double uk = fma((double)k, T.du, T.u0);
    const double x = (u - uk) * T.idu;
    const double y = (th - (double)l * T.dth) * T.idth;
    const Hb bx = hermite_basis(x), by = hermite_basis(y);
    const double rk0 = exp(uk), rk1 = exp(fma((double)(k + 1), T.du, T.u0));
    const double sdu0 = rk0 * T.du, sdu1 = rk1 * T.du;
    const size_t plane = (size_t)T.nr * T.nth * 4;
    const double* base = INTER ? T.inter + ((size_t)k * T.nth + l) * 20 : T.tab + ((size_t)k * T.nth + l) * 4;
    const size_t cstep = INTER ? 4 : plane, lstep = INTER ? 20 : 4, kstep = (size_t)T.nth * lstep;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const double* e00 = base + c * cstep;          // (k, l)
        const double* e01 = e00 + lstep;               // (k, l+1)
        const double* e10 = e00 + kstep;               // (k+1, l)
        const double* e11 = e10 + lstep;               // (k+1, l+1)
        const double4 c00 = *reinterpret_cast<const double4*>(e00);
        const double4 c01 = *reinterpret_cast<const double4*>(e01);
        const double4 c10 = *reinterpret_cast<const double4*>(e10);
        const double4 c11 = *reinterpret_cast<const double4*>(e11);
        // per corner: value, u-slope and theta-slope in cell units, cross term
        const double F00 = c00.x, U00 = c00.y * sdu0, V00 = c00.z * T.dth, X00 = c00.w * sdu0 * T.dth;
        const double F01 = c01.x, U01 = c01.y * sdu0, V01 = c01.z * T.dth, X01 = c01.w * sdu0 * T.dth;
        const double F10 = c10.x, U10 = c10.y * sdu1, V10 = c10.z * T.dth, X10 = c10.w * sdu1 * T.dth;
        const double F11 = c11.x, U11 = c11.y * sdu1, V11 = c11.z * T.dth, X11 = c11.w * sdu1 * T.dth;
        // collapse the theta direction first: A_i(y) = sum_j (F p_j(y) + V m_j(y)), B_i(y) = same for U, X
        const double A0 = F00 * by.p0 + V00 * by.m0 + F01 * by.p1 + V01 * by.m1;
        const double A1 = F10 * by.p0 + V10 * by.m0 + F11 * by.p1 + V11 * by.m1;
        const double B0 = U00 * by.p0 + X00 * by.m0 + U01 * by.p1 + X01 * by.m1;
        const double B1 = U10 * by.p0 + X10 * by.m0 + U11 * by.p1 + X11 * by.m1;
        g[c] = A0 * bx.p0 + B0 * bx.m0 + A1 * bx.p1 + B1 * bx.m1;
        if (WITH_DERIVS) {
            const double dA0 = F00 * by.dp0 + V00 * by.dm0 + F01 * by.dp1 + V01 * by.dm1;
            const double dA1 = F10 * by.dp0 + V10 * by.dm0 + F11 * by.dp1 + V11 * by.dm1;
            const double dB0 = U00 * by.dp0 + X00 * by.dm0 + U01 * by.dp1 + X01 * by.dm1;
            const double dB1 = U10 * by.dp0 + X10 * by.dm0 + U11 * by.dp1 + X11 * by.dm1;
            const double gx = A0 * bx.dp0 + B0 * bx.dm0 + A1 * bx.dp1 + B1 * bx.dm1;
            const double gy = dA0 * bx.p0 + dB0 * bx.m0 + dA1 * bx.p1 + dB1 * bx.m1;
            gr[c] = gx * T.idu / r;
            gt[c] = gy * T.idth;
        }
    }
    // restore the sin^2 factor of g_tphi and g_phph
    double s, cth;
    sincos64(th, &s, &cth);
    const double s2 = s * s, ds2 = 2.0 * s * cth;
    if (WITH_DERIVS) {
        gt[1] = fma(ds2, g[1], s2 * gt[1]);
        gr[1] *= s2;
        gt[4] = fma(ds2, g[4], s2 * gt[4]);
        gr[4] *= s2;
    }
    g[1] *= s2;
    g[4] *= s2;
}

// Generic right-hand side of Eqs. (2)-(3) for a metric of the form of Eq. (6),
// on the interleaved copy (T.inter must be set):
// dx^mu = g^{mu nu} p_nu and dp_mu = 1/2 (d_mu g_ab) dx^a dx^b (the same as
// -1/2 (d_mu g^{ab}) p_a p_b, since d g^{-1} = -g^{-1} (d g) g^{-1}).
__device__ __forceinline__ void table_rhs64(const TableView& T, double r, double th, double pr, double pth,
                                            double pt, double pph, Deriv<double>& d, double& H, double& cth,
                                            double& sth)
{
    double g[5], gr[5], gt[5];
    table_metric<true, true>(T, r, th, g, gr, gt);
    const double idet = rcp64(fma(g[0], g[4], -g[1] * g[1]));
    const double Gtt = g[4] * idet, Gtp = -g[1] * idet, Gpp = g[0] * idet;
    const double Grr = rcp64(g[2]), Ghh = rcp64(g[3]);
    d.t = fma(Gtt, pt, Gtp * pph);
    d.ph = fma(Gtp, pt, Gpp * pph);
    d.r = Grr * pr;
    d.th = Ghh * pth;
    d.pr = 0.5 * (gr[0] * d.t * d.t + 2.0 * gr[1] * d.t * d.ph + gr[2] * d.r * d.r + gr[3] * d.th * d.th +
                  gr[4] * d.ph * d.ph);
    d.pth = 0.5 * (gt[0] * d.t * d.t + 2.0 * gt[1] * d.t * d.ph + gt[2] * d.r * d.r + gt[3] * d.th * d.th +
                   gt[4] * d.ph * d.ph);
    H = 0.5 * (d.t * pt + d.ph * pph + d.r * pr + d.th * pth);
    sincos64(th, &sth, &cth);
}

}  // namespace tartarus
