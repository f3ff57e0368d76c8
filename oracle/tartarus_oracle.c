/*
 * tartarus_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for
 * backward ray tracing of null geodesics through Kerr spacetime.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header, table or constant generator with the
 * HIP path.
 *
 * What it follows (TARTARUS, Bambague & Larranaga):
 *   - Sec. 2.1, Eqs. (1)-(3): H = 1/2 g^{mu nu} p_mu p_nu and Hamilton's
 *     equations on the 8-D state q = [t, r, theta, phi, p_t, p_r, p_theta, p_phi].
 *   - Sec. 2.2, Eqs. (4)-(10): celestial coordinates -> local momentum ->
 *     ZAMO tetrad projection at the observer (t=0, r=D, theta=iota, phi=0).
 *   - Sec. 2.3, Eqs. (11)-(12): Page-Thorne flux and the cubic roots.
 *   - Sec. 2.4, Eqs. (13)-(16): redshift g and I_obs = g^4 I_em.
 *   - Sec. 3.2: Dormand-Prince, Cash-Karp and Fehlberg 5(4) pairs with local
 *     extrapolation and embedded error estimate; Gragg-Bulirsch-Stoer
 *     modified-midpoint extrapolation with error-controlled macro-steps;
 *     a fixed-step symmetric (generalized Stormer-)Verlet scheme;
 *     horizon / escape / equatorial-disk events
 *     refined by bisection on the step's cubic Hermite interpolant to about
 *     1e-12 in the affine parameter (for the extrapolation, whose macro-steps
 *     are too long for a cubic, by bisection on its own solution over the
 *     partial step).
 *   - Sec. 4.1, Eq. (17): the constraint residual |H| at every accepted step.
 *
 * Readings where the paper is silent (kept identical on the HIP side, each
 * written out where it is used): the tetrad's e_(t)^phi component, the pixel
 * grid, the sign flip used for backward tracing, the step-size controller,
 * the failure limits, the event rules and the bisection count, the
 * rounding floor of the error estimates, the extrapolation's substep
 * sequence, column count, error estimate, power-of-two step factor and event
 * location, the
 * Verlet scheme for a non-separable Hamiltonian and its step, the emitter's
 * Keplerian angular velocity, the a = 0 guard in the flux sum.
 *
 * The metric derivatives come from hyper-dual arithmetic (exact first and
 * mixed second derivatives of the closed-form covariant components), and the
 * right-hand side is Eq. (3) literally, with the derivative of the inverse
 * metric formed as -g^{-1} (d g) g^{-1}.
 */
#include "tartarus_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NSTATE 8
enum { T_ = 0, R_ = 1, TH_ = 2, PH_ = 3, PT_ = 4, PR_ = 5, PTH_ = 6, PPH_ = 7 };
/* order of the five stored metric components (Eq. (6)) */
enum { G_TT = 0, G_TP = 1, G_RR = 2, G_HH = 3, G_PP = 4 };

/* ------------------------------------------------------------------ */
/* Hyper-dual numbers: value, d/dr, d/dtheta, d2/(dr dtheta).          */
/* ------------------------------------------------------------------ */
typedef struct { double v, r, t, rt; } hd;

static hd hd_c(double c) { hd z = {c, 0.0, 0.0, 0.0}; return z; }
static hd hd_add(hd x, hd y) { hd z = {x.v + y.v, x.r + y.r, x.t + y.t, x.rt + y.rt}; return z; }
static hd hd_sub(hd x, hd y) { hd z = {x.v - y.v, x.r - y.r, x.t - y.t, x.rt - y.rt}; return z; }
static hd hd_scale(hd x, double c) { hd z = {c * x.v, c * x.r, c * x.t, c * x.rt}; return z; }
static hd hd_mul(hd x, hd y)
{
    hd z;
    z.v = x.v * y.v;
    z.r = x.r * y.v + x.v * y.r;
    z.t = x.t * y.v + x.v * y.t;
    z.rt = x.rt * y.v + x.r * y.t + x.t * y.r + x.v * y.rt;
    return z;
}
/* apply a scalar function with derivatives f0, f1, f2 at x.v (chain rule) */
static hd hd_fn(hd x, double f0, double f1, double f2)
{
    hd z;
    z.v = f0;
    z.r = f1 * x.r;
    z.t = f1 * x.t;
    z.rt = f1 * x.rt + f2 * x.r * x.t;
    return z;
}
static hd hd_inv(hd x) { double i = 1.0 / x.v; return hd_fn(x, i, -i * i, 2.0 * i * i * i); }
static hd hd_div(hd x, hd y) { return hd_mul(x, hd_inv(y)); }
static hd hd_sin(hd x) { return hd_fn(x, sin(x.v), cos(x.v), -sin(x.v)); }
static hd hd_cos(hd x) { return hd_fn(x, cos(x.v), -sin(x.v), -cos(x.v)); }

/* ------------------------------------------------------------------ */
/* Kerr metric in Boyer-Lindquist coordinates (textbook closed form;    */
/* the paper's kerr.py module, Sec. 3.1, in the form of Eq. (6)).       */
/* Writes the five components g_tt, g_tphi, g_rr, g_thth, g_phph, and   */
/* g_tphi / sin^2, g_phph / sin^2 (the smooth forms that are tabulated). */
/* ------------------------------------------------------------------ */
static void kerr_components_hd(double a, double r, double th, hd g[5], hd tg[5])
{
    hd R = {r, 1.0, 0.0, 0.0};
    hd TH = {th, 0.0, 1.0, 0.0};
    hd s = hd_sin(TH), c = hd_cos(TH);
    hd s2 = hd_mul(s, s), c2 = hd_mul(c, c);
    hd r2 = hd_mul(R, R);
    hd a2 = hd_c(a * a);
    hd Sigma = hd_add(r2, hd_mul(a2, c2));
    hd Delta = hd_add(hd_sub(r2, hd_scale(R, 2.0)), a2);
    hd two_r_over_S = hd_div(hd_scale(R, 2.0), Sigma);

    hd gtt = hd_sub(two_r_over_S, hd_c(1.0));                 /* -(1 - 2r/Sigma)          */
    hd ttp = hd_scale(two_r_over_S, -a);                      /* g_tphi / s^2 = -2ar/Sigma */
    hd grr = hd_div(Sigma, Delta);
    hd ghh = Sigma;
    hd tpp = hd_add(hd_add(r2, a2), hd_mul(hd_scale(two_r_over_S, a * a), s2)); /* g_phph / s^2 */

    tg[G_TT] = gtt; tg[G_TP] = ttp; tg[G_RR] = grr; tg[G_HH] = ghh; tg[G_PP] = tpp;
    g[G_TT] = gtt; g[G_TP] = hd_mul(ttp, s2); g[G_RR] = grr; g[G_HH] = ghh; g[G_PP] = hd_mul(tpp, s2);
}

/* Covariant components (value, d_r, d_theta) of analytic Kerr. */
static void kerr_metric(double a, double r, double th, double g[5], double gr[5], double gth[5])
{
    hd G[5], T[5];
    kerr_components_hd(a, r, th, G, T);
    for (int i = 0; i < 5; ++i) { g[i] = G[i].v; gr[i] = G[i].r; gth[i] = G[i].t; }
}

/* ------------------------------------------------------------------ */
/* Tabulated metric: table[comp][k][l][4] = (f, df/dr, df/dth, d2f/drdth)  */
/* of the smooth components (g_tt, g_tphi/s^2, g_rr, g_thth, g_phph/s^2)  */
/* at r_k = exp(u_k), u_k = ln r_min + k du, theta_l = l dth.             */
/* Interpolated by a tensor-product cubic Hermite patch in (u = ln r, th). */
/* ------------------------------------------------------------------ */
void or_build_kerr_table(double a, int nr, int nth, double r_min, double r_max, double* table)
{
    double u0 = log(r_min), du = (log(r_max) - log(r_min)) / (double)(nr - 1);
    double dth = M_PI / (double)(nth - 1);
    for (int k = 0; k < nr; ++k) {
        double r = exp(u0 + (double)k * du);
        for (int l = 0; l < nth; ++l) {
            double th = (double)l * dth;
            hd G[5], T[5];
            kerr_components_hd(a, r, th, G, T);
            for (int c = 0; c < 5; ++c) {
                double* e = table + (((size_t)c * nr + k) * nth + l) * 4;
                e[0] = T[c].v; e[1] = T[c].r; e[2] = T[c].t; e[3] = T[c].rt;
            }
        }
    }
}

/* 1-D cubic Hermite basis: value weights P0, P1 and slope weights M0, M1, plus d/dx. */
static void hermite_basis(double x, double P[2], double M[2], double dP[2], double dM[2])
{
    double x2 = x * x, x3 = x2 * x;
    P[0] = 2.0 * x3 - 3.0 * x2 + 1.0;  dP[0] = 6.0 * x2 - 6.0 * x;
    P[1] = -2.0 * x3 + 3.0 * x2;       dP[1] = -6.0 * x2 + 6.0 * x;
    M[0] = x3 - 2.0 * x2 + x;          dM[0] = 3.0 * x2 - 4.0 * x + 1.0;
    M[1] = x3 - x2;                    dM[1] = 3.0 * x2 - 2.0 * x;
}

/* Interpolated smooth component c at (r, th): value, d/dr, d/dth. */
static void table_component(const or_metric* m, int c, double r, double th, double* f, double* fr, double* fth)
{
    int nr = m->nr, nth = m->nth;
    double u0 = log(m->r_min), du = (log(m->r_max) - log(m->r_min)) / (double)(nr - 1);
    double dth = M_PI / (double)(nth - 1);
    double u = log(r);
    int k = (int)floor((u - u0) / du);
    if (k < 0) k = 0;
    if (k > nr - 2) k = nr - 2;
    int l = (int)floor(th / dth);
    if (l < 0) l = 0;
    if (l > nth - 2) l = nth - 2;
    double x = (u - (u0 + (double)k * du)) / du;
    double y = (th - (double)l * dth) / dth;
    double Px[2], Mx[2], dPx[2], dMx[2], Py[2], My[2], dPy[2], dMy[2];
    hermite_basis(x, Px, Mx, dPx, dMx);
    hermite_basis(y, Py, My, dPy, dMy);
    double v = 0.0, vx = 0.0, vy = 0.0;
    for (int i = 0; i < 2; ++i) {
        double rk = exp(u0 + (double)(k + i) * du);
        for (int j = 0; j < 2; ++j) {
            const double* e = m->table + (((size_t)c * nr + (k + i)) * nth + (l + j)) * 4;
            double F = e[0];
            double Fu = rk * e[1] * du;          /* df/du = r df/dr, scaled to the cell */
            double Ft = e[2] * dth;
            double Fut = rk * e[3] * du * dth;
            v  += F * Px[i] * Py[j]  + Fu * Mx[i] * Py[j]  + Ft * Px[i] * My[j]  + Fut * Mx[i] * My[j];
            vx += F * dPx[i] * Py[j] + Fu * dMx[i] * Py[j] + Ft * dPx[i] * My[j] + Fut * dMx[i] * My[j];
            vy += F * Px[i] * dPy[j] + Fu * Mx[i] * dPy[j] + Ft * Px[i] * dMy[j] + Fut * Mx[i] * dMy[j];
        }
    }
    *f = v;
    *fr = vx / du / r;    /* d/dr = (1/r) d/du */
    *fth = vy / dth;
}

static void table_metric(const or_metric* m, double r, double th, double g[5], double gr[5], double gth[5])
{
    double f[5], fr[5], ft[5];
    for (int c = 0; c < 5; ++c) table_component(m, c, r, th, &f[c], &fr[c], &ft[c]);
    double s = sin(th), co = cos(th), s2 = s * s, ds2 = 2.0 * s * co;
    for (int c = 0; c < 5; ++c) { g[c] = f[c]; gr[c] = fr[c]; gth[c] = ft[c]; }
    /* restore the sin^2 factor of the two azimuthal components */
    g[G_TP] = s2 * f[G_TP]; gr[G_TP] = s2 * fr[G_TP]; gth[G_TP] = ds2 * f[G_TP] + s2 * ft[G_TP];
    g[G_PP] = s2 * f[G_PP]; gr[G_PP] = s2 * fr[G_PP]; gth[G_PP] = ds2 * f[G_PP] + s2 * ft[G_PP];
}

static void metric_eval(const or_metric* m, double r, double th, double g[5], double gr[5], double gth[5])
{
    if (m->kind == 1) table_metric(m, r, th, g, gr, gth);
    else kerr_metric(m->a, r, th, g, gr, gth);
}

/* 4x4 matrix of the five components (indices t, r, theta, phi). */
static void full4(const double g[5], double G[4][4])
{
    memset(G, 0, sizeof(double) * 16);
    G[0][0] = g[G_TT]; G[0][3] = G[3][0] = g[G_TP];
    G[1][1] = g[G_RR]; G[2][2] = g[G_HH]; G[3][3] = g[G_PP];
}

/* Inverse of a metric of the form of Eq. (6): 2x2 (t,phi) block plus diagonal. */
static void inverse4(const double g[5], double Gi[4][4])
{
    memset(Gi, 0, sizeof(double) * 16);
    double det = g[G_TT] * g[G_PP] - g[G_TP] * g[G_TP];
    Gi[0][0] = g[G_PP] / det;
    Gi[0][3] = Gi[3][0] = -g[G_TP] / det;
    Gi[3][3] = g[G_TT] / det;
    Gi[1][1] = 1.0 / g[G_RR];
    Gi[2][2] = 1.0 / g[G_HH];
}

/* Eq. (1): H = 1/2 g^{mu nu} p_mu p_nu. */
static double hamiltonian_m(const or_metric* m, const double* q)
{
    double g[5], gr[5], gt[5], Gi[4][4];
    metric_eval(m, q[R_], q[TH_], g, gr, gt);
    inverse4(g, Gi);
    const double* p = q + 4;
    double H = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) H += Gi[i][j] * p[i] * p[j];
    return 0.5 * H;
}

/* Eqs. (2)-(3): dx^mu/dl = g^{mu nu} p_nu, dp_mu/dl = -1/2 (d_mu g^{ab}) p_a p_b,
 * with d_mu g^{-1} = -g^{-1} (d_mu g) g^{-1}; t and phi are cyclic. */
static void rhs_m(const or_metric* m, const double* q, double* dq)
{
    double g[5], gr[5], gt[5], Gi[4][4];
    metric_eval(m, q[R_], q[TH_], g, gr, gt);
    inverse4(g, Gi);
    const double* p = q + 4;
    for (int mu = 0; mu < 4; ++mu) {
        double s = 0.0;
        for (int nu = 0; nu < 4; ++nu) s += Gi[mu][nu] * p[nu];
        dq[mu] = s;
    }
    dq[PT_] = 0.0;
    dq[PPH_] = 0.0;
    for (int which = 0; which < 2; ++which) {
        double dG[4][4], tmp[4][4], dGi[4][4];
        full4(which == 0 ? gr : gt, dG);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += dG[i][k] * Gi[k][j];
                tmp[i][j] = s;
            }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += Gi[i][k] * tmp[k][j];
                dGi[i][j] = -s;
            }
        double acc = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) acc += dGi[i][j] * p[i] * p[j];
        dq[which == 0 ? PR_ : PTH_] = -0.5 * acc;
    }
}

/* ------------------------------------------------------------------ */
/* Radii of the hole (textbook Kerr; the paper names EH and ISCO as     */
/* metric-supplied boundaries, Sec. 3.1).                               */
/* ------------------------------------------------------------------ */
double or_horizon(double a) { return 1.0 + sqrt(1.0 - a * a); }

/* Prograde innermost stable circular orbit (Bardeen, Press & Teukolsky 1972). */
double or_isco(double a)
{
    double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    double z2 = sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

/* ------------------------------------------------------------------ */
/* Emitter model (Secs. 2.3-2.4).                                       */
/* ------------------------------------------------------------------ */

/* Eq. (11) with roots from Eq. (12); zero outside the disk's radial range.
 * x_2 = 0 when a = 0 makes its term 0/0; its limit is 0, so the term is
 * dropped when |x_2| < 1e-12. */
double or_nt_flux(double a, double r_in, double r_out, double r)
{
    if (!(r >= r_in && r <= r_out)) return 0.0;
    double x = sqrt(r), x0 = sqrt(r_in);
    double ac = acos(a);
    double xi[3];
    xi[0] = 2.0 * cos((ac - M_PI) / 3.0);
    xi[1] = 2.0 * cos((ac + M_PI) / 3.0);
    xi[2] = -2.0 * cos(ac / 3.0);
    double bracket = x - x0 - 1.5 * a * log(x / x0);
    for (int i = 0; i < 3; ++i) {
        if (fabs(xi[i]) < 1e-12) continue;
        double prod = 1.0;
        for (int j = 0; j < 3; ++j)
            if (j != i) prod *= (xi[i] - xi[j]);
        double coef = 3.0 * (xi[i] - a) * (xi[i] - a) / (xi[i] * prod);
        bracket -= coef * log((x - xi[i]) / (x0 - xi[i]));
    }
    return 3.0 / (2.0 * x * x * x * x * (x * x * x - 3.0 * x + 2.0 * a)) * bracket;
}

/* Eq. (15): g = p_t / (u^t (p_t + Omega p_phi)), with u^t from Eq. (14) at
 * theta = pi/2 and the prograde Keplerian Omega = 1/(r^{3/2} + a). */
double or_redshift(double a, double r, double p_t, double p_phi)
{
    /* covariant components exactly in the equatorial plane: sin = 1, cos = 0 */
    double g[5];
    double Sigma = r * r;
    g[G_TT] = -(1.0 - 2.0 * r / Sigma);
    g[G_TP] = -2.0 * a * r / Sigma;
    g[G_PP] = r * r + a * a + 2.0 * a * a * r / Sigma;
    double Om = 1.0 / (pow(r, 1.5) + a);
    double ut = 1.0 / sqrt(-g[G_TT] - 2.0 * Om * g[G_TP] - Om * Om * g[G_PP]);
    return p_t / (ut * (p_t + Om * p_phi));
}

/* ------------------------------------------------------------------ */
/* Camera and initial conditions (Sec. 2.2, Eqs. (4)-(10)).             */
/* ------------------------------------------------------------------ */

/* Pixel grid reading: inclusive linspace over each window, pixel (i, j) at
 * index j*nx + i.  Backward-tracing reading: Eq. (4) describes the photon
 * arriving at the observer (p^(r) > 0); the stored momenta are negated so
 * that integrating with increasing lambda retraces it toward the hole. */
void or_initial_state(const or_metric* m, const or_camera* cam, int i, int j, double* q)
{
    double D = cam->r_obs, iota = cam->theta_obs;
    double al = cam->nx > 1 ? cam->alpha_min + (double)i * (cam->alpha_max - cam->alpha_min) / (double)(cam->nx - 1)
                            : cam->alpha_min;
    double be = cam->ny > 1 ? cam->beta_min + (double)j * (cam->beta_max - cam->beta_min) / (double)(cam->ny - 1)
                            : cam->beta_min;
    double g[5], gr[5], gt[5];
    metric_eval(m, D, iota, g, gr, gt);
    double omega = -g[G_TP] / g[G_PP];                          /* frame dragging       */
    double e_tt = 1.0 / sqrt(-g[G_TT] + omega * omega * g[G_PP]); /* Eq. (7)            */
    double e_tp = omega * e_tt;                                  /* ZAMO e_(t)^phi      */
    double e_rr = 1.0 / sqrt(g[G_RR]);                           /* Eq. (8)            */
    double e_hh = 1.0 / sqrt(g[G_HH]);                           /* Eq. (9)            */
    double e_pp = 1.0 / sqrt(g[G_PP]);                           /* Eq. (10)           */
    /* Eq. (4) */
    double pl_t = 1.0;
    double pl_r = sqrt(1.0 - (al * al + be * be) / (D * D));
    double pl_h = be / D;
    double pl_p = -al / D;
    /* Eq. (5) */
    double pu_t = e_tt * pl_t;
    double pu_r = e_rr * pl_r;
    double pu_h = e_hh * pl_h;
    double pu_p = e_tp * pl_t + e_pp * pl_p;
    /* lower the index with Eq. (6) */
    double p_t = g[G_TT] * pu_t + g[G_TP] * pu_p;
    double p_r = g[G_RR] * pu_r;
    double p_h = g[G_HH] * pu_h;
    double p_p = g[G_TP] * pu_t + g[G_PP] * pu_p;
    q[T_] = 0.0; q[R_] = D; q[TH_] = iota; q[PH_] = 0.0;
    q[PT_] = -p_t; q[PR_] = -p_r; q[PTH_] = -p_h; q[PPH_] = -p_p;
}

/* ------------------------------------------------------------------ */
/* Embedded Runge-Kutta 5(4) pairs (Sec. 3.2): Dormand & Prince (1980),  */
/* Cash & Karp (1990), Fehlberg (1969).  The fifth-order weights         */
/* propagate the solution, the embedded fourth-order weights give the    */
/* error estimate.  Each pair is stored as seven stages: the six of the  */
/* method and a seventh evaluation f(y5) at the new point (the first     */
/* stage of Dormand-Prince's next step; for the two six-stage pairs the  */
/* derivative the next step starts from and the event interpolant uses). */
/* Row 6 of A is therefore b, and only Dormand-Prince's embedded weights */
/* give the seventh evaluation a nonzero weight.                         */
/* ------------------------------------------------------------------ */
static const double RK_C[3][7] = {
    {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0},
    {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0, 1.0},
    {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0, 1.0}};
static const double RK_A[3][7][6] = {
    {{0, 0, 0, 0, 0, 0},
     {1.0 / 5.0, 0, 0, 0, 0, 0},
     {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
     {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
     {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
     {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
     {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}},
    {{0, 0, 0, 0, 0, 0},
     {1.0 / 5.0, 0, 0, 0, 0, 0},
     {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
     {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0, 0},
     {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0, 0},
     {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0, 0},
     {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0}},
    {{0, 0, 0, 0, 0, 0},
     {1.0 / 4.0, 0, 0, 0, 0, 0},
     {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0, 0},
     {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0, 0},
     {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0, 0},
     {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0, 0},
     {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0}}};
/* fifth-order weights (propagate: local extrapolation) */
static const double RK_B[3][7] = {
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0},
    {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0, 0.0},
    {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0, 0.0}};
/* embedded fourth-order weights (error estimate) */
static const double RK_BS[3][7] = {
    {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0},
    {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0, 277.0 / 14336.0, 1.0 / 4.0, 0.0},
    {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0, 0.0}};

void or_rk_tableau(int method, double* c, double* a, double* b, double* bstar)
{
    for (int i = 0; i < 7; ++i) {
        c[i] = RK_C[method][i];
        b[i] = RK_B[method][i];
        bstar[i] = RK_BS[method][i];
        for (int j = 0; j < 6; ++j) a[i * 6 + j] = RK_A[method][i][j];
    }
}

void or_dp45_tableau(double* c, double* a, double* b, double* bstar) { or_rk_tableau(0, c, a, b, bstar); }

typedef void (*rhs_fn)(void* ctx, const double* y, double* dy);

/* Rounding floor of an embedded pair's error estimate (a reading: the paper
 * gives no controller).  The estimate h sum_j (b_j - b*_j) k_j of a component
 * rounds to a few ulps of h |b - b*|_1 max(|k_n|, |k_n+1|); far from the hole
 * the first steps' estimates are that rounding alone (a cancellation of ~1e9
 * in the angular components), and a step factor taken from them differs
 * between two correct FP64 evaluations by ~1e-7, enough for a later estimate
 * to fall on the other side of 1.  A component whose estimate is at most
 * RK_FLOOR_ULPS of that scale, capped at RK_FLOOR_TOL of its tolerance scale,
 * is taken as zero.  (The extrapolation has its own floor, GBS_FLOOR_*.) */
#define RK_FLOOR_ULPS 262144.0       /* 2^18 */
#define RK_FLOOR_TOL 0.01

/* One attempted step of size h from y with k1 = f(y): writes the fifth-order
 * solution, the error vector (b - b*) h k with the rounding floor applied for
 * the tolerance (atol, rtol) (rtol = atol = 0: no floor), and k7 = f(y5). */
static void rk_attempt(int method, int n, rhs_fn f, void* ctx, const double* y, const double* k1, double h,
                       double atol, double rtol, double* y5, double* err, double* k7)
{
    const double(*A)[6] = RK_A[method];
    const double* B = RK_B[method];
    const double* BS = RK_BS[method];
    double k[7][NSTATE > 16 ? NSTATE : 16];
    double Y[16];
    for (int d = 0; d < n; ++d) k[0][d] = k1[d];
    for (int s = 1; s < 6; ++s) {
        for (int d = 0; d < n; ++d) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += A[s][j] * k[j][d];
            Y[d] = y[d] + h * acc;
        }
        f(ctx, Y, k[s]);
    }
    for (int d = 0; d < n; ++d) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += B[j] * k[j][d];
        y5[d] = y[d] + h * acc;
    }
    f(ctx, y5, k[6]);
    double enorm1 = 0.0;
    for (int j = 0; j < 7; ++j) enorm1 += fabs(B[j] - BS[j]);
    for (int d = 0; d < n; ++d) {
        double acc = 0.0;
        for (int j = 0; j < 7; ++j) acc += (B[j] - BS[j]) * k[j][d];
        err[d] = h * acc;
        k7[d] = k[6][d];
        double floor_ = RK_FLOOR_ULPS * DBL_EPSILON * enorm1 * fabs(h) * fmax(fabs(k[0][d]), fabs(k[6][d]));
        double cap = RK_FLOOR_TOL * (atol + rtol * fmax(fabs(y[d]), fabs(y5[d])));
        if (cap < floor_) floor_ = cap;
        if (fabs(err[d]) <= floor_) err[d] = 0.0;
    }
}

/* Test hook: fixed-step steps of a 5(4) pair on a user ODE (y' = f(y), n <= 16). */
typedef void (*or_user_rhs)(const double* y, double* dy, int n);
struct user_ctx { or_user_rhs f; int n; };
static void user_tramp(void* ctx, const double* y, double* dy)
{
    struct user_ctx* u = (struct user_ctx*)ctx;
    u->f(y, dy, u->n);
}
void or_rk_fixed(int method, int n, or_user_rhs f, double* y, double h, int nsteps, double* last_err)
{
    struct user_ctx u = {f, n};
    double k1[16], y5[16], e[16], k7[16];
    f(y, k1, n);
    for (int s = 0; s < nsteps; ++s) {
        rk_attempt(method, n, user_tramp, &u, y, k1, h, 0.0, 0.0, y5, e, k7);
        for (int d = 0; d < n; ++d) { y[d] = y5[d]; k1[d] = k7[d]; last_err[d] = e[d]; }
    }
}

void or_dp45_fixed(int n, or_user_rhs f, double* y, double h, int nsteps, double* last_err)
{
    or_rk_fixed(0, n, f, y, h, nsteps, last_err);
}

/* ------------------------------------------------------------------ */
/* Gragg-Bulirsch-Stoer extrapolation (Sec. 3.2): a macro-step of size  */
/* H is covered K times by Gragg's modified midpoint rule, the j-th time */
/* with n_j = 2j equal substeps; each result T[j][1] has an error        */
/* expansion in even powers of the substep H/n_j, and Richardson         */
/* extrapolation to zero substep in (H/n)^2 fills the tableau            */
/* (Aitken-Neville form)                                                 */
/*   T[j][k+1] = T[j][k] + (T[j][k] - T[j-1][k]) / ((n_j/n_{j-k})^2 - 1). */
/* The diagonal T[K][K] propagates the solution and the difference to    */
/* T[K][K-1] is the error estimate driving the macro-step control.       */
/* The sweeps and the tableau carry increments z - y (the extrapolation  */
/* is linear, so this is the same scheme), which keeps the rounding of   */
/* the estimate at the size of the step's change instead of the state's. */
/* ------------------------------------------------------------------ */
#define GBS_KMAX 8

static int gbs_substeps(int j) { return 2 * j; }

/* Gragg's modified midpoint rule on increments: m substeps of size hs = H/m
 * from y, where k1 = f(y):  d_0 = 0,  d_1 = hs f(y),  d_{i+1} = d_{i-1} +
 * 2 hs f(y + d_i), followed by the smoothing step (d_m + d_{m-1} + hs f(y +
 * d_m)) / 2; out = the smoothed increment. */
static void modified_midpoint(int n, rhs_fn f, void* ctx, const double* y, const double* k1, double H, int m,
                              double* out)
{
    double hs = H / (double)m;
    double dprev[16], d[16], dnext[16], z[16], dz[16];
    for (int q = 0; q < n; ++q) {
        dprev[q] = 0.0;
        d[q] = hs * k1[q];
    }
    for (int i = 1; i < m; ++i) {
        for (int q = 0; q < n; ++q) z[q] = y[q] + d[q];
        f(ctx, z, dz);
        for (int q = 0; q < n; ++q) dnext[q] = dprev[q] + 2.0 * hs * dz[q];
        for (int q = 0; q < n; ++q) { dprev[q] = d[q]; d[q] = dnext[q]; }
    }
    for (int q = 0; q < n; ++q) z[q] = y[q] + d[q];
    f(ctx, z, dz);
    for (int q = 0; q < n; ++q) out[q] = 0.5 * (dprev[q] + d[q] + hs * dz[q]);
}

/* Rounding floor of the extrapolation's error estimate (a reading: the
 * paper gives no controller).  Far from the hole the truncation error of a
 * macro-step falls below the rounding of the difference T[K][K] - T[K][K-1],
 * and a step factor taken from rounding noise differs between any two
 * correct FP64 evaluations.  A component whose estimate is at most
 * GBS_FLOOR_ULPS ulps of the largest increment of that component among the
 * sweeps, capped at GBS_FLOOR_TOL of its tolerance scale, is taken as zero;
 * the threshold sits far above the rounding noise (tens of ulps), so both
 * evaluations fall on the same side of it, and the cap keeps the tolerance's
 * meaning at tight tolerances. */
#define GBS_FLOOR_ULPS 262144.0      /* 2^18 */
#define GBS_FLOOR_TOL 0.01

/* One macro-step with K columns from y (k1 = f(y)): writes T[K][K], the error
 * vector T[K][K] - T[K][K-1] with the rounding floor applied for the
 * tolerance (atol, rtol) (rtol = atol = 0: no floor), and f(T[K][K]) (knew
 * may be NULL). */
static void gbs_attempt(int K, int n, rhs_fn f, void* ctx, const double* y, const double* k1, double H,
                        double atol, double rtol, double* ynew, double* err, double* knew)
{
    double T[GBS_KMAX][GBS_KMAX][16];
    double big[16];
    for (int d = 0; d < n; ++d) big[d] = 0.0;
    for (int j = 1; j <= K; ++j) {
        modified_midpoint(n, f, ctx, y, k1, H, gbs_substeps(j), T[j - 1][0]);
        for (int d = 0; d < n; ++d) big[d] = fmax(big[d], fabs(T[j - 1][0][d]));
        for (int k = 1; k < j; ++k) {
            double ratio = (double)gbs_substeps(j) / (double)gbs_substeps(j - k);
            double den = ratio * ratio - 1.0;
            for (int d = 0; d < n; ++d)
                T[j - 1][k][d] = T[j - 1][k - 1][d] + (T[j - 1][k - 1][d] - T[j - 2][k - 1][d]) / den;
        }
    }
    for (int d = 0; d < n; ++d) {
        ynew[d] = y[d] + T[K - 1][K - 1][d];
        double e = T[K - 1][K - 1][d] - T[K - 1][K - 2][d];
        double floor_ = GBS_FLOOR_ULPS * DBL_EPSILON * big[d];
        double cap = GBS_FLOOR_TOL * (atol + rtol * fmax(fabs(y[d]), fabs(ynew[d])));
        if (cap < floor_) floor_ = cap;
        err[d] = fabs(e) <= floor_ ? 0.0 : e;
    }
    if (knew) f(ctx, ynew, knew);
}

/* Columns of the extrapolation used to trace rays (orders 2K and 2K - 2). */
int or_gbs_columns(void) { return OR_GBS_COLUMNS; }

/* Test hook: fixed macro-steps with K columns (2 <= K <= 8) on a user ODE. */
void or_gbs_fixed(int K, int n, or_user_rhs f, double* y, double h, int nsteps, double* last_err)
{
    struct user_ctx u = {f, n};
    double k1[16], yn[16], e[16], kn[16];
    if (K < 2 || K > GBS_KMAX) return;
    f(y, k1, n);
    for (int s = 0; s < nsteps; ++s) {
        gbs_attempt(K, n, user_tramp, &u, y, k1, h, 0.0, 0.0, yn, e, kn);
        for (int d = 0; d < n; ++d) { y[d] = yn[d]; k1[d] = kn[d]; last_err[d] = e[d]; }
    }
}

/* ------------------------------------------------------------------ */
/* Verlet (Sec. 3.2): fixed step, time-reversible, symmetric.  H(x, p) = */
/* 1/2 g^{ab}(x) p_a p_b does not split into a kinetic and a potential   */
/* part, so the scheme is the symmetric generalization of Stormer-Verlet */
/* to such Hamiltonians: an implicit half step in the momenta, a         */
/* trapezoidal step in the positions, an explicit closing half step:     */
/*   p' = p - (h/2) dH/dx(x, p')                                         */
/*   x+ = x + (h/2) [dH/dp(x, p') + dH/dp(x+, p')]                       */
/*   p+ = p' - (h/2) dH/dx(x+, p')                                       */
/* (for H = T(p) + V(x) this is the classical velocity Verlet step).     */
/* The map is symplectic and symmetric, so H stays bounded.  The two     */
/* implicit stages are solved by fixed-point iteration from an explicit  */
/* predictor, to a relative change of VERLET_ITER_TOL; a stage that does */
/* not converge has (for this step) no solution near the current one,    */
/* which happens close to the horizon, where dH/dx grows like 1/Delta.   */
/* The state is [x (n/2 components), p (n/2 components)] and f returns   */
/* [dH/dp, -dH/dx].                                                      */
/* ------------------------------------------------------------------ */
#define VERLET_MAX_ITER 50
#define VERLET_ITER_TOL 1e-14

/* One step from y (fy = f(y)); returns 0 when an implicit stage does not
 * converge within VERLET_MAX_ITER iterations. */
static int verlet_step(int n, rhs_fn f, void* ctx, const double* y, const double* fy, double h, double* ynew)
{
    int d = n / 2;
    double z[16] = {0.0}, fz[16], ph[8], v0[8], xk[8];
    /* stage 1: p' = p + (h/2) [-dH/dx](x, p'), predictor p + (h/2) [-dH/dx](x, p) */
    for (int i = 0; i < d; ++i) ph[i] = y[d + i] + 0.5 * h * fy[d + i];
    int conv = 0;
    for (int it = 0; it < VERLET_MAX_ITER && !conv; ++it) {
        for (int i = 0; i < d; ++i) { z[i] = y[i]; z[d + i] = ph[i]; }
        f(ctx, z, fz);
        double dmax = 0.0, vmax = 0.0;
        int finite = 1;
        for (int i = 0; i < d; ++i) {
            double pn = y[d + i] + 0.5 * h * fz[d + i];
            finite = finite && isfinite(pn);
            dmax = fmax(dmax, fabs(pn - ph[i]));
            vmax = fmax(vmax, fabs(pn));
            ph[i] = pn;
        }
        /* (fmax ignores a NaN operand, so a non-finite iterate is excluded explicitly) */
        conv = finite && dmax <= VERLET_ITER_TOL * fmax(1.0, vmax);
    }
    if (!conv) return 0;
    /* stage 2: x+ = x + (h/2) [dH/dp(x, p') + dH/dp(x+, p')], predictor x + h dH/dp(x, p') */
    for (int i = 0; i < d; ++i) { z[i] = y[i]; z[d + i] = ph[i]; }
    f(ctx, z, fz);
    for (int i = 0; i < d; ++i) { v0[i] = fz[i]; xk[i] = y[i] + h * v0[i]; }
    conv = 0;
    for (int it = 0; it < VERLET_MAX_ITER && !conv; ++it) {
        for (int i = 0; i < d; ++i) { z[i] = xk[i]; z[d + i] = ph[i]; }
        f(ctx, z, fz);
        double dmax = 0.0, vmax = 0.0;
        int finite = 1;
        for (int i = 0; i < d; ++i) {
            double xn = y[i] + 0.5 * h * (v0[i] + fz[i]);
            finite = finite && isfinite(xn);
            dmax = fmax(dmax, fabs(xn - xk[i]));
            vmax = fmax(vmax, fabs(xn));
            xk[i] = xn;
        }
        conv = finite && dmax <= VERLET_ITER_TOL * fmax(1.0, vmax);
    }
    if (!conv) return 0;
    /* stage 3: p+ = p' + (h/2) [-dH/dx](x+, p') */
    for (int i = 0; i < d; ++i) { z[i] = xk[i]; z[d + i] = ph[i]; }
    f(ctx, z, fz);
    for (int i = 0; i < d; ++i) {
        ynew[i] = xk[i];
        ynew[d + i] = ph[i] + 0.5 * h * fz[d + i];
    }
    return 1;
}

/* Test hook: nsteps fixed Verlet steps on a Hamiltonian system y = [x, p]
 * (n even, <= 16); returns the number of steps completed. */
int or_verlet_fixed(int n, or_user_rhs f, double* y, double h, int nsteps)
{
    struct user_ctx u = {f, n};
    double fy[16], yn[16];
    for (int s = 0; s < nsteps; ++s) {
        f(y, fy, n);
        if (!verlet_step(n, user_tramp, &u, y, fy, h, yn)) return s;
        for (int d = 0; d < n; ++d) y[d] = yn[d];
    }
    return nsteps;
}

/* ------------------------------------------------------------------ */
/* Dense output and event location (Sec. 3.2).                          */
/* ------------------------------------------------------------------ */

/* Cubic Hermite interpolant of one component on [l_n, l_n + h] at s in [0,1]. */
double or_hermite(double s, double y0, double d0, double y1, double d1, double h)
{
    double s2 = s * s, s3 = s2 * s;
    double h00 = 2.0 * s3 - 3.0 * s2 + 1.0;
    double h10 = s3 - 2.0 * s2 + s;
    double h01 = -2.0 * s3 + 3.0 * s2;
    double h11 = s3 - s2;
    return h00 * y0 + h10 * h * d0 + h01 * y1 + h11 * h * d1;
}

/* Number of halvings: the smallest n >= 0 with h / 2^n <= tol (exact). */
int or_bisect_count(double h, double tol)
{
    int n = 0;
    double w = h;
    while (w > tol && n < 1100) { w *= 0.5; ++n; }
    return n;
}

enum { EV_DISK = 0, EV_HORIZON = 1, EV_ESCAPE = 2 };

typedef struct {
    const double *y0, *y1, *k1, *k7;
    double h;
    const or_metric* reint;   /* non-NULL: the extrapolation's own solution */
} step_ctx;

static void kerr_rhs_tramp(void* ctx, const double* y, double* dy);

/* Component comp of the step's solution at lambda_n + s h.  The 5(4) pairs
 * and Verlet read it off the cubic Hermite interpolant.  A macro-step of the
 * extrapolation spans up to hundreds of M, over which a cubic is accurate to
 * ~1e-3 only; there the point is one macro-step of length s h from the
 * step's start (the same sweeps and columns, without error control). */
static double interp(const step_ctx* st, int comp, double s)
{
    if (st->reint) {
        double ys[NSTATE], es[NSTATE];
        if (s == 0.0) return st->y0[comp];
        gbs_attempt(OR_GBS_COLUMNS, NSTATE, kerr_rhs_tramp, (void*)st->reint, st->y0, st->k1, s * st->h, 0.0, 0.0,
                    ys, es, NULL);
        return ys[comp];
    }
    return or_hermite(s, st->y0[comp], st->k1[comp], st->y1[comp], st->k7[comp], st->h);
}

/* Event functions C(lambda, q) of Sec. 3.2 on the interpolant. */
static double event_value(const step_ctx* st, int ev, double s, double r_stop, double r_esc)
{
    if (ev == EV_HORIZON) return interp(st, R_, s) - r_stop;
    if (ev == EV_ESCAPE) return interp(st, R_, s) - r_esc;
    return cos(interp(st, TH_, s));
}

/* Bisection on the sign of the event function: the half that keeps the
 * start's strict sign becomes the new lower end; the root is the midpoint of
 * the final bracket. */
static double locate(const step_ctx* st, int ev, double start_val, double r_stop, double r_esc, double tol)
{
    int n = or_bisect_count(st->h, tol);
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < n; ++it) {
        double mid = 0.5 * (lo + hi);
        double v = event_value(st, ev, mid, r_stop, r_esc);
        int same = start_val > 0.0 ? (v > 0.0) : (v < 0.0);
        if (same) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------ */
/* One ray.                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    int cls, n_hits, n_cross, n_accept, n_reject;
    double final_rtp[3], h_drift, h_gate, intensity;
    double hit_r[3], hit_g[3], hit_flux[3], hit_lambda[3];
    int hit_order[3];
} ray_result;

static void kerr_rhs_tramp(void* ctx, const double* y, double* dy) { rhs_m((const or_metric*)ctx, y, dy); }

static int all_finite(const double* y)
{
    for (int d = 0; d < NSTATE; ++d)
        if (!isfinite(y[d])) return 0;
    return 1;
}

/* The largest power of two not above x (x > 0, finite): the extrapolation's
 * step factor (a reading, with its rounding floor: steps stay h0 * 2^k, so
 * two correct FP64 evaluations, whose error estimates differ by rounding,
 * take the same step sizes unless an estimate lies within rounding of a
 * power-of-two boundary of the factor or of the acceptance threshold). */
static double pow2_floor(double x)
{
    int e;
    frexp(x, &e);
    return ldexp(1.0, e - 1);
}

/* Integrate one ray from the initial state y0 with first step h0.  When rec
 * is non-NULL the accepted states (the initial one first) are recorded, up to
 * rec_cap of them, with their affine parameters. */
static void trace_from(const or_metric* m, const double* y0, double h0, const or_disk* disk,
                       const or_solver* sv, ray_result* out, double* rec, double* rec_l, int rec_cap,
                       int* rec_n)
{
    memset(out, 0, sizeof(*out));
    double a = m->a;
    double rp = or_horizon(a);
    double r_stop = sv->horizon_factor * rp;
    if (m->kind == 1 && m->r_min > r_stop) r_stop = m->r_min;   /* table's inner edge */
    double r_esc = sv->r_escape;
    double r_gate = 1.5 * rp;
    int max_hits = disk ? disk->max_hits : 0;
    if (max_hits > OR_MAX_HITS) max_hits = OR_MAX_HITS;
    int opaque = disk && disk->opaque && max_hits > 0;
    int intrinsic = disk && disk->shading == OR_SHADE_INTRINSIC;
    double r_in = 0.0, r_out = 0.0;
    if (max_hits > 0) {
        r_in = disk->r_in > 0.0 ? disk->r_in : or_isco(a);
        r_out = disk->r_out;
    }

    double y[NSTATE], k1[NSTATE], y5[NSTATE], e[NSTATE], k7[NSTATE];
    memcpy(y, y0, sizeof(y));
    rhs_m(m, y, k1);
    double lambda = 0.0;
    double h = h0;
    int rejected_prev = 0;
    int nrec = 0;
    if (rec && nrec < rec_cap) { memcpy(rec, y, sizeof(y)); rec_l[0] = 0.0; nrec = 1; }

    /* controller exponent -1/(p+1) with p the order of the error estimate:
     * 4 for the Runge-Kutta pairs, 2K - 2 for the extrapolation */
    double expo = sv->method == OR_METHOD_GBS ? -1.0 / (2.0 * OR_GBS_COLUMNS - 1.0) : -0.2;
    double H0 = fabs(hamiltonian_m(m, y));
    out->h_drift = H0;
    out->h_gate = y[R_] >= r_gate ? H0 : 0.0;
    out->cls = OR_FAILED;

    for (;;) {
        if ((int64_t)out->n_accept + out->n_reject >= sv->max_steps) break;
        double err;
        if (sv->method == OR_METHOD_VERLET) {
            /* fixed step, no error control: every converged step is taken */
            if (!verlet_step(NSTATE, kerr_rhs_tramp, (void*)m, y, k1, h, y5)) break;
            rhs_m(m, y5, k7);
            err = 0.0;
        } else {
            if (sv->method == OR_METHOD_GBS)
                gbs_attempt(OR_GBS_COLUMNS, NSTATE, kerr_rhs_tramp, (void*)m, y, k1, h, sv->atol, sv->rtol, y5, e,
                            k7);
            else
                rk_attempt(sv->method, NSTATE, kerr_rhs_tramp, (void*)m, y, k1, h, sv->atol, sv->rtol, y5, e, k7);
            /* RMS error norm over all eight components */
            double acc = 0.0;
            for (int d = 0; d < NSTATE; ++d) {
                double sc = sv->atol + sv->rtol * fmax(fabs(y[d]), fabs(y5[d]));
                double z = e[d] / sc;
                acc += z * z;
            }
            err = sqrt(acc / (double)NSTATE);
        }
        if (!(err <= 1.0)) {
            /* rejected (a NaN or infinite error also lands here) */
            out->n_reject++;
            double fac = isnan(err) ? 0.2 : fmax(0.2, 0.9 * pow(err, expo));
            if (sv->method == OR_METHOD_GBS) fac = pow2_floor(fac);
            h *= fac;
            rejected_prev = 1;
            if (h < 1e-14 * fmax(1.0, fabs(lambda))) break;
            continue;
        }
        out->n_accept++;
        if (!all_finite(y5)) break;

        /* events on the accepted step [lambda, lambda + h] */
        step_ctx st = {y, y5, k1, k7, h, sv->method == OR_METHOD_GBS ? m : NULL};
        double ev_s[3];
        int ev_kind[3], nev = 0;
        double ch0 = y[R_] - r_stop, ch1 = y5[R_] - r_stop;
        if (ch0 > 0.0 && ch1 <= 0.0) {
            ev_s[nev] = locate(&st, EV_HORIZON, ch0, r_stop, r_esc, sv->event_tol);
            ev_kind[nev++] = EV_HORIZON;
        }
        double ce0 = y[R_] - r_esc, ce1 = y5[R_] - r_esc;
        if (ce0 < 0.0 && ce1 >= 0.0) {
            ev_s[nev] = locate(&st, EV_ESCAPE, ce0, r_stop, r_esc, sv->event_tol);
            ev_kind[nev++] = EV_ESCAPE;
        }
        if (max_hits > 0) {
            double c0 = cos(y[TH_]), c1 = cos(y5[TH_]);
            if ((c0 > 0.0 && c1 <= 0.0) || (c0 < 0.0 && c1 >= 0.0)) {
                ev_s[nev] = locate(&st, EV_DISK, c0, r_stop, r_esc, sv->event_tol);
                ev_kind[nev++] = EV_DISK;
            }
        }
        /* root order; on a tie the disk crossing comes first */
        for (int p = 1; p < nev; ++p)
            for (int q = p; q > 0; --q) {
                int swap = ev_s[q] < ev_s[q - 1] || (ev_s[q] == ev_s[q - 1] && ev_kind[q] == EV_DISK);
                if (!swap) break;
                double ts = ev_s[q]; ev_s[q] = ev_s[q - 1]; ev_s[q - 1] = ts;
                int tk = ev_kind[q]; ev_kind[q] = ev_kind[q - 1]; ev_kind[q - 1] = tk;
            }
        int terminal = -1;
        double term_s = 0.0;
        for (int p = 0; p < nev; ++p) {
            double s = ev_s[p];
            if (ev_kind[p] == EV_DISK) {
                out->n_cross++;
                double rr = interp(&st, R_, s);
                if (rr >= r_in && rr <= r_out && out->n_hits < max_hits) {
                    int k = out->n_hits++;
                    double g = or_redshift(a, rr, y[PT_], y[PPH_]);
                    double F = or_nt_flux(a, r_in, r_out, rr);
                    double g2 = g * g;
                    out->hit_r[k] = rr;
                    out->hit_g[k] = g;
                    /* Eq. (16); the intrinsic map drops the shift (Fig. KerrUHD b) */
                    out->hit_flux[k] = intrinsic ? F : g2 * g2 * F;
                    out->hit_lambda[k] = lambda + s * h;
                    out->hit_order[k] = out->n_cross;
                    out->intensity += out->hit_flux[k];
                    if (opaque) {
                        /* optically thick disk (Sec. 2.3): the ray ends on it */
                        terminal = EV_DISK;
                        term_s = s;
                        break;
                    }
                }
            } else {
                terminal = ev_kind[p];
                term_s = s;
                break;
            }
        }

        /* constraint residual, Eq. (17), at the accepted state */
        double Hn = fabs(hamiltonian_m(m, y5));
        if (Hn > out->h_drift) out->h_drift = Hn;
        if (y5[R_] >= r_gate && Hn > out->h_gate) out->h_gate = Hn;

        if (rec && nrec < rec_cap) {
            memcpy(rec + (size_t)nrec * NSTATE, y5, sizeof(y5));
            rec_l[nrec] = lambda + h;
            ++nrec;
        }
        if (terminal >= 0) {
            out->cls = terminal == EV_HORIZON ? OR_CAPTURED : terminal == EV_ESCAPE ? OR_ESCAPED : OR_ON_DISK;
            out->final_rtp[0] = interp(&st, R_, term_s);
            out->final_rtp[1] = interp(&st, TH_, term_s);
            out->final_rtp[2] = interp(&st, PH_, term_s);
            if (rec_n) *rec_n = nrec;
            return;
        }

        /* elementary controller: safety 0.9, factor in [0.2, 10], no growth
         * on the step right after a rejection */
        double fmax_ = rejected_prev ? 1.0 : 10.0;
        double fac = err == 0.0 ? fmax_ : fmin(fmax_, fmax(0.2, 0.9 * pow(err, expo)));
        if (sv->method == OR_METHOD_VERLET) fac = 1.0;
        if (sv->method == OR_METHOD_GBS) fac = pow2_floor(fac);
        lambda += h;
        for (int d = 0; d < NSTATE; ++d) { y[d] = y5[d]; k1[d] = k7[d]; }
        h *= fac;
        rejected_prev = 0;
    }
    out->cls = OR_FAILED;
    out->final_rtp[0] = y[R_];
    out->final_rtp[1] = y[TH_];
    out->final_rtp[2] = y[PH_];
    if (rec_n) *rec_n = nrec;
}

static void trace_ray(const or_metric* m, const or_camera* cam, const or_disk* disk, const or_solver* sv,
                      int i, int j, ray_result* out)
{
    double y0[NSTATE];
    or_initial_state(m, cam, i, j, y0);
    trace_from(m, y0, sv->h0_frac * cam->r_obs, disk, sv, out, NULL, NULL, 0, NULL);
}

/* ------------------------------------------------------------------ */
/* Exported entry points.                                               */
/* ------------------------------------------------------------------ */
double or_hamiltonian(const or_metric* m, const double* q) { return hamiltonian_m(m, q); }
void or_rhs(const or_metric* m, const double* q, double* dq) { rhs_m(m, q, dq); }
void or_metric_eval(const or_metric* m, double r, double th, double* g, double* gr, double* gth)
{
    metric_eval(m, r, th, g, gr, gth);
}
/* hyper-dual components for tests: out[5][4] = (f, f_r, f_th, f_rth) of the smooth components */
void or_kerr_smooth_components(double a, double r, double th, double* out)
{
    hd G[5], T[5];
    kerr_components_hd(a, r, th, G, T);
    for (int c = 0; c < 5; ++c) { out[4 * c] = T[c].v; out[4 * c + 1] = T[c].r; out[4 * c + 2] = T[c].t; out[4 * c + 3] = T[c].rt; }
}

/* Trace the listed rays (global id = c*nx*ny + j*nx + i over ncams cameras with
 * the same nx, ny); ray_ids == NULL traces all of them.  Outputs are indexed by
 * position in the list. */
int or_trace(const or_metric* m, const or_camera* cams, int ncams, const or_disk* disk, const or_solver* sv,
             const int64_t* ray_ids, int64_t n, const or_outputs* o, int nthreads)
{
    int64_t per = (int64_t)cams[0].nx * cams[0].ny;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    (void)ncams;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t idx = 0; idx < n; ++idx) {
        int64_t id = ray_ids ? ray_ids[idx] : idx;
        int c = (int)(id / per);
        int64_t pix = id % per;
        const or_camera* cam = &cams[c];
        int i = (int)(pix % cam->nx), j = (int)(pix / cam->nx);
        ray_result rr;
        trace_ray(m, cam, disk, sv, i, j, &rr);
        o->cls[idx] = rr.cls;
        o->n_hits[idx] = rr.n_hits;
        for (int k = 0; k < 3; ++k) {
            o->final_rtp[3 * idx + k] = rr.final_rtp[k];
            o->hit_r[3 * idx + k] = rr.hit_r[k];
            o->hit_g[3 * idx + k] = rr.hit_g[k];
            o->hit_flux[3 * idx + k] = rr.hit_flux[k];
            o->hit_lambda[3 * idx + k] = rr.hit_lambda[k];
            o->hit_order[3 * idx + k] = rr.hit_order[k];
        }
        o->h_drift[idx] = rr.h_drift;
        o->h_gate[idx] = rr.h_gate;
        o->intensity[idx] = rr.intensity;
        o->n_accept[idx] = rr.n_accept;
        o->n_reject[idx] = rr.n_reject;
        o->n_cross[idx] = rr.n_cross;
    }
    return 0;
}

/* One ray from an arbitrary initial state, recording its accepted states
 * (test hook for the constraint and conservation checks).  res[] receives
 * cls, n_hits, n_accept, n_reject, n_cross; resd[] receives final r, theta,
 * phi, h_drift, h_gate, intensity, then hit_r[3], hit_g[3], hit_flux[3],
 * hit_lambda[3]. */
void or_trace_path(const or_metric* m, const double* q0, double h0, const or_disk* disk, const or_solver* sv,
                   double* states, double* lambdas, int cap, int* n_states, int* res, double* resd)
{
    ray_result rr;
    trace_from(m, q0, h0, disk, sv, &rr, states, lambdas, cap, n_states);
    res[0] = rr.cls; res[1] = rr.n_hits; res[2] = rr.n_accept; res[3] = rr.n_reject; res[4] = rr.n_cross;
    resd[0] = rr.final_rtp[0]; resd[1] = rr.final_rtp[1]; resd[2] = rr.final_rtp[2];
    resd[3] = rr.h_drift; resd[4] = rr.h_gate; resd[5] = rr.intensity;
    for (int k = 0; k < 3; ++k) {
        resd[6 + k] = rr.hit_r[k]; resd[9 + k] = rr.hit_g[k];
        resd[12 + k] = rr.hit_flux[k]; resd[15 + k] = rr.hit_lambda[k];
    }
}

/* Classic fixed-step fourth-order Runge-Kutta step (brute-force cross-check of
 * the adaptive integrator; not part of the traced method). */
void or_rk4_step(const or_metric* m, const double* q, double h, double* out)
{
    double k1[NSTATE], k2[NSTATE], k3[NSTATE], k4[NSTATE], Y[NSTATE];
    rhs_m(m, q, k1);
    for (int d = 0; d < NSTATE; ++d) Y[d] = q[d] + 0.5 * h * k1[d];
    rhs_m(m, Y, k2);
    for (int d = 0; d < NSTATE; ++d) Y[d] = q[d] + 0.5 * h * k2[d];
    rhs_m(m, Y, k3);
    for (int d = 0; d < NSTATE; ++d) Y[d] = q[d] + h * k3[d];
    rhs_m(m, Y, k4);
    for (int d = 0; d < NSTATE; ++d) out[d] = q[d] + h / 6.0 * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
}

/* Many RK4 steps of size h_frac * r (step proportional to radius, no error
 * control), stopping before r leaves [r_lo, r_hi] or cos(theta) changes sign.
 * Returns the number of steps taken; q is advanced in place. */
int or_rk4_run(const or_metric* m, double* q, double h_frac, double r_lo, double r_hi, int max_steps,
               int stop_on_equator)
{
    double y[NSTATE];
    int n = 0;
    for (; n < max_steps; ++n) {
        or_rk4_step(m, q, h_frac * q[R_], y);
        if (y[R_] < r_lo || y[R_] > r_hi) break;
        if (stop_on_equator && ((cos(q[TH_]) > 0.0) != (cos(y[TH_]) > 0.0))) break;
        memcpy(q, y, sizeof(y));
    }
    return n;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
