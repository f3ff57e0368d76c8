// trace_kernel.hip -- the persistent ray-queue integrator (gfx950) and the
// passes around it.
//
// A trace is a short sequence of launches on one stream:
//   1. job_setup: per camera / request, the observer's metric and ZAMO tetrad
//      (Sec. 2.2), r_+, the disk's inner edge and the Page-Thorne constants.
//   2. order_keys / order_scan / order_scatter (traces of >= 4096 rays by
//      default): the cost-ordered queue, rays nearest the critical curve first.
//   3. trace_persistent<KIND, PREC, METHOD, SERVE>: one lane integrates one ray at a
//      time.  A wavefront takes ray ids from a global atomic queue head; when
//      a lane's ray terminates, the lane is refilled, so divergent step counts
//      do not leave lanes idle until the slowest ray of the wave is done.  Per
//      ray: camera initial conditions, steps of the chosen method (Sec. 3.2:
//      Dormand-Prince, Cash-Karp or Fehlberg 5(4) with the elementary
//      controller, Gragg-Bulirsch-Stoer extrapolation, or fixed-step Verlet),
//      the constraint residual |H| at each accepted state (Sec. 4.1), and the
//      detection of horizon / escape / equatorial events on accepted steps.
//      The integrator leaves each event's step (its cubic Hermite data) in
//      the ray's record instead of locating it, except where a crossing
//      straddles a disk edge.
//   4. finish_kernel: one thread per ray locates the recorded roots on the
//      same cubics, writes every output, and shades the disk hits with g
//      (Eq. (15)) and g^4 F(r) (Eqs. (11), (16)).
// Per-ray arithmetic never depends on other lanes, so results are
// bit-identical for every launch shape, queue order and batch composition.
//
// KIND 0 is analytic Kerr, 1 the tabulated metric.  PREC = 0 evaluates every
// stage in FP64; PREC = 1 evaluates the stages of far-field steps in FP32
// (stages32) while the state update, error norm, controller, events and
// shading stay FP64.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "order.hpp"
#include "kerr.hpp"
#include "kerr32.hpp"
#include "table.hpp"

namespace tartarus {

// Dormand & Prince (1980) 5(4) coefficients.
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0, A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0, A64 = 49.0 / 176.0,
                 A65 = -5103.0 / 18656.0;
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0, B5 = -2187.0 / 6784.0,
                 B6 = 11.0 / 84.0;
// error weights b - b* (fifth minus embedded fourth order)
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0, E5 = -17253.0 / 339200.0,
                 E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;

// The two six-stage 5(4) pairs of Sec. 3.2 (Cash & Karp 1990, Fehlberg 1969):
// stage matrix a, fifth-order weights b (propagated) and error weights
// e = b - b* (b* the embedded fourth-order weights).  f(y5) closes each step
// as the next step's first stage and the event interpolant's end slope.
enum { METHOD_DP45 = 0, METHOD_CK45 = 1, METHOD_RKF45 = 2, METHOD_GBS = 3, METHOD_VERLET = 4 };

template <int M>
struct Pair;

template <>
struct Pair<METHOD_CK45> {
    static constexpr double a[6][5] = {{0, 0, 0, 0, 0},
                                       {1.0 / 5.0, 0, 0, 0, 0},
                                       {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
                                       {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
                                       {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
                                       {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0,
                                        253.0 / 4096.0}};
    static constexpr double b[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
    static constexpr double e[6] = {37.0 / 378.0 - 2825.0 / 27648.0, 0.0, 250.0 / 621.0 - 18575.0 / 48384.0,
                                    125.0 / 594.0 - 13525.0 / 55296.0, 0.0 - 277.0 / 14336.0,
                                    512.0 / 1771.0 - 1.0 / 4.0};
};

template <>
struct Pair<METHOD_RKF45> {
    static constexpr double a[6][5] = {{0, 0, 0, 0, 0},
                                       {1.0 / 4.0, 0, 0, 0, 0},
                                       {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
                                       {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
                                       {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
                                       {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
    static constexpr double b[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};
    static constexpr double e[6] = {16.0 / 135.0 - 25.0 / 216.0, 0.0, 6656.0 / 12825.0 - 1408.0 / 2565.0,
                                    28561.0 / 56430.0 - 2197.0 / 4104.0, -9.0 / 50.0 + 1.0 / 5.0, 2.0 / 55.0};
};

// Rows of a pair's tableau as compile-time weight functions over the six
// stage slopes: stage S's a[S][.], the propagated b and the error e.
template <class P, int S>
struct RowA {
    static constexpr double w(int j) { return j < 5 ? P::a[S][j] : 0.0; }
};
template <class P>
struct RowB {
    static constexpr double w(int j) { return P::b[j]; }
};
template <class P>
struct RowE {
    static constexpr double w(int j) { return P::e[j]; }
};

// sum_j w(j) k[j] over the nonzero compile-time weights of Row: the first term
// a product, the rest fused in index order.  Zero weights generate no code and
// no test (the row and the index are template arguments).
template <class Row, int J = 0, bool STARTED = false>
__device__ __forceinline__ double weighted(const double (&k)[6], double acc = 0.0)
{
    if constexpr (J == 6) {
        return acc;
    } else if constexpr (Row::w(J) == 0.0) {
        return weighted<Row, J + 1, STARTED>(k, acc);
    } else if constexpr (!STARTED) {
        return weighted<Row, J + 1, true>(k, Row::w(J) * k[J]);
    } else {
        return weighted<Row, J + 1, true>(k, fma(Row::w(J), k[J], acc));
    }
}

enum { CLS_ESCAPED = 0, CLS_CAPTURED = 1, CLS_FAILED = 2, CLS_ON_DISK = 3 };

struct Ray {
    double t, r, th, ph, pr, pth, pt, pph;
    Deriv<double> k;   // right-hand side at the current state (first same as last)
    double cth, sth;   // cos(theta) and sin(theta) at the current state
    double lam, h;
    double hmax, hgate;
    double a, rp;      // spin and horizon radius r_+
    float guard_r, guard_th;  // mixed precision: FP32 only while |p_r| >= guard_r and |p_theta| >= guard_th
    int n_acc, n_rej, n_f32, n_cross, n_hits, rej_prev, max_hits, job;
    int k32;           // R.k was evaluated in FP32 (mixed precision)
    int opaque;        // the first crossing on the disk ends the ray
    long long local;
    double* rec;       // this ray's record for the finishing pass
    double r_in, r_out;  // disk radii
};

// Solver settings a ray is traced with.  A one-shot trace takes them from the
// launch (every ray of the trace shares them, so they stay wave-uniform); a
// serving epoch takes each ray's from its request, so requests of different
// tolerances and precisions share the epoch.
struct RaySettings {
    double rtol, atol, horizon_factor, r_escape, event_tol;
    int max_steps;   // attempts allowed, clamped to the int range (attempts are counted in int)
    int allow32;   // mixed precision: FP32 stages allowed where the regime test passes
};

// What every ray of a one-shot trace shares (one metric, one solver), read
// once per wavefront from the first job's constants, so it stays in scalar
// registers: the spin and its square, the radius from which the constraint
// gate counts and the horizon event's radius.  Serving epochs form these per
// ray from the ray's own request.
struct TraceUniform {
    Spin spin;
    double gate_r, r_stop;
};

__device__ __forceinline__ TraceUniform trace_uniform(const LaunchArgs& A)
{
    const JobConst& C = A.jc[0];
    return {{A.jobs[0].a, C.a2}, C.gate_r, C.r_stop};
}

__device__ __forceinline__ int clamp_steps(long long n)
{
    return n > 0x7fffffffLL ? 0x7fffffff : (int)n;
}

__device__ __forceinline__ RaySettings launch_settings(const LaunchArgs& A)
{
    return {A.rtol, A.atol, A.horizon_factor, A.r_escape, A.event_tol, clamp_steps(A.max_steps), 1};
}

__device__ __forceinline__ RaySettings job_settings(const DevJob& J)
{
    return {J.rtol, J.atol, J.horizon_factor, J.r_escape, J.event_tol, clamp_steps(J.max_steps), J.allow32};
}

// max(|a|, |b|) in one instruction.  fmax of values the compiler cannot prove
// canonical (loop-carried state) first canonicalizes one operand, a second
// instruction; the operands here come from arithmetic, so they are never
// signalling NaNs, and for a quiet NaN the hardware maximum returns the other
// operand, as fmax does.
__device__ __forceinline__ double max_abs(double a, double b)
{
    double m;
    asm("v_max_f64 %0, |%1|, |%2|" : "=v"(m) : "v"(a), "v"(b));
    return m;
}

template <int KIND>
struct MetricOps {
    TableView T;
    // coef: where the analytic right-hand side takes its sine/cosine
    // coefficients from (immediates unless a stage loop passes SinCosLoad)
    // Right-hand side at (r, th, pr, pth); also H, cos(th) and sin(th).
    template <class Coef = SinCosImm>
    __device__ __forceinline__ void rhs_sc(Spin a, double r, double th, double pr, double pth, double pt, double pph,
                                           Deriv<double>& d, double& H, double& c, double& s, Coef coef = {}) const
    {
        if (KIND == 0)
            kerr_rhs64(a, r, th, pr, pth, pt, pph, d, H, c, s, coef);
        else
            table_rhs64(T, r, th, pr, pth, pt, pph, d, H, c, s);
    }
    template <class Coef = SinCosImm>
    __device__ __forceinline__ void rhs(Spin a, double r, double th, double pr, double pth, double pt, double pph,
                                        Deriv<double>& d, double& H, double& c, Coef coef = {}) const
    {
        double s;
        rhs_sc(a, r, th, pr, pth, pt, pph, d, H, c, s, coef);
    }
    // The same at a stage point near the step's start (th0, with sine s0 and
    // cosine c0): where |th - th0| <= dmax the analytic metric takes sin and
    // cos of th from those of th0 by the angle-sum identities, elsewhere from
    // th itself.  Returns cos(th) in c.
    template <class Coef, class Shift>
    __device__ __forceinline__ void rhs_near(Spin a, double r, double th, double th0, double s0, double c0,
                                             double dmax, double pr, double pth, double pt, double pph,
                                             Deriv<double>& d, double& H, double& c, Coef coef, Shift shift) const
    {
        if constexpr (KIND == 0) {
            const double dt = th - th0;
            double sn, cs;
            if (fabs(dt) <= dmax)
                sincos_shift(s0, c0, dt, sn, cs, shift);
            else
                sincos64_with(th, &sn, &cs, coef);
            kerr_rhs64_trig(a, r, sn * sn, cs * cs, sn * cs, pr, pth, pt, pph, d, H);
            c = cs;
        } else {
            rhs(a, r, th, pr, pth, pt, pph, d, H, c);
        }
    }
    __device__ __forceinline__ void metric(double a, double r, double th, double g[5]) const
    {
        if (KIND == 0) {
            kerr_metric64(a, r, th, g);
        } else {
            double gr[5], gt[5];
            table_metric<false, false>(T, r, th, g, gr, gt);
        }
    }
};

// ---------------------------------------------------------------------------
// per-job constants
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void job_setup(const DevJob* jobs, JobConst* jc, int njobs, const double* table, int nr, int nth,
                          double r_min, double r_max)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    const DevJob& J = jobs[j];
    MetricOps<KIND> M;
    if (KIND == 1) M.T = make_table_view(table, nr, nth, r_min, r_max);
    JobConst C;
    M.metric(J.a, J.r_obs, J.theta_obs, C.g);
    // ZAMO tetrad (Eqs. (7)-(10)); e_(t)^phi = omega e_(t)^t with omega = -g_tphi / g_phph
    const double omega = -C.g[1] / C.g[4];
    C.ett = 1.0 / sqrt(fma(omega * omega, C.g[4], -C.g[0]));
    C.etp = omega * C.ett;
    C.err = 1.0 / sqrt(C.g[2]);
    C.ehh = 1.0 / sqrt(C.g[3]);
    C.epp = 1.0 / sqrt(C.g[4]);
    double s, c;
    sincos64(J.theta_obs, &s, &c);
    C.c2_obs = c * c;
    C.is2_obs = 1.0 / (s * s);
    C.rp = horizon_radius(J.a);
    C.r_in = J.disk_r_in > 0.0 ? J.disk_r_in : isco_radius(J.a);
    C.x0 = sqrt(C.r_in);
    nt_flux_constants(J.a, C.xi, C.coef);
    C.a2 = J.a * J.a;
    C.gate_r = 1.5 * C.rp;
    C.r_stop = J.horizon_factor * C.rp;
    if (KIND == 1 && r_min > C.r_stop) C.r_stop = r_min;
    jc[j] = C;
}

// Covariant momentum of pixel (alpha, beta) (Eqs. (4)-(5) and the lowering with
// Eq. (6)), negated for backward tracing.  Shared by the integrator and the
// shading pass so both obtain the same p_t, p_phi.
__device__ __forceinline__ void pixel_momentum(const JobConst& C, double D, double al, double be, double p[4])
{
    const double iD = 1.0 / D;
    const double plr = sqrt(1.0 - (al * al + be * be) * (iD * iD));
    const double put = C.ett;
    const double pur = C.err * plr;
    const double puh = C.ehh * (be * iD);
    const double pup = fma(C.epp, -al * iD, C.etp);
    p[0] = -fma(C.g[0], put, C.g[1] * pup);
    p[1] = -(C.g[2] * pur);
    p[2] = -(C.g[3] * puh);
    p[3] = -fma(C.g[1], put, C.g[4] * pup);
}

__device__ __forceinline__ void pixel_coords(const DevJob& J, long long pix, double& al, double& be)
{
    const int i = (int)(pix % J.nx), j = (int)(pix / J.nx);
    al = J.nx > 1 ? J.alpha_min + (double)i * (J.alpha_max - J.alpha_min) / (double)(J.nx - 1) : J.alpha_min;
    be = J.ny > 1 ? J.beta_min + (double)j * (J.beta_max - J.beta_min) / (double)(J.ny - 1) : J.beta_min;
}

// ---------------------------------------------------------------------------
// event location on the step's cubic Hermite interpolant
// ---------------------------------------------------------------------------
// y(s) = y0 + s (h d0 + s (c2 + s c3)), s in [0, 1], the Hermite interpolant
// through (y_n, h k1) and (y_n+1, h k7) in monomial form.
struct Cubic {
    double y0, c1, c2, c3;
    __device__ __forceinline__ Cubic(double y0_, double d0, double y1, double d1, double h)
    {
        y0 = y0_;
        c1 = h * d0;
        c2 = fma(3.0, y1 - y0_, -h * fma(2.0, d0, d1));
        c3 = fma(2.0, y0_ - y1, h * (d0 + d1));
    }
    __device__ __forceinline__ double at(double s) const { return fma(s, fma(s, fma(s, c3, c2), c1), y0); }
    __device__ __forceinline__ double slope(double s) const { return fma(s, fma(3.0 * s, c3, 2.0 * c2), c1); }
};

// Root of y(s) = target in (0, 1]: y(0) lies strictly on the start side
// ("above": y > target) and y(1) does not.  The bracket [lo, hi] always keeps
// the start side at lo; each iteration takes a Newton step on the cubic when it
// stays inside the bracket and bisects otherwise.  Stops when the Newton
// correction or the bracket is below tol in the affine parameter (tol is set
// below the event tolerance).  At most 64 iterations.
__device__ __forceinline__ double locate_root(const Cubic& p, double target, bool above, double h, double tol)
{
    double lo = 0.0, hi = 1.0;
    const double f0 = p.y0 - target, f1 = p.at(1.0) - target;
    double s = (f0 != f1) ? f0 / (f0 - f1) : 0.5;
    if (!(s > 0.0 && s < 1.0)) s = 0.5;
    for (int it = 0; it < 64; ++it) {
        const double f = p.at(s) - target;
        const bool same = above ? (f > 0.0) : (f < 0.0);
        if (same)
            lo = s;
        else
            hi = s;
        if ((hi - lo) * h <= tol) return 0.5 * (lo + hi);
        double sn = s - f / p.slope(s);
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) * h <= 0.25 * tol) return sn;
        s = sn;
    }
    return 0.5 * (lo + hi);
}

// Equatorial crossing for polar angles outside (-pi/2, 3pi/2), where the sign
// of cos(theta) is not the sign of pi/2 - theta: plain bisection on cos.
__device__ __noinline__ double locate_equator_wide(const Cubic& p, bool north_start, double h, double tol)
{
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 80 && (hi - lo) * h > tol; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double v = cos(p.at(mid));
        const bool same = north_start ? (v > 0.0) : (v < 0.0);
        lo = same ? mid : lo;
        hi = same ? hi : mid;
    }
    return 0.5 * (lo + hi);
}

// Job of global ray index gid: binary search over the first ray of each job
// (serving: over the directory of live entries).  The persistent kernel keeps a
// copy of the search keys in LDS when they fit (kLdsJobs), so a refill does not
// wait on a chain of dependent global loads.
constexpr int kLdsJobs = 1024;

struct JobDir {
    const long long* begin;   // LDS copy, or null: search the global tables
    const int* job;
    int n;
};

__device__ __forceinline__ int find_job(const LaunchArgs& A, const JobDir& D, long long gid)
{
    if (D.begin) {
        int lo = 0, hi = D.n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (D.begin[mid] <= gid)
                lo = mid;
            else
                hi = mid - 1;
        }
        return D.job[lo];
    }
    if (A.dir_begin) {
        int lo = 0, hi = A.ndir - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.dir_begin[mid] <= gid)
                lo = mid;
            else
                hi = mid - 1;
        }
        return A.dir_job[lo];
    }
    int lo = 0, hi = A.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.jobs[mid].ray_begin <= gid)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// one ray
// ---------------------------------------------------------------------------
// Returns false when the ray's job has been cancelled (serving): then the ray
// is not traced.
// Absolute ray index of queue position q in a serving epoch whose queue runs
// over segments (the unstarted rays of each live request, in hand-out order):
// binary search for the segment k with seg_q[k] <= q < seg_q[k + 1].
__device__ __forceinline__ long long segment_ray(const LaunchArgs& A, long long q)
{
    int lo = 0, hi = A.nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.seg_q[mid] <= q)
            lo = mid;
        else
            hi = mid - 1;
    }
    return A.seg_ray[lo] + (q - A.seg_q[lo]);
}

// Pixel of queue position q when a camera's rays are handed out by 8 x 8 tiles:
// tile rows of 8 pixel rows (the last one h = ny - 8 ty rows high), tiles
// row-major within a tile row (each 8 wide but the last, nx - 8 tx), pixels
// row-major within a tile.  Tile (tx, ty) starts at 8 ty nx + 8 tx h.
__device__ __forceinline__ long long tile_pixel(long long q, int nx, int ny)
{
    const long long band = 8ll * nx;
    long long ty = q / band;
    const long long ty_last = (ny - 1) / 8;
    if (ty > ty_last) ty = ty_last;
    const long long h = ny - 8 * ty < 8 ? ny - 8 * ty : 8;
    const long long r = q - ty * band;
    long long tx = r / (8 * h);
    const long long tx_last = (nx - 1) / 8;
    if (tx > tx_last) tx = tx_last;
    const long long inner = r - tx * 8 * h;
    const long long w = nx - 8 * tx < 8 ? nx - 8 * tx : 8;
    const long long jj = inner / w, ii = inner - jj * w;
    return (8 * ty + jj) * nx + 8 * tx + ii;
}

template <int KIND>
__device__ bool ray_init(Ray& R, long long gid, const LaunchArgs& A, const JobDir& D, const MetricOps<KIND>& M)
{
    const int jb = find_job(A, D, gid);
    const DevJob& J = A.jobs[jb];
    const JobConst& C = A.jc[jb];
    const long long pos = gid - J.ray_begin;
    const long long pix = A.tile ? tile_pixel(pos, J.nx, J.ny) : pos;
    double al, be, p[4];
    pixel_coords(J, pix, al, be);
    pixel_momentum(C, J.r_obs, al, be, p);
    R.t = 0.0;
    R.r = J.r_obs;
    R.th = J.theta_obs;
    R.ph = 0.0;
    R.pt = p[0];
    R.pr = p[1];
    R.pth = p[2];
    R.pph = p[3];
    R.a = J.a;
    R.rp = C.rp;
    R.k32 = 0;
    // Carter's constant from the initial state sets the polar turning-point guard
    const double Q = fma(R.pth, R.pth, C.c2_obs * fma(R.pph * R.pph, C.is2_obs, -(R.a * R.a * R.pt * R.pt)));
    R.guard_th = (float)(A.turn_th * sqrt(fmax(Q, 1e-12)));
    R.guard_r = (float)(A.turn_r * fabs(R.pt));
    double H;
    M.rhs_sc(spin_of(R.a), R.r, R.th, R.pr, R.pth, R.pt, R.pph, R.k, H, R.cth, R.sth);
    R.hmax = fabs(H);
    R.hgate = R.r >= 1.5 * R.rp ? fabs(H) : 0.0;
    R.lam = 0.0;
    R.h = J.h0_frac * J.r_obs;
    R.n_acc = R.n_rej = R.n_f32 = R.n_cross = R.n_hits = R.rej_prev = 0;
    R.max_hits = J.max_hits;
    R.opaque = J.disk_flags & DISK_OPAQUE;
    R.job = jb;
    R.local = pix;
    R.rec = J.rec + pix * REC_DOUBLES;
    R.r_in = C.r_in;
    R.r_out = J.disk_r_out;
    return !J.cancelled;
}

// The ray's counters and classification go to its record; the finishing pass
// turns the record into outputs.  code: terminal kind | 4 * equator crossed in
// the terminal step (REC_CODE).
__device__ void ray_finish(const Ray& R, const LaunchArgs& A, int cls, int code)
{
    double* rec = R.rec;
    rec[REC_CODE] = (double)code;
    rec[REC_HMAX] = R.hmax;
    rec[REC_HGATE] = R.hgate;
    int* iv = reinterpret_cast<int*>(rec + REC_INTS);
    iv[0] = cls;
    iv[1] = R.n_hits;
    iv[2] = R.n_acc;
    iv[3] = R.n_rej;
    iv[4] = R.n_f32;
    iv[5] = R.n_cross;
    (void)A;
}

// A ray that ends where it stands (no terminal root to locate).
__device__ void ray_fail(const Ray& R, const LaunchArgs& A)
{
    R.rec[REC_TERM + 0] = R.r;
    R.rec[REC_TERM + 4] = R.th;
    R.rec[REC_TERM + 8] = R.ph;
    ray_finish(R, A, CLS_FAILED, 0);
}

// Equatorial crossing on the step's polar cubic (root of theta = pi/2, or of
// cos(theta) = 0 where theta has left (-pi/2, 3pi/2)).
__device__ __forceinline__ double equator_root(const Cubic& pth, double th0, double th1, double cth0, double h,
                                               double tol)
{
    const bool wide = !(th0 > -M_PI_2 && th0 < 1.5 * M_PI && th1 > -M_PI_2 && th1 < 1.5 * M_PI);
    return wide ? locate_equator_wide(pth, cth0 > 0.0, h, tol) : locate_root(pth, M_PI_2, cth0 < 0.0, h, tol);
}

// The step that ends a ray, for the finishing pass to locate its root on:
// r, theta, phi as (y0, dy0/dlam, y1, dy1/dlam), h, lam, the target radius of
// a radial event, cos(theta0).
__device__ __forceinline__ void terminal_step(const Ray& R, double h, const Deriv<double>& y5,
                                              const Deriv<double>& k7, double target)
{
    double* t = R.rec + REC_TERM;
    t[0] = R.r;
    t[1] = R.k.r;
    t[2] = y5.r;
    t[3] = k7.r;
    t[4] = R.th;
    t[5] = R.k.th;
    t[6] = y5.th;
    t[7] = k7.th;
    t[8] = R.ph;
    t[9] = R.k.ph;
    t[10] = y5.ph;
    t[11] = k7.ph;
    t[12] = h;
    t[13] = R.lam;
    t[14] = target;
    t[15] = R.cth;
}

// An equatorial crossing of an opaque disk's ray (Sec. 2.3, optically thick):
// it counts, and returns whether it lies on the disk, which ends the ray.  The
// step's radial Bernstein hull decides without a root unless it straddles an
// edge of the disk; the finishing pass locates the crossing either way (same
// cubic, same root finder).
__device__ __forceinline__ bool opaque_hit(Ray& R, double h, const Deriv<double>& y5, const Deriv<double>& k7,
                                           double tol)
{
    R.n_cross++;
    const double b1 = fma(h * (1.0 / 3.0), R.k.r, R.r), b2 = fma(-h * (1.0 / 3.0), k7.r, y5.r);
    const double lo = fmin(fmin(R.r, y5.r), fmin(b1, b2)), hi = fmax(fmax(R.r, y5.r), fmax(b1, b2));
    constexpr double m = 1e-12;
    if (hi < R.r_in * (1.0 - m) || lo > R.r_out * (1.0 + m)) return false;
    if (lo >= R.r_in * (1.0 + m) && hi <= R.r_out * (1.0 - m)) return true;
    const Cubic pth(R.th, R.k.th, y5.th, k7.th, h);
    const double sd = equator_root(pth, R.th, y5.th, R.cth, h, tol);
    const double rr = Cubic(R.r, R.k.r, y5.r, k7.r, h).at(sd);
    return rr >= R.r_in && rr <= R.r_out;
}

// An equatorial crossing on a step that does not end the ray.  It counts, and
// it takes the next free hit slot when it lies on the disk.  Where the step's
// radial cubic stays inside the disk's radii (its Bernstein control points
// bound it) the decision needs no root: the slot keeps the step and the
// finishing pass locates the crossing.  Where it stays outside, nothing is
// recorded.  Only steps that straddle an edge of the disk locate the root here.
__device__ __forceinline__ void disk_crossing(Ray& R, double h, const Deriv<double>& y5, const Deriv<double>& k7,
                                              double tol)
{
    R.n_cross++;
    if (R.n_hits >= R.max_hits) return;
    const double b1 = fma(h * (1.0 / 3.0), R.k.r, R.r), b2 = fma(-h * (1.0 / 3.0), k7.r, y5.r);
    const double lo = fmin(fmin(R.r, y5.r), fmin(b1, b2)), hi = fmax(fmax(R.r, y5.r), fmax(b1, b2));
    constexpr double m = 1e-12;   // margin for rounding of the cubic evaluated at the root
    if (hi < R.r_in * (1.0 - m) || lo > R.r_out * (1.0 + m)) return;
    double* sl = R.rec + REC_SLOT0 + REC_SLOT_LEN * R.n_hits;
    if (lo >= R.r_in * (1.0 + m) && hi <= R.r_out * (1.0 - m)) {
        sl[0] = R.r;
        sl[1] = R.k.r;
        sl[2] = y5.r;
        sl[3] = k7.r;
        sl[4] = R.th;
        sl[5] = R.k.th;
        sl[6] = y5.th;
        sl[7] = k7.th;
        sl[8] = h;
        sl[9] = R.lam;
        sl[10] = R.cth;
    } else {
        const Cubic pth(R.th, R.k.th, y5.th, k7.th, h);
        const double sd = equator_root(pth, R.th, y5.th, R.cth, h, tol);
        const double rr = Cubic(R.r, R.k.r, y5.r, k7.r, h).at(sd);
        if (!(rr >= R.r_in && rr <= R.r_out)) return;
        sl[0] = rr;
        sl[8] = 0.0;
        sl[9] = fma(sd, h, R.lam);
    }
    reinterpret_cast<int*>(R.rec + REC_INTS)[6 + R.n_hits] = R.n_cross;
    R.n_hits++;
}

// ---- mixed precision ------------------------------------------------------
// The regime is decided per ray from its own state only (never from its
// wavefront), so a ray's arithmetic is the same in any batch.  FP32 stages are
// used where r >= r_switch_factor * r_+ at the start of the step, away from
// radial and polar turning points, away from the polar axis, and where the
// FP32 rounding of the error estimate stays well below the tolerance.  Near
// the axis sin(theta) is small and p_phi / sin^2(theta) large, and theta
// rounded to FP32 leaves sin^2(theta) with a relative error of order
// 1e-7 / sin(theta): the FP32 error estimate of p_theta then sits above the
// tolerance and the step collapses (rays of zero angular momentum cross the
// axis; |cos(theta)| <= 0.995 keeps them in FP64 there).
//
// Noise floor: a stage slope evaluated in FP32 carries a relative error of a
// few FP32 ulps, so the estimate h sum_j e_j k_j of component i carries about
// |e|_2 * 4 * 2^-24 * h |k_i| of rounding (|e|_2 = 0.0798 for the
// Dormand-Prince error weights).  FP32 stages are used only where that is at
// most half of the component's tolerance scale atol + rtol |y_i|, i.e.
// h |k_i| <= kNoiseRatio (atol + rtol |y_i|); otherwise an FP32 attempt would
// be rejected on rounding noise and the step driven down to the noise level.
// The same bound keeps the FP32 rounding of the state update below the
// tolerance.  At tight tolerances the test leaves FP32 off almost everywhere.
constexpr double kDp45ErrNorm = 0.07976;                          // |b - b*|_2
constexpr double kNoiseRatio = 0.5 / (kDp45ErrNorm * 4.0 * 0x1p-24);   // ~2.6e7

__device__ __forceinline__ bool fp32_noise_ok(double hk, double y, double atol, double rtol)
{
    return fabs(hk) <= kNoiseRatio * fma(rtol, fabs(y), atol);
}

__device__ __forceinline__ bool far_field(const Ray& R, const LaunchArgs& A, const RaySettings& P)
{
    const double h = R.h, atol = P.atol, rtol = P.rtol;
    return P.allow32 && R.r >= A.r_switch_factor * R.rp && R.cth * R.cth <= 0.99 && fabs(R.pr) >= (double)R.guard_r &&
           fabs(R.pth) >= (double)R.guard_th && fp32_noise_ok(h * R.k.r, R.r, atol, rtol) &&
           fp32_noise_ok(h * R.k.th, R.th, atol, rtol) && fp32_noise_ok(h * R.k.ph, R.ph, atol, rtol) &&
           fp32_noise_ok(h * R.k.pr, R.pr, atol, rtol) && fp32_noise_ok(h * R.k.pth, R.pth, atol, rtol);
}

// One attempted DP45 step whose six new stage evaluations run in FP32 (on-shell
// far-field form, kerr32.hpp).  The stage increments are summed in FP32 and
// added to the FP64 state; the t component carries only delta_t in FP32 and
// its constant part -p_t h is added in FP64.  The error vector feeds the FP64
// norm; H(y5) and cos(theta5) are evaluated in FP64 for the constraint monitor
// and the event tests.
__device__ __forceinline__ void stages32(const Ray& R, double h, Deriv<double>& y5, Deriv<double>& k7d,
                                         Deriv<double>& e, double& H5, double& c5, double& s5)
{
    const float a = (float)R.a, hf = (float)h;
    const float r0 = (float)R.r, th0 = (float)R.th, pr0 = (float)R.pr, pth0 = (float)R.pth;
    const float pt = (float)R.pt, pph = (float)R.pph;
    Deriv<float> k1;
    k1.t = (float)(R.k.t + R.pt);
    k1.r = (float)R.k.r;
    k1.th = (float)R.k.th;
    k1.ph = (float)R.k.ph;
    k1.pr = (float)R.k.pr;
    k1.pth = (float)R.k.pth;
    Deriv<float> k2, k3, k4, k5, k6, k7;
    const float a21 = (float)A21, a31 = (float)A31, a32 = (float)A32, a41 = (float)A41, a42 = (float)A42,
                a43 = (float)A43, a51 = (float)A51, a52 = (float)A52, a53 = (float)A53, a54 = (float)A54,
                a61 = (float)A61, a62 = (float)A62, a63 = (float)A63, a64 = (float)A64, a65 = (float)A65;
    kerr_rhs32(a, fmaf(hf, a21 * k1.r, r0), fmaf(hf, a21 * k1.th, th0), fmaf(hf, a21 * k1.pr, pr0),
               fmaf(hf, a21 * k1.pth, pth0), pt, pph, k2);
#define TT_S3(c, y) fmaf(hf, fmaf(a32, k2.c, a31 * k1.c), y)
    kerr_rhs32(a, TT_S3(r, r0), TT_S3(th, th0), TT_S3(pr, pr0), TT_S3(pth, pth0), pt, pph, k3);
#define TT_S4(c, y) fmaf(hf, fmaf(a43, k3.c, fmaf(a42, k2.c, a41 * k1.c)), y)
    kerr_rhs32(a, TT_S4(r, r0), TT_S4(th, th0), TT_S4(pr, pr0), TT_S4(pth, pth0), pt, pph, k4);
#define TT_S5(c, y) fmaf(hf, fmaf(a54, k4.c, fmaf(a53, k3.c, fmaf(a52, k2.c, a51 * k1.c))), y)
    kerr_rhs32(a, TT_S5(r, r0), TT_S5(th, th0), TT_S5(pr, pr0), TT_S5(pth, pth0), pt, pph, k5);
#define TT_S6(c, y) fmaf(hf, fmaf(a65, k5.c, fmaf(a64, k4.c, fmaf(a63, k3.c, fmaf(a62, k2.c, a61 * k1.c)))), y)
    kerr_rhs32(a, TT_S6(r, r0), TT_S6(th, th0), TT_S6(pr, pr0), TT_S6(pth, pth0), pt, pph, k6);
    const float b1 = (float)B1, b3 = (float)B3, b4 = (float)B4, b5 = (float)B5, b6 = (float)B6;
#define TT_INC(c) (double)(hf * fmaf(b6, k6.c, fmaf(b5, k5.c, fmaf(b4, k4.c, fmaf(b3, k3.c, b1 * k1.c)))))
    y5.t = fma(-h, R.pt, R.t) + TT_INC(t);
    y5.r = R.r + TT_INC(r);
    y5.th = R.th + TT_INC(th);
    y5.ph = R.ph + TT_INC(ph);
    y5.pr = R.pr + TT_INC(pr);
    y5.pth = R.pth + TT_INC(pth);
    kerr_rhs32(a, (float)y5.r, (float)y5.th, (float)y5.pr, (float)y5.pth, pt, pph, k7);
    const float e1 = (float)E1, e3 = (float)E3, e4 = (float)E4, e5 = (float)E5, e6 = (float)E6, e7 = (float)E7;
#define TT_E32(c) (double)(hf * fmaf(e7, k7.c, fmaf(e6, k6.c, fmaf(e5, k5.c, fmaf(e4, k4.c, fmaf(e3, k3.c, e1 * k1.c))))))
    e.t = TT_E32(t);
    e.r = TT_E32(r);
    e.th = TT_E32(th);
    e.ph = TT_E32(ph);
    e.pr = TT_E32(pr);
    e.pth = TT_E32(pth);
    k7d.t = (double)k7.t - R.pt;
    k7d.r = (double)k7.r;
    k7d.th = (double)k7.th;
    k7d.ph = (double)k7.ph;
    k7d.pr = (double)k7.pr;
    k7d.pth = (double)k7.pth;
    H5 = kerr_H64(R.a, y5.r, y5.th, y5.pr, y5.pth, R.pt, R.pph, c5, s5);
#undef TT_S3
#undef TT_S4
#undef TT_S5
#undef TT_S6
#undef TT_INC
#undef TT_E32
}

// One attempted DP45 step with FP64 stages.  Writes the fifth-order state y5
// (dynamic components), k7 = f(y5), H(y5), cos(theta5) and the error vector.
// The FP64 DP45 coefficients in constant memory, read with scalar loads one
// stage's worth at a time.  FP64 VALU instructions cannot encode a 64-bit
// literal, so written as immediates every coefficient costs two s_mov per
// attempt; held across the loop they exceed the SGPR file and spill.  A
// constant-memory pointer passed through an empty asm cannot be hoisted out of
// the integration loop, so each stage's loads stay next to their use
// (measured: 2 % off the 512 x 512, a = 0.9 trace at rtol 3e-10 with one
// wavefront per SIMD).  The tabulated metric keeps immediates: its cell
// gather already fills the SGPR file, and the loads made it spill more.
typedef const __attribute__((address_space(4))) double ConstDouble;
constexpr double kDp45[26] = {A21, A31, A32, A41, A42, A43, A51, A52, A53, A54, A61, A62, A63, A64, A65,
                              B1,  B3,  B4,  B5,  B6,  E1,  E3,  E4,  E5,  E6,  E7};
__constant__ double kDp45Coef[26] = {A21, A31, A32, A41, A42, A43, A51, A52, A53, A54, A61, A62, A63, A64, A65,
                                     B1,  B3,  B4,  B5,  B6,  E1,  E3,  E4,  E5,  E6,  E7};
__device__ __forceinline__ ConstDouble* opaque_const(ConstDouble* p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// Where stages64 takes the coefficients from: scalar loads (LOAD) or
// immediates.  next() starts a new stage's group of loads.
template <bool LOAD>
struct Dp45Source {
    ConstDouble* p = (ConstDouble*)kDp45Coef;
    __device__ __forceinline__ void next()
    {
        if constexpr (LOAD) p = opaque_const(p);
    }
    __device__ __forceinline__ double operator[](int i) const { return LOAD ? p[i] : kDp45[i]; }
};

// The sincos64 coefficients in constant memory: the stage loop reads them once
// per attempt (two scalar loads) through an opaque pointer, and all six
// right-hand sides of the attempt share the loaded values.
__constant__ double kSinCos64Const[16] = {kSinCos64[0],  kSinCos64[1],  kSinCos64[2],  kSinCos64[3],
                                          kSinCos64[4],  kSinCos64[5],  kSinCos64[6],  kSinCos64[7],
                                          kSinCos64[8],  kSinCos64[9],  kSinCos64[10], kSinCos64[11],
                                          kSinCos64[12], kSinCos64[13], kSinCos64[14], kSinCos64[15]};
struct SinCosLoad {
    ConstDouble* p;
    __device__ double operator()(int i) const { return p[i]; }
};

// The angle-shift coefficients, loaded the same way once per attempt.
__constant__ double kShift64Const[6] = {kShift64[0], kShift64[1], kShift64[2], kShift64[3], kShift64[4], kShift64[5]};
struct ShiftLoad {
    ConstDouble* p;
    __device__ double operator()(int i) const { return p[i]; }
};

// The analytic metric's stages load the sine/cosine coefficients; the
// tabulated metric does not evaluate them in its right-hand side.
template <int KIND>
__device__ __forceinline__ auto sincos_source()
{
    if constexpr (KIND == 0)
        return SinCosLoad{opaque_const((ConstDouble*)kSinCos64Const)};
    else
        return SinCosImm{};
}
template <int KIND>
__device__ __forceinline__ void stages64(const Ray& R, const MetricOps<KIND>& M, Spin a, double h, Deriv<double>& y5,
                                         Deriv<double>& k7, Deriv<double>& e, double& H5, double& c5, double& s5)
{
    const Deriv<double>& k1 = R.k;
    Deriv<double> k2, k3, k4, k5, k6;
    double Hd, cd;
    const auto sc = sincos_source<KIND>();
    // stages 2-6 take sin and cos of their polar angle from the step's start
    // where it is within 1/16 and within half of |sin(theta0)| of it (the
    // latter keeps the sine's relative accuracy near the poles)
    const double dmax = fmin(0.0625, 0.5 * fabs(R.sth));
    const ShiftLoad shift{opaque_const((ConstDouble*)kShift64Const)};
#define TT_RHS(th_, r_, pr_, pth_, k_) \
    M.rhs_near(a, r_, th_, R.th, R.sth, R.cth, dmax, pr_, pth_, R.pt, R.pph, k_, Hd, cd, sc, shift)
    Dp45Source<KIND == 0> K;
    K.next();
    {
        const double A21 = K[0];
        TT_RHS(fma(h, A21 * k1.th, R.th), fma(h, A21 * k1.r, R.r), fma(h, A21 * k1.pr, R.pr),
               fma(h, A21 * k1.pth, R.pth), k2);
    }
    K.next();
    {
        const double A31 = K[1], A32 = K[2];
#define TT_S3(c) fma(h, fma(A32, k2.c, A31 * k1.c), R.c)
        TT_RHS(TT_S3(th), TT_S3(r), TT_S3(pr), TT_S3(pth), k3);
    }
    K.next();
    {
        const double A41 = K[3], A42 = K[4], A43 = K[5];
#define TT_S4(c) fma(h, fma(A43, k3.c, fma(A42, k2.c, A41 * k1.c)), R.c)
        TT_RHS(TT_S4(th), TT_S4(r), TT_S4(pr), TT_S4(pth), k4);
    }
    K.next();
    {
        const double A51 = K[6], A52 = K[7], A53 = K[8], A54 = K[9];
#define TT_S5(c) fma(h, fma(A54, k4.c, fma(A53, k3.c, fma(A52, k2.c, A51 * k1.c))), R.c)
        TT_RHS(TT_S5(th), TT_S5(r), TT_S5(pr), TT_S5(pth), k5);
    }
    K.next();
    {
        const double A61 = K[10], A62 = K[11], A63 = K[12], A64 = K[13], A65 = K[14];
#define TT_S6(c) fma(h, fma(A65, k5.c, fma(A64, k4.c, fma(A63, k3.c, fma(A62, k2.c, A61 * k1.c)))), R.c)
        TT_RHS(TT_S6(th), TT_S6(r), TT_S6(pr), TT_S6(pth), k6);
    }
    K.next();
    {
        const double B1 = K[15], B3 = K[16], B4 = K[17], B5 = K[18], B6 = K[19];
#define TT_Y5(c) fma(h, fma(B6, k6.c, fma(B5, k5.c, fma(B4, k4.c, fma(B3, k3.c, B1 * k1.c)))), R.c)
        y5.t = TT_Y5(t);
        y5.r = TT_Y5(r);
        y5.th = TT_Y5(th);
        y5.ph = TT_Y5(ph);
        y5.pr = TT_Y5(pr);
        y5.pth = TT_Y5(pth);
    }
    // the step's end from its own angle: the next step starts from its sin and cos
    M.rhs_sc(a, y5.r, y5.th, y5.pr, y5.pth, R.pt, R.pph, k7, H5, c5, s5, sc);
    K.next();
    {
        const double E1 = K[20], E3 = K[21], E4 = K[22], E5 = K[23], E6 = K[24], E7 = K[25];
#define TT_E(c) h * fma(E7, k7.c, fma(E6, k6.c, fma(E5, k5.c, fma(E4, k4.c, fma(E3, k3.c, E1 * k1.c)))))
        e.t = TT_E(t);
        e.r = TT_E(r);
        e.th = TT_E(th);
        e.ph = TT_E(ph);
        e.pr = TT_E(pr);
        e.pth = TT_E(pth);
    }
#undef TT_RHS
#undef TT_S3
#undef TT_S4
#undef TT_S5
#undef TT_S6
#undef TT_Y5
#undef TT_E
}

// One attempted step of a six-stage pair (Cash-Karp or Fehlberg) with FP64
// stages: the same outputs as stages64.
// Stage slopes of a six-stage pair, by component.
struct SixSlopes {
    double t[6], r[6], th[6], ph[6], pr[6], pth[6];
};

// Stages S..5 of a six-stage pair: the stage argument from the compile-time
// row a[S] (zero weights drop out), then its slope.
template <int KIND, class P, int S, class Coef>
__device__ __forceinline__ void six_stage(const Ray& R, const MetricOps<KIND>& M_, Spin a, double h, SixSlopes& k, Coef sc)
{
    if constexpr (S < 6) {
        using W = RowA<P, S>;
        Deriv<double> ks;
        double Hd, cd;
        M_.rhs(a, fma(h, weighted<W>(k.r), R.r), fma(h, weighted<W>(k.th), R.th), fma(h, weighted<W>(k.pr), R.pr),
               fma(h, weighted<W>(k.pth), R.pth), R.pt, R.pph, ks, Hd, cd, sc);
        k.t[S] = ks.t;
        k.r[S] = ks.r;
        k.th[S] = ks.th;
        k.ph[S] = ks.ph;
        k.pr[S] = ks.pr;
        k.pth[S] = ks.pth;
        six_stage<KIND, P, S + 1>(R, M_, a, h, k, sc);
    }
}

template <int KIND, int M>
__device__ __forceinline__ void stages64_six(const Ray& R, const MetricOps<KIND>& M_, Spin a, double h, Deriv<double>& y5,
                                             Deriv<double>& k7, Deriv<double>& e, double& H5, double& c5, double& s5)
{
    using P = Pair<M>;
    // component-wise stage derivatives k.c[stage] for the dynamic components
    SixSlopes k;
    k.t[0] = R.k.t;
    k.r[0] = R.k.r;
    k.th[0] = R.k.th;
    k.ph[0] = R.k.ph;
    k.pr[0] = R.k.pr;
    k.pth[0] = R.k.pth;
    const auto sc = sincos_source<KIND>();
    six_stage<KIND, P, 1>(R, M_, a, h, k, sc);
    using B = RowB<P>;
    y5.t = fma(h, weighted<B>(k.t), R.t);
    y5.r = fma(h, weighted<B>(k.r), R.r);
    y5.th = fma(h, weighted<B>(k.th), R.th);
    y5.ph = fma(h, weighted<B>(k.ph), R.ph);
    y5.pr = fma(h, weighted<B>(k.pr), R.pr);
    y5.pth = fma(h, weighted<B>(k.pth), R.pth);
    M_.rhs_sc(a, y5.r, y5.th, y5.pr, y5.pth, R.pt, R.pph, k7, H5, c5, s5, sc);
    using E = RowE<P>;
    e.t = h * weighted<E>(k.t);
    e.r = h * weighted<E>(k.r);
    e.th = h * weighted<E>(k.th);
    e.ph = h * weighted<E>(k.ph);
    e.pr = h * weighted<E>(k.pr);
    e.pth = h * weighted<E>(k.pth);
}

// Gragg-Bulirsch-Stoer extrapolation (Sec. 3.2).  A macro-step h is covered
// kGbsColumns times by Gragg's modified midpoint rule, row i (0-based) with
// n_i = 2(i+1) substeps and the final smoothing step; Richardson extrapolation
// in (h/n)^2 (Aitken-Neville) turns row i's midpoint result into
//   T[i][k+1] = T[i][k] + (T[i][k] - T[i-1][k]) / ((n_i / n_{i-k-1})^2 - 1).
// T[K-1][K-1] propagates; T[K-1][K-1] - T[K-1][K-2] is the error estimate, of
// order 2K - 2, so the controller's exponent is -1/(2K - 1).
constexpr int kGbsColumns = 6;

struct GbsWeights {
    double w[kGbsColumns][kGbsColumns - 1];   // 1 / ((n_i / n_{i-k-1})^2 - 1), zero for k >= i
};

constexpr GbsWeights make_gbs_weights()
{
    GbsWeights g{};
    for (int i = 0; i < kGbsColumns; ++i)
        for (int k = 0; k < kGbsColumns - 1; ++k) {
            if (k < i) {
                const double ratio = (double)(2 * (i + 1)) / (double)(2 * (i - k));
                g.w[i][k] = 1.0 / (ratio * ratio - 1.0);
            } else {
                g.w[i][k] = 0.0;
            }
        }
    return g;
}

__constant__ GbsWeights kGbsW = make_gbs_weights();

// Rounding floor of the extrapolation's error estimate: a component whose
// estimate is at most kGbsFloorUlps ulps of the largest increment of that
// component among the sweeps, capped at kGbsFloorTol of its tolerance scale,
// counts as zero.  Far from the hole the truncation error of a macro-step lies
// below the rounding of T[K-1][K-1] - T[K-1][K-2]; a step factor taken from
// that noise would differ between any two correct FP64 evaluations.  The
// threshold sits far above the noise (tens of ulps), so both fall on the same
// side of it; the cap keeps the tolerance's meaning at tight tolerances.
constexpr double kGbsFloorUlps = 262144.0;   // 2^18
constexpr double kGbsFloorTol = 0.01;

__device__ __forceinline__ double gbs_floor(double e, double big, double y0, double y1, double atol, double rtol)
{
    const double fl = fmin(kGbsFloorUlps * 0x1p-52 * big, kGbsFloorTol * fma(rtol, max_abs(y0, y1), atol));
    return fabs(e) <= fl ? 0.0 : e;
}

// One macro-step of the extrapolation with FP64 stages: the same outputs as
// stages64 (y5 = y + T[K-1][K-1], k7 = f(y5), H(y5), cos(theta5), error
// vector with the rounding floor for (atol, rtol); atol = rtol = 0: none).
// The sweeps and the tableau carry increments z - y (the extrapolation is
// linear, so this is the same scheme), which keeps the rounding of the
// estimate at the size of the step's change instead of the state's.
// The row and substep loops are uniform across the wavefront (every lane runs
// the same substep counts), so one inlined right-hand side serves all 42
// substep evaluations.  Rows are folded into the tableau in place, all
// kGbsColumns entries per row: entries past the row's own take a zero weight
// and copy their left neighbour, so register indices stay compile-time.
template <int KIND>
__device__ __forceinline__ void stages64_gbs(const Ray& R, const MetricOps<KIND>& M, Spin a, double h, double atol,
                                             double rtol, Deriv<double>& y5, Deriv<double>& k7, Deriv<double>& e,
                                             double& H5, double& c5, double& s5)
{
    constexpr int K = kGbsColumns;
    double Tt[K], Tr[K], Tth[K], Tph[K], Tpr[K], Tpth[K];
#pragma unroll
    for (int k = 0; k < K; ++k) Tt[k] = Tr[k] = Tth[k] = Tph[k] = Tpr[k] = Tpth[k] = 0.0;
    double bt = 0.0, br = 0.0, bth = 0.0, bph = 0.0, bpr = 0.0, bpth = 0.0;   // largest |sweep increment|
#pragma unroll 1
    for (int i = 0; i < K; ++i) {
        const int n = 2 * (i + 1);
        const double hs = h / (double)n;
        const double h2 = 2.0 * hs;
        // d_0 = 0 (in e_), d_1 = hs f(y) (in o_); d_{m+1} = d_{m-1} + 2 hs f(y + d_m).
        // n is even, so the substeps go in pairs: each pair updates the even
        // then the odd sequence in place, and no value changes registers.
        double et = 0.0, er = 0.0, eth = 0.0, eph = 0.0, epr = 0.0, epth = 0.0;
        double ot = hs * R.k.t, orr = hs * R.k.r, oth = hs * R.k.th;
        double oph = hs * R.k.ph, opr = hs * R.k.pr, opth = hs * R.k.pth;
        Deriv<double> dz;
        for (int m = 1;; m += 2) {
            double Hd, cd;
            M.rhs(a, R.r + orr, R.th + oth, R.pr + opr, R.pth + opth, R.pt, R.pph, dz, Hd, cd);
            et = fma(h2, dz.t, et); er = fma(h2, dz.r, er); eth = fma(h2, dz.th, eth);
            eph = fma(h2, dz.ph, eph); epr = fma(h2, dz.pr, epr); epth = fma(h2, dz.pth, epth);
            M.rhs(a, R.r + er, R.th + eth, R.pr + epr, R.pth + epth, R.pt, R.pph, dz, Hd, cd);
            if (m + 1 == n) break;
            ot = fma(h2, dz.t, ot); orr = fma(h2, dz.r, orr); oth = fma(h2, dz.th, oth);
            oph = fma(h2, dz.ph, oph); opr = fma(h2, dz.pr, opr); opth = fma(h2, dz.pth, opth);
        }
        // smoothing: (d_n + d_{n-1} + hs f(y + d_n)) / 2, with d_n in e_ and d_{n-1} in o_
        double vt = 0.5 * (ot + fma(hs, dz.t, et)), vr = 0.5 * (orr + fma(hs, dz.r, er));
        double vth = 0.5 * (oth + fma(hs, dz.th, eth)), vph = 0.5 * (oph + fma(hs, dz.ph, eph));
        double vpr = 0.5 * (opr + fma(hs, dz.pr, epr)), vpth = 0.5 * (opth + fma(hs, dz.pth, epth));
        bt = fmax(bt, fabs(vt)); br = fmax(br, fabs(vr)); bth = fmax(bth, fabs(vth));
        bph = fmax(bph, fabs(vph)); bpr = fmax(bpr, fabs(vpr)); bpth = fmax(bpth, fabs(vpth));
        // fold into the tableau
#pragma unroll
        for (int k = 0; k < K - 1; ++k) {
            const double w = kGbsW.w[i][k];
            const double ut = fma(vt - Tt[k], w, vt), ur = fma(vr - Tr[k], w, vr);
            const double uth = fma(vth - Tth[k], w, vth), uph = fma(vph - Tph[k], w, vph);
            const double upr = fma(vpr - Tpr[k], w, vpr), upth = fma(vpth - Tpth[k], w, vpth);
            Tt[k] = vt; Tr[k] = vr; Tth[k] = vth; Tph[k] = vph; Tpr[k] = vpr; Tpth[k] = vpth;
            vt = ut; vr = ur; vth = uth; vph = uph; vpr = upr; vpth = upth;
        }
        Tt[K - 1] = vt; Tr[K - 1] = vr; Tth[K - 1] = vth; Tph[K - 1] = vph; Tpr[K - 1] = vpr; Tpth[K - 1] = vpth;
    }
    y5.t = R.t + Tt[K - 1];
    y5.r = R.r + Tr[K - 1];
    y5.th = R.th + Tth[K - 1];
    y5.ph = R.ph + Tph[K - 1];
    y5.pr = R.pr + Tpr[K - 1];
    y5.pth = R.pth + Tpth[K - 1];
    e.t = gbs_floor(Tt[K - 1] - Tt[K - 2], bt, R.t, y5.t, atol, rtol);
    e.r = gbs_floor(Tr[K - 1] - Tr[K - 2], br, R.r, y5.r, atol, rtol);
    e.th = gbs_floor(Tth[K - 1] - Tth[K - 2], bth, R.th, y5.th, atol, rtol);
    e.ph = gbs_floor(Tph[K - 1] - Tph[K - 2], bph, R.ph, y5.ph, atol, rtol);
    e.pr = gbs_floor(Tpr[K - 1] - Tpr[K - 2], bpr, R.pr, y5.pr, atol, rtol);
    e.pth = gbs_floor(Tpth[K - 1] - Tpth[K - 2], bpth, R.pth, y5.pth, atol, rtol);
    M.rhs_sc(a, y5.r, y5.th, y5.pr, y5.pth, R.pt, R.pph, k7, H5, c5, s5);
}

// Verlet (Sec. 3.2): a fixed step of the generalized Stormer-Verlet scheme for
// the non-separable H(x, p) = 1/2 g^{ab}(x) p_a p_b, symmetric and symplectic:
//   p' = p - (h/2) dH/dx(x, p')                      (implicit in p')
//   x+ = x + (h/2) [dH/dp(x, p') + dH/dp(x+, p')]    (implicit in x+)
//   p+ = p' - (h/2) dH/dx(x+, p')
// Both implicit stages iterate to a fixed point from an explicit predictor,
// stopping once the largest change of a component is at most 1e-14 of
// max(1, largest component).  p_t and p_phi never change (dH/dt = dH/dphi = 0)
// but enter the size of the momenta.  Returns false when a stage has not
// converged after kVerletMaxIter iterations (near the horizon, where dH/dx
// grows like 1/Delta, the stage has no solution close to the current state
// for a fixed step).  Lanes iterate independently; the loops end for every
// lane after at most kVerletMaxIter passes.
constexpr int kVerletMaxIter = 50;
constexpr double kVerletTol = 1e-14;

template <int KIND>
__device__ __forceinline__ bool stages_verlet(const Ray& R, const MetricOps<KIND>& M, Spin a, double h, Deriv<double>& y5,
                                              Deriv<double>& k7, double& H5, double& c5, double& s5)
{
    const double hh = 0.5 * h;
    Deriv<double> d;
    double Hd, cd;
    // stage 1
    double pr = fma(hh, R.k.pr, R.pr), pth = fma(hh, R.k.pth, R.pth);
    const double pconst = fmax(fabs(R.pt), fabs(R.pph));
    bool conv = false;
    for (int it = 0; it < kVerletMaxIter && !conv; ++it) {
        M.rhs(a, R.r, R.th, pr, pth, R.pt, R.pph, d, Hd, cd);
        const double npr = fma(hh, d.pr, R.pr), npth = fma(hh, d.pth, R.pth);
        const double dmax = fmax(fabs(npr - pr), fabs(npth - pth));
        const double vmax = fmax(fmax(fabs(npr), fabs(npth)), pconst);
        pr = npr;
        pth = npth;
        // fmax drops a NaN operand: a non-finite iterate never counts as converged
        conv = isfinite(npr) && isfinite(npth) && dmax <= kVerletTol * fmax(1.0, vmax);
    }
    if (!conv) return false;
    // stage 2
    M.rhs(a, R.r, R.th, pr, pth, R.pt, R.pph, d, Hd, cd);
    const double v0t = d.t, v0r = d.r, v0th = d.th, v0ph = d.ph;
    double xt = fma(h, v0t, R.t), xr = fma(h, v0r, R.r), xth = fma(h, v0th, R.th), xph = fma(h, v0ph, R.ph);
    conv = false;
    for (int it = 0; it < kVerletMaxIter && !conv; ++it) {
        M.rhs(a, xr, xth, pr, pth, R.pt, R.pph, d, Hd, cd);
        const double nt = fma(hh, v0t + d.t, R.t), nr = fma(hh, v0r + d.r, R.r);
        const double nth = fma(hh, v0th + d.th, R.th), nph = fma(hh, v0ph + d.ph, R.ph);
        const double dmax = fmax(fmax(fabs(nt - xt), fabs(nr - xr)), fmax(fabs(nth - xth), fabs(nph - xph)));
        const double vmax = fmax(fmax(fabs(nt), fabs(nr)), fmax(fabs(nth), fabs(nph)));
        xt = nt;
        xr = nr;
        xth = nth;
        xph = nph;
        conv = isfinite(nt) && isfinite(nr) && isfinite(nth) && isfinite(nph) &&
               dmax <= kVerletTol * fmax(1.0, vmax);
    }
    if (!conv) return false;
    // stage 3
    M.rhs(a, xr, xth, pr, pth, R.pt, R.pph, d, Hd, cd);
    y5.t = xt;
    y5.r = xr;
    y5.th = xth;
    y5.ph = xph;
    y5.pr = fma(hh, d.pr, pr);
    y5.pth = fma(hh, d.pth, pth);
    M.rhs_sc(a, y5.r, y5.th, y5.pr, y5.pth, R.pt, R.pph, k7, H5, c5, s5);
    return true;
}

// Scaled error of one component, e / (atol + rtol max(|y0|, |y1|)).
__device__ __forceinline__ double err_ratio(double e, double y0, double y1, double atol, double rtol)
{
    return e * rcp64_coarse(fma(rtol, max_abs(y0, y1), atol));
}

// Sum of squares of the six scaled errors, the first squared and the others
// added by fused multiply-adds in this order.  (Written out, z0 z0 + z1 z1 lets
// the compiler fuse either product, and which one it picks can change with
// unrelated code; the explicit form rounds the same in every build.)
__device__ __forceinline__ double sum_sq6(double z0, double z1, double z2, double z3, double z4, double z5)
{
    return fma(z5, z5, fma(z4, z4, fma(z3, z3, fma(z2, z2, fma(z1, z1, z0 * z0)))));
}

// Rounding floor of an embedded pair's error estimate.  The estimate
// h sum_j (b_j - b*_j) k_j of a component rounds to a few ulps of
// h |b - b*|_1 max(|k_n|, |k_n+1|); far from the hole the first steps'
// estimates are that rounding alone (a ~1e9-fold cancellation in the angular
// components), and a step factor taken from them differs between two correct
// FP64 evaluations by ~1e-7, enough for a later estimate to fall on the other
// side of 1.  A component whose estimate is at most kPairFloorUlps of that
// scale, capped at kPairFloorTol of its tolerance scale, counts as zero.
constexpr double kPairFloorUlps = 262144.0;   // 2^18
constexpr double kPairFloorTol = 0.01;

template <int M>
struct PairErrNorm1;
template <>
struct PairErrNorm1<METHOD_DP45> {
    static constexpr double value = E1 - E3 + E4 - E5 + E6 - E7;   // |b - b*|_1
};
template <int M>
struct PairErrNorm1 {
    static constexpr double sum(int j) { return j == 6 ? 0.0 : (Pair<M>::e[j] < 0 ? -Pair<M>::e[j] : Pair<M>::e[j]) + sum(j + 1); }
    static constexpr double value = sum(0);
};

// Scaled error of one component with the rounding floor: contributes nothing
// to the sum of squares when |e| <= min(c max(|k0|, |k1|), kPairFloorTol sc),
// c = kPairFloorUlps ulp |b - b*|_1 |h|.  A floored ratio keeps its low word
// and loses its high word, a subnormal below 2^-1022 whose square, and so its
// term in sum_sq6, rounds to exactly zero: one select instead of two.
__device__ __forceinline__ double err_ratio_floor(double e, double c, double k0, double k1, double y0, double y1,
                                                  double atol, double rtol)
{
    const double sc = fma(rtol, max_abs(y0, y1), atol);
    const double fl = fmin(c * max_abs(k0, k1), kPairFloorTol * sc);
    const double z = e * rcp64_coarse(sc);
    return __hiloint2double(fabs(e) <= fl ? 0 : __double2hiint(z), __double2loint(z));
}

// y^N for a compile-time N >= 1 by repeated squaring.
template <int N>
__device__ __forceinline__ double ipow(double y)
{
    if constexpr (N == 1) {
        return y;
    } else if constexpr (N % 2 == 0) {
        const double h = ipow<N / 2>(y);
        return h * h;
    } else {
        return ipow<N - 1>(y) * y;
    }
}

// x^(-1/P) on the range step_factor passes in: an FP32 estimate refined by
// two Newton steps on y^-P = x (y <- y ((P + 1) - x y^P) / P), which take the
// ~1e-7 relative error of the estimate below an ulp of the double result.
// The estimate uses the hardware log2 and exp2 directly: x, its logarithm
// scaled by -1/P and the result are normal floats there (x in [1e-24, 1e16]),
// where the library functions' denormal handling returns the same values.
template <int P>
__device__ __forceinline__ double pow_m_inv(double x)
{
    double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)x) * (-1.0f / (float)P));
#pragma unroll
    for (int i = 0; i < 2; ++i) y = y * fma(-x, ipow<P>(y), (double)(P + 1)) * (1.0 / (double)P);
    return y;
}

// Step-size factor of the elementary controller from the squared error norm
// err2 = err^2: min(fmx, max(0.2, 0.9 err^(-1/P))) = min(fmx, max(0.2,
// 0.9 err2^(-1/(2P)))), P = 5 for the 5(4) pairs and 2K - 1 for the
// extrapolation (working on err^2 saves the square root).  The power is taken
// of err2 clamped to [1e-24, 1e16], the range its estimate covers: at the ends
// 0.9 err2^(-1/(2P)) is at least 11 and at most 0.17 for both P, beyond the
// factor's own clamps, so clamping err2 never changes the factor and no branch
// is needed.  fmin drops a NaN operand, so a NaN err2 clamps to the upper end
// and gets the smallest factor, 0.2.
template <int P>
__device__ __forceinline__ double step_factor(double err2, double fmx)
{
    const double x = fmax(fmin(err2, 1e16), 1e-24);
    return fmin(fmx, fmax(0.2, 0.9 * pow_m_inv<2 * P>(x)));
}

// Event search of the extrapolation.  A macro-step spans up to hundreds of M,
// over which the step's cubic Hermite interpolant is accurate to ~1e-3 only,
// so an event root is located on the method's own solution: a probe at s is
// one macro-step of length s h from the step's start (the same sweeps and
// columns, without error control).  The search runs across iterations of the
// persistent loop: after an accepted macro-step with an event the ray stays at
// the step's start, and each of its following iterations is one probe through
// the same stages64_gbs call as an attempt, so a wavefront runs that code once
// per iteration whatever its lanes are doing (a probe inside the attempt's
// iteration would run with one lane active while the others wait).  Newton's
// method from the cubic's root, safeguarded by the bracket [lo, hi] (the start
// side at lo): the terminal root first, then an equatorial crossing in the
// same step (it counts when it is not after the terminal root); after a
// crossing that does not end the ray, a last probe at s = 1 rebuilds the
// step's end, bit for bit as the attempt produced it, and the ray advances.
struct GbsSearch {
    double h;          // the accepted macro-step being searched
    double lo, hi, s;  // bracket and current probe, in units of h
    double target;     // radial target of the terminal event
    double fac;        // the controller's factor for the step after it
    double s_disk;     // the cubic's equatorial root: where the disk search starts
    int phase;         // 0 attempts; 1 terminal root; 2 equatorial root; 3 rebuild the step's end
    int flags;         // 1 horizon, 2 escape, 4 equator crossed; probes of this search above bit 8
};
constexpr int kGbsMaxProbes = 64;

__device__ __forceinline__ void gbs_search_start(GbsSearch& S, double s0)
{
    S.lo = 0.0;
    S.hi = 1.0;
    S.s = (s0 > 0.0 && s0 <= 1.0) ? s0 : 0.5;
    S.flags &= 0xff;
}

// The ray moves to the end of its accepted step.
__device__ __forceinline__ void advance(Ray& R, double h, double fac, const Deriv<double>& y5, const Deriv<double>& k7,
                                        double c5, double s5, bool used32)
{
    R.lam += h;
    R.t = y5.t;
    R.r = y5.r;
    R.th = y5.th;
    R.ph = y5.ph;
    R.pr = y5.pr;
    R.pth = y5.pth;
    R.k = k7;
    R.k32 = used32 ? 1 : 0;
    R.cth = c5;
    R.sth = s5;
    R.h = h * fac;
    R.rej_prev = 0;
}

// One probe of an event search, with the solution y at s and its slope k.
// Returns true when the ray has ended.
__device__ bool gbs_probe(Ray& R, GbsSearch& S, const LaunchArgs& A, const RaySettings& P, const Deriv<double>& y,
                          const Deriv<double>& k, double c, double s_end)
{
    if (S.phase == 3) {
        advance(R, S.h, S.fac, y, k, c, s_end, false);
        S.phase = 0;
        return false;
    }
    const bool disk = S.phase == 2;
    double g, dg;
    if (disk) {
        double sn, cs;
        sincos64(y.th, &sn, &cs);
        g = cs;
        dg = -sn * k.th * S.h;
    } else {
        g = y.r - S.target;
        dg = k.r * S.h;
    }
    const bool above = disk ? R.cth > 0.0 : R.r - S.target > 0.0;
    if (above ? g > 0.0 : g < 0.0)
        S.lo = S.s;
    else
        S.hi = S.s;
    double sn = S.s - g / dg;
    if (!(sn > S.lo && sn < S.hi)) sn = 0.5 * (S.lo + S.hi);   // also a zero or non-finite slope
    const double tol = 0.125 * P.event_tol;
    S.flags += 256;
    if (!(fabs(sn - S.s) * S.h <= tol || (S.hi - S.lo) * S.h <= tol || (S.flags >> 8) >= kGbsMaxProbes)) {
        S.s = sn;
        return false;
    }
    // the root is S.s, within tol in lambda; y is the solution there
    const int cls = (S.flags & 1) ? CLS_CAPTURED : CLS_ESCAPED;
    double* term = R.rec + REC_TERM;
    if (!disk) {
        term[0] = y.r;
        term[4] = y.th;
        term[8] = y.ph;
        term[13] = S.s;
        if (S.flags & 4) {
            S.phase = 2;
            gbs_search_start(S, S.s_disk);
            return false;
        }
        ray_finish(R, A, cls, 0);
        return true;
    }
    const bool terminal = (S.flags & 3) != 0;
    if (!terminal || S.s <= term[13]) {
        R.n_cross++;
        if (y.r >= R.r_in && y.r <= R.r_out && R.n_hits < R.max_hits) {
            double* sl = R.rec + REC_SLOT0 + REC_SLOT_LEN * R.n_hits;
            sl[0] = y.r;
            sl[8] = 0.0;
            sl[9] = fma(S.s, S.h, R.lam);
            reinterpret_cast<int*>(R.rec + REC_INTS)[6 + R.n_hits] = R.n_cross;
            R.n_hits++;
            if (R.opaque) {
                term[0] = y.r;
                term[4] = y.th;
                term[8] = y.ph;
                ray_finish(R, A, CLS_ON_DISK, 0);
                return true;
            }
        }
    }
    if (terminal) {
        ray_finish(R, A, cls, 0);
        return true;
    }
    S.phase = 3;
    S.s = 1.0;
    return false;
}

// The largest power of two not above x (x > 0, finite): the extrapolation's
// step factor, so its steps stay h0 2^k and an estimate's rounding moves them
// only where it straddles a power-of-two boundary of the factor.
__device__ __forceinline__ double pow2_floor(double x)
{
    return __longlong_as_double(__double_as_longlong(x) & (long long)0xfff0000000000000ull);
}

// One attempt; returns true when the ray has terminated (outputs written).
// (S: the extrapolation's event search; unused by the other methods.)
template <int KIND, int PREC, int METHOD, int SERVE>
__device__ bool ray_step(Ray& R, GbsSearch& S, const LaunchArgs& A, const RaySettings& P, const MetricOps<KIND>& M,
                         const TraceUniform& U)
{
    // a one-shot trace's rays share the metric and the solver: their spin
    // constants and radii come wave-uniform from the launch
    const Spin K = SERVE ? spin_of(R.a) : U.spin;
    bool probe = false;
    if constexpr (METHOD == METHOD_GBS) probe = S.phase != 0;
    if (!probe && R.n_acc + R.n_rej >= P.max_steps) {
        ray_fail(R, A);
        return true;
    }
    const double h = probe ? S.s * S.h : R.h;
    Deriv<double> y5, k7, e;
    double H5, c5, s5;
    bool used32 = false;
    double fac = 1.0;
    if constexpr (METHOD == METHOD_VERLET) {
        // fixed step, no error control: a converged step is always taken
        if (!stages_verlet<KIND>(R, M, K, h, y5, k7, H5, c5, s5)) {
            ray_fail(R, A);
            return true;
        }
    } else {
        if (PREC == 1 && KIND == 0 && far_field(R, A, P)) {
            stages32(R, h, y5, k7, e, H5, c5, s5);
            used32 = true;
        } else {
            if (PREC == 1 && R.k32) {
                // leaving the FP32 regime: re-evaluate the first stage in FP64
                double Hd;
                M.rhs_sc(K, R.r, R.th, R.pr, R.pth, R.pt, R.pph, R.k, Hd, R.cth, R.sth);
                R.k32 = 0;
            }
            if constexpr (METHOD == METHOD_DP45)
                stages64<KIND>(R, M, K, h, y5, k7, e, H5, c5, s5);
            else if constexpr (METHOD == METHOD_GBS)
                // one call site for attempts and probes (a probe has no error control)
                stages64_gbs<KIND>(R, M, K, h, probe ? 0.0 : P.atol, probe ? 0.0 : P.rtol, y5, k7, e, H5, c5, s5);
            else
                stages64_six<KIND, METHOD>(R, M, K, h, y5, k7, e, H5, c5, s5);
        }
        if constexpr (METHOD == METHOD_GBS) {
            if (probe) return gbs_probe(R, S, A, P, y5, k7, c5, s5);
        }
        R.n_f32 += used32 ? 1 : 0;
        const double atol = P.atol, rtol = P.rtol;
        double acc;
        if constexpr (METHOD == METHOD_GBS) {
            // (the extrapolation applies its own floor in stages64_gbs)
            acc = sum_sq6(err_ratio(e.t, R.t, y5.t, atol, rtol), err_ratio(e.r, R.r, y5.r, atol, rtol),
                          err_ratio(e.th, R.th, y5.th, atol, rtol), err_ratio(e.ph, R.ph, y5.ph, atol, rtol),
                          err_ratio(e.pr, R.pr, y5.pr, atol, rtol), err_ratio(e.pth, R.pth, y5.pth, atol, rtol));
        } else {
            const double c = kPairFloorUlps * 0x1p-52 * PairErrNorm1<METHOD>::value * fabs(h);
            acc = sum_sq6(err_ratio_floor(e.t, c, R.k.t, k7.t, R.t, y5.t, atol, rtol),
                          err_ratio_floor(e.r, c, R.k.r, k7.r, R.r, y5.r, atol, rtol),
                          err_ratio_floor(e.th, c, R.k.th, k7.th, R.th, y5.th, atol, rtol),
                          err_ratio_floor(e.ph, c, R.k.ph, k7.ph, R.ph, y5.ph, atol, rtol),
                          err_ratio_floor(e.pr, c, R.k.pr, k7.pr, R.pr, y5.pr, atol, rtol),
                          err_ratio_floor(e.pth, c, R.k.pth, k7.pth, R.pth, y5.pth, atol, rtol));
        }
        // p_t and p_phi have zero error (their derivatives vanish identically)
        const double err2 = acc * 0.125;   // squared RMS error over the 8 components
        // elementary controller, evaluated once for both outcomes: after a
        // rejection (or for one) the step may not grow
        const bool ok = err2 <= 1.0;
        constexpr int P = METHOD == METHOD_GBS ? 2 * kGbsColumns - 1 : 5;
        fac = step_factor<P>(err2, (ok && !R.rej_prev) ? 10.0 : 1.0);   // 0.2 for a NaN err2
        if constexpr (METHOD == METHOD_GBS) fac = pow2_floor(fac);
        if (!ok) {
            // rejected; a NaN or infinite error also lands here
            R.n_rej++;
            R.h = h * fac;
            R.rej_prev = 1;
            if (R.h < 1e-14 * fmax(1.0, fabs(R.lam))) {
                ray_fail(R, A);
                return true;
            }
            return false;
        }
    }
    R.n_acc++;
    if (!(isfinite(y5.t) && isfinite(y5.r) && isfinite(y5.th) && isfinite(y5.ph) && isfinite(y5.pr) &&
          isfinite(y5.pth))) {
        ray_fail(R, A);
        return true;
    }

    // ---- constraint residual (Eq. (17)) at the accepted state
    const double aH = fabs(H5);
    R.hmax = max_abs(R.hmax, aH);   // (both non-negative)
    if (y5.r >= (SERVE ? 1.5 * R.rp : U.gate_r)) R.hgate = max_abs(R.hgate, aH);

    // ---- events on the accepted step [lam, lam + h]
    double r_stop = U.r_stop;
    if constexpr (SERVE) {
        r_stop = P.horizon_factor * R.rp;
        if (KIND == 1 && A.tab_r_min > r_stop) r_stop = A.tab_r_min;
    }
    const double r_esc = P.r_escape;
    const bool hz = (R.r - r_stop > 0.0) && (y5.r - r_stop <= 0.0);
    const bool es = (R.r - r_esc < 0.0) && (y5.r - r_esc >= 0.0);
    const bool dk = R.max_hits > 0 && ((R.cth > 0.0 && c5 <= 0.0) || (R.cth < 0.0 && c5 >= 0.0));
    if constexpr (METHOD == METHOD_GBS) {
        if (hz | es | dk) {
            // the ray stays at the step's start while its events are searched
            S.h = h;
            S.fac = fac;
            S.flags = (hz ? 1 : 0) | (es ? 2 : 0) | (dk ? 4 : 0);
            S.s_disk = 0.5;
            if (dk) S.s_disk = equator_root(Cubic(R.th, R.k.th, y5.th, k7.th, h), R.th, y5.th, R.cth, h, 1e-6 * h);
            if (hz | es) {
                S.phase = 1;
                S.target = hz ? r_stop : r_esc;
                gbs_search_start(S, locate_root(Cubic(R.r, R.k.r, y5.r, k7.r, h), S.target, hz, h, 1e-6 * h));
            } else {
                S.phase = 2;
                gbs_search_start(S, S.s_disk);
            }
            return false;
        }
    } else if (hz | es) {
        // terminal step: the finishing pass locates the root (and a crossing
        // of the equator before it) on the step's cubics; at most one radial
        // event brackets a root in one step
        terminal_step(R, h, y5, k7, hz ? r_stop : r_esc);
        ray_finish(R, A, hz ? CLS_CAPTURED : CLS_ESCAPED, (hz ? 1 : 2) | (dk ? 4 : 0));
        return true;
    }
    if (METHOD != METHOD_GBS && dk) {
        if (R.opaque) {
            if (opaque_hit(R, h, y5, k7, 0.125 * P.event_tol)) {
                terminal_step(R, h, y5, k7, 0.0);
                ray_finish(R, A, CLS_ON_DISK, 8);
                return true;
            }
        } else {
            disk_crossing(R, h, y5, k7, 0.125 * P.event_tol);
        }
    }

    advance(R, h, fac, y5, k7, c5, s5, used32);
    return false;
}

__device__ __forceinline__ unsigned long long lanemask_lt()
{
    const unsigned int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

static_assert(sizeof(Ray) % sizeof(double) == 0 && sizeof(GbsSearch) % sizeof(double) == 0, "parked in doubles");
static_assert(sizeof(Ray) + sizeof(GbsSearch) <= SLOT_DOUBLES * sizeof(double), "parked ray state must fit a slot");

// A lane's ray, and for the extrapolation its event search, to and from its slot.
template <int METHOD>
__device__ __forceinline__ void park(const Ray& R, const GbsSearch& S, double* slot)
{
    const double* src = reinterpret_cast<const double*>(&R);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Ray) / sizeof(double)); ++i) slot[i] = src[i];
    if constexpr (METHOD == METHOD_GBS) {
        const double* ss = reinterpret_cast<const double*>(&S);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(GbsSearch) / sizeof(double)); ++i) slot[sizeof(Ray) / sizeof(double) + i] = ss[i];
    }
}

template <int METHOD>
__device__ __forceinline__ void unpark(Ray& R, GbsSearch& S, const double* slot)
{
    double* dst = reinterpret_cast<double*>(&R);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Ray) / sizeof(double)); ++i) dst[i] = slot[i];
    if constexpr (METHOD == METHOD_GBS) {
        double* sd = reinterpret_cast<double*>(&S);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(GbsSearch) / sizeof(double)); ++i) sd[i] = slot[sizeof(Ray) / sizeof(double) + i];
    }
}

// Serving: the rays of each job still to finish are counted down on the
// device.  Lanes whose ray ended this iteration (finished, failed or dropped
// with a cancelled job) carry its job in `done`; one atomic per job and
// wavefront iteration subtracts them, instead of one per ray on a single
// counter.
__device__ __forceinline__ void count_done(const LaunchArgs& A, int& done)
{
    unsigned long long m = __ballot(done >= 0);
    while (m) {
        const int leader = __ffsll((long long)m) - 1;
        const int j = __shfl(done, leader);
        const unsigned long long same = __ballot(done == j);
        if ((int)__lane_id() == leader) atomicSub(A.remaining + j * kRemainingStride, (unsigned int)__popcll(same));
        if (done == j) done = -1;
        m &= ~same;
    }
}

// SERVE = 1: the serving epochs' instance, which resumes parked rays, parks
// those that use up the epoch's attempt budget and counts finished rays down per
// request; SERVE = 0: one-shot traces, without that machinery (a ray that can
// be parked at any iteration keeps every field of its state live, 190 VGPRs
// against 160 for the Dormand-Prince FP64 instance).
//
// Occupancy target: at most 2 waves per SIMD (up to 256 VGPRs), or 3 (168) for
// the one-shot analytic Dormand-Prince instances: the FP64 one fits without
// spills; the mixed one spills 13 VGPRs outside its stage blocks and still runs
// 6 % faster at 3 waves than at 2 on a 2048x2048 image.  One wave per SIMD is
// fastest on small images (a lone wavefront keeps the long rays' critical path
// short); more give large images more throughput.  The autotuner picks.
template <int KIND, int PREC, int METHOD, int SERVE>
struct WavesPerEU {
    static constexpr int value = (!SERVE && KIND == 0 && METHOD == METHOD_DP45) ? 3 : 2;
};

template <int KIND, int PREC, int METHOD, int SERVE>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(WavesPerEU<KIND, PREC, METHOD, SERVE>::value))) trace_persistent(LaunchArgs A)
{
    MetricOps<KIND> M;
    if (KIND == 1) {
        M.T = make_table_view(A.table, A.nr, A.nth, A.tab_r_min, A.tab_r_max);
        M.T.inter = A.table_inter;
    }
    // job directory in LDS
    __shared__ long long s_begin[kLdsJobs];
    __shared__ int s_job[kLdsJobs];
    JobDir D;
    D.n = A.dir_begin ? A.ndir : A.njobs;
    D.begin = nullptr;
    D.job = nullptr;
    if (D.n <= kLdsJobs) {
        for (int i = threadIdx.x; i < D.n; i += blockDim.x) {
            s_begin[i] = A.dir_begin ? A.dir_begin[i] : A.jobs[i].ray_begin;
            s_job[i] = A.dir_begin ? A.dir_job[i] : i;
        }
        __syncthreads();
        D.begin = s_begin;
        D.job = s_job;
    }
    Ray R;
    GbsSearch S;
    S.phase = 0;
    RaySettings P = launch_settings(A);   // serving: each ray's request's, set with the ray
    TraceUniform U{};
    if constexpr (!SERVE) U = trace_uniform(A);
    bool active = false;
    bool parked = false;       // serving: this launch's epoch has ended for the lane
    bool exhausted = false;
    int done = -1;             // serving: job of a ray that ended this iteration
    long long iter = 0;        // serving: wavefront iterations with work this launch
    const long long slot = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if constexpr (SERVE) {
        if (A.slots && A.slot_live[slot]) {
            unpark<METHOD>(R, S, A.slots + slot * SLOT_DOUBLES);
            A.slot_live[slot] = 0u;
            P = job_settings(A.jobs[R.job]);
            active = !A.jobs[R.job].cancelled;
            if (!active) done = R.job;
        }
        if (A.remaining) count_done(A, done);
    }
    // this wavefront's current chunk of ray ids [next, end) (wave-uniform values)
    long long next = 0, end = 0;
    const long long n_rays = A.total_rays - A.first_ray;
    for (;;) {
        if (__any(active)) {
            if (active) {
                active = !ray_step<KIND, PREC, METHOD, SERVE>(R, S, A, P, M, U);
                if (!active) done = R.job;
            }
            if constexpr (SERVE) {
                // An epoch is step_budget iterations of the wavefront: then every
                // lane parks its ray at once.  (A per-lane attempt budget let
                // lanes that had waited for a refill run on alone at the end of
                // the epoch, with the rest of the wavefront idle.)
                if (A.slots && A.step_budget > 0 && ++iter >= A.step_budget) {
                    if (active) {
                        park<METHOD>(R, S, A.slots + slot * SLOT_DOUBLES);
                        A.slot_live[slot] = 1u;
                        active = false;
                    }
                    parked = true;
                }
                if (A.remaining) count_done(A, done);
            }
        }
        if (!exhausted) {
            const unsigned long long need = __ballot(!active && !parked);
            const int nneed = __popcll(need);
            if (nneed > 0 && (nneed >= A.refill_min || !__any(active))) {
                const int rank = __popcll(need & lanemask_lt());
                long long id = -1;
                const long long avail = end - next;
                if (!active && !parked && rank < avail) id = next + rank;
                const int taken = (int)(avail < nneed ? avail : nneed);
                next += taken;
                const int rem = nneed - taken;
                if (rem > 0) {
                    // One-shot traces fetch a chunk and keep the rest for later
                    // refills.  In serving epochs a wavefront may exit with all
                    // lanes parked, so it fetches exactly the ids it hands out:
                    // an id taken from the queue is never left unassigned.
                    const long long fetch = (SERVE && A.slots) ? (long long)rem : (A.chunk > rem ? A.chunk : rem);
                    const int leader = __ffsll((long long)need) - 1;
                    unsigned long long c0 = 0;
                    if ((int)__lane_id() == leader) c0 = atomicAdd(A.head, (unsigned long long)fetch);
                    c0 = __shfl(c0, leader);
                    if ((long long)c0 >= n_rays) {
                        exhausted = true;
                        next = end = 0;
                    } else {
                        next = (long long)c0;
                        end = next + fetch < n_rays ? next + fetch : n_rays;
                        const long long r2 = rank - taken;
                        if (!active && !parked && r2 >= 0 && r2 < end - next) id = next + r2;
                        const long long got = (end - next) < rem ? (end - next) : rem;
                        next += got;
                    }
                }
                if (id >= 0) {
                    long long gid;
                    if (A.nseg > 0) {
                        gid = segment_ray(A, id);
                    } else {
                        if (A.order) id = (long long)A.order[id];
                        gid = A.first_ray + id;
                    }
                    active = ray_init<KIND>(R, gid, A, D, M);
                    if constexpr (SERVE) P = job_settings(A.jobs[R.job]);
                    S.phase = 0;
                    if (!active) done = R.job;
                }
                if constexpr (SERVE) {
                    if (A.remaining) count_done(A, done);
                }
            }
        }
        if (!__any(active)) {
            if (exhausted || !__any(!parked)) break;
        }

    }
}

// ---------------------------------------------------------------------------
// finishing pass: event roots, outputs, and shading (g and g^4 F(r))
// ---------------------------------------------------------------------------
// int32 field i of a record header held in registers (REC_INTS: two per
// double, the lower address in the low half).
__device__ __forceinline__ int rec_int(const double* hd, int i)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(hd[REC_INTS + (i >> 1)]);
    return (int)(unsigned)((i & 1) ? (b >> 32) : b);
}

// One thread per ray.  Locates the crossings and the terminal root the
// integrator left in the ray's record (same cubics and root finders as on the
// integrator side, so the results do not depend on where a root was found),
// writes every output of the ray, then shades its disk hits with Eqs. (11)
// and (15).  blockIdx.y selects the job (job0 + blockIdx.y); x covers its rays.
__global__ void finish_kernel(const DevJob* jobs, const JobConst* jc, int job0)
{
    const int jb = job0 + blockIdx.y;
    const DevJob& J = jobs[jb];
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= J.ray_count) return;
    if (J.cancelled) return;
    const JobConst& C = jc[jb];
    const double* rec = J.rec + q * REC_DOUBLES;
    // the header as one run of 16-byte loads issued together, so each of its
    // two lines is fetched once (reads spread over the code below would let
    // other waves evict a line between them)
    double hd[REC_HEAD];
#pragma unroll
    for (int i = 0; i < REC_HEAD; i += 2) {
        const double2 v = *reinterpret_cast<const double2*>(rec + i);
        hd[i] = v.x;
        hd[i + 1] = v.y;
    }
    const double tol = 0.125 * J.event_tol;
    int n = rec_int(hd, 1);
    int n_cross = rec_int(hd, 5);
    double hr[3] = {0.0, 0.0, 0.0}, hl[3] = {0.0, 0.0, 0.0};
    int ho[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= n) break;
        const double* sl = rec + REC_SLOT0 + REC_SLOT_LEN * k;
        if (sl[8] > 0.0) {
            const double h = sl[8];
            const Cubic pth(sl[4], sl[5], sl[6], sl[7], h);
            const double sd = equator_root(pth, sl[4], sl[6], sl[10], h, tol);
            hr[k] = Cubic(sl[0], sl[1], sl[2], sl[3], h).at(sd);
            hl[k] = fma(sd, h, sl[9]);
        } else {
            hr[k] = sl[0];
            hl[k] = sl[9];
        }
        ho[k] = rec_int(hd, 6 + k);
    }
    const double* t = hd + REC_TERM;
    const int code = (int)hd[REC_CODE];
    int cls = rec_int(hd, 0);
    double fr = t[0], fth = t[4], fph = t[8];
    if (code & 11) {
        const double h = t[12];
        const Cubic pr(t[0], t[1], t[2], t[3], h);
        const Cubic pth(t[4], t[5], t[6], t[7], h);
        // code 8: the crossing itself ends the ray (opaque disk); it was
        // counted in the integrator and lies on the disk
        double s_end = (code & 8) ? equator_root(pth, t[4], t[6], t[15], h, tol)
                                  : locate_root(pr, t[14], (code & 3) == 1, h, tol);
        bool hit = (code & 8) != 0;
        double s_disk = s_end;
        if (code & 4) {
            // a crossing at or before the terminal root counts, one after it does not
            s_disk = equator_root(pth, t[4], t[6], t[15], h, tol);
            if (s_disk <= s_end) {
                n_cross++;
                const double rr = pr.at(s_disk);
                hit = n < J.max_hits && rr >= C.r_in && rr <= J.disk_r_out;
                if (hit && (J.disk_flags & DISK_OPAQUE)) {
                    // the opaque disk comes first: the ray ends on it
                    s_end = s_disk;
                    cls = CLS_ON_DISK;
                }
            }
        }
        if (hit) {
            const double rr = pr.at(s_disk);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k == n) {
                    hr[k] = rr;
                    hl[k] = fma(s_disk, h, t[13]);
                    ho[k] = n_cross;
                }
            n++;
        }
        fr = pr.at(s_end);
        fth = pth.at(s_end);
        fph = Cubic(t[8], t[9], t[10], t[11], h).at(s_end);
    }
    J.cls[q] = cls;
    J.n_hits[q] = n;
    J.final_rtp[3 * q + 0] = fr;
    J.final_rtp[3 * q + 1] = fth;
    J.final_rtp[3 * q + 2] = fph;
    J.h_drift[q] = hd[REC_HMAX];
    J.h_gate[q] = hd[REC_HGATE];
    J.n_accept[q] = rec_int(hd, 2);
    J.n_reject[q] = rec_int(hd, 3);
    J.n_fp32[q] = rec_int(hd, 4);
    J.n_cross[q] = n_cross;
    double inten = 0.0;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    if (n > 0) {
        double al, be;
        pixel_coords(J, q, al, be);
        pixel_momentum(C, J.r_obs, al, be, p);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double g = 0.0, flux = 0.0;
        if (k < n) {
            g = redshift(J.a, hr[k], p[0], p[3]);
            const double F = nt_flux_pre(J.a, C.x0, C.xi, C.coef, hr[k]);
            const double g2 = g * g;
            flux = (J.disk_flags & DISK_INTRINSIC) ? F : g2 * g2 * F;
            inten += flux;
        }
        J.hit_r[3 * q + k] = hr[k];
        J.hit_g[3 * q + k] = g;
        J.hit_flux[3 * q + k] = flux;
        J.hit_lambda[3 * q + k] = hl[k];
        J.hit_order[3 * q + k] = ho[k];
    }
    J.intensity[q] = inten;
}

}  // namespace tartarus

using namespace tartarus;

// ---------------------------------------------------------------------------
// cost-ordered work queue: rays nearest the critical curve are handed out first
// ---------------------------------------------------------------------------
// Adds each valid lane to hist[k] with one LDS atomic per distinct k in the
// wavefront (neighbouring rays mostly share a bucket; one atomic per lane on
// 32 counters serialised) and returns the lane's rank: the count before it,
// in the atomic's order between wavefronts and in lane order within one.
// Every lane of the wavefront must call it.
__device__ __forceinline__ unsigned int wave_bucket_add(unsigned int* hist, int k, bool valid)
{
    unsigned long long todo = __ballot(valid);
    unsigned int rank = 0u;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int kk = __shfl(k, leader);
        const unsigned long long same = __ballot(valid && k == kk);
        unsigned int base = 0u;
        if ((int)__lane_id() == leader) base = atomicAdd(&hist[kk], (unsigned int)__popcll(same));
        base = __shfl(base, leader);
        if (valid && k == kk) rank = base + (unsigned int)__popcll(same & lanemask_lt());
        todo &= ~same;
    }
    return rank;
}

// The passes below give each block a run of `per` consecutive rays (a
// multiple of the block size) and keep one histogram per block in LDS: the
// global bucket counters then take a few thousand atomics per trace instead
// of one per bucket and 256 rays (same-address atomics serialise in L2).
constexpr int kOrderMaxBlocks = 2048;

// Pass 1: bucket of every ray (from its constants of motion) and the bucket
// histogram.  LDS histogram per block, then one global add per non-empty
// bucket.
__global__ void __launch_bounds__(256) order_keys_kernel(const DevJob* jobs, const JobConst* jc, int njobs,
                                                         long long total, long long per, unsigned char* key,
                                                         unsigned int* count)
{
    __shared__ unsigned int hist[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0u;
    __syncthreads();
    const long long r0 = blockIdx.x * per;
    const long long r1 = r0 + per < total ? r0 + per : total;
    for (long long g0 = r0; g0 < r1; g0 += blockDim.x) {
        const long long gid = g0 + threadIdx.x;
        int k = 0;
        if (gid < r1) {
            int lo = 0, hi = njobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].ray_begin <= gid)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const DevJob& J = jobs[lo];
            const JobConst& C = jc[lo];
            double al, be, p[4];
            pixel_coords(J, gid - J.ray_begin, al, be);
            pixel_momentum(C, J.r_obs, al, be, p);
            // b = L / E and q = Q / E^2 are unchanged by the backward-tracing sign flip
            const double ipt = 1.0 / p[0];
            const double b = -p[3] * ipt;
            const double Q = fma(p[2], p[2], C.c2_obs * (p[3] * p[3] * C.is2_obs - J.a * J.a * p[0] * p[0]));
            k = cost_bucket(J.a, b, Q * ipt * ipt, C.rp);
            key[gid] = (unsigned char)k;
        }
        wave_bucket_add(hist, k, gid < r1);
    }
    __syncthreads();
    if (threadIdx.x < kOrderBuckets && hist[threadIdx.x]) atomicAdd(&count[threadIdx.x], hist[threadIdx.x]);
}

// Pass 2: start of each bucket in the queue, highest bucket first.
__global__ void order_scan_kernel(const unsigned int* count, unsigned int* cursor)
{
    if (threadIdx.x != 0) return;
    unsigned int run = 0u;
    for (int k = kOrderBuckets - 1; k >= 0; --k) {
        cursor[k] = run;
        run += count[k];
    }
}

// Pass 3: scatter ray indices to their bucket's range.  A block counts its
// run's buckets, reserves its share of each bucket's range with one global
// atomic, then places its rays.  The order inside a bucket depends on atomic
// timing, which only changes when a ray is traced.
__global__ void __launch_bounds__(256) order_scatter_kernel(const unsigned char* key, unsigned int* cursor,
                                                            long long total, long long per, unsigned int* order)
{
    __shared__ unsigned int hist[kOrderBuckets], base[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0u;
    __syncthreads();
    const long long r0 = blockIdx.x * per;
    const long long r1 = r0 + per < total ? r0 + per : total;
    for (long long g0 = r0; g0 < r1; g0 += blockDim.x) {
        const long long gid = g0 + threadIdx.x;
        wave_bucket_add(hist, gid < r1 ? (int)key[gid] : 0, gid < r1);
    }
    __syncthreads();
    if (threadIdx.x < kOrderBuckets) {
        base[threadIdx.x] = hist[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], hist[threadIdx.x]) : 0u;
        hist[threadIdx.x] = 0u;
    }
    __syncthreads();
    for (long long g0 = r0; g0 < r1; g0 += blockDim.x) {
        const long long gid = g0 + threadIdx.x;
        const int k = gid < r1 ? (int)key[gid] : 0;
        const unsigned int rank = wave_bucket_add(hist, k, gid < r1);
        if (gid < r1) order[base[k] + rank] = (unsigned int)gid;
    }
}

// The three passes; count and cursor (kOrderBuckets entries each) must be zero
// on entry to the first one.
extern "C" hipError_t tartarus_launch_order(const LaunchArgs* args, long long total, unsigned char* key,
                                            unsigned int* count, unsigned int* cursor, unsigned int* order,
                                            hipStream_t stream)
{
    if (total <= 0) return hipSuccess;
    if (total > 0xffffffffll) return hipErrorInvalidValue;
    // runs of `per` rays (a multiple of 256), at most kOrderMaxBlocks of them
    const long long groups = (total + 255) / 256;
    const long long want = groups < kOrderMaxBlocks ? groups : kOrderMaxBlocks;
    const long long per = (groups + want - 1) / want * 256;
    const long long blocks = (total + per - 1) / per;
    hipLaunchKernelGGL(order_keys_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, args->jobs, args->jc,
                       args->njobs, total, per, key, count);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(64), 0, stream, count, cursor);
    hipLaunchKernelGGL(order_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, key, cursor, total, per,
                       order);
    return hipGetLastError();
}

extern "C" hipError_t tartarus_launch_setup(int kind, const LaunchArgs* args, hipStream_t stream)
{
    const int n = args->njobs;
    const int blocks = (n + 63) / 64;
    if (kind == 0)
        hipLaunchKernelGGL((job_setup<0>), dim3(blocks), dim3(64), 0, stream, args->jobs, (JobConst*)args->jc, n,
                           nullptr, 0, 0, 0.0, 0.0);
    else
        hipLaunchKernelGGL((job_setup<1>), dim3(blocks), dim3(64), 0, stream, args->jobs, (JobConst*)args->jc, n,
                           args->table, args->nr, args->nth, args->tab_r_min, args->tab_r_max);
    return hipGetLastError();
}

// The integrator instance for (metric kind, precision, method); null if there
// is none.  Mixed precision and the tabulated metric are provided with
// Dormand-Prince only (a tabulated six-stage instance keeps all six stage
// derivatives next to the table patch and spills heavily).
static const void* trace_kernel_for(int kind, int prec, int method, int serve)
{
    if (serve) {
        // serving takes analytic Kerr requests
        if (kind == 0 && prec == 0 && method == 0) return (const void*)trace_persistent<0, 0, 0, 1>;
        if (kind == 0 && prec == 0 && method == 1) return (const void*)trace_persistent<0, 0, 1, 1>;
        if (kind == 0 && prec == 0 && method == 2) return (const void*)trace_persistent<0, 0, 2, 1>;
        if (kind == 0 && prec == 1 && method == 0) return (const void*)trace_persistent<0, 1, 0, 1>;
        if (kind == 0 && prec == 0 && method == 3) return (const void*)trace_persistent<0, 0, 3, 1>;
        if (kind == 0 && prec == 0 && method == 4) return (const void*)trace_persistent<0, 0, 4, 1>;
        return nullptr;
    }
    if (kind == 0 && prec == 0 && method == 0) return (const void*)trace_persistent<0, 0, 0, 0>;
    if (kind == 0 && prec == 0 && method == 1) return (const void*)trace_persistent<0, 0, 1, 0>;
    if (kind == 0 && prec == 0 && method == 2) return (const void*)trace_persistent<0, 0, 2, 0>;
    if (kind == 0 && prec == 1 && method == 0) return (const void*)trace_persistent<0, 1, 0, 0>;
    if (kind == 0 && prec == 0 && method == 3) return (const void*)trace_persistent<0, 0, 3, 0>;
    if (kind == 0 && prec == 0 && method == 4) return (const void*)trace_persistent<0, 0, 4, 0>;
    if (kind == 1 && prec == 0 && method == 0) return (const void*)trace_persistent<1, 0, 0, 0>;
    return nullptr;
}

// The serving instance runs when the launch parks rays (args->slots).
extern "C" hipError_t tartarus_launch_trace(int kind, int prec, int method, const LaunchArgs* args, int grid,
                                            int block, hipStream_t stream)
{
    const void* f = trace_kernel_for(kind, prec, method, args->slots != nullptr);
    if (!f) return hipErrorInvalidValue;
    void* params[] = {(void*)args};
    return hipLaunchKernel(f, dim3(grid), dim3(block), params, 0, stream);
}

extern "C" hipError_t tartarus_occupancy(int kind, int prec, int method, int serve, int block, int* blocks_per_cu)
{
    const void* f = trace_kernel_for(kind, prec, method, serve);
    if (!f) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, 0);
}

// Finishing pass for jobs [job0, job0 + njobs), each with at most max_rays rays.
extern "C" hipError_t tartarus_launch_finish(const LaunchArgs* args, int job0, int njobs, long long max_rays,
                                             hipStream_t stream)
{
    if (njobs <= 0 || max_rays <= 0) return hipSuccess;
    const long long bx = (max_rays + 255) / 256;
    if (bx > 0x7fffffffll || njobs > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(finish_kernel, dim3((unsigned)bx, (unsigned)njobs), dim3(256), 0, stream, args->jobs, args->jc,
                       job0);
    return hipGetLastError();
}

// Interleave the caller's table by grid point for the integrator (table.hpp):
// one thread per (node, component), 4 doubles each.
__global__ void table_interleave_kernel(const double* table, long long nodes, double* inter)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= nodes * 5) return;
    const long long node = i / 5;
    const int c = (int)(i - node * 5);
    const double4 v = *reinterpret_cast<const double4*>(table + ((size_t)c * nodes + node) * 4);
    *reinterpret_cast<double4*>(inter + (size_t)i * 4) = v;
}

extern "C" hipError_t tartarus_launch_table_interleave(const LaunchArgs* args, double* inter, hipStream_t stream)
{
    const long long nodes = (long long)args->nr * args->nth;
    if (nodes <= 0) return hipErrorInvalidValue;
    const long long blocks = (nodes * 5 + 255) / 256;
    if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(table_interleave_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, args->table, nodes,
                       inter);
    return hipGetLastError();
}
