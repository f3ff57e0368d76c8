/*
 * tartarus.h -- C ABI of the MI355X (gfx950) Kerr null-geodesic ray tracer.
 *
 * One null geodesic is traced backward from every pixel of a camera at
 * distance r_obs through Kerr spacetime (Boyer-Lindquist coordinates, units
 * G = c = M = 1), following the TARTARUS method (Bambague & Larranaga):
 *   - initial momenta from the celestial coordinates (alpha, beta) projected
 *     on the ZAMO tetrad at the observer (Sec. 2.2, Eqs. (4)-(10));
 *   - Hamilton's equations of H = 1/2 g^{mu nu} p_mu p_nu (Sec. 2.1, Eqs. (1)-(3)),
 *     on the 8-D state q = [t, r, theta, phi, p_t, p_r, p_theta, p_phi];
 *   - an adaptive embedded Dormand-Prince 5(4) step with per-ray error control
 *     (Sec. 3.2); the paper's other integrators (Cash-Karp and Fehlberg 5(4),
 *     Gragg-Bulirsch-Stoer, fixed-step Verlet) through tartarus_solver.method;
 *   - horizon, escape and equatorial-disk events located on the step's cubic
 *     Hermite interpolant (Sec. 3.2);
 *   - Novikov-Thorne shading g^4 F(r) at each recorded disk crossing
 *     (Secs. 2.3-2.4, Eqs. (11)-(16));
 *   - the constraint residual |H| at every accepted step (Sec. 4.1, Eq. (17)).
 *
 * Every step of the path runs in HIP kernels on the device.  All pointers to
 * bulk data (tables, outputs) are DEVICE pointers owned by the caller (for
 * example torch tensors); the library never frees caller memory.  Structs
 * passed by pointer are read during the call only.  No function throws; each
 * returns a tartarus_status, and on a negative status tartarus_last_error()
 * returns a message for the calling thread.
 *
 * Readings of points the paper leaves open (applied identically by the
 * library and documented per field below):
 *   - pixel grid: inclusive linspace, alpha_i = alpha_min + i (alpha_max -
 *     alpha_min) / (nx - 1), same for beta with j; pixel (i, j) of camera c is
 *     ray index c*nx*ny + j*nx + i;
 *   - the tetrad's e_(t)^phi = omega e_(t)^t (ZAMO);
 *   - backward tracing stores the negated momenta of Eq. (4)-(5) and integrates
 *     with increasing lambda (same spatial path; g is unchanged);
 *   - step control: RMS norm over the 8 components with scale atol + rtol *
 *     max(|y_n|, |y_n+1|); accept iff err <= 1 (NaN rejects); new step
 *     h * min(fmax, max(0.2, 0.9 err^(-1/p))), p = 5 for the 5(4) pairs and
 *     11 for the extrapolation, fmax = 10, or 1 right after a rejection; first
 *     step h0_frac * r_obs.  A component whose error estimate lies within its
 *     own rounding (2^18 ulps of h |b - b*|_1 max(|k_n|, |k_n+1|) for a pair,
 *     of the largest sweep increment for the extrapolation, capped at 1 % of
 *     the component's tolerance scale) counts as zero, so that step sequences
 *     do not depend on rounding order; the extrapolation's step factor is
 *     rounded down to a power of two;
 *   - events on each accepted step: horizon when r falls to horizon_factor *
 *     r_+ (or the table's inner radius, if larger), escape when r rises to
 *     r_escape, disk crossing when cos(theta) changes sign; the root is
 *     located on the step's cubic Hermite interpolant to well within
 *     event_tol in lambda (safeguarded Newton iteration on the cubic, bracket
 *     kept; the paper bisects to ~1e-12, and the two roots differ by less than
 *     that); for the extrapolation, whose macro-steps are too long for a cubic,
 *     on the method's own solution (sub-steps re-integrated from the step's
 *     start, the cubic's root as first guess);
 *   - emitter: prograde Keplerian Omega = 1 / (r^{3/2} + a); the first up to
 *     max_hits (<= 3) crossings inside [r_in, r_out] are recorded; the ray
 *     continues to a terminal event unless the disk is opaque.
 */
#ifndef TARTARUS_H
#define TARTARUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TARTARUS_OK = 0,
    TARTARUS_E_INVALID = -1,   /* an argument is out of range or a required pointer is NULL  */
    TARTARUS_E_NOMEM = -2,     /* device or host allocation failed                          */
    TARTARUS_E_DEVICE = -3,    /* a HIP call failed, or no usable gfx950 device              */
    TARTARUS_E_TOO_LARGE = -4, /* a request can never fit the HBM budget                    */
    TARTARUS_E_NOT_FOUND = -5, /* unknown ticket                                            */
    TARTARUS_E_AGAIN = -6      /* not ready yet (serving)                                   */
} tartarus_status;

/* Ray classes written to outputs.cls. */
#define TARTARUS_ESCAPED 0
#define TARTARUS_CAPTURED 1
#define TARTARUS_FAILED 2
#define TARTARUS_ON_DISK 3   /* ended on an opaque disk (tartarus_disk.opaque) */

#define TARTARUS_METRIC_KERR 0
#define TARTARUS_METRIC_TABLE 1
#define TARTARUS_PREC_FP64 0
#define TARTARUS_PREC_MIXED 1

/* Background metric (Sec. 3.1: analytic Kerr, or a numerically supplied metric
 * of the stationary axisymmetric form of Eq. (6)).
 * kind = TARTARUS_METRIC_KERR: analytic Kerr with spin a, 0 <= a < 1.
 * kind = TARTARUS_METRIC_TABLE: table is a DEVICE array of doubles laid out as
 *   table[c][k][l][4], c = 0..4 over (g_tt, g_tphi / sin^2 theta, g_rr,
 *   g_thth, g_phph / sin^2 theta), k = 0..nr-1 over r_k = exp(ln r_min + k du),
 *   du = ln(r_max / r_min) / (nr - 1), l = 0..nth-1 over theta_l = l pi / (nth - 1),
 *   and the last index over (f, df/dr, df/dtheta, d2f/dr dtheta).  It is
 *   interpolated by a bicubic Hermite patch in (ln r, theta).  The emitter
 *   model (Omega, u^t, F) uses the Kerr closed forms with spin a.  Rays that
 *   reach r_min are classed CAPTURED.  nr, nth >= 4; 0 < r_min < r_max. */
typedef struct {
    int kind;
    double a;
    const double* table;
    int nr, nth;
    double r_min, r_max;
} tartarus_metric;

/* Observer (Sec. 2.2): distance r_obs = D, inclination theta_obs in (0, pi),
 * phi_obs = t_obs = 0; an nx x ny pixel grid over the (alpha, beta) window.
 * Requires alpha^2 + beta^2 < r_obs^2 at every pixel, nx, ny >= 1. */
typedef struct {
    double r_obs, theta_obs;
    int nx, ny;
    double alpha_min, alpha_max, beta_min, beta_max;
} tartarus_camera;

/* Thin Novikov-Thorne disk in theta = pi/2 (Sec. 2.3).  r_in <= 0 selects the
 * prograde ISCO.  max_hits in 0..3; 0 disables the disk event.
 * opaque = 0: crossings do not stop the ray; the first max_hits crossings on
 *   the disk are recorded and later ones counted.  opaque = 1 (optically
 *   thick, Sec. 2.3; needs max_hits >= 1): the first crossing on the disk ends
 *   the ray there, cls = TARTARUS_ON_DISK, final_rtp = the crossing point.
 * shading = TARTARUS_SHADE_OBSERVED: hit_flux = g^4 F(r_em) (Eq. (16));
 *   TARTARUS_SHADE_INTRINSIC: hit_flux = F(r_em), the map with the redshift
 *   and beaming switched off (Fig. KerrUHD b); hit_g is reported either way. */
#define TARTARUS_SHADE_OBSERVED 0
#define TARTARUS_SHADE_INTRINSIC 1
typedef struct {
    double r_in;
    double r_out;
    int max_hits;
    int opaque;
    int shading;
} tartarus_disk;

/* Integrator settings (Sec. 3.2).  rtol > 0, atol > 0, h0_frac > 0,
 * horizon_factor >= 1, r_obs < r_escape <= 1e15, event_tol > 0, max_steps >= 1
 * (attempted steps, accepted + rejected).  precision: TARTARUS_PREC_FP64, or
 * TARTARUS_PREC_MIXED (Runge-Kutta stages evaluated in FP32 in the far field,
 * r >= 10 r_+ away from turning points and the axis, on steps whose FP32
 * rounding stays below half the tolerance: h |k_i| <= 2.6e7 (atol + rtol |y_i|)
 * for every component; state sums, error norm, controller, events and shading
 * stay FP64.  Below rtol 5e-10 no far-field step passes that test, and a mixed
 * trace runs the FP64 arithmetic throughout, n_fp32 = 0).
 * method (Sec. 3.2): an embedded 5(4) pair, TARTARUS_METHOD_DP45
 * (Dormand-Prince), TARTARUS_METHOD_CK45 (Cash-Karp) or TARTARUS_METHOD_RKF45
 * (Fehlberg), each propagating the fifth-order solution with the step
 * controlled by the embedded fourth-order estimate; or TARTARUS_METHOD_GBS,
 * Gragg-Bulirsch-Stoer extrapolation: per macro-step six modified-midpoint
 * sweeps with 2, 4, ..., 12 substeps, Richardson extrapolation in h^2 to order
 * 12 of the sweeps' increments y - y_n, the difference to the order-10 entry
 * as error estimate (42 right-hand sides per attempt, against 6 for a pair);
 * or TARTARUS_METHOD_VERLET, the
 * symmetric, symplectic generalized Stormer-Verlet scheme with the FIXED step
 * h0_frac * r_obs and no error control (rtol and atol are not used; every
 * step counts as accepted).  Its two implicit stages are solved by fixed-point
 * iteration; a ray whose stage does not converge (close to the horizon, where
 * dH/dx grows like 1/Delta, a fixed step eventually has no nearby solution)
 * ends FAILED at its current state.  Fixed steps resolve the strong field
 * only if they are small (~0.01 M near the hole), so Verlet traces take
 * 1e5-1e6 steps per ray from a distant camera; with horizon_factor >= 1.05
 * the captured rays of a spin-0.9 hole reach the stop radius at h <= 0.01.
 * For every method, h0_frac and max_steps keep their meaning (an attempt is
 * one macro-step or one fixed step), and events are located as described at
 * the top of this file.  Mixed precision and the tabulated metric need DP45. */
enum {
    TARTARUS_METHOD_DP45 = 0,
    TARTARUS_METHOD_CK45 = 1,
    TARTARUS_METHOD_RKF45 = 2,
    TARTARUS_METHOD_GBS = 3,
    TARTARUS_METHOD_VERLET = 4
};
typedef struct {
    double rtol, atol, h0_frac, horizon_factor, r_escape, event_tol;
    int64_t max_steps;
    int precision;
    int method;
} tartarus_solver;

/* Caller-owned DEVICE output buffers, one entry per ray (ray index as above);
 * arrays marked [3] hold three doubles / ints per ray (hit slots).  All are
 * required.  Unused hit slots are written as zero. */
typedef struct {
    int32_t* cls;          /* TARTARUS_ESCAPED / CAPTURED / FAILED / ON_DISK          */
    int32_t* n_hits;       /* recorded disk hits, 0..max_hits                        */
    double* final_rtp;     /* [3] r, theta, phi at the terminal event (FAILED: last state) */
    double* h_drift;       /* max |H| over the accepted states (Eq. (17))            */
    double* h_gate;        /* max |H| over accepted states with r >= 1.5 r_+         */
    double* hit_r;         /* [3] emission radius                                    */
    double* hit_g;         /* [3] redshift factor g, Eq. (15)                         */
    double* hit_flux;      /* [3] g^4 F(r), Eqs. (11), (16)                           */
    double* hit_lambda;    /* [3] affine parameter of the crossing                   */
    int32_t* hit_order;    /* [3] which equatorial crossing (1-based) the hit was    */
    double* intensity;     /* sum of hit_flux over the recorded hits                 */
    int32_t* n_accept;     /* accepted steps                                         */
    int32_t* n_reject;     /* rejected steps                                         */
    int32_t* n_fp32;       /* attempts whose stages ran in FP32 (mixed precision)    */
    int32_t* n_cross;      /* equatorial crossings seen (recorded or not)            */
} tartarus_outputs;

/* Launch shape of the persistent integrator.  Any value <= 0 means "use the
 * tuned or default choice".  Results are bit-identical for every launch shape
 * and queue order (rays never share arithmetic).
 *
 * order: TARTARUS_ORDER_PIXEL hands rays out in pixel order (camera by camera,
 * row-major); TARTARUS_ORDER_COST first sorts them into buckets by how close
 * they pass to the critical curve (the spherical photon orbits, which the
 * rays that take the most steps wind around) and starts the closest first, so
 * that the longest rays do not start last and finish alone; TARTARUS_ORDER_TILE
 * hands them out by 8 x 8 pixel tiles (tiles row-major, pixels row-major in a
 * tile; ragged edge tiles are smaller), so that a wavefront's rays are
 * neighbours on the sky and follow similar paths.  The default (0) is COST
 * for traces of at least 4096 rays, else PIXEL. */
enum { TARTARUS_ORDER_DEFAULT = 0, TARTARUS_ORDER_PIXEL = 1, TARTARUS_ORDER_COST = 2, TARTARUS_ORDER_TILE = 3 };

typedef struct {
    int block_threads;     /* 64, 128 or 256                                        */
    int blocks_per_cu;     /* resident workgroups per compute unit; default: 1 when the trace has fewer than 8 rays per lane of one block per CU, else the occupancy maximum */
    int chunk;             /* least ray ids a wavefront takes per fetch; ids beyond its idle lanes wait in it (1 = none wait) */
    int refill_min;        /* idle lanes that trigger a refill (1..64)              */
    int order;             /* TARTARUS_ORDER_*                                      */
} tartarus_launch;

/* Select the device and set the HBM budget (bytes) for the serving queue
 * (0 = 8 GiB).  Must be called before any other call except
 * tartarus_last_error and tartarus_validate.  Returns E_DEVICE if the device is
 * not gfx950. */
int tartarus_init(int device, size_t hbm_budget_bytes);

/* Release the library's device memory and stop the serving thread.  Call it
 * before the process exits (and before the HIP runtime is torn down) when
 * tartarus_submit has been used: a serving thread still running at exit keeps
 * the device busy.  The Python binding registers it with atexit. */
int tartarus_shutdown(void);

/* Check the arguments of a trace without touching the device (same checks as
 * tartarus_trace, outputs excluded). */
int tartarus_validate(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                      const tartarus_disk* disk, const tartarus_solver* solver);

/* Trace every pixel of ncams cameras (all with the same nx, ny) into outputs,
 * asynchronously on hip_stream (a hipStream_t; NULL = the null stream).  The
 * call enqueues the work and returns; results are valid once the stream has
 * completed.  Buffers must stay alive until then.  Not for HIP graph capture:
 * the job table is staged in pinned slots that later calls reuse. */
int tartarus_trace(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                   const tartarus_disk* disk, const tartarus_solver* solver,
                   const tartarus_outputs* out, void* hip_stream);

/* As tartarus_trace with an explicit launch shape (NULL = tuned/default). */
int tartarus_trace_launch(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                          const tartarus_disk* disk, const tartarus_solver* solver,
                          const tartarus_outputs* out, const tartarus_launch* launch, void* hip_stream);

/* Allocation-free trace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  As tartarus_trace_launch for the analytic Kerr metric, but the
 * library's working memory for the call (job table, job constants, queue head,
 * cost-order keys and counters, per-ray records) comes from one fixed array
 * per device of TARTARUS_NOALLOC_SCRATCH_BYTES, which the library holds from
 * its load until the process ends; the call itself allocates nothing (no
 * hipMalloc, hipFree or pinned host memory) and copies the job table by
 * kernel argument.  Limits: ncams <= TARTARUS_NOALLOC_MAX_CAMERAS and
 * ncams * nx * ny <= TARTARUS_NOALLOC_MAX_RAYS (else TARTARUS_E_TOO_LARGE);
 * metric kind TARTARUS_METRIC_KERR only (else TARTARUS_E_INVALID).  Every call
 * on one device uses that device's one array, and a call leaves its contents
 * behind: calls that overlap on a device (on two streams, or on one stream
 * while another call's work is still running elsewhere) race and corrupt each
 * other's results; calls in order on one stream are safe.  Not counted by
 * tartarus_kernel_timing.  Results are bit-identical to tartarus_trace_launch
 * with the same arguments (same kernels). */
#define TARTARUS_NOALLOC_MAX_RAYS 262144
#define TARTARUS_NOALLOC_MAX_CAMERAS 64
#define TARTARUS_NOALLOC_SCRATCH_BYTES (135561216ull)   /* 129.3 MiB */
int tartarus_trace_noalloc(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                           const tartarus_disk* disk, const tartarus_solver* solver,
                           const tartarus_outputs* out, const tartarus_launch* launch, void* hip_stream);

/* Time candidate launch shapes on the given trace (synchronously, on
 * hip_stream; each candidate is the best of three runs), keep the fastest for
 * this (metric kind, precision, method) for the rest of the process, and write
 * it to *best.  The outputs hold the last run's results. */
int tartarus_autotune(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                      const tartarus_disk* disk, const tartarus_solver* solver,
                      const tartarus_outputs* out, void* hip_stream, tartarus_launch* best);

/* Integrator timing, for benchmarks and profilers.  While it is enabled, each
 * launch of the persistent integrator that tartarus_trace,
 * tartarus_trace_launch or tartarus_autotune enqueue is bracketed by a pair of
 * HIP events recorded on the trace's stream; the ordering and finishing
 * kernels of the trace fall outside the pair, and serving epochs are not
 * timed.  tartarus_kernel_time waits for the recorded launches, writes the sum
 * of their durations (milliseconds) and their number, and starts both sums
 * afresh.  Disabling stops the recording; launches recorded before stay
 * readable.  enable: 0 or 1 (else E_INVALID); NULL outputs: E_INVALID; both
 * return E_DEVICE before tartarus_init.  The event pairs are the library's and
 * are reused. */
int tartarus_kernel_timing(int enable);
int tartarus_kernel_time(double* total_ms, long long* launches);

/* Fill a caller-owned DEVICE table (layout of tartarus_metric.table, nr*nth*20
 * doubles) from the analytic Kerr metric with spin a, on hip_stream. */
int tartarus_build_kerr_table(double a, int nr, int nth, double r_min, double r_max, double* table,
                              void* hip_stream);

/* ---- serving: continuous batching of image requests ------------------------
 * tartarus_submit queues one image request (one camera) and returns a ticket
 * at once.  A scheduler thread admits queued requests in arrival order while
 * their output bytes plus the library's ray-slot arena fit the HBM budget,
 * and traces all admitted requests together on one device queue in epochs;
 * requests arriving while others run join at the next epoch.  Per-ray results
 * are bit-identical to tartarus_trace of the same request alone.  Tolerances,
 * step settings and precision are the request's own; the integration method
 * is the session's (the first request's: a request with another method gets
 * E_INVALID).  Requests use the analytic Kerr metric (a tabulated metric gets
 * E_INVALID; trace it with tartarus_trace).  Output buffers must stay alive
 * until poll reports done or cancel returns. */

/* Hand-out order of the serving queue's unstarted rays, applied from the next
 * epoch on: TARTARUS_SERVE_SMALLEST_FIRST (default) gives lanes to the rays of
 * the admitted request with the fewest rays not yet handed out first, so small
 * images finish within a few epochs of their arrival while large ones run
 * behind them;
 * TARTARUS_SERVE_ARRIVAL hands them out in admission order.  Rays already on
 * a lane always run to their end, and results do not depend on the order.
 * E_INVALID for another value, E_DEVICE before tartarus_init. */
#define TARTARUS_SERVE_SMALLEST_FIRST 0
#define TARTARUS_SERVE_ARRIVAL 1
int tartarus_serving_order(int order);

int tartarus_submit(const tartarus_metric* metric, const tartarus_camera* cam, const tartarus_disk* disk,
                    const tartarus_solver* solver, const tartarus_outputs* out, uint64_t* ticket);

/* *state: 0 queued, 1 running, 2 done (outputs complete).  Ticket records are
 * kept until tartarus_shutdown. */
int tartarus_poll(uint64_t ticket, int* state);

/* Block until the ticket is done (or timeout_ms elapses: E_AGAIN). */
int tartarus_wait(uint64_t ticket, int64_t timeout_ms);

/* Remove a queued or running request.  Its outputs are left incomplete. */
int tartarus_cancel(uint64_t ticket);

/* Latency stamps of a ticket in nanoseconds of a monotonic host clock:
 * stamps[0] submit, [1] admitted, [2] done (0 while not reached). */
int tartarus_ticket_times(uint64_t ticket, int64_t stamps[3]);

/* Message for the last non-OK status returned on this thread. */
const char* tartarus_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
