/*
 * tartarus_oracle.h -- declarations of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle exists to check the HIP library; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no code, header, table or constant with the HIP path.
 *
 * Units: geometric, G = c = M = 1; Boyer-Lindquist coordinates (t, r, theta, phi).
 * State layout (the paper's 8-D phase-space array, Sec. 2.1):
 *     q = [t, r, theta, phi, p_t, p_r, p_theta, p_phi]
 */
#ifndef TARTARUS_ORACLE_H
#define TARTARUS_ORACLE_H
#include <stdint.h>

#define OR_ESCAPED 0
#define OR_CAPTURED 1
#define OR_FAILED 2
#define OR_ON_DISK 3       /* ended on an opaque disk */
#define OR_MAX_HITS 3

typedef struct {
    int kind;              /* 0 analytic Kerr, 1 bicubic table                      */
    double a;              /* spin; also used by the emitter model for kind 1       */
    const double* table;   /* host array [5][nr][nth][4] (kind 1)                   */
    int nr, nth;
    double r_min, r_max;
} or_metric;

typedef struct {
    double r_obs, theta_obs;
    int nx, ny;
    double alpha_min, alpha_max, beta_min, beta_max;
} or_camera;

#define OR_SHADE_OBSERVED 0   /* hit flux g^4 F (Eq. (16))                          */
#define OR_SHADE_INTRINSIC 1  /* hit flux F: redshift and beaming off (Fig. KerrUHD b) */

typedef struct {
    double r_in;           /* <= 0 means r_ISCO                                      */
    double r_out;
    int max_hits;          /* 0..3; 0 = no disk                                      */
    int opaque;            /* 1: the first crossing on the disk ends the ray         */
    int shading;           /* OR_SHADE_OBSERVED or OR_SHADE_INTRINSIC                */
} or_disk;

/* method: 0 Dormand-Prince, 1 Cash-Karp, 2 Fehlberg 5(4) pair, 3 Gragg-
 * Bulirsch-Stoer extrapolation with OR_GBS_COLUMNS columns, 4 Verlet with the
 * fixed step h0_frac * r_obs (Sec. 3.2). */
#define OR_METHOD_GBS 3
#define OR_METHOD_VERLET 4
#define OR_GBS_COLUMNS 6
typedef struct {
    double rtol, atol, h0_frac, horizon_factor, r_escape, event_tol;
    int64_t max_steps;
    int32_t method;
    int32_t pad;
} or_solver;

/* Structure-of-arrays outputs, indexed by position in the traced ray list. */
typedef struct {
    int32_t* cls;
    int32_t* n_hits;
    double* final_rtp;     /* [n][3]  */
    double* h_drift;       /* max |H| over accepted states                        */
    double* h_gate;        /* max |H| over accepted states with r >= 1.5 r_+       */
    double* hit_r;         /* [n][3]  */
    double* hit_g;         /* [n][3]  */
    double* hit_flux;      /* [n][3]  */
    double* hit_lambda;    /* [n][3]  */
    int32_t* hit_order;    /* [n][3]  */
    double* intensity;
    int32_t* n_accept;
    int32_t* n_reject;
    int32_t* n_cross;      /* equatorial crossings seen (recorded or not)        */
} or_outputs;

#endif
