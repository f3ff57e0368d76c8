// internal.hpp -- structures shared by the host runtime and the HIP kernels.
#pragma once

#include <stdint.h>

namespace tartarus {

// One camera (trace) or one image request (serving): a contiguous range of
// global ray indices with its own parameters and output pointers (already
// offset to the job's first ray).
struct DevJob {
    long long ray_begin;
    long long ray_count;
    int nx, ny;
    int max_hits;
    int disk_flags;                 // DISK_OPAQUE | DISK_INTRINSIC
    double a;
    double r_obs, theta_obs;
    double alpha_min, alpha_max, beta_min, beta_max;
    double disk_r_in, disk_r_out;   // r_in <= 0: prograde ISCO
    int32_t* cls;
    int32_t* n_hits;
    double* final_rtp;
    double* h_drift;
    double* h_gate;
    double* hit_r;
    double* hit_g;
    double* hit_flux;
    double* hit_lambda;
    int32_t* hit_order;
    double* intensity;
    int32_t* n_accept;
    int32_t* n_reject;
    int32_t* n_fp32;
    int32_t* n_cross;
    unsigned int* remaining;        // serving: rays still running (may be null)
    int cancelled;                  // serving: drop the job's rays without writing outputs
    int pad1;
    double* rec;                    // [ray_count][REC_DOUBLES] integrator -> finishing pass records
    double event_tol;               // event location tolerance (affine parameter)
    // the request's solver settings (serving traces each ray with its own
    // request's; a one-shot trace's kernels take them from the launch)
    double rtol, atol, h0_frac, horizon_factor, r_escape;
    long long max_steps;
    int allow32;                    // mixed precision: FP32 stages allowed (tolerance permitting)
    int pad2;
};

// Per-ray record the integrator leaves for the finishing pass (doubles).  The
// fields every ray needs come first, in REC_HEAD doubles (192 bytes, within
// the record's first two 128-byte lines), so the finishing pass reads them as
// one contiguous run; the hit slots follow and are read only for rays that
// hit the disk.
// Terminal step at REC_TERM: r, th, phi as (y0, dy0/dlam, y1, dy1/dlam) each,
// then h, lam, target radius, cos(th0); for rays that end without a terminal
// root (failed) only the three y0 are meaningful.  REC_CODE: terminal kind
// (0 none, 1 horizon, 2 escape) + 4 if the equator was crossed in that step,
// or 8: the step's equatorial crossing is on an opaque disk and ends the ray.
// REC_INTS: int32 cls, n_hits, n_accept, n_reject, n_fp32, n_cross, order[3].
// Crossing slot k (k < 3) at REC_SLOT0 + REC_SLOT_LEN * k: r0, kr0, r1, kr1,
// th0, kth0, th1, kth1, h, lam, cos(th0) of the step that crossed the equator
// on the disk (h = 0: already located, r0 = radius, lam = affine parameter of
// the crossing).
constexpr int DISK_OPAQUE = 1;     // the first crossing on the disk ends the ray
constexpr int DISK_INTRINSIC = 2;  // hit flux F instead of g^4 F
constexpr int REC_TERM = 0;
constexpr int REC_CODE = 16;
constexpr int REC_HMAX = 17;
constexpr int REC_HGATE = 18;
constexpr int REC_INTS = 19;       // 9 int32 in doubles 19..23
constexpr int REC_HEAD = 24;
constexpr int REC_SLOT0 = REC_HEAD;
constexpr int REC_SLOT_LEN = 11;
constexpr int REC_DOUBLES = 64;    // 512 bytes: records stay aligned to 128-byte lines
static_assert(REC_SLOT0 + 3 * REC_SLOT_LEN <= REC_DOUBLES, "record overflow");
static_assert(REC_HEAD % 2 == 0, "the header is read in 16-byte pieces");

// Per-job constants computed on the device by the set-up kernel before a
// trace: the observer's metric and ZAMO tetrad (Sec. 2.2), the horizon
// radius, the disk's inner edge and the Page-Thorne roots and coefficients
// (Sec. 2.3).
struct JobConst {
    double g[5];                    // covariant metric at the observer
    double ett, etp, err, ehh, epp; // tetrad components e_(t)^t, e_(t)^phi, e_(r)^r, e_(th)^th, e_(ph)^ph
    double c2_obs, is2_obs;         // cos^2 and 1 / sin^2 of the inclination
    double rp;                      // horizon radius r_+
    double r_in, x0;                // disk inner edge (r_ISCO if not given) and sqrt(r_in)
    double xi[3], coef[3];          // roots of x^3 - 3x + 2a and their Page-Thorne coefficients
    double a2;                      // a^2
    double gate_r;                  // 1.5 r_+: the constraint gate counts states at r >= gate_r
    double r_stop;                  // horizon event radius: horizon_factor r_+ (tabulated: at least the table's r_min)
};

// Per-launch uniform parameters.
struct LaunchArgs {
    const DevJob* jobs;
    const JobConst* jc;
    int njobs;
    int chunk;                      // ray ids fetched per wavefront
    int refill_min;                 // idle lanes that trigger a refill
    int pad0;
    long long total_rays;           // global ray indices run over [first_ray, total_rays)
    long long first_ray;
    unsigned long long* head;       // global queue head (relative to first_ray)
    double rtol, atol, h0_frac, event_tol;
    double horizon_factor, r_escape;
    long long max_steps;
    // tabulated metric (kind 1)
    const double* table;
    int nr, nth;
    double tab_r_min, tab_r_max;
    // mixed precision regime thresholds
    double r_switch_factor;         // FP32 stages only where r >= factor * r_+
    double turn_r, turn_th;         // turning-point guards (fractions)
    // serving epochs: resume / park ray state (null for one-shot traces)
    double* slots;                  // [nslot][SLOT_DOUBLES] parked state, slot = global lane id
    long long step_budget;          // serving: wavefront iterations per launch, then every lane parks (<= 0: none)
    unsigned int* slot_live;        // [nslot] 1 if a parked ray lives in the slot
    // serving: directory from global ray index to job-table entry, sorted by begin
    const long long* dir_begin;     // null: look up jobs[].ray_begin directly
    const int* dir_job;
    int ndir;
    int tile;                       // 1: queue positions run over 8 x 8 pixel tiles of each camera
    // queue position -> ray index (relative to first_ray); null: identity
    const unsigned int* order;
    // serving: rays still to finish, per job-table entry, one per
    // kRemainingStride words (null: not counted)
    unsigned int* remaining;
    // tabulated metric interleaved by grid point (the integrator reads this)
    const double* table_inter;
    // serving: queue positions run over nseg segments, segment k covering
    // positions [seg_q[k], seg_q[k+1]) and rays seg_ray[k] + (q - seg_q[k])
    // (absolute ray indices); nseg = 0: rays first_ray + q
    const long long* seg_q;         // [nseg + 1]
    const long long* seg_ray;       // [nseg]
    int nseg;
    int pad3;
};

// Serving: each job-table entry's count of unfinished rays sits on a
// 128-byte line of its own (every wavefront iteration that ends a ray
// subtracts from its job's count; counts sharing a line made those atomics
// contend).
constexpr int kRemainingStride = 32;   // unsigned ints

constexpr int SLOT_DOUBLES = 40;   // a parked ray (32 doubles) and its event search (8)

constexpr long long align256(long long b) { return (b + 255) / 256 * 256; }

// Byte layout of the fixed working memory of the allocation-free trace
// (tartarus_trace_noalloc): job table, job constants, queue head, cost-order
// counters, keys and order, per-ray records; each part 256-byte aligned.
struct NoallocLayout {
    static constexpr long long max_rays = 262144;   // TARTARUS_NOALLOC_MAX_RAYS
    static constexpr int max_cameras = 64;          // TARTARUS_NOALLOC_MAX_CAMERAS
    static constexpr int buckets = 32;              // counters of the cost-ordered queue (kOrderBuckets)
    static constexpr long long jobs = 0;
    static constexpr long long jc = jobs + align256(max_cameras * (long long)sizeof(DevJob));
    static constexpr long long head = jc + align256(max_cameras * (long long)sizeof(JobConst));
    static constexpr long long count = head + 256;
    static constexpr long long key = count + align256(2 * buckets * 4);
    static constexpr long long order = key + align256(max_rays);
    static constexpr long long rec = order + align256(4 * max_rays);
    static constexpr long long bytes = rec + max_rays * REC_DOUBLES * 8;
};

}  // namespace tartarus
