// host_logic.hpp -- the host-only parts of the runtime: argument validation,
// job-table and launch-argument filling, the launch-shape rules, and the
// serving scheduler's bookkeeping (record-buffer pool, HBM-budget admission,
// epoch queue segments).  No HIP types or calls: this unit also builds with a
// plain C++ compiler, so it can run under the address and undefined-behaviour
// sanitizers on the host.
#pragma once

#include <cstddef>
#include <map>
#include <string>
#include <vector>

#include "../../include/tartarus.h"
#include "internal.hpp"

namespace tartarus {
namespace host {

// Thread-local message of the last non-OK status (tartarus_last_error).
int fail(int code, const std::string& msg);
const char* last_error();

// Argument checks of the C ABI (tartarus.h documents each rule).
int check_metric(const tartarus_metric* m, int precision, int method);
int check_camera(const tartarus_camera& c, const tartarus_solver* s);
int check_solver(const tartarus_solver* s);
int check_disk(const tartarus_disk* d);
int check_outputs(const tartarus_outputs* o);
int validate_all(const tartarus_metric* metric, const tartarus_camera* cams, int ncams, const tartarus_disk* disk,
                 const tartarus_solver* solver);

// Default mixed-precision regime: FP32 stages where r >= 10 r_+, away from
// radial (|p_r| < 0.05 |p_t|) and polar (|p_theta| < 0.05 sqrt(Q)) turning points.
constexpr double kDefaultSwitch = 10.0;
constexpr double kDefaultTurnR = 0.05;
constexpr double kDefaultTurnTh = 0.05;

// Mixed precision uses FP32 stages only where their rounding stays below the
// tolerance (the integrator's per-step test: h |k_i| <= 2.6e7 (atol + rtol
// |y_i|) for every component).  Far from the hole the controller's steps have
// h / r ~ rtol^(1/5), so the test fails for every far-field step once
// rtol^(1/5) > 2.6e7 rtol, i.e. below rtol ~ 5e-10; there a mixed trace runs the
// FP64 instance (the same arithmetic, without the per-step test).
constexpr double kMixedMinRtol = 5e-10;
inline int kernel_precision(const tartarus_solver* s)
{
    return (s->precision == TARTARUS_PREC_MIXED && s->rtol >= kMixedMinRtol) ? TARTARUS_PREC_MIXED : TARTARUS_PREC_FP64;
}

// One camera or request as a device job-table entry: ray range [begin, begin +
// nx ny), outputs offset by `offset` rays, records at rec.
void fill_job(DevJob& J, const tartarus_metric* m, const tartarus_camera& c, const tartarus_disk* d,
              const tartarus_solver* s, const tartarus_outputs* o, long long begin, long long offset, double* rec);
// Uniform launch parameters of a trace (queue and serving fields left zero).
void fill_args(LaunchArgs& A, const tartarus_metric* m, const tartarus_solver* s);

// Launch shape: the request's positive fields override the base (tuned or
// default) shape, then the fields are checked.  occ is the kernel's
// resident-block limit per CU for the chosen block size; n_rays > 0 (a one-shot
// trace) lets an unset blocks_per_cu fall to 1 when the trace has fewer than
// kRaysPerLaneForFullOccupancy rays per lane of one block per CU.
constexpr long long kRaysPerLaneForFullOccupancy = 8;
int merge_shape(const tartarus_launch& base, const tartarus_launch* req, tartarus_launch& L);
int finish_shape(tartarus_launch& L, int occ, long long n_rays, int cus, int& grid);

// ---- serving ----------------------------------------------------------------
constexpr size_t kRecordBytes = REC_DOUBLES * sizeof(double);

// Outputs of one ray (cls, n_hits, n_accept, n_reject, n_fp32, n_cross int32;
// final_rtp[3], h_drift, h_gate, intensity double; hit_r, hit_g, hit_flux,
// hit_lambda [3] double; hit_order[3] int32).
constexpr size_t kOutputBytesPerRay = 6 * 4 + 6 * 8 + 12 * 8 + 3 * 4;

// Freed record buffers kept for reuse (a hipFree between epochs would
// synchronize the device), by capacity in rays.  A request of n rays reuses
// the smallest pooled buffer of n..4n rays.
class RecordPool {
public:
    // Capacity of the buffer take_pooled(n) would return; 0 if none fits.
    long long pooled_capacity(long long n) const;
    // Remove that buffer from the pool (null if none fits).
    void* take_pooled(long long n, long long& cap);
    // Keep a buffer of cap rays while the pool stays within limit bytes
    // (returns false: the caller frees it).
    bool give(void* p, long long cap, size_t limit);
    // Empty the pool; the caller frees the returned buffers.
    std::vector<void*> drain();
    size_t bytes() const { return bytes_; }
    bool empty() const { return pool_.empty(); }

private:
    std::multimap<long long, void*> pool_;
    size_t bytes_ = 0;
};

// Device bytes a request holds while admitted: its outputs and its record
// buffer of rec_cap rays.
inline size_t held_bytes(long long nrays, long long rec_cap)
{
    return (size_t)nrays * kOutputBytesPerRay + (size_t)rec_cap * kRecordBytes;
}

// Whether a request of nrays, with a record buffer of rec_cap rays (taken from
// the pool when pooled), fits the HBM budget next to the bytes held by
// admitted requests, the pooled buffers and the slot arena.
bool admission_fits(size_t used, size_t pool_bytes, size_t arena, size_t budget, long long nrays, long long rec_cap,
                    bool pooled);

// A request that can never be admitted: its outputs and exact-size records
// with the arena exceed the budget.
inline bool never_fits(long long nrays, size_t arena, size_t budget)
{
    return held_bytes(nrays, nrays) + arena > budget;
}

// Epoch queue: the unstarted rays of each live request as one segment, the
// cancelled first (so their rays drain at once), then fewest unstarted rays
// first (TARTARUS_SERVE_SMALLEST_FIRST) or by first ray (TARTARUS_SERVE_ARRIVAL).
struct SegmentSource {
    int entry;
    int cancelled;
    long long nrays, started, ray_begin;
};
struct Segment {
    int entry;
    long long ray;      // absolute index of the segment's first ray
    long long q_begin;  // first queue position
    long long count;
};
std::vector<Segment> build_segments(const std::vector<SegmentSource>& live, int order);
// Rays handed out from each segment when the queue head stopped at `taken`
// (positions are consumed in segment order).
std::vector<long long> consumed_per_segment(const std::vector<Segment>& segs, long long taken);

}  // namespace host
}  // namespace tartarus
