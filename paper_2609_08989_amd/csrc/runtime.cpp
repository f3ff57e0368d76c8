// runtime.cpp -- host side of the C ABI declared in include/tartarus.h.
//
// The host validates arguments, copies them into a device job table (one entry
// per camera or request) and launches the persistent integrator; it performs
// none of the ray arithmetic.  Serving (submit / poll) runs a scheduler thread
// that admits requests by HBM budget and traces them together in epochs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/tartarus.h"
#include "host_logic.hpp"
#include "internal.hpp"
#include "order.hpp"

using namespace tartarus;
using namespace tartarus::host;

extern "C" hipError_t tartarus_launch_trace(int kind, int prec, int method, const LaunchArgs* args, int grid, int block,
                                            hipStream_t stream);
extern "C" hipError_t tartarus_launch_setup(int kind, const LaunchArgs* args, hipStream_t stream);
extern "C" hipError_t tartarus_launch_finish(const LaunchArgs* args, int job0, int njobs, long long max_rays,
                                            hipStream_t stream);
extern "C" hipError_t tartarus_occupancy(int kind, int prec, int method, int serve, int block, int* blocks_per_cu);
extern "C" hipError_t tartarus_launch_build_table(double a, int nr, int nth, double r_min, double r_max,
                                                  double* table, hipStream_t stream);
extern "C" hipError_t tartarus_launch_order(const LaunchArgs* args, long long total, unsigned char* key,
                                            unsigned int* count, unsigned int* cursor, unsigned int* order,
                                            hipStream_t stream);
extern "C" hipError_t tartarus_launch_table_interleave(const LaunchArgs* args, double* inter, hipStream_t stream);
extern "C" hipError_t tartarus_launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t stream);
extern "C" hipError_t tartarus_launch_fill_u64(unsigned long long* p, unsigned long long v, long long n,
                                               hipStream_t stream);
extern "C" hipError_t tartarus_noalloc_scratch(int device, void** ptr);
extern "C" hipError_t tartarus_launch_job_upload(const DevJob* job, DevJob* dst, hipStream_t stream);

namespace {

int hip_fail(hipError_t e, const char* what)
{
    return fail(TARTARUS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

// Per-call launch resources.  A trace copies its job table through pinned host
// memory into a device table and resets a queue head, then launches; the slot
// is reused only after the event recorded behind that launch has completed, so
// calls stay asynchronous without a host buffer outliving its copy.
struct Slot {
    DevJob* djobs = nullptr;
    DevJob* hjobs = nullptr;             // pinned
    JobConst* djc = nullptr;             // per-job constants (device, written by the set-up kernel)
    int cap = 0;
    unsigned long long* head = nullptr;
    unsigned char* ord = nullptr;        // cost-ordered queue: order[n] u32, key[n] u8, count and cursor
    size_t ord_cap = 0;                  // bytes
    double* rec = nullptr;               // per-ray records for the finishing pass
    size_t rec_cap = 0;                  // rays
    double* inter = nullptr;             // tabulated metric interleaved by grid point
    size_t inter_cap = 0;                // doubles
    hipEvent_t ev = nullptr;
    bool pending = false;
};
constexpr int kSlots = 16;
constexpr long long kCostOrderMin = 4096;  // default: cost-ordered queue from this many rays on

struct Device {
    bool ready = false;
    int id = 0;
    int cus = 0;
    size_t budget = 0;
    std::mutex mu;                       // guards the slots and the tuning table
    Slot slots[kSlots];
    int next_slot = 0;
    std::map<int, tartarus_launch> tuned;  // key: tune_key(kind, precision, method)
    // integrator timing (tartarus_kernel_timing): an event pair around each
    // integrator launch while on; pairs are read back by tartarus_kernel_time
    bool ktime_on = false;
    unsigned char* scratch = nullptr;    // device address of the allocation-free trace's array
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ktime_pending, ktime_spare;
};
Device g_dev;

// Drains the recorded integrator event pairs into (total ms, launches).
int ktime_collect(double& total_ms, long long& launches)
{
    total_ms = 0.0;
    launches = 0;
    // a pair leaves the pending list only once it has been read, so an error
    // part-way leaves the unread pairs pending and none in both lists
    while (!g_dev.ktime_pending.empty()) {
        const auto pr = g_dev.ktime_pending.front();
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        total_ms += ms;
        ++launches;
        g_dev.ktime_pending.erase(g_dev.ktime_pending.begin());
        g_dev.ktime_spare.push_back(pr);
    }
    return TARTARUS_OK;
}

int take_slot(int njobs, Slot*& out)
{
    Slot& S = g_dev.slots[g_dev.next_slot];
    g_dev.next_slot = (g_dev.next_slot + 1) % kSlots;
    if (S.pending) {
        HIP_TRY(hipEventSynchronize(S.ev));
        S.pending = false;
    }
    if (!S.ev) HIP_TRY(hipEventCreateWithFlags(&S.ev, hipEventDisableTiming));
    if (!S.head) HIP_TRY(hipMalloc(&S.head, sizeof(unsigned long long)));
    if (njobs > S.cap) {
        if (S.djobs) (void)hipFree(S.djobs);
        if (S.hjobs) (void)hipHostFree(S.hjobs);
        if (S.djc) (void)hipFree(S.djc);
        S.djobs = nullptr;
        S.hjobs = nullptr;
        S.djc = nullptr;
        S.cap = 0;
        const int cap = std::max(njobs, 64);
        if (hipMalloc(&S.djobs, sizeof(DevJob) * cap) != hipSuccess) return fail(TARTARUS_E_NOMEM, "job table allocation failed");
        if (hipMalloc(&S.djc, sizeof(JobConst) * cap) != hipSuccess) return fail(TARTARUS_E_NOMEM, "job constants allocation failed");
        if (hipHostMalloc(&S.hjobs, sizeof(DevJob) * cap, hipHostMallocDefault) != hipSuccess)
            return fail(TARTARUS_E_NOMEM, "pinned job table allocation failed");
        S.cap = cap;
    }
    out = &S;
    return TARTARUS_OK;
}

int tune_key(int kind, int prec, int method) { return (kind * 2 + prec) * 8 + method; }

tartarus_launch default_launch(int kind, int prec, int method)
{
    auto it = g_dev.tuned.find(tune_key(kind, prec, method));
    if (it != g_dev.tuned.end()) return it->second;
    tartarus_launch L;
    L.block_threads = 256;
    L.blocks_per_cu = 0;
    L.chunk = 1;
    L.refill_min = 4;
    L.order = TARTARUS_ORDER_DEFAULT;
    return L;
}

// Resolve a launch request against the tuned or default shape (the rules are
// in host_logic.cpp); n_rays > 0 is a one-shot trace of that many rays.  The
// caller holds g_dev.mu (the tuning table).
int resolve_launch(int kind, int prec, int method, const tartarus_launch* req, tartarus_launch& L, int& grid,
                   long long n_rays = 0, int serve = 0)
{
    int rc = merge_shape(default_launch(kind, prec, method), req, L);
    if (rc) return rc;
    int occ = 0;
    HIP_TRY(tartarus_occupancy(kind, prec, method, serve, L.block_threads, &occ));
    return finish_shape(L, occ, n_rays, g_dev.cus, grid);
}

// Device memory one trace works in.
struct TraceMem {
    DevJob* djobs;                  // job table, already filled on the stream
    JobConst* djc;                  // per-job constants (written by job_setup)
    unsigned long long* head;       // queue head
    unsigned int* order;            // cost-ordered queue: order[n], then
    unsigned char* key;             //   key[n],
    unsigned int* count;            //   count[kOrderBuckets], cursor[kOrderBuckets]
    double* inter;                  // tabulated metric interleaved by grid point
};

bool cost_ordered(const tartarus_launch& L, long long n)
{
    return n <= 0xffffffffll &&
           (L.order == TARTARUS_ORDER_COST || (L.order == TARTARUS_ORDER_DEFAULT && n >= kCostOrderMin));
}

// The device part of a trace, on the stream, after the job table: queue head,
// set-up, (table interleave,) cost order, integrator (bracketed by an event
// pair when timed), finishing pass.
int launch_sequence(const tartarus_metric* metric, const tartarus_solver* solver, const tartarus_launch& L, int grid,
                    int ncams, long long per, const TraceMem& M, bool timed, hipStream_t stream)
{
    const int kind = metric->kind, prec = kernel_precision(solver), method = solver->method;
    HIP_TRY(tartarus_launch_fill_u64(M.head, 0ull, 1, stream));
    LaunchArgs A;
    fill_args(A, metric, solver);
    A.jobs = M.djobs;
    A.jc = M.djc;
    A.njobs = ncams;
    A.chunk = L.chunk;
    A.refill_min = L.refill_min;
    A.first_ray = 0;
    A.total_rays = per * ncams;
    A.head = M.head;
    HIP_TRY(tartarus_launch_setup(kind, &A, stream));
    if (kind == TARTARUS_METRIC_TABLE) {
        HIP_TRY(tartarus_launch_table_interleave(&A, M.inter, stream));
        A.table_inter = M.inter;
    }
    const long long n = A.total_rays;
    if (cost_ordered(L, n)) {
        unsigned int* cursor = M.count + kOrderBuckets;
        HIP_TRY(tartarus_launch_fill_u32(M.count, 0u, kOrderBuckets, stream));
        HIP_TRY(tartarus_launch_order(&A, n, M.key, M.count, cursor, M.order, stream));
        A.order = M.order;
    }
    A.tile = L.order == TARTARUS_ORDER_TILE ? 1 : 0;
    if (timed) {
        std::pair<hipEvent_t, hipEvent_t> kt(nullptr, nullptr);
        if (!g_dev.ktime_spare.empty()) {
            kt = g_dev.ktime_spare.back();
            g_dev.ktime_spare.pop_back();
        } else {
            HIP_TRY(hipEventCreate(&kt.first));
            const hipError_t e = hipEventCreate(&kt.second);
            if (e != hipSuccess) {
                (void)hipEventDestroy(kt.first);
                return hip_fail(e, "hipEventCreate");
            }
        }
        // the pair goes back to the pool if the launch cannot be enqueued
        hipError_t e = hipEventRecord(kt.first, stream);
        if (e == hipSuccess) e = tartarus_launch_trace(kind, prec, method, &A, grid, L.block_threads, stream);
        if (e == hipSuccess) e = hipEventRecord(kt.second, stream);
        if (e != hipSuccess) {
            g_dev.ktime_spare.push_back(kt);
            return hip_fail(e, "integrator launch");
        }
        g_dev.ktime_pending.push_back(kt);
    } else {
        HIP_TRY(tartarus_launch_trace(kind, prec, method, &A, grid, L.block_threads, stream));
    }
    for (int c0 = 0; c0 < ncams; c0 += 65535)
        HIP_TRY(tartarus_launch_finish(&A, c0, std::min(65535, ncams - c0), per, stream));
    return TARTARUS_OK;
}

// Enqueue one trace (no validation) on the stream, with the per-call slot's
// growable buffers.
int enqueue_trace(const tartarus_metric* metric, const tartarus_camera* cams, int ncams, const tartarus_disk* disk,
                  const tartarus_solver* solver, const tartarus_outputs* out, const tartarus_launch* launch,
                  hipStream_t stream)
{
    const int kind = metric->kind, prec = kernel_precision(solver), method = solver->method;
    tartarus_launch L;
    int grid = 0;
    const long long n_rays = (long long)cams[0].nx * cams[0].ny * ncams;
    int rc = resolve_launch(kind, prec, method, launch, L, grid, n_rays);
    if (rc) return rc;
    Slot* S = nullptr;
    if ((rc = take_slot(ncams, S))) return rc;
    const long long per = (long long)cams[0].nx * cams[0].ny;
    const size_t nrec = (size_t)per * ncams;
    if (nrec > S->rec_cap) {
        if (S->rec) (void)hipFree(S->rec);
        S->rec = nullptr;
        S->rec_cap = 0;
        HIP_TRY(hipMalloc(&S->rec, nrec * REC_DOUBLES * sizeof(double)));
        S->rec_cap = nrec;
    }
    TraceMem M{S->djobs, S->djc, S->head, nullptr, nullptr, nullptr, nullptr};
    if (kind == TARTARUS_METRIC_TABLE) {
        const size_t need = (size_t)metric->nr * metric->nth * 20;
        if (need > S->inter_cap) {
            if (S->inter) (void)hipFree(S->inter);
            S->inter = nullptr;
            S->inter_cap = 0;
            HIP_TRY(hipMalloc(&S->inter, need * sizeof(double)));
            S->inter_cap = need;
        }
        M.inter = S->inter;
    }
    if (cost_ordered(L, n_rays)) {
        const size_t key_bytes = ((size_t)n_rays + 255) / 256 * 256;
        const size_t need = (size_t)n_rays * 4 + key_bytes + 2 * kOrderBuckets * sizeof(unsigned int);
        if (need > S->ord_cap) {
            if (S->ord) (void)hipFree(S->ord);
            S->ord = nullptr;
            S->ord_cap = 0;
            HIP_TRY(hipMalloc(&S->ord, need));
            S->ord_cap = need;
        }
        M.order = reinterpret_cast<unsigned int*>(S->ord);
        M.key = S->ord + (size_t)n_rays * 4;
        M.count = reinterpret_cast<unsigned int*>(M.key + key_bytes);
    }
    for (int c = 0; c < ncams; ++c)
        fill_job(S->hjobs[c], metric, cams[c], disk, solver, out, c * per, c * per, S->rec + (size_t)c * per * REC_DOUBLES);
    HIP_TRY(hipMemcpyAsync(S->djobs, S->hjobs, sizeof(DevJob) * ncams, hipMemcpyHostToDevice, stream));
    if ((rc = launch_sequence(metric, solver, L, grid, ncams, per, M, g_dev.ktime_on, stream))) return rc;
    HIP_TRY(hipEventRecord(S->ev, stream));
    S->pending = true;
    return TARTARUS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported
// ---------------------------------------------------------------------------
extern "C" const char* tartarus_last_error(void) { return last_error(); }

extern "C" int tartarus_validate(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                                 const tartarus_disk* disk, const tartarus_solver* solver)
{
    return validate_all(metric, cams, ncams, disk, solver);
}

extern "C" int tartarus_init(int device, size_t hbm_budget_bytes)
{
    std::lock_guard<std::mutex> lk(g_dev.mu);
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(TARTARUS_E_DEVICE, "no HIP device");
    if (device < 0 || device >= n) return fail(TARTARUS_E_INVALID, "device index out of range");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(TARTARUS_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950");
    if (g_dev.ready && g_dev.id == device) {
        g_dev.budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)8 << 30;
        return TARTARUS_OK;
    }
    // the allocation-free trace's working memory on this device (current now)
    void* scratch = nullptr;
    HIP_TRY(tartarus_noalloc_scratch(device, &scratch));
    g_dev.id = device;
    g_dev.scratch = static_cast<unsigned char*>(scratch);
    g_dev.cus = prop.multiProcessorCount;
    g_dev.budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)8 << 30;
    g_dev.ready = true;
    return TARTARUS_OK;
}

extern "C" int tartarus_trace_launch(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                                     const tartarus_disk* disk, const tartarus_solver* solver,
                                     const tartarus_outputs* out, const tartarus_launch* launch, void* hip_stream)
{
    int rc = validate_all(metric, cams, ncams, disk, solver);
    if (rc) return rc;
    if ((rc = check_outputs(out))) return rc;
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    HIP_TRY(hipSetDevice(g_dev.id));
    return enqueue_trace(metric, cams, ncams, disk, solver, out, launch, (hipStream_t)hip_stream);
}

extern "C" int tartarus_trace(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                              const tartarus_disk* disk, const tartarus_solver* solver, const tartarus_outputs* out,
                              void* hip_stream)
{
    return tartarus_trace_launch(metric, cams, ncams, disk, solver, out, nullptr, hip_stream);
}

static_assert(NoallocLayout::bytes == TARTARUS_NOALLOC_SCRATCH_BYTES, "header states the scratch size");
static_assert(NoallocLayout::max_rays == TARTARUS_NOALLOC_MAX_RAYS, "header states the ray limit");
static_assert(NoallocLayout::max_cameras == TARTARUS_NOALLOC_MAX_CAMERAS, "header states the camera limit");
static_assert(NoallocLayout::buckets == kOrderBuckets, "cost-order counters");

extern "C" int tartarus_trace_noalloc(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                                      const tartarus_disk* disk, const tartarus_solver* solver,
                                      const tartarus_outputs* out, const tartarus_launch* launch, void* hip_stream)
{
    int rc = validate_all(metric, cams, ncams, disk, solver);
    if (rc) return rc;
    if ((rc = check_outputs(out))) return rc;
    if (metric->kind != TARTARUS_METRIC_KERR)
        return fail(TARTARUS_E_INVALID, "the allocation-free trace takes the analytic Kerr metric");
    using NL = NoallocLayout;
    if (ncams > NL::max_cameras) return fail(TARTARUS_E_TOO_LARGE, "more cameras than the allocation-free trace holds");
    const long long per = (long long)cams[0].nx * cams[0].ny;
    if (per * ncams > NL::max_rays) return fail(TARTARUS_E_TOO_LARGE, "more rays than the allocation-free trace holds");
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready || !g_dev.scratch) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    HIP_TRY(hipSetDevice(g_dev.id));
    hipStream_t stream = (hipStream_t)hip_stream;
    tartarus_launch L;
    int grid = 0;
    if ((rc = resolve_launch(metric->kind, kernel_precision(solver), solver->method, launch, L, grid, per * ncams)))
        return rc;
    unsigned char* b = g_dev.scratch;
    TraceMem M{reinterpret_cast<DevJob*>(b + NL::jobs), reinterpret_cast<JobConst*>(b + NL::jc),
               reinterpret_cast<unsigned long long*>(b + NL::head), reinterpret_cast<unsigned int*>(b + NL::order),
               b + NL::key, reinterpret_cast<unsigned int*>(b + NL::count), nullptr};
    double* rec = reinterpret_cast<double*>(b + NL::rec);
    for (int c = 0; c < ncams; ++c) {
        DevJob J;
        fill_job(J, metric, cams[c], disk, solver, out, c * per, c * per, rec + (size_t)c * per * REC_DOUBLES);
        HIP_TRY(tartarus_launch_job_upload(&J, M.djobs + c, stream));
    }
    return launch_sequence(metric, solver, L, grid, ncams, per, M, false, stream);
}

extern "C" int tartarus_build_kerr_table(double a, int nr, int nth, double r_min, double r_max, double* table,
                                         void* hip_stream)
{
    if (!(std::isfinite(a) && a >= 0.0 && a < 1.0)) return fail(TARTARUS_E_INVALID, "spin a must be in [0, 1)");
    if (nr < 4 || nth < 4) return fail(TARTARUS_E_INVALID, "table needs nr, nth >= 4");
    if (!(std::isfinite(r_min) && r_min > 0.0) || !(r_max > r_min) || !std::isfinite(r_max))
        return fail(TARTARUS_E_INVALID, "table needs 0 < r_min < r_max");
    if (!table) return fail(TARTARUS_E_INVALID, "table is NULL");
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    HIP_TRY(hipSetDevice(g_dev.id));
    HIP_TRY(tartarus_launch_build_table(a, nr, nth, r_min, r_max, table, (hipStream_t)hip_stream));
    return TARTARUS_OK;
}

// ---------------------------------------------------------------------------
// autotuner: coordinate search over the launch shape on the caller's workload
// ---------------------------------------------------------------------------
namespace {

// Best of kTuneRepeats traces with launch shape L: a single run varies by a
// few percent from launch to launch, enough to mislead a coordinate search.
constexpr int kTuneRepeats = 3;

int time_trace(const tartarus_metric* metric, const tartarus_camera* cams, int ncams, const tartarus_disk* disk,
               const tartarus_solver* solver, const tartarus_outputs* out, const tartarus_launch& L,
               hipStream_t stream, float& ms)
{
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    ms = 0.f;
    for (int rep = 0; rep < kTuneRepeats; ++rep) {
        HIP_TRY(hipEventRecord(e0, stream));
        int rc = enqueue_trace(metric, cams, ncams, disk, solver, out, &L, stream);
        if (rc) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (rep == 0 || t < ms) ms = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return TARTARUS_OK;
}

}  // namespace

extern "C" int tartarus_autotune(const tartarus_metric* metric, const tartarus_camera* cams, int ncams,
                                 const tartarus_disk* disk, const tartarus_solver* solver,
                                 const tartarus_outputs* out, void* hip_stream, tartarus_launch* best)
{
    int rc = validate_all(metric, cams, ncams, disk, solver);
    if (rc) return rc;
    if ((rc = check_outputs(out))) return rc;
    if (!best) return fail(TARTARUS_E_INVALID, "best is NULL");
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    HIP_TRY(hipSetDevice(g_dev.id));
    hipStream_t stream = (hipStream_t)hip_stream;
    const int kind = metric->kind, prec = kernel_precision(solver), method = solver->method;
    g_dev.tuned.erase(tune_key(kind, prec, method));
    tartarus_launch cur = default_launch(kind, prec, method);
    int grid = 0;
    if ((rc = resolve_launch(kind, prec, method, &cur, cur, grid))) return rc;
    if (cur.order == TARTARUS_ORDER_DEFAULT) {
        // report the order the default stands for on this trace
        long long n = 0;
        for (int c = 0; c < ncams; ++c) n += (long long)cams[c].nx * cams[c].ny;
        cur.order = n >= kCostOrderMin ? TARTARUS_ORDER_COST : TARTARUS_ORDER_PIXEL;
    }
    float best_ms = 0.f;
    if ((rc = time_trace(metric, cams, ncams, disk, solver, out, cur, stream, best_ms))) return rc;  // warm-up
    if ((rc = time_trace(metric, cams, ncams, disk, solver, out, cur, stream, best_ms))) return rc;
    const int blocks[] = {64, 128, 256};
    const int chunks[] = {1, 16, 64, 256, 1024};
    const int refills[] = {1, 8, 16, 32, 48};
    for (int pass = 0; pass < 2; ++pass) {
        for (int b : blocks) {
            tartarus_launch L = cur;
            L.block_threads = b;
            L.blocks_per_cu = 0;
            int g2 = 0;
            if (resolve_launch(kind, prec, method, &L, L, g2)) continue;
            float ms = 0.f;
            if ((rc = time_trace(metric, cams, ncams, disk, solver, out, L, stream, ms))) return rc;
            if (ms < best_ms) { best_ms = ms; cur = L; }
        }
        int occ = 0;
        HIP_TRY(tartarus_occupancy(kind, prec, method, 0, cur.block_threads, &occ));
        for (int bpc = 1; bpc <= occ; ++bpc) {
            tartarus_launch L = cur;
            L.blocks_per_cu = bpc;
            float ms = 0.f;
            if ((rc = time_trace(metric, cams, ncams, disk, solver, out, L, stream, ms))) return rc;
            if (ms < best_ms) { best_ms = ms; cur = L; }
        }
        for (int c : chunks) {
            tartarus_launch L = cur;
            L.chunk = c;
            float ms = 0.f;
            if ((rc = time_trace(metric, cams, ncams, disk, solver, out, L, stream, ms))) return rc;
            if (ms < best_ms) { best_ms = ms; cur = L; }
        }
        for (int f : refills) {
            tartarus_launch L = cur;
            L.refill_min = f;
            float ms = 0.f;
            if ((rc = time_trace(metric, cams, ncams, disk, solver, out, L, stream, ms))) return rc;
            if (ms < best_ms) { best_ms = ms; cur = L; }
        }
        for (int o : {(int)TARTARUS_ORDER_PIXEL, (int)TARTARUS_ORDER_COST, (int)TARTARUS_ORDER_TILE}) {
            tartarus_launch L = cur;
            L.order = o;
            float ms = 0.f;
            if ((rc = time_trace(metric, cams, ncams, disk, solver, out, L, stream, ms))) return rc;
            if (ms < best_ms) { best_ms = ms; cur = L; }
        }
    }
    g_dev.tuned[tune_key(kind, prec, method)] = cur;
    *best = cur;
    return TARTARUS_OK;
}

namespace {
void server_stop();
}

extern "C" int tartarus_shutdown(void)
{
    server_stop();
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready) return TARTARUS_OK;
    (void)hipSetDevice(g_dev.id);
    for (Slot& S : g_dev.slots) {
        if (S.pending) (void)hipEventSynchronize(S.ev);
        if (S.djobs) (void)hipFree(S.djobs);
        if (S.hjobs) (void)hipHostFree(S.hjobs);
        if (S.djc) (void)hipFree(S.djc);
        if (S.head) (void)hipFree(S.head);
        if (S.ord) (void)hipFree(S.ord);
        if (S.rec) (void)hipFree(S.rec);
        if (S.inter) (void)hipFree(S.inter);
        if (S.ev) (void)hipEventDestroy(S.ev);
        S = Slot();
    }
    g_dev.tuned.clear();
    for (auto* v : {&g_dev.ktime_pending, &g_dev.ktime_spare}) {
        for (auto& pr : *v) {
            (void)hipEventSynchronize(pr.second);
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        v->clear();
    }
    g_dev.ktime_on = false;
    g_dev.ready = false;
    return TARTARUS_OK;
}

extern "C" int tartarus_kernel_timing(int enable)
{
    if (enable != 0 && enable != 1) return fail(TARTARUS_E_INVALID, "enable must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    g_dev.ktime_on = enable == 1;
    return TARTARUS_OK;
}

extern "C" int tartarus_kernel_time(double* total_ms, long long* launches)
{
    if (!total_ms || !launches) return fail(TARTARUS_E_INVALID, "total_ms and launches must not be NULL");
    std::lock_guard<std::mutex> lk(g_dev.mu);
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    HIP_TRY(hipSetDevice(g_dev.id));
    return ktime_collect(*total_ms, *launches);
}

// ---------------------------------------------------------------------------
// serving: continuous batching of image requests
//
// Requests are admitted in arrival order while their output bytes plus the
// ray-slot arena fit the HBM budget (and a request-table entry is free).  All
// admitted requests share one device queue of global ray indices; the
// persistent kernel runs in epochs of a bounded number of wavefront
// iterations, parks unfinished rays in their lane's slot (exact bits) and resumes them in
// the next epoch, so requests that arrive while others are on the device join
// at the next epoch boundary and their rays overlap with the running ones.
// ---------------------------------------------------------------------------
namespace {

constexpr int kMaxEntries = 256;        // request-table entries (requests in flight)
constexpr long long kEpochIterations = 192;  // wavefront iterations (attempts) per epoch

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    tartarus_metric metric;
    tartarus_camera cam;
    tartarus_disk disk;
    tartarus_solver solver;
    tartarus_outputs out;
    long long nrays = 0;
    size_t held = 0;        // device bytes counted against the budget while admitted
    int state = 0;          // 0 queued, 1 running, 2 done
    int entry = -1;
    long long ray_begin = 0;
    double* rec = nullptr;  // device records of its rays while admitted
    long long rec_rays = 0; // capacity of rec in rays
    long long started = 0;  // rays already handed out to lanes
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    bool cancel_req = false, cancel_sent = false, cancel_acked = false;
    bool too_large = false;  // can never fit the budget next to the slot arena
};

// Per-epoch scheduling state: one device block and its pinned host mirror.
// Before each epoch the host writes the whole block with one copy (request
// table, queue head reset to zero, each entry's count of unfinished rays, the
// directory of live entries and the queue segments), and after it reads back
// head and counts with another: as separate small copies they cost ~13 us of
// stream time each between two epochs.  The host mirror of the counts equals
// the device's whenever the host writes it (it was read back after the
// previous epoch and only fresh entries change).  The queue head and the
// counts each start a 256-byte line of their own: every wavefront's refill
// adds to the head and every wavefront iteration subtracts from counts, and
// sharing one line made those atomics contend (epochs 7 % slower).
struct EpochBlock {
    DevJob jobs[kMaxEntries];
    alignas(256) unsigned long long head;
    alignas(256) unsigned int remaining[kMaxEntries * kRemainingStride];
    int dir_job[kMaxEntries];
    long long dir_begin[kMaxEntries];
    long long seg_q[kMaxEntries + 1];
    long long seg_ray[kMaxEntries];
};

struct Server {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    bool running = false;
    bool have_solver = false;
    tartarus_solver solver;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    uint64_t entry_ticket[kMaxEntries] = {};
    size_t used_bytes = 0;
    long long next_ray = 0;    // global ray indices assigned to admitted requests so far
    int serve_order = TARTARUS_SERVE_SMALLEST_FIRST;
    long long* dseg_q = nullptr;    // epoch queue segments (see LaunchArgs)
    long long* dseg_ray = nullptr;
    long long* hseg_q = nullptr;
    long long* hseg_ray = nullptr;
    int seg_entry[kMaxEntries] = {};
    // device resources (owned by the scheduler thread once started); the
    // per-epoch arrays below point into dblk (device) and hblk (pinned host)
    bool dev_ready = false;
    hipStream_t stream = nullptr;
    EpochBlock* dblk = nullptr;
    EpochBlock* hblk = nullptr;
    bool jobs_dirty = true;           // the host's request table differs from the device's
    // finishing passes of the requests the last epoch completed run on fstream
    // beside the next epoch; fin_ev marks their end, fin_pending their entries
    hipStream_t fstream = nullptr;
    hipEvent_t fin_ev = nullptr;
    std::vector<int> fin_pending;
    DevJob* djobs = nullptr;
    DevJob* hjobs = nullptr;
    JobConst* djc = nullptr;
    unsigned int* dremaining = nullptr;
    unsigned int* hremaining = nullptr;
    long long* ddir_begin = nullptr;
    int* ddir_job = nullptr;
    long long* hdir_begin = nullptr;
    int* hdir_job = nullptr;
    double* slots = nullptr;
    unsigned int* slot_live = nullptr;
    unsigned long long* dhead = nullptr;
    unsigned long long* hhead = nullptr;
    long long nslots = 0;
    int grid = 0, block = 0;
    size_t arena_bytes = 0;
    // freed per-request record buffers kept for reuse (hipFree would
    // synchronize the device between epochs), counted against the budget
    RecordPool rec_pool;
    std::string dev_error;
};
Server g_srv;

// Free every pooled record buffer (hipFree synchronizes the device; done only
// when admission needs the memory).
void rec_pool_release(Server& S)
{
    for (void* p : S.rec_pool.drain()) (void)hipFree(p);
}

// Return a request's record buffer to the pool (kept while the pool stays under
// a quarter of the HBM budget, else freed).
void rec_give(Server& S, double* p, long long cap)
{
    if (!S.rec_pool.give(p, cap, g_dev.budget / 4)) (void)hipFree(p);
}

int server_alloc(int prec, int method)
{
    Server& S = g_srv;
    HIP_TRY(hipSetDevice(g_dev.id));
    HIP_TRY(hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&S.fstream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&S.fin_ev, hipEventDisableTiming));
    S.fin_pending.clear();
    S.jobs_dirty = true;
    tartarus_launch L;
    int grid = 0;
    {
        // the tuning table is shared with tartarus_autotune
        std::lock_guard<std::mutex> dlk(g_dev.mu);
        int rc = resolve_launch(TARTARUS_METRIC_KERR, prec, method, nullptr, L, grid, 0, 1);
        if (rc) return rc;
    }
    S.grid = grid;
    S.block = L.block_threads;
    S.nslots = (long long)grid * L.block_threads;
    HIP_TRY(hipMalloc(&S.dblk, sizeof(EpochBlock)));
    HIP_TRY(hipHostMalloc(&S.hblk, sizeof(EpochBlock), hipHostMallocDefault));
    HIP_TRY(hipMalloc(&S.djc, sizeof(JobConst) * kMaxEntries));
    // device addresses of the block's parts: offsets from its base (nothing is
    // dereferenced on the host)
    char* const db = reinterpret_cast<char*>(S.dblk);
    S.djobs = reinterpret_cast<DevJob*>(db + offsetof(EpochBlock, jobs));
    S.dhead = reinterpret_cast<unsigned long long*>(db + offsetof(EpochBlock, head));
    S.dremaining = reinterpret_cast<unsigned int*>(db + offsetof(EpochBlock, remaining));
    S.ddir_job = reinterpret_cast<int*>(db + offsetof(EpochBlock, dir_job));
    S.ddir_begin = reinterpret_cast<long long*>(db + offsetof(EpochBlock, dir_begin));
    S.dseg_q = reinterpret_cast<long long*>(db + offsetof(EpochBlock, seg_q));
    S.dseg_ray = reinterpret_cast<long long*>(db + offsetof(EpochBlock, seg_ray));
    S.hjobs = S.hblk->jobs;
    S.hhead = &S.hblk->head;
    S.hremaining = S.hblk->remaining;
    S.hdir_job = S.hblk->dir_job;
    S.hdir_begin = S.hblk->dir_begin;
    S.hseg_q = S.hblk->seg_q;
    S.hseg_ray = S.hblk->seg_ray;
    HIP_TRY(hipMalloc(&S.slots, sizeof(double) * SLOT_DOUBLES * S.nslots));
    HIP_TRY(hipMalloc(&S.slot_live, sizeof(unsigned int) * S.nslots));
    std::memset(S.hblk, 0, sizeof(EpochBlock));
    HIP_TRY(tartarus_launch_fill_u32(S.slot_live, 0u, S.nslots, S.stream));
    HIP_TRY(hipMemcpyAsync(S.dblk, S.hblk, sizeof(EpochBlock), hipMemcpyHostToDevice, S.stream));
    HIP_TRY(hipStreamSynchronize(S.stream));
    S.arena_bytes = sizeof(double) * SLOT_DOUBLES * S.nslots + sizeof(unsigned int) * S.nslots +
                    (sizeof(DevJob) + 16) * kMaxEntries;
    S.dev_ready = true;
    return TARTARUS_OK;
}

void server_free()
{
    Server& S = g_srv;
    if (S.stream) (void)hipStreamSynchronize(S.stream);
    if (S.fstream) (void)hipStreamSynchronize(S.fstream);
    (void)hipFree(S.dblk);
    (void)hipHostFree(S.hblk);
    (void)hipFree(S.djc);
    (void)hipFree(S.slots);
    (void)hipFree(S.slot_live);
    rec_pool_release(S);
    if (S.stream) (void)hipStreamDestroy(S.stream);
    if (S.fstream) (void)hipStreamDestroy(S.fstream);
    if (S.fin_ev) (void)hipEventDestroy(S.fin_ev);
    S.fstream = nullptr; S.fin_ev = nullptr;
    S.fin_pending.clear();
    S.dblk = nullptr; S.hblk = nullptr;
    S.djobs = nullptr; S.djc = nullptr; S.hjobs = nullptr; S.dremaining = nullptr; S.hremaining = nullptr;
    S.ddir_begin = nullptr; S.ddir_job = nullptr; S.hdir_begin = nullptr; S.hdir_job = nullptr;
    S.dseg_q = nullptr; S.dseg_ray = nullptr; S.hseg_q = nullptr; S.hseg_ray = nullptr;
    S.slots = nullptr; S.slot_live = nullptr; S.dhead = nullptr; S.hhead = nullptr; S.stream = nullptr;
    S.dev_ready = false;
}

bool any_live(const Server& S)
{
    for (int e = 0; e < kMaxEntries; ++e)
        if (S.entry_ticket[e]) return true;
    return false;
}

void finish_request(Server& S, uint64_t ticket, Request& R)
{
    R.state = 2;
    R.t_done = now_ns();
    if (R.entry >= 0) {
        S.entry_ticket[R.entry] = 0;
        S.hjobs[R.entry].cancelled = 0;
        R.entry = -1;
        S.used_bytes -= R.held;
        R.held = 0;
    }
    if (R.rec) {
        rec_give(S, R.rec, R.rec_rays);
        R.rec = nullptr;
    }
    (void)ticket;
}

// Completes the requests whose finishing pass went to fstream after the last
// epoch: waits for it, then marks them done.  Called with lk released;
// returns with it released.
int complete_finished(Server& S, std::unique_lock<std::mutex>& lk)
{
    if (S.fin_pending.empty()) return TARTARUS_OK;
    HIP_TRY(hipEventSynchronize(S.fin_ev));
    lk.lock();
    for (int e : S.fin_pending) {
        const uint64_t t = S.entry_ticket[e];
        finish_request(S, t, S.reqs[t]);
    }
    // (finish_request clears the entries' cancel flags on the host only: a
    // freed entry is not read on the device until an admission refills it,
    // which marks the table for copying)
    S.fin_pending.clear();
    S.done_cv.notify_all();
    lk.unlock();
    return TARTARUS_OK;
}

bool finishing(const Server& S, int e)
{
    return std::find(S.fin_pending.begin(), S.fin_pending.end(), e) != S.fin_pending.end();
}

// One scheduling round: admit, run one epoch, collect completions.  The
// finishing passes of the requests an epoch completes run on their own stream
// while the next epoch traces; those requests are marked done when their pass
// has ended.
int server_round(std::unique_lock<std::mutex>& lk)
{
    Server& S = g_srv;
    // ---- admission (arrival order; head-of-line blocking keeps it FIFO)
    std::vector<int> fresh;
    while (!S.queue.empty()) {
        const uint64_t t = S.queue.front();
        Request& R = S.reqs[t];
        if (never_fits(R.nrays, S.arena_bytes, g_dev.budget)) {
            // submit checked against an estimate of the arena; this one never fits
            S.queue.pop_front();
            R.too_large = true;
            R.state = 2;
            R.t_done = now_ns();
            continue;
        }
        int entry = -1;
        for (int e = 0; e < kMaxEntries; ++e)
            if (!S.entry_ticket[e]) { entry = e; break; }
        if (entry < 0) break;
        // records: a pooled buffer of n..4n rays if there is one, else a new one
        // of n; the pool's buffers count against the budget, and are released
        // when the request would fit without them
        long long cap = S.rec_pool.pooled_capacity(R.nrays);
        bool pooled = cap > 0;
        if (!pooled) cap = R.nrays;
        if (!admission_fits(S.used_bytes, S.rec_pool.bytes(), S.arena_bytes, g_dev.budget, R.nrays, cap, pooled)) {
            if (S.rec_pool.empty() ||
                !admission_fits(S.used_bytes, 0, S.arena_bytes, g_dev.budget, R.nrays, R.nrays, false))
                break;   // waits for running requests to release memory
            rec_pool_release(S);
            pooled = false;
            cap = R.nrays;
        }
        if (pooled) {
            R.rec = (double*)S.rec_pool.take_pooled(R.nrays, cap);
        } else if (hipMalloc(&R.rec, (size_t)cap * kRecordBytes) != hipSuccess) {
            (void)hipGetLastError();
            R.rec = nullptr;
        }
        R.rec_rays = cap;
        if (!R.rec) {
            if (any_live(S)) break;   // retried once running requests have released memory
            S.queue.pop_front();      // nothing else holds device memory: it never fits
            R.too_large = true;
            R.state = 2;
            R.t_done = now_ns();
            continue;
        }
        S.queue.pop_front();
        R.entry = entry;
        R.ray_begin = S.next_ray;
        S.next_ray += R.nrays;
        R.held = held_bytes(R.nrays, R.rec_rays);
        S.used_bytes += R.held;
        R.state = 1;
        R.t_admit = now_ns();
        S.entry_ticket[entry] = t;
        fill_job(S.hjobs[entry], &R.metric, R.cam, &R.disk, &R.solver, &R.out, R.ray_begin, 0, R.rec);
        S.hjobs[entry].remaining = S.dremaining + entry * kRemainingStride;
        S.hjobs[entry].cancelled = 0;
        S.hremaining[entry * kRemainingStride] = (unsigned int)R.nrays;
        fresh.push_back(entry);
    }
    // ---- cancellations become visible to the kernel from this epoch on
    std::vector<uint64_t> sent;
    for (int e = 0; e < kMaxEntries; ++e) {
        const uint64_t t = S.entry_ticket[e];
        if (!t) continue;
        Request& R = S.reqs[t];
        if (R.cancel_req && !R.cancel_sent) {
            S.hjobs[e].cancelled = 1;
            R.cancel_sent = true;
            sent.push_back(t);
        }
    }
    // ---- directory of live entries sorted by first ray
    int nd = 0;
    std::vector<std::pair<long long, int>> dir;
    for (int e = 0; e < kMaxEntries; ++e)
        if (S.entry_ticket[e]) dir.push_back({S.hjobs[e].ray_begin, e});
    std::sort(dir.begin(), dir.end());
    for (auto& d : dir) {
        S.hdir_begin[nd] = d.first;
        S.hdir_job[nd] = d.second;
        ++nd;
    }
    if (nd == 0) return TARTARUS_OK;
    if (!fresh.empty() || !sent.empty()) S.jobs_dirty = true;
    // ---- nothing to trace but finishing passes in flight: wait for those
    bool tracing = false;
    for (int e = 0; e < kMaxEntries; ++e)
        if (S.entry_ticket[e] && !finishing(S, e)) tracing = true;
    if (!tracing) {
        lk.unlock();
        const int rc = complete_finished(S, lk);
        lk.lock();
        return rc;
    }
    // ---- this epoch's queue: the unstarted rays of every live request, one
    // segment each (ordering rules in host_logic.cpp)
    std::vector<SegmentSource> live;
    for (int e = 0; e < kMaxEntries; ++e) {
        const uint64_t t = S.entry_ticket[e];
        if (!t) continue;
        const Request& R = S.reqs[t];
        live.push_back({e, S.hjobs[e].cancelled, R.nrays, R.started, R.ray_begin});
    }
    const std::vector<Segment> segv = build_segments(live, S.serve_order);
    const int nseg = (int)segv.size();
    S.hseg_q[0] = 0;
    for (int k = 0; k < nseg; ++k) {
        S.seg_entry[k] = segv[k].entry;
        S.hseg_ray[k] = segv[k].ray;
        S.hseg_q[k + 1] = segv[k].q_begin + segv[k].count;
    }
    const long long total = S.hseg_q[nseg];
    const tartarus_solver sv = S.solver;
    // the mixed-precision instance when a live request may use FP32 stages;
    // its FP64 path traces the other requests with the FP64 instance's arithmetic
    int eprec = TARTARUS_PREC_FP64;
    for (int e = 0; e < kMaxEntries; ++e)
        if (S.entry_ticket[e] && !S.hjobs[e].cancelled && S.hjobs[e].allow32) eprec = TARTARUS_PREC_MIXED;
    lk.unlock();

    // the request table when it changed (after the finishing passes in flight,
    // which read it), then the rest of the block in one copy: head = 0, the
    // counts (fresh entries set above, the others as read back after the last
    // epoch), directory and segments
    if (S.jobs_dirty) {
        if (!S.fin_pending.empty()) HIP_TRY(hipStreamWaitEvent(S.stream, S.fin_ev, 0));
        HIP_TRY(hipMemcpyAsync(S.djobs, S.hjobs, sizeof(DevJob) * kMaxEntries, hipMemcpyHostToDevice, S.stream));
        S.jobs_dirty = false;
    }
    *S.hhead = 0ull;
    constexpr size_t kDown = sizeof(EpochBlock) - offsetof(EpochBlock, head);
    HIP_TRY(hipMemcpyAsync(S.dhead, S.hhead, kDown, hipMemcpyHostToDevice, S.stream));
    LaunchArgs A;
    tartarus_metric m0;
    std::memset(&m0, 0, sizeof(m0));
    fill_args(A, &m0, &sv);
    A.jobs = S.djobs;
    A.jc = S.djc;
    A.njobs = kMaxEntries;
    A.chunk = 1;
    A.refill_min = 4;
    A.first_ray = 0;
    A.total_rays = total;
    A.seg_q = S.dseg_q;
    A.seg_ray = S.dseg_ray;
    A.nseg = nseg;
    A.head = S.dhead;
    A.slots = S.slots;
    A.slot_live = S.slot_live;
    A.step_budget = kEpochIterations;
    if (const char* e = std::getenv("TARTARUS_EPOCH_ATTEMPTS")) {   // experiment override
        const long long v = std::atoll(e);
        if (v > 0) A.step_budget = v;
    }
    A.dir_begin = S.ddir_begin;
    A.dir_job = S.ddir_job;
    A.ndir = nd;
    A.remaining = S.dremaining;
    if (!fresh.empty()) HIP_TRY(tartarus_launch_setup(TARTARUS_METRIC_KERR, &A, S.stream));
    HIP_TRY(tartarus_launch_trace(TARTARUS_METRIC_KERR, eprec, sv.method, &A, S.grid, S.block, S.stream));
    // head and counts in one copy back (with the padding between them)
    constexpr size_t kBack = offsetof(EpochBlock, remaining) + sizeof(EpochBlock::remaining) - offsetof(EpochBlock, head);
    HIP_TRY(hipMemcpyAsync(S.hhead, S.dhead, kBack, hipMemcpyDeviceToHost, S.stream));
    // the last epoch's completed requests, while this one traces
    if (const int rc = complete_finished(S, lk)) return rc;
    HIP_TRY(hipStreamSynchronize(S.stream));
    // requests whose rays have all finished: their finishing pass (disk
    // crossings, shading, outputs) on fstream; the records are complete, the
    // stream having been synchronized
    std::vector<int> done;
    for (int e = 0; e < kMaxEntries; ++e)
        if (S.entry_ticket[e] && !finishing(S, e) && S.hremaining[e * kRemainingStride] == 0) done.push_back(e);
    if (!done.empty()) {
        for (int e : done) HIP_TRY(tartarus_launch_finish(&A, e, 1, S.hjobs[e].ray_count, S.fstream));
        HIP_TRY(hipEventRecord(S.fin_ev, S.fstream));
        S.fin_pending = done;
    }

    lk.lock();
    // the queue was consumed in segment order
    const std::vector<long long> used = consumed_per_segment(segv, std::min((long long)*S.hhead, total));
    for (int k = 0; k < nseg; ++k) S.reqs[S.entry_ticket[S.seg_entry[k]]].started += used[k];
    for (uint64_t t : sent) S.reqs[t].cancel_acked = true;
    S.done_cv.notify_all();
    return TARTARUS_OK;
}

void server_main()
{
    Server& S = g_srv;
    std::unique_lock<std::mutex> lk(S.mu);
    if (!S.dev_ready) {
        // the launch shape must suit both serving instances an epoch may run
        // (mixed precision needs at least the FP64 instance's registers)
        const int prec = S.solver.method == TARTARUS_METHOD_DP45 ? TARTARUS_PREC_MIXED : TARTARUS_PREC_FP64;
        int rc = server_alloc(prec, S.solver.method);
        if (rc) {
            S.dev_error = tartarus_last_error();
            S.running = false;
            S.done_cv.notify_all();
            return;
        }
    }
    while (S.running) {
        if (S.queue.empty() && !any_live(S)) {
            S.cv.wait(lk, [&] { return !S.running || !S.queue.empty() || any_live(S); });
            continue;
        }
        int rc = server_round(lk);
        if (rc) {
            // (a device call failed with lk released)
            if (!lk.owns_lock()) lk.lock();
            S.dev_error = tartarus_last_error();
            S.running = false;
            S.done_cv.notify_all();
            break;
        }
    }
    // finishing passes still in flight complete their requests
    if (S.dev_error.empty() && !S.fin_pending.empty()) {
        lk.unlock();
        const int rc = complete_finished(S, lk);
        lk.lock();
        if (rc) {
            S.dev_error = tartarus_last_error();
            S.done_cv.notify_all();
        }
    }
}



}  // namespace

extern "C" int tartarus_serving_order(int order)
{
    if (order != TARTARUS_SERVE_SMALLEST_FIRST && order != TARTARUS_SERVE_ARRIVAL)
        return fail(TARTARUS_E_INVALID, "unknown serving order");
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    std::lock_guard<std::mutex> lk(g_srv.mu);
    g_srv.serve_order = order;
    return TARTARUS_OK;
}

extern "C" int tartarus_submit(const tartarus_metric* metric, const tartarus_camera* cam, const tartarus_disk* disk,
                               const tartarus_solver* solver, const tartarus_outputs* out, uint64_t* ticket)
{
    int rc = validate_all(metric, cam, 1, disk, solver);
    if (rc) return rc;
    if ((rc = check_outputs(out))) return rc;
    if (!ticket) return fail(TARTARUS_E_INVALID, "ticket is NULL");
    if (metric->kind != TARTARUS_METRIC_KERR) return fail(TARTARUS_E_INVALID, "serving takes analytic Kerr requests");
    if (!g_dev.ready) return fail(TARTARUS_E_DEVICE, "tartarus_init has not been called");
    Server& S = g_srv;
    std::unique_lock<std::mutex> lk(S.mu);
    if (!S.dev_error.empty()) return fail(TARTARUS_E_DEVICE, "serving stopped after a device error: " + S.dev_error);
    if (S.have_solver && S.solver.method != solver->method)
        return fail(TARTARUS_E_INVALID, "requests of one serving session must share the integration method");
    Request R;
    R.metric = *metric;
    R.cam = *cam;
    R.disk = *disk;
    R.solver = *solver;
    R.out = *out;
    R.nrays = (long long)cam->nx * cam->ny;
    // the slot arena is allocated when the scheduler starts; estimate it beforehand
    const size_t arena = S.dev_ready ? S.arena_bytes : (size_t)g_dev.cus * 768 * (SLOT_DOUBLES * 8 + 4);
    if (never_fits(R.nrays, arena, g_dev.budget))
        return fail(TARTARUS_E_TOO_LARGE, "request needs more than the HBM budget");
    if (R.nrays > 0xffffffffll) return fail(TARTARUS_E_TOO_LARGE, "request has too many rays");
    R.t_submit = now_ns();
    const uint64_t t = S.next_ticket++;
    S.reqs[t] = R;
    S.queue.push_back(t);
    if (!S.have_solver) {
        S.solver = *solver;
        S.have_solver = true;
    }
    if (!S.running) {
        if (S.th.joinable()) S.th.join();
        S.running = true;
        S.th = std::thread(server_main);
    }
    S.cv.notify_all();
    *ticket = t;
    return TARTARUS_OK;
}

extern "C" int tartarus_poll(uint64_t ticket, int* state)
{
    if (!state) return fail(TARTARUS_E_INVALID, "state is NULL");
    Server& S = g_srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(TARTARUS_E_NOT_FOUND, "unknown ticket");
    if (!S.dev_error.empty() && it->second.state != 2) return fail(TARTARUS_E_DEVICE, S.dev_error);
    if (it->second.too_large) return fail(TARTARUS_E_TOO_LARGE, "request does not fit the HBM budget");
    *state = it->second.state;
    return TARTARUS_OK;
}

extern "C" int tartarus_wait(uint64_t ticket, int64_t timeout_ms)
{
    Server& S = g_srv;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(TARTARUS_E_NOT_FOUND, "unknown ticket");
    auto pred = [&] { return S.reqs[ticket].state == 2 || !S.dev_error.empty(); };
    if (timeout_ms < 0)
        S.done_cv.wait(lk, pred);
    else if (!S.done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
        return fail(TARTARUS_E_AGAIN, "request not done yet");
    if (S.reqs[ticket].state != 2) return fail(TARTARUS_E_DEVICE, S.dev_error);
    if (S.reqs[ticket].too_large) return fail(TARTARUS_E_TOO_LARGE, "request does not fit the HBM budget");
    return TARTARUS_OK;
}

extern "C" int tartarus_cancel(uint64_t ticket)
{
    Server& S = g_srv;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(TARTARUS_E_NOT_FOUND, "unknown ticket");
    Request& R = it->second;
    if (R.state == 2) return TARTARUS_OK;
    if (R.state == 0) {
        S.queue.erase(std::find(S.queue.begin(), S.queue.end(), ticket));
        R.state = 2;
        R.t_done = now_ns();
        S.done_cv.notify_all();
        return TARTARUS_OK;
    }
    // running: from the next epoch on its rays are dropped without writing
    // outputs; return once such an epoch has completed (or the request ended)
    R.cancel_req = true;
    S.cv.notify_all();
    S.done_cv.wait(lk, [&] { return S.reqs[ticket].cancel_acked || S.reqs[ticket].state == 2 || !S.dev_error.empty(); });
    return TARTARUS_OK;
}

extern "C" int tartarus_ticket_times(uint64_t ticket, int64_t stamps[3])
{
    if (!stamps) return fail(TARTARUS_E_INVALID, "stamps is NULL");
    Server& S = g_srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(TARTARUS_E_NOT_FOUND, "unknown ticket");
    stamps[0] = it->second.t_submit;
    stamps[1] = it->second.t_admit;
    stamps[2] = it->second.t_done;
    return TARTARUS_OK;
}

namespace {
void server_stop()
{
    Server& S = g_srv;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.running = false;
        S.cv.notify_all();
    }
    if (S.th.joinable()) S.th.join();
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stream) (void)hipStreamSynchronize(S.stream);
    for (auto& kv : S.reqs)
        if (kv.second.rec) {
            (void)hipFree(kv.second.rec);
            kv.second.rec = nullptr;
        }
    if (S.dev_ready) server_free();
    S.queue.clear();
    S.reqs.clear();
    for (auto& e : S.entry_ticket) e = 0;
    S.used_bytes = 0;
    S.next_ray = 0;
    S.serve_order = TARTARUS_SERVE_SMALLEST_FIRST;
    S.have_solver = false;
    S.dev_error.clear();
}
}  // namespace
