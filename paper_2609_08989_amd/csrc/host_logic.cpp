// host_logic.cpp -- host-only parts of the runtime (see host_logic.hpp).
#include "host_logic.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <tuple>

namespace tartarus {
namespace host {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

const char* last_error() { return g_err.c_str(); }

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_metric(const tartarus_metric* m, int precision, int method)
{
    if (!m) return fail(TARTARUS_E_INVALID, "metric is NULL");
    if (!(std::isfinite(m->a) && m->a >= 0.0 && m->a < 1.0)) return fail(TARTARUS_E_INVALID, "spin a must be in [0, 1)");
    if (m->kind == TARTARUS_METRIC_TABLE) {
        if (!m->table) return fail(TARTARUS_E_INVALID, "tabulated metric needs a table");
        if (m->nr < 4 || m->nth < 4) return fail(TARTARUS_E_INVALID, "table needs nr, nth >= 4");
        if (!finite_pos(m->r_min) || !(m->r_max > m->r_min) || !std::isfinite(m->r_max))
            return fail(TARTARUS_E_INVALID, "table needs 0 < r_min < r_max");
        if (precision != TARTARUS_PREC_FP64)
            return fail(TARTARUS_E_INVALID, "the tabulated metric is traced in FP64 only");
        if (method != TARTARUS_METHOD_DP45)
            return fail(TARTARUS_E_INVALID, "the tabulated metric is traced with Dormand-Prince 5(4) only");
    } else if (m->kind != TARTARUS_METRIC_KERR) {
        return fail(TARTARUS_E_INVALID, "unknown metric kind");
    }
    return TARTARUS_OK;
}

int check_camera(const tartarus_camera& c, const tartarus_solver* s)
{
    if (!finite_pos(c.r_obs)) return fail(TARTARUS_E_INVALID, "r_obs must be > 0");
    if (!(std::isfinite(c.theta_obs) && c.theta_obs > 0.0 && c.theta_obs < M_PI))
        return fail(TARTARUS_E_INVALID, "theta_obs must be in (0, pi)");
    if (c.nx < 1 || c.ny < 1) return fail(TARTARUS_E_INVALID, "nx, ny must be >= 1");
    const double w[4] = {c.alpha_min, c.alpha_max, c.beta_min, c.beta_max};
    for (double v : w)
        if (!std::isfinite(v)) return fail(TARTARUS_E_INVALID, "non-finite image window");
    const double am = std::max(std::fabs(c.alpha_min), std::fabs(c.alpha_max));
    const double bm = std::max(std::fabs(c.beta_min), std::fabs(c.beta_max));
    if (!(am * am + bm * bm < c.r_obs * c.r_obs)) return fail(TARTARUS_E_INVALID, "image window must satisfy alpha^2 + beta^2 < r_obs^2");
    if (s && !(s->r_escape > c.r_obs)) return fail(TARTARUS_E_INVALID, "r_escape must exceed r_obs");
    if ((long long)c.nx * c.ny > (1ll << 40)) return fail(TARTARUS_E_INVALID, "image too large");
    return TARTARUS_OK;
}

int check_solver(const tartarus_solver* s)
{
    if (!s) return fail(TARTARUS_E_INVALID, "solver is NULL");
    if (!finite_pos(s->rtol)) return fail(TARTARUS_E_INVALID, "rtol must be > 0");
    if (!finite_pos(s->atol)) return fail(TARTARUS_E_INVALID, "atol must be > 0");
    if (!finite_pos(s->h0_frac)) return fail(TARTARUS_E_INVALID, "h0_frac must be > 0");
    if (!(std::isfinite(s->horizon_factor) && s->horizon_factor >= 1.0))
        return fail(TARTARUS_E_INVALID, "horizon_factor must be >= 1");
    if (!(finite_pos(s->r_escape) && s->r_escape <= 1e15))
        return fail(TARTARUS_E_INVALID, "r_escape must be in (0, 1e15]");
    if (!finite_pos(s->event_tol)) return fail(TARTARUS_E_INVALID, "event_tol must be > 0");
    if (s->max_steps < 1) return fail(TARTARUS_E_INVALID, "max_steps must be >= 1");
    if (s->precision != TARTARUS_PREC_FP64 && s->precision != TARTARUS_PREC_MIXED)
        return fail(TARTARUS_E_INVALID, "unknown precision");
    if (s->method < TARTARUS_METHOD_DP45 || s->method > TARTARUS_METHOD_VERLET)
        return fail(TARTARUS_E_INVALID,
                    "unknown method (0 Dormand-Prince, 1 Cash-Karp, 2 Fehlberg, 3 Gragg-Bulirsch-Stoer, 4 Verlet)");
    if (s->precision == TARTARUS_PREC_MIXED && s->method != TARTARUS_METHOD_DP45)
        return fail(TARTARUS_E_INVALID, "mixed precision is provided with Dormand-Prince 5(4) only");
    return TARTARUS_OK;
}

int check_disk(const tartarus_disk* d)
{
    if (!d) return fail(TARTARUS_E_INVALID, "disk is NULL");
    if (d->max_hits < 0 || d->max_hits > 3) return fail(TARTARUS_E_INVALID, "max_hits must be in 0..3");
    if (d->opaque != 0 && d->opaque != 1) return fail(TARTARUS_E_INVALID, "disk opaque must be 0 or 1");
    if (d->opaque && d->max_hits < 1) return fail(TARTARUS_E_INVALID, "an opaque disk needs max_hits >= 1");
    if (d->shading != TARTARUS_SHADE_OBSERVED && d->shading != TARTARUS_SHADE_INTRINSIC)
        return fail(TARTARUS_E_INVALID, "unknown disk shading");
    if (d->max_hits > 0) {
        if (!std::isfinite(d->r_in) || !std::isfinite(d->r_out)) return fail(TARTARUS_E_INVALID, "non-finite disk radii");
        if (!(d->r_out > 0.0)) return fail(TARTARUS_E_INVALID, "disk r_out must be > 0");
        if (d->r_in > 0.0 && !(d->r_out > d->r_in)) return fail(TARTARUS_E_INVALID, "disk needs r_out > r_in");
    }
    return TARTARUS_OK;
}

int check_outputs(const tartarus_outputs* o)
{
    if (!o) return fail(TARTARUS_E_INVALID, "outputs is NULL");
    const void* p[] = {o->cls, o->n_hits, o->final_rtp, o->h_drift, o->h_gate, o->hit_r, o->hit_g, o->hit_flux,
                       o->hit_lambda, o->hit_order, o->intensity, o->n_accept, o->n_reject, o->n_fp32, o->n_cross};
    for (const void* q : p)
        if (!q) return fail(TARTARUS_E_INVALID, "an output buffer is NULL");
    return TARTARUS_OK;
}

int validate_all(const tartarus_metric* metric, const tartarus_camera* cams, int ncams, const tartarus_disk* disk,
                 const tartarus_solver* solver)
{
    int rc;
    if ((rc = check_solver(solver))) return rc;
    if ((rc = check_metric(metric, solver->precision, solver->method))) return rc;
    if ((rc = check_disk(disk))) return rc;
    if (!cams || ncams < 1) return fail(TARTARUS_E_INVALID, "need at least one camera");
    for (int c = 0; c < ncams; ++c) {
        if ((rc = check_camera(cams[c], solver))) return rc;
        if (cams[c].nx != cams[0].nx || cams[c].ny != cams[0].ny)
            return fail(TARTARUS_E_INVALID, "all cameras of a trace must share nx, ny");
    }
    return TARTARUS_OK;
}

void fill_job(DevJob& J, const tartarus_metric* m, const tartarus_camera& c, const tartarus_disk* d,
              const tartarus_solver* s, const tartarus_outputs* o, long long begin, long long offset, double* rec)
{
    std::memset(&J, 0, sizeof(J));
    J.ray_begin = begin;
    J.ray_count = (long long)c.nx * c.ny;
    J.nx = c.nx;
    J.ny = c.ny;
    J.max_hits = d->max_hits;
    J.disk_flags = (d->opaque ? DISK_OPAQUE : 0) | (d->shading == TARTARUS_SHADE_INTRINSIC ? DISK_INTRINSIC : 0);
    J.a = m->a;
    J.r_obs = c.r_obs;
    J.theta_obs = c.theta_obs;
    J.alpha_min = c.alpha_min;
    J.alpha_max = c.alpha_max;
    J.beta_min = c.beta_min;
    J.beta_max = c.beta_max;
    J.disk_r_in = d->r_in;
    J.disk_r_out = d->r_out;
    J.cls = o->cls + offset;
    J.n_hits = o->n_hits + offset;
    J.final_rtp = o->final_rtp + 3 * offset;
    J.h_drift = o->h_drift + offset;
    J.h_gate = o->h_gate + offset;
    J.hit_r = o->hit_r + 3 * offset;
    J.hit_g = o->hit_g + 3 * offset;
    J.hit_flux = o->hit_flux + 3 * offset;
    J.hit_lambda = o->hit_lambda + 3 * offset;
    J.hit_order = o->hit_order + 3 * offset;
    J.intensity = o->intensity + offset;
    J.n_accept = o->n_accept + offset;
    J.n_reject = o->n_reject + offset;
    J.n_fp32 = o->n_fp32 + offset;
    J.n_cross = o->n_cross + offset;
    J.remaining = nullptr;
    J.rec = rec;
    J.event_tol = s->event_tol;
    J.rtol = s->rtol;
    J.atol = s->atol;
    J.h0_frac = s->h0_frac;
    J.horizon_factor = s->horizon_factor;
    J.r_escape = s->r_escape;
    J.max_steps = s->max_steps;
    J.allow32 = kernel_precision(s) == TARTARUS_PREC_MIXED ? 1 : 0;
}

void fill_args(LaunchArgs& A, const tartarus_metric* m, const tartarus_solver* s)
{
    std::memset(&A, 0, sizeof(A));
    A.rtol = s->rtol;
    A.atol = s->atol;
    A.h0_frac = s->h0_frac;
    A.event_tol = s->event_tol;
    A.horizon_factor = s->horizon_factor;
    A.r_escape = s->r_escape;
    A.max_steps = s->max_steps;
    A.r_switch_factor = kDefaultSwitch;
    A.turn_r = kDefaultTurnR;
    A.turn_th = kDefaultTurnTh;
    // experiment overrides of the mixed-precision regime
    if (const char* e = std::getenv("TARTARUS_MIXED_SWITCH")) {
        const double v = std::atof(e);
        if (v > 0.0) A.r_switch_factor = v;
    }
    if (const char* e = std::getenv("TARTARUS_MIXED_TURN_R")) A.turn_r = std::atof(e);
    if (const char* e = std::getenv("TARTARUS_MIXED_TURN_TH")) A.turn_th = std::atof(e);
    if (m->kind == TARTARUS_METRIC_TABLE) {
        A.table = m->table;
        A.nr = m->nr;
        A.nth = m->nth;
        A.tab_r_min = m->r_min;
        A.tab_r_max = m->r_max;
    }
}

int merge_shape(const tartarus_launch& base, const tartarus_launch* req, tartarus_launch& L)
{
    // req may point at L itself: read the request before L is overwritten
    tartarus_launch r{};
    if (req) r = *req;
    L = base;
    if (req) {
        if (r.block_threads > 0) L.block_threads = r.block_threads;
        if (r.blocks_per_cu > 0) L.blocks_per_cu = r.blocks_per_cu;
        if (r.chunk > 0) L.chunk = r.chunk;
        if (r.refill_min > 0) L.refill_min = r.refill_min;
        if (r.order > 0) L.order = r.order;
    }
    if (L.order < 0 || L.order > TARTARUS_ORDER_TILE) return fail(TARTARUS_E_INVALID, "unknown queue order");
    if (L.block_threads != 64 && L.block_threads != 128 && L.block_threads != 256)
        return fail(TARTARUS_E_INVALID, "block_threads must be 64, 128 or 256");
    if (L.refill_min < 1 || L.refill_min > 64) return fail(TARTARUS_E_INVALID, "refill_min must be in 1..64");
    if (L.chunk < 1) return fail(TARTARUS_E_INVALID, "chunk must be >= 1");
    return TARTARUS_OK;
}

// With few rays per lane the longest rays set the kernel time and a lone
// wavefront per SIMD runs them fastest; with many, a second wavefront's
// throughput wins (measured: one block of 256 per CU on a 512^2 image, two on
// 1024^2 and 2048^2 images).
int finish_shape(tartarus_launch& L, int occ, long long n_rays, int cus, int& grid)
{
    if (occ < 1) return fail(TARTARUS_E_DEVICE, "kernel cannot be resident with this block size");
    if (cus < 1) return fail(TARTARUS_E_DEVICE, "no compute units");
    if (L.blocks_per_cu <= 0 && n_rays > 0 && n_rays < kRaysPerLaneForFullOccupancy * (long long)cus * L.block_threads)
        L.blocks_per_cu = 1;
    if (L.blocks_per_cu <= 0 || L.blocks_per_cu > occ) L.blocks_per_cu = occ;
    grid = cus * L.blocks_per_cu;
    return TARTARUS_OK;
}

long long RecordPool::pooled_capacity(long long n) const
{
    auto it = pool_.lower_bound(n);
    return (it != pool_.end() && it->first <= 4 * n) ? it->first : 0;
}

void* RecordPool::take_pooled(long long n, long long& cap)
{
    auto it = pool_.lower_bound(n);
    if (it == pool_.end() || it->first > 4 * n) return nullptr;
    void* p = it->second;
    cap = it->first;
    bytes_ -= (size_t)cap * kRecordBytes;
    pool_.erase(it);
    return p;
}

bool RecordPool::give(void* p, long long cap, size_t limit)
{
    const size_t b = (size_t)cap * kRecordBytes;
    if (bytes_ + b > limit) return false;
    pool_.emplace(cap, p);
    bytes_ += b;
    return true;
}

std::vector<void*> RecordPool::drain()
{
    std::vector<void*> v;
    v.reserve(pool_.size());
    for (auto& kv : pool_) v.push_back(kv.second);
    pool_.clear();
    bytes_ = 0;
    return v;
}

bool admission_fits(size_t used, size_t pool_bytes, size_t arena, size_t budget, long long nrays, long long rec_cap,
                    bool pooled)
{
    // a pooled buffer moves from the pool to the request: counted once
    const size_t pool_after = pooled ? pool_bytes - (size_t)rec_cap * kRecordBytes : pool_bytes;
    const size_t total = used + pool_after + held_bytes(nrays, rec_cap) + arena;
    return total <= budget;
}

std::vector<Segment> build_segments(const std::vector<SegmentSource>& live, int order)
{
    std::vector<std::tuple<int, long long, long long, int, long long, long long>> keyed;
    keyed.reserve(live.size());
    for (const SegmentSource& s : live) {
        if (s.started >= s.nrays) continue;
        const long long key = order == TARTARUS_SERVE_SMALLEST_FIRST ? s.nrays - s.started : s.ray_begin;
        keyed.emplace_back(s.cancelled ? 0 : 1, key, s.ray_begin, s.entry, s.ray_begin + s.started,
                           s.nrays - s.started);
    }
    std::sort(keyed.begin(), keyed.end());
    std::vector<Segment> segs;
    segs.reserve(keyed.size());
    long long q = 0;
    for (auto& k : keyed) {
        segs.push_back({std::get<3>(k), std::get<4>(k), q, std::get<5>(k)});
        q += std::get<5>(k);
    }
    return segs;
}

std::vector<long long> consumed_per_segment(const std::vector<Segment>& segs, long long taken)
{
    std::vector<long long> c(segs.size(), 0);
    for (size_t k = 0; k < segs.size() && taken > 0; ++k) {
        c[k] = std::min(taken, segs[k].count);
        taken -= c[k];
    }
    return c;
}

}  // namespace host
}  // namespace tartarus
