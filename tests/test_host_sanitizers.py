"""The host-only C/C++ of the project under AddressSanitizer and
UndefinedBehaviorSanitizer, built with g++/gcc for the CPU (no device code):

* the runtime's host logic (csrc/host_logic.cpp): argument validation on valid
  and invalid inputs, job-table and launch-argument filling, the launch-shape
  rules, and a simulated serving session driving the record-buffer pool, the
  HBM-budget admission and the epoch queue segments through thousands of
  random admissions and completions, with the budget invariant checked at
  every step;
* the CPU oracle (oracle/tartarus_oracle.c) tracing small images with every
  integrator, the disk variants and the tabulated metric.

Any sanitizer report aborts the driver (-fno-sanitize-recover=all); leaks are
reported at exit."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_08989_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "host_logic.hpp"
extern "C" {
#include "tartarus_oracle.h"
int or_trace(const or_metric* m, const or_camera* cams, int ncams, const or_disk* disk, const or_solver* sv,
             const int64_t* ray_ids, int64_t n, const or_outputs* o, int nthreads);
void or_build_kerr_table(double a, int nr, int nth, double r_min, double r_max, double* table);
double or_horizon(double a);
}

using namespace tartarus;
using namespace tartarus::host;

static int g_fail = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("CHECK failed at line %d: %s\n", __LINE__, #c);       \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

static tartarus_camera cam0()
{
    tartarus_camera c;
    c.r_obs = 1000.0; c.theta_obs = 1.0; c.nx = 16; c.ny = 12;
    c.alpha_min = -20.0; c.alpha_max = 20.0; c.beta_min = -15.0; c.beta_max = 15.0;
    return c;
}
static tartarus_solver sv0()
{
    tartarus_solver s;
    s.rtol = 1e-8; s.atol = 1e-10; s.h0_frac = 0.01; s.horizon_factor = 1.01; s.r_escape = 1100.0;
    s.event_tol = 1e-12; s.max_steps = 1000000; s.precision = 0; s.method = 0;
    return s;
}

static void validation()
{
    tartarus_metric m{}; m.kind = 0; m.a = 0.9;
    tartarus_camera c = cam0();
    tartarus_disk d{}; d.r_in = 0.0; d.r_out = 20.0; d.max_hits = 3;
    tartarus_solver s = sv0();
    CHECK(validate_all(&m, &c, 1, &d, &s) == TARTARUS_OK);
    struct Bad { const char* what; int code; };
    auto expect = [&](int rc, int code) { CHECK(rc == code); CHECK(std::strlen(last_error()) > 0); };
    { tartarus_metric b = m; b.a = 1.0; expect(validate_all(&b, &c, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_metric b = m; b.a = NAN; expect(validate_all(&b, &c, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_metric b = m; b.kind = 7; expect(validate_all(&b, &c, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_metric b = m; b.kind = 1; expect(validate_all(&b, &c, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_camera b = c; b.theta_obs = 0.0; expect(validate_all(&m, &b, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_camera b = c; b.nx = 0; expect(validate_all(&m, &b, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_camera b = c; b.alpha_max = 2000.0; expect(validate_all(&m, &b, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_camera b = c; b.beta_min = INFINITY; expect(validate_all(&m, &b, 1, &d, &s), TARTARUS_E_INVALID); }
    { tartarus_camera b[2] = {c, c}; b[1].nx = 17; expect(validate_all(&m, b, 2, &d, &s), TARTARUS_E_INVALID); }
    expect(validate_all(&m, &c, 0, &d, &s), TARTARUS_E_INVALID);
    expect(validate_all(&m, nullptr, 1, &d, &s), TARTARUS_E_INVALID);
    expect(validate_all(&m, &c, 1, nullptr, &s), TARTARUS_E_INVALID);
    expect(validate_all(&m, &c, 1, &d, nullptr), TARTARUS_E_INVALID);
    expect(validate_all(nullptr, &c, 1, &d, &s), TARTARUS_E_INVALID);
    { tartarus_solver b = s; b.rtol = 0.0; expect(validate_all(&m, &c, 1, &d, &b), TARTARUS_E_INVALID); }
    { tartarus_solver b = s; b.r_escape = 900.0; expect(validate_all(&m, &c, 1, &d, &b), TARTARUS_E_INVALID); }
    { tartarus_solver b = s; b.max_steps = 0; expect(validate_all(&m, &c, 1, &d, &b), TARTARUS_E_INVALID); }
    { tartarus_solver b = s; b.method = 9; expect(validate_all(&m, &c, 1, &d, &b), TARTARUS_E_INVALID); }
    { tartarus_solver b = s; b.precision = 1; b.method = 3; expect(validate_all(&m, &c, 1, &d, &b), TARTARUS_E_INVALID); }
    { tartarus_disk b = d; b.max_hits = 4; expect(validate_all(&m, &c, 1, &b, &s), TARTARUS_E_INVALID); }
    { tartarus_disk b = d; b.opaque = 1; b.max_hits = 0; expect(validate_all(&m, &c, 1, &b, &s), TARTARUS_E_INVALID); }
    { tartarus_disk b = d; b.r_in = 30.0; expect(validate_all(&m, &c, 1, &b, &s), TARTARUS_E_INVALID); }
    tartarus_outputs o{};
    expect(check_outputs(&o), TARTARUS_E_INVALID);
    expect(check_outputs(nullptr), TARTARUS_E_INVALID);
}

static void filling()
{
    tartarus_metric m{}; m.kind = 0; m.a = 0.5;
    tartarus_camera c = cam0();
    tartarus_disk d{}; d.r_out = 20.0; d.max_hits = 2; d.opaque = 1; d.shading = 1;
    tartarus_solver s = sv0();
    std::vector<int32_t> i32(1000); std::vector<double> f64(3000);
    tartarus_outputs o;
    o.cls = o.n_hits = o.hit_order = o.n_accept = o.n_reject = o.n_fp32 = o.n_cross = i32.data();
    o.final_rtp = o.h_drift = o.h_gate = o.hit_r = o.hit_g = o.hit_flux = o.hit_lambda = o.intensity = f64.data();
    DevJob J;
    fill_job(J, &m, c, &d, &s, &o, 384, 192, nullptr);
    CHECK(J.ray_begin == 384 && J.ray_count == 192 && J.nx == 16 && J.ny == 12);
    CHECK(J.cls == i32.data() + 192 && J.final_rtp == f64.data() + 576 && J.hit_order == i32.data() + 576);
    CHECK(J.disk_flags == (DISK_OPAQUE | DISK_INTRINSIC) && J.max_hits == 2 && J.event_tol == 1e-12);
    // the request's own solver settings, and FP32 stages only for mixed
    // precision at a tolerance where they can pass the rounding test
    CHECK(J.rtol == s.rtol && J.atol == s.atol && J.h0_frac == s.h0_frac && J.max_steps == s.max_steps);
    CHECK(J.horizon_factor == s.horizon_factor && J.r_escape == s.r_escape && J.allow32 == 0);
    { tartarus_solver b = s; b.precision = 1; fill_job(J, &m, c, &d, &b, &o, 0, 0, nullptr); CHECK(J.allow32 == 1); }
    { tartarus_solver b = s; b.precision = 1; b.rtol = 1e-10; fill_job(J, &m, c, &d, &b, &o, 0, 0, nullptr);
      CHECK(J.allow32 == 0 && kernel_precision(&b) == TARTARUS_PREC_FP64); }
    LaunchArgs A;
    fill_args(A, &m, &s);
    CHECK(A.rtol == 1e-8 && A.table == nullptr && A.r_switch_factor == kDefaultSwitch && A.slots == nullptr);
}

static void shapes()
{
    std::mt19937_64 rng(7);
    tartarus_launch base{256, 0, 1, 4, 0};
    for (int it = 0; it < 2000; ++it) {
        tartarus_launch req{(int)(rng() % 300) - 10, (int)(rng() % 6) - 1, (int)(rng() % 2000) - 5,
                            (int)(rng() % 80) - 5, (int)(rng() % 6) - 1};
        tartarus_launch L;
        const int rc = merge_shape(base, (it % 7) ? &req : nullptr, L);
        if (rc != TARTARUS_OK) continue;
        CHECK(L.block_threads == 64 || L.block_threads == 128 || L.block_threads == 256);
        CHECK(L.refill_min >= 1 && L.refill_min <= 64 && L.chunk >= 1 && L.order >= 0 && L.order <= 3);
        int grid = 0;
        const int occ = 1 + (int)(rng() % 4);
        const long long n = (long long)(rng() % 5000000);
        if (finish_shape(L, occ, n, 256, grid) == TARTARUS_OK) {
            CHECK(L.blocks_per_cu >= 1 && L.blocks_per_cu <= occ && grid == 256 * L.blocks_per_cu);
        }
    }
    tartarus_launch L = base;
    CHECK(merge_shape(base, &L, L) == TARTARUS_OK);   // request aliasing the result
    int grid = 0;
    CHECK(finish_shape(L, 0, 10, 256, grid) == TARTARUS_E_DEVICE);
}

// A serving session with a fake device allocator: every admitted request holds
// its outputs and a record buffer; finished ones return the buffer to the pool.
static void serving()
{
    std::mt19937_64 rng(11);
    const size_t budget = (size_t)8 << 30;
    const size_t arena = (size_t)256 * 768 * (SLOT_DOUBLES * 8 + 4);
    RecordPool pool;
    struct Live { long long n, cap; void* rec; size_t held; };
    std::vector<Live> live;
    std::vector<long long> queue;
    size_t used = 0;
    long long allocs = 0, frees = 0, admitted = 0;
    const long long res[5] = {64, 128, 256, 512, 1024};
    for (int step = 0; step < 20000; ++step) {
        if (rng() % 3 != 0) {
            const long long r = res[rng() % 5];
            queue.push_back(r * r);
        }
        // admission, arrival order
        while (!queue.empty()) {
            const long long n = queue.front();
            if (never_fits(n, arena, budget)) { queue.erase(queue.begin()); continue; }
            long long cap = pool.pooled_capacity(n);
            bool pooled = cap > 0;
            if (!pooled) cap = n;
            if (!admission_fits(used, pool.bytes(), arena, budget, n, cap, pooled)) {
                if (pool.empty() || !admission_fits(used, 0, arena, budget, n, n, false)) break;
                for (void* p : pool.drain()) { std::free(p); ++frees; }
                pooled = false;
                cap = n;
            }
            void* rec;
            if (pooled) {
                long long got = 0;
                rec = pool.take_pooled(n, got);
                CHECK(rec != nullptr && got == cap && got >= n && got <= 4 * n);
            } else {
                rec = std::malloc(16);
                ++allocs;
            }
            const size_t h = held_bytes(n, cap);
            used += h;
            live.push_back({n, cap, rec, h});
            queue.erase(queue.begin());
            ++admitted;
            CHECK(used + pool.bytes() + arena <= budget);
        }
        // completions
        if (!live.empty() && rng() % 2 == 0) {
            const size_t k = rng() % live.size();
            used -= live[k].held;
            if (!pool.give(live[k].rec, live[k].cap, budget / 4)) { std::free(live[k].rec); ++frees; }
            live.erase(live.begin() + (long)k);
        }
        CHECK(pool.bytes() <= budget / 4);
        CHECK(used + pool.bytes() + arena <= budget);
        // the epoch queue over the live requests
        if (step % 50 == 0 && !live.empty()) {
            std::vector<SegmentSource> src;
            long long begin = 0;
            for (size_t k = 0; k < live.size(); ++k) {
                const long long started = (long long)(rng() % (unsigned long long)(live[k].n + 1));
                src.push_back({(int)k, (int)(rng() % 5 == 0), live[k].n, started, begin});
                begin += live[k].n;
            }
            for (int order = 0; order < 2; ++order) {
                const std::vector<Segment> segs = build_segments(src, order);
                long long q = 0, total = 0;
                for (auto& s : src) total += s.nrays - s.started;
                for (size_t k = 0; k < segs.size(); ++k) {
                    CHECK(segs[k].q_begin == q && segs[k].count > 0);
                    const SegmentSource& s = src[(size_t)segs[k].entry];
                    CHECK(segs[k].ray == s.ray_begin + s.started && segs[k].count == s.nrays - s.started);
                    if (k > 0) {
                        const SegmentSource& p = src[(size_t)segs[k - 1].entry];
                        CHECK(p.cancelled >= s.cancelled || p.cancelled == 1);
                        if (order == 0 && p.cancelled == s.cancelled)
                            CHECK(p.nrays - p.started <= s.nrays - s.started);
                    }
                    q += segs[k].count;
                }
                CHECK(q == total);
                const long long taken = total ? (long long)(rng() % (unsigned long long)(total + 10)) : 0;
                const std::vector<long long> c = consumed_per_segment(segs, taken);
                long long sum = 0;
                for (size_t k = 0; k < c.size(); ++k) { CHECK(c[k] >= 0 && c[k] <= segs[k].count); sum += c[k]; }
                CHECK(sum == (taken < total ? taken : total));
            }
        }
    }
    for (auto& l : live) { std::free(l.rec); ++frees; }
    for (void* p : pool.drain()) { std::free(p); ++frees; }
    CHECK(allocs == frees);
    CHECK(admitted > 1000);
    std::printf("serving: %lld admitted, %lld record allocations\n", admitted, allocs);
}

static void oracle_images()
{
    or_camera c{1000.0, 1.0, 9, 7, -12.0, 12.0, -9.0, 9.0};
    or_disk d{0.0, 20.0, 3, 0, 0};
    const int n = 63;
    std::vector<int32_t> cls(n), nh(n), ho(3 * n), na(n), nr(n), nc(n);
    std::vector<double> frtp(3 * n), hd(n), hg(n), hr(3 * n), hgg(3 * n), hf(3 * n), hl(3 * n), in(n);
    or_outputs o{cls.data(), nh.data(), frtp.data(), hd.data(), hg.data(), hr.data(), hgg.data(), hf.data(),
                 hl.data(), ho.data(), in.data(), na.data(), nr.data(), nc.data()};
    const int nr_ = 48, nth = 24;
    const double rmin = 1.1 * or_horizon(0.7), rmax = 2000.0;
    std::vector<double> table((size_t)5 * nr_ * nth * 4);
    or_build_kerr_table(0.7, nr_, nth, rmin, rmax, table.data());
    struct Case { int kind; int method; double h0; int opaque; int shading; double hf; };
    const Case cases[] = {{0, 0, 0.01, 0, 0, 1.01}, {0, 1, 0.01, 0, 0, 1.01}, {0, 2, 0.01, 1, 0, 1.01},
                          {0, 3, 0.01, 0, 1, 1.01}, {1, 0, 0.01, 0, 0, 1.01}};
    for (const Case& k : cases) {
        or_metric m{k.kind, k.kind ? 0.7 : 0.9, k.kind ? table.data() : nullptr, nr_, nth, rmin, rmax};
        or_solver s{1e-8, 1e-10, k.h0, k.hf, 1100.0, 1e-12, 1000000, k.method, 0};
        or_disk dk = d;
        dk.opaque = k.opaque;
        dk.shading = k.shading;
        or_trace(&m, &c, 1, &dk, &s, nullptr, n, &o, 1);
        for (int i = 0; i < n; ++i) {
            CHECK(cls[i] >= 0 && cls[i] <= 3 && cls[i] != 2);
            CHECK(std::isfinite(frtp[3 * i]) && std::isfinite(hd[i]) && nh[i] >= 0 && nh[i] <= 3);
        }
    }
    // Verlet: a few rays from r = 100 with a fixed step
    or_camera cv{100.0, 1.0, 3, 2, -8.0, 8.0, -6.0, 6.0};
    or_metric m{0, 0.9, nullptr, 0, 0, 0.0, 0.0};
    or_solver s{1e-8, 1e-10, 0.05 / 100.0, 1.05, 110.0, 1e-12, 1000000, 4, 0};
    or_trace(&m, &cv, 1, &d, &s, nullptr, 6, &o, 1);
    for (int i = 0; i < 6; ++i) CHECK(cls[i] >= 0 && cls[i] <= 2);
}

int main()
{
    validation();
    filling();
    shapes();
    serving();
    oracle_images();
    std::printf("failures: %d\n", g_fail);
    return g_fail ? 1 : 0;
}
"""


def _have_sanitizers(d):
    src = os.path.join(d, "probe.cpp")
    open(src, "w").write("int main() { return 0; }\n")
    r = subprocess.run(["g++", *SAN, src, "-o", os.path.join(d, "probe")], capture_output=True, text=True)
    return r.returncode == 0


@pytest.mark.slow
def test_host_code_and_oracle_under_asan_and_ubsan():
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    d = tempfile.mkdtemp()
    try:
        if not _have_sanitizers(d):
            pytest.skip("the host compiler has no address / undefined-behaviour sanitizer runtime")
        drv = os.path.join(d, "driver.cpp")
        open(drv, "w").write(DRIVER)
        orc_o = os.path.join(d, "oracle.o")
        subprocess.run(["gcc", *SAN, "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-c",
                        os.path.join(ROOT, "oracle", "tartarus_oracle.c"), "-o", orc_o], check=True)
        exe = os.path.join(d, "driver")
        subprocess.run(["g++", *SAN, "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "oracle"), drv,
                        os.path.join(CSRC, "host_logic.cpp"), orc_o, "-o", exe, "-lm"], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        print(r.stdout[-2000:], r.stderr[-4000:])
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "failures: 0" in r.stdout
    finally:
        shutil.rmtree(d, ignore_errors=True)
