#!/usr/bin/env python3
"""Benchmark of the Kerr null-geodesic tracer on one MI355X.

Headline workload: Kerr a = 0.998, observer at r = 1000 M and 17 deg
inclination, a 2048 x 2048 camera over alpha, beta in [-20, 20] M, a
Novikov-Thorne disk from r_ISCO to 30 M with up to 3 recorded crossings
(synthetic camera grid, no data; 4,194,304 rays).  One "step" is one full
trace of the image (camera initial conditions, Dormand-Prince 5(4)
integration, events, shading) through the C ABI; inputs are generated on the
device, so the timed region reads nothing from the host.

The metric is rays/s at |H| <= 1e-8: before anything is timed, the image is
traced (untimed) at rtol in {1e-8, 3e-9, 1e-9, 3e-10, 1e-10} (atol = rtol /
100), and further along 7e-11, 5e-11, 3e-11, 2e-11, 1e-11 (the 1-2-3-5-7
steps of a decade) if none of those passes, in FP64 and in mixed precision, and the constraint gate (max |H| over accepted states with
r >= 1.5 r_+, every non-failed ray) is read off the outputs.  The headline value is FP64 at the loosest tolerance whose gate
holds; mixed precision is timed at that same tolerance and at its own loosest
passing tolerance (or reported with its gate fraction where none passes).
The roofline entry prices the integrator kernel's algorithmic FP64 work
(per-ray attempt counts x FLOPs per attempt) against the FP64 vector peak,
over the kernel's own launch duration (HIP events the library records on the
trace's stream).  The CPU baseline is the plain FP64 oracle on a seeded
sample of the same image's pixels, on all host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/sec at |H|≤1e-8 (FP64 vs mixed, same GPU); p50/p99 image latency"
HEADLINE = "kerr0998_2048"
HEADLINE_NAME = "kerr_a0.998_i17deg_r1000_2048x2048_disk_isco_to_30M"
GATE_RTOLS = (1e-8, 3e-9, 1e-9, 3e-10, 1e-10)
GATE_RTOLS_BEYOND = (7e-11, 5e-11, 3e-11, 2e-11, 1e-11)   # searched only when no listed tolerance passes
GATE_H = 1e-8
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
GATHER_BYTES_PER_RHS = 640
PEAK_L2_TBS = 8 * 16 * 128 * 2.4e9 / 1e12   # 39.3 TB/s, derived from the L2 organisation
PEAK_FP32_TFLOPS = 78.6     # non-packed FP32 (packed FP32 is disabled in this build)

# Algorithmic FLOPs (FMA = 2, division / sqrt / transcendental = 1) of the
# analytic-Kerr FP64 path, counted from the formulas the kernel evaluates:
FLOP_RHS = 72               # one right-hand side incl. H
FLOP_ATTEMPT = 6 * FLOP_RHS + 140 + 66 + 72 + 38 + 5 + 6   # stages, y5, error, norm, controller, events = 759
FLOP_RAY_INIT = 130         # observer metric, tetrad, first right-hand side
FLOP_EVENT = 300            # Hermite set-up + ~40 bisection iterations
FLOP_HIT = 120              # Omega, u^t, g, Page-Thorne flux

HERE = os.path.dirname(os.path.abspath(__file__))
SHAPE_KEYS = ("block_threads", "blocks_per_cu", "chunk", "refill_min", "order")
COUNTER_FILE = os.path.join(HERE, "profiles", "trace_persistent_fp64_kerr0998_2048.counters.json")


def solver_at(w: dict, rtol: float) -> dict:
    return dict(w["solver"], rtol=rtol, atol=rtol / 100.0)


def algorithmic_flops(out: dict) -> float:
    att = out["n_accept"].astype(np.float64) + out["n_reject"]
    return float(att.sum() * FLOP_ATTEMPT + len(att) * (FLOP_RAY_INIT + FLOP_EVENT)
                 + out["n_cross"].sum() * FLOP_EVENT + out["n_hits"].sum() * FLOP_HIT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def kernel_source_hash() -> str:
    """sha256 over the device sources with comments and blank lines removed;
    counters measured on other code are stale."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "paper_2609_08989_amd", "csrc", "*.h*")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            code = _COMMENT.sub("", fh.read())
        h.update("\n".join(ln.rstrip() for ln in code.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def committed_counters():
    """The headline kernel's committed rocprofv3 figures, if they were taken on
    these kernel sources; else None."""
    try:
        with open(COUNTER_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    return t if t.get("source_sha256") == kernel_source_hash() else None


def gate_stats(o: dict) -> dict:
    ok = o["cls"] != 2
    hg = o["h_gate"][ok]
    return {"h_gate_max": float(hg.max()) if hg.size else 0.0,
            "frac_le_1e-8": float(np.mean(hg <= GATE_H)) if hg.size else 1.0,
            "holds": bool(hg.size == 0 or hg.max() <= GATE_H),
            "failed_rays": int((~ok).sum())}


def attempts_histogram(att) -> dict:
    """Attempted steps per ray: quantiles and counts per power-of-two bin
    (key k counts rays with 2^k <= attempts < 2^(k+1))."""
    att = np.asarray(att, dtype=np.int64)
    q = {f"p{p}": float(np.percentile(att, p)) for p in (0, 10, 50, 90, 99, 100)}
    k = np.floor(np.log2(np.maximum(att, 1))).astype(int)
    q["log2_bins"] = {str(int(b)): int(c) for b, c in zip(*np.unique(k, return_counts=True))}
    return q


def shape(L):
    return [L.block_threads, L.blocks_per_cu, L.chunk, L.refill_min, L.order]


def time_leg(T, torch, args_tuple, out, steps, warmup, launch=None):
    """Wall time of `steps` traces (bracketed by device synchronizations), the
    median duration of one trace (HIP events on the trace's stream between
    consecutive traces), and the mean duration of the integrator launches (the
    event pair the library records around each one)."""
    for _ in range(warmup):
        T.tartarus_trace(*args_tuple, out, launch=launch)
    torch.cuda.synchronize()
    T.tartarus_kernel_time()                 # drop anything recorded before
    T.tartarus_kernel_timing(True)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(st)
    for k in range(steps):
        T.tartarus_trace(*args_tuple, out, launch=launch)
        ev[k + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tartarus_kernel_timing(False)
    kernel_total_ms, launches = T.tartarus_kernel_time()
    assert launches == steps, (launches, steps)
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return wall, kernel_total_ms / launches, float(np.median(per))


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, solver, seconds: float, label: str) -> dict:
    import oracle
    oracle.build(force=False)
    cam = w["cameras"][0]
    n_img = cam["nx"] * cam["ny"]
    m, c = oracle.make_metric(w["a"]), oracle.make_camera(cam)
    d, s = oracle.make_disk(w["disk"]), oracle.make_solver(solver)
    rng = np.random.default_rng(0)
    probe = rng.choice(n_img, 1024, replace=False)
    t = time.perf_counter()
    oracle.trace(m, c, d, s, ray_ids=probe)
    rate = 1024 / max(time.perf_counter() - t, 1e-6)
    n = int(min(n_img, max(2048, rate * seconds)))
    ids = rng.choice(n_img, n, replace=False)
    t = time.perf_counter()
    oracle.trace(m, c, d, s, ray_ids=ids)
    dt = time.perf_counter() - t
    return {"value": n / dt, "unit": "rays/s", "cores": oracle.max_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} seeded-random pixels of the {label} image (rtol={solver['rtol']:g}, "
                      f"atol={solver['atol']:g}), plain FP64 C oracle, OpenMP over pixels, {dt:.1f} s"}


class Scene:
    """One image workload on the device: its C-ABI arguments and outputs."""

    def __init__(self, T, W, name, nx=None):
        self.T, self.name = T, name
        self.w = W.WORKLOADS[name] if nx is None else W.scaled(name, nx)
        self.cams = [T.make_camera(c) for c in self.w["cameras"]]
        self.n = sum(c["nx"] * c["ny"] for c in self.w["cameras"])
        self.metric = T.make_metric(self.w["a"])
        self.disk = T.make_disk(self.w["disk"])
        self.out = T.alloc_outputs(self.n)

    def args(self, rtol=None, prec=0, **solver_kw):
        sv = dict(self.w["solver"]) if rtol is None else solver_at(self.w, rtol)
        sv.update(solver_kw)
        return (self.metric, self.cams, self.disk, self.T.make_solver(sv, prec))

    def trace(self, la, launch=None):
        import torch
        self.T.tartarus_trace(*la, self.out, launch=launch)
        torch.cuda.synchronize()
        return self.T.to_numpy(self.out)


def leg_record(T, torch, S, la, steps, warmup, launch=None, extra=None) -> dict:
    wl, km, med = time_leg(T, torch, la, S.out, steps, warmup, launch)
    o = T.to_numpy(S.out)
    att = o["n_accept"] + o["n_reject"]
    rec = {"rays": S.n, "rays_per_s": S.n * steps / wl, "median_trace_ms": med, "kernel_ms": km,
           "attempts_per_ray": float(att.mean()),
           "fp32_attempt_frac": float(o["n_fp32"].sum() / max(att.sum(), 1)),
           "gate": gate_stats(o)}
    if launch is not None:
        rec["launch"] = dict(zip(SHAPE_KEYS, shape(launch)))
    if extra:
        rec.update(extra)
    return rec


def gather_roofline(rec: dict, n_rays: int) -> dict:
    """Table bytes the tabulated integrator gathers per second: 640 B per
    right-hand side (2 x 2 nodes x 5 components x 4 doubles), six right-hand
    sides per attempt and one per ray, over the integrator's launch time.  The
    gathers are served by L2 (94 % hits in the tabulated-kernel profile); the
    peak is the L2 read bandwidth of 8 XCDs x 16 channels x 128 B per clock at
    2.4 GHz."""
    rhs = rec["attempts_per_ray"] * n_rays * 6 + n_rays
    achieved = rhs * GATHER_BYTES_PER_RHS / (rec["kernel_ms"] * 1e-3) / 1e12
    return {"bound": "l2", "achieved": achieved, "peak": PEAK_L2_TBS, "unit": "TB/s", "frac": achieved / PEAK_L2_TBS,
            "bytes_per_rhs": GATHER_BYTES_PER_RHS, "rhs_per_launch": rhs}


def gate_search(T, S, prec):
    """Untimed traces at each listed tolerance: the gate per tolerance and the
    loosest tolerance whose gate holds; when none of the listed ones does, the
    search goes on down the 1-2-3-5-7 steps from 7e-11 to 1e-11 (None if no
    tolerance passes)."""
    table, first = {}, None
    for rtol in GATE_RTOLS + GATE_RTOLS_BEYOND:
        if rtol in GATE_RTOLS_BEYOND and first is not None:
            break
        o = S.trace(S.args(rtol, prec))
        g = gate_stats(o)
        table[f"{rtol:g}"] = g
        log(f"bench: gate {S.name} {'mixed' if prec else 'fp64'} rtol {rtol:g}: max {g['h_gate_max']:.3e} "
            f"frac {g['frac_le_1e-8']:.4f}")
        if g["holds"] and first is None:
            first = rtol
    return table, first


def tabulated_scene(T, torch, W):
    """The 64-camera batch on the tabulated a = 0.7 metric (table built on the
    device from analytic Kerr) and the launch shape measured best for it."""
    w = W.WORKLOADS["tabulated07_64cams"]
    t = w["table"]
    r_min = t["r_min_over_rplus"] * (1.0 + np.sqrt(1.0 - w["a"] ** 2))
    tab = torch.zeros(5 * t["nr"] * t["nth"] * 4, dtype=torch.float64, device="cuda")
    T.tartarus_build_kerr_table(w["a"], t["nr"], t["nth"], r_min, t["r_max"], tab)
    S = Scene(T, W, "tabulated07_64cams")
    S.metric = T.make_metric(w["a"], tab, t["nr"], t["nth"], r_min, t["r_max"])
    S.table = tab                # keeps the table alive with the scene
    return S, T.make_launch(256, 2, 1, 4, T.ORDER_PIXEL)


def workload_legs(T, torch, W, steps, autotune: bool) -> dict:
    """Other image workloads at their config tolerance (rtol 1e-8): the
    Schwarzschild shadow, the paper's OSIRIS calibration scene, the paper's
    Table 1 scene (Schwarzschild with the disk at D = 100) at 512^2, 1024^2 and
    2048^2, and the 64-camera tabulated-metric batch.  Each image scene is
    autotuned first (untimed); the tabulated batch (0.7 s a launch) uses the
    shape measured best for it (256 threads, 2 blocks per CU, pixel order)."""
    legs = {}
    for name, nx in (("schwarzschild_64", None), ("osiris_1024", None), ("schwarzschild_disk_100", 512),
                     ("schwarzschild_disk_100", 1024), ("schwarzschild_disk_100", 2048)):
        S = Scene(T, W, name, nx)
        la = S.args()
        log("bench: workload", name, nx or "")
        launch = T.tartarus_autotune(*la, S.out) if autotune else None
        key = name if nx is None else f"{name}_{nx}"
        legs[key] = leg_record(T, torch, S, la, steps, 1, launch)
        del S
    S, launch = tabulated_scene(T, torch, W)
    log("bench: workload tabulated07_64cams")
    rec = leg_record(T, torch, S, S.args(), 2, 1, launch)
    rec["gather_roofline"] = gather_roofline(rec, S.n)
    legs["tabulated07_64cams"] = rec
    return legs


def method_legs(T, torch, W, steps, gate_rtol_c2) -> dict:
    """The 512^2 a = 0.9 image (the Kerr scene with the disk at 60 deg): DP45 at
    its gate tolerance, the other 5(4) pairs, Gragg-Bulirsch-Stoer and Verlet."""
    legs = {}
    S = Scene(T, W, "kerr09_512")
    la = S.args(gate_rtol_c2)
    launch = T.tartarus_autotune(*la, S.out)
    legs["kerr09_512_fp64_gate"] = leg_record(T, torch, S, la, steps, 2, launch, {"rtol": gate_rtol_c2})
    for prec in (0, 1):
        legs[f"kerr09_512_{'mixed' if prec else 'fp64'}_rtol1e-8"] = leg_record(T, torch, S, S.args(1e-8, prec),
                                                                                 steps, 2)
    for mname, mcode in (("ck45", T.METHOD_CK45), ("rkf45", T.METHOD_RKF45)):
        log("bench: leg", mname)
        legs[f"kerr09_512_{mname}_rtol1e-8"] = leg_record(T, torch, S, S.args(1e-8, 0, method=mcode), steps, 2)
    for mname, rtol in (("gbs_rtol1e-8", 1e-8), ("gbs_at_dp45_gate_rtol", gate_rtol_c2), ("gbs_rtol1e-12", 1e-12),
                        ("fp64_rtol1e-12", 1e-12)):
        log("bench: leg", mname)
        kw = {"method": T.METHOD_GBS} if mname.startswith("gbs") else {}
        legs[f"kerr09_512_{mname}"] = leg_record(T, torch, S, S.args(rtol, 0, **kw), steps, 2)
    # fixed-step Verlet (Sec. 3.2): h = 0.01 on a 256^2 image of the same scene,
    # stop at 1.05 r_+ (where its implicit stages still converge), two launches
    V = Scene(T, W, "kerr09_512", 256)
    sv = dict(method=T.METHOD_VERLET, h0_frac=0.01 / V.w["cameras"][0]["r_obs"], horizon_factor=1.05)
    log("bench: leg verlet_h0.01_256")
    rec = leg_record(T, torch, V, V.args(None, 0, **sv), 2, 1)
    o = T.to_numpy(V.out)
    rec["steps_per_s"] = float(o["n_accept"].sum()) * 2 / (V.n * 2 / rec["rays_per_s"])
    legs["kerr09_512_verlet_h0.01_256"] = rec
    return legs


def serving_leg(T, torch, W, n_requests: int, rtol: float, loads=(0.5, 0.8, 0.95), budget_gib: int = 8,
                arrival_order_load: float = 0.8) -> dict:
    """Poisson streams of image requests (resolution uniform over 64^2..1024^2,
    spin, inclination, disk size drawn per request) submitted at their arrival
    times through tartarus_submit under an HBM budget that makes admission
    bind; latency = done - submit per request.  One session per precision
    (FP64, mixed), both at the given tolerance.  The offered load is a fraction
    of the session's own throughput, measured on a burst of 48 requests from
    the same distribution (another seed) after a warm-up burst, beside the rate
    of the same requests traced one by one; stream k uses seed k.  The queue
    hands out the smallest admitted request's rays first; one more FP64 stream,
    at arrival_order_load with the seed of that load, runs with arrival order
    for comparison."""
    sv_at = lambda r: dict(r["solver"], rtol=rtol, atol=rtol / 100.0)
    mean_rays = float(np.mean([r * r for r in W.RESOLUTIONS]))
    result = {"requests_per_load": n_requests, "rtol": rtol, "atol": rtol / 100.0, "hbm_budget_gib": budget_gib,
              "note": "latency = completion - submission; first 10 requests of each stream are warm-up; "
                      "load = fraction of the session's burst capacity; smallest request first unless noted"}
    for prec in (T.PREC_FP64, T.PREC_MIXED):
        pname = "mixed" if prec else "fp64"
        mk = lambda r: (T.make_metric(r["a"]), T.make_camera(r["camera"]), T.make_disk(r["disk"]),
                        T.make_solver(sv_at(r), prec))
        T.tartarus_shutdown()
        T.tartarus_init(0, budget_gib << 30)
        burst = W.request_stream(1000, 48, 1e9)
        bouts = [T.alloc_outputs(r["camera"]["nx"] * r["camera"]["ny"]) for r in burst]
        burst_rays = sum(r["camera"]["nx"] * r["camera"]["ny"] for r in burst)
        # the same requests traced one by one (context for the session's rate)
        for r, o in zip(burst[:4], bouts):
            T.tartarus_trace(*mk(r), o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r, o in zip(burst, bouts):
            T.tartarus_trace(*mk(r), o)
        torch.cuda.synchronize()
        one_shot = burst_rays / (time.perf_counter() - t0)
        # a warm-up burst starts the scheduler and fills the record pool; the
        # session's capacity is then timed on the burst
        warm = W.request_stream(999, 16, 1e9)
        wouts = [T.alloc_outputs(r["camera"]["nx"] * r["camera"]["ny"]) for r in warm]
        for t in [T.tartarus_submit(*mk(r), o) for r, o in zip(warm, wouts)]:
            T.tartarus_wait(t, 120000)
        del wouts
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in [T.tartarus_submit(*mk(r), o) for r, o in zip(burst, bouts)]:
            T.tartarus_wait(t, 120000)
        capacity = burst_rays / (time.perf_counter() - t0)
        del bouts
        runs = []
        plan = [(seed, load, T.SERVE_SMALLEST_FIRST) for seed, load in enumerate(loads)]
        if prec == T.PREC_FP64 and arrival_order_load in loads:
            plan.append((loads.index(arrival_order_load), arrival_order_load, T.SERVE_ARRIVAL))
        for seed, load, policy in plan:
            T.tartarus_serving_order(policy)
            rate = load * capacity / mean_rays
            reqs = W.request_stream(seed, n_requests, rate)
            outs = [T.alloc_outputs(r["camera"]["nx"] * r["camera"]["ny"]) for r in reqs]
            torch.cuda.synchronize()
            log("bench: serving", pname, "load", load, "requests", n_requests, "order", policy)
            tickets = []
            t0 = time.perf_counter()
            for r, o in zip(reqs, outs):
                delay = r["arrival_s"] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                tickets.append(T.tartarus_submit(*mk(r), o))
            for t in tickets:
                T.tartarus_wait(t, 120000)
            stamps = np.array([T.tartarus_ticket_times(t) for t in tickets], dtype=np.float64)
            lat_ms = (stamps[:, 2] - stamps[:, 0]) * 1e-6
            warm = 10 if len(lat_ms) > 20 else 0
            rays = sum(r["camera"]["nx"] * r["camera"]["ny"] for r in reqs)
            span = (stamps[:, 2].max() - stamps[:, 0].min()) * 1e-9
            cls = [T.to_numpy({"cls": o["cls"], "h_gate": o["h_gate"]}) for o in outs]
            failed = int(sum(int((c["cls"] == 2).sum()) for c in cls))
            hg = np.concatenate([c["h_gate"][c["cls"] != 2] for c in cls])
            runs.append({"load": load, "seed": seed, "requests": len(reqs), "arrival_rate_per_s": rate,
                         "order": "smallest_first" if policy == T.SERVE_SMALLEST_FIRST else "arrival",
                         "p50_latency_ms": float(np.percentile(lat_ms[warm:], 50)),
                         "p99_latency_ms": float(np.percentile(lat_ms[warm:], 99)),
                         "max_latency_ms": float(lat_ms[warm:].max()), "rays_per_s": rays / span,
                         "failed_rays": failed, "gate_frac_le_1e-8": float(np.mean(hg <= GATE_H)),
                         "gate_h_max": float(hg.max())})
            del outs
        result[pname] = {"capacity_rays_per_s": capacity, "one_shot_rays_per_s": one_shot, "by_load": runs}
    T.tartarus_shutdown()
    T.tartarus_init(0, 0)
    T.tartarus_serving_order(T.SERVE_SMALLEST_FIRST)
    ref = min((x for x in result["fp64"]["by_load"] if x["order"] == "smallest_first"),
              key=lambda x: abs(x["load"] - 0.8))
    result.update({"p50_latency_ms": ref["p50_latency_ms"], "p99_latency_ms": ref["p99_latency_ms"],
                   "load": ref["load"], "precision": "fp64"})
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="time only the headline and mixed legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true", help="use the default launch shape")
    ap.add_argument("--launch", default="", help="force the launch shape block,blocks_per_cu,chunk,refill_min[,order]")
    ap.add_argument("--rtol", type=float, default=0.0, help="skip the gate search and use this rtol")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="with --only-headline: the precision of the traced headline")
    ap.add_argument("--only-headline", action="store_true",
                    help="trace the headline image only (for profilers): no search, no legs")
    ap.add_argument("--only-tabulated", action="store_true",
                    help="trace the 64-camera tabulated batch only (for profilers)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-latency leg")
    ap.add_argument("--only-serving", action="store_true",
                    help="run the serving-latency leg only (for profilers), at --rtol or the headline's gate 7e-11")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one device copy of this many MiB (calibrates FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(on several GPUs the tracer would shard by pixel rows or by requests)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2609_08989_amd import tartarus as T

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nb}))
        return

    T.tartarus_init(0, 0)
    if args.only_serving:
        rec = serving_leg(T, torch, W, n_requests=args.serving_requests, rtol=args.rtol or 7e-11)
        print(json.dumps({"only_serving": rec}))
        return
    if args.only_tabulated:
        S, launch = tabulated_scene(T, torch, W)
        rec = leg_record(T, torch, S, S.args(), args.steps, args.warmup, launch)
        print(json.dumps({"only_tabulated": rec}))
        return
    S = Scene(T, W, HEADLINE)
    forced = T.make_launch(*[int(v) for v in args.launch.split(",")]) if args.launch else None

    if args.only_headline:
        prec = T.PREC_MIXED if args.precision == "mixed" else T.PREC_FP64
        la = S.args(args.rtol or 3e-10, prec)
        log("bench: headline only", args.precision, args.rtol or 3e-10, args.launch)
        rec = leg_record(T, torch, S, la, args.steps, args.warmup, forced)
        print(json.dumps({"only_headline": rec}))
        return

    # ---- the gate: loosest listed tolerance whose |H| <= 1e-8 gate holds
    if args.rtol:
        gates, gate_rtol = {}, args.rtol
        gates_mixed, gate_rtol_mixed = {}, None
    else:
        gates, gate_rtol = gate_search(T, S, T.PREC_FP64)
        gates_mixed, gate_rtol_mixed = gate_search(T, S, T.PREC_MIXED)
        if gate_rtol is None:
            gate_rtol = GATE_RTOLS[-1]
    la = S.args(gate_rtol, T.PREC_FP64)
    tuned = {}
    launch = forced
    if launch is None and not args.no_autotune:
        log("bench: autotune fp64")
        launch = T.tartarus_autotune(*la, S.out)     # untimed: part of the warm-up
    if launch is not None:
        tuned["fp64"] = shape(launch)
    log("bench: headline leg (fp64, rtol %g)" % gate_rtol, tuned)
    wall, kern_ms, med_ms = time_leg(T, torch, la, S.out, args.steps, args.warmup, launch)
    o = T.to_numpy(S.out)
    n = S.n
    value = n * args.steps / wall
    flops = algorithmic_flops(o)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    att = o["n_accept"] + o["n_reject"]
    g = gate_stats(o)
    cnt = committed_counters()
    executed, traffic, occupancy = None, None, None
    if cnt is not None:
        ex = float(cnt["executed_fp64_flop"])
        executed = {"flop_per_launch": ex, "achieved": ex / (kern_ms * 1e-3) / 1e12,
                    "frac": ex / (kern_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                    "note": "FP64 VALU instructions x 64 lanes x lane efficiency from the committed counters "
                            "(FMA = 2), over this run's kernel time"}
        traffic = float(cnt["fetch_bytes"] + cnt["write_bytes"])
        occupancy = {"mean_resident_waves_per_simd": cnt.get("mean_resident_waves_per_simd"),
                     "max_waves_per_simd": cnt.get("max_waves_per_simd"), "vgprs": cnt.get("vgprs"),
                     "counter_launch_shape": cnt.get("launch"), "counter_rtol": cnt.get("rtol")}
    if launch is not None:
        sh = dict(zip(SHAPE_KEYS, shape(launch)))
        occupancy = dict(occupancy or {}, launched_waves_per_simd=sh["block_threads"] // 64 * sh["blocks_per_cu"] / 4.0)
    result = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": HEADLINE_NAME, "rays": n, "rtol": gate_rtol, "atol": gate_rtol / 100.0,
                   "precision": "fp64", "median_trace_ms": med_ms,
                   "gate": g, "gate_by_rtol_fp64": gates, "gate_by_rtol_mixed": gates_mixed,
                   "gate_rtol_fp64": gate_rtol, "gate_rtol_mixed": gate_rtol_mixed,
                   "attempts_per_ray": float(att.mean()), "attempts_histogram": attempts_histogram(att)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "trace_persistent<0,0,0> (analytic Kerr, FP64, Dormand-Prince)",
                     "kernel_ms": kern_ms, "flop_per_launch": flops, "flop_per_attempt": FLOP_ATTEMPT,
                     "executed": executed, "occupancy": occupancy},
    }

    # ---- mixed precision on the same image: at FP64's gate tolerance, at its own
    legs = {}
    mixed_launch = None
    la_m = S.args(gate_rtol, T.PREC_MIXED)
    if forced is None and not args.no_autotune:
        log("bench: autotune mixed")
        mixed_launch = T.tartarus_autotune(*la_m, S.out)
        tuned["mixed"] = shape(mixed_launch)
    legs["mixed_at_fp64_gate_rtol"] = leg_record(T, torch, S, la_m, args.steps, args.warmup, mixed_launch or forced,
                                                 {"rtol": gate_rtol})
    if gate_rtol_mixed is not None and gate_rtol_mixed != gate_rtol:
        legs["mixed_at_own_gate_rtol"] = leg_record(T, torch, S, S.args(gate_rtol_mixed, T.PREC_MIXED), args.steps,
                                                    args.warmup, mixed_launch or forced, {"rtol": gate_rtol_mixed})
    for rtol in (1e-8,):
        for prec in (T.PREC_FP64, T.PREC_MIXED):
            log("bench: leg rtol", rtol, "mixed" if prec else "fp64")
            legs[f"{'mixed' if prec else 'fp64'}_rtol{rtol:g}"] = leg_record(
                T, torch, S, S.args(rtol, prec), args.steps, args.warmup,
                (mixed_launch if prec else launch) or forced, {"rtol": rtol})
    legs["mixed_over_fp64_at_fp64_gate_rtol"] = legs["mixed_at_fp64_gate_rtol"]["rays_per_s"] / value
    legs["mixed_over_fp64_rtol1e-8"] = legs["mixed_rtol1e-08"]["rays_per_s"] / legs["fp64_rtol1e-08"]["rays_per_s"]
    del S
    torch.cuda.empty_cache()

    if not args.no_extra:
        legs.update(method_legs(T, torch, W, args.steps, 3e-10))
        legs.update(workload_legs(T, torch, W, 3, autotune=not args.no_autotune))
    result["legs"] = legs

    if not args.no_serving:
        log("bench: serving leg")
        result["serving"] = serving_leg(T, torch, W, n_requests=args.serving_requests, rtol=gate_rtol)
    if tuned:
        result["launch_shape"] = {k: dict(zip(SHAPE_KEYS, v)) for k, v in tuned.items()}
    if not args.no_cpu:
        log("bench: cpu baseline")
        result["cpu_baseline"] = cpu_baseline(W.WORKLOADS[HEADLINE], solver_at(W.WORKLOADS[HEADLINE], gate_rtol),
                                              args.cpu_seconds, "2048x2048 a = 0.998")
    print(json.dumps(result))


if __name__ == "__main__":
    main()
